// Alpha-beta units with all four orbitals virtual (the vv|vv ladder of the
// alpha-beta class; two electrons per spin) as a block-sparse product on
// FP64 matrix cores.
//
// For spectators x (alpha) and y (beta) and virtual q, s
//   T[(q, s)][(x, y, v)] = sgn(q - x) sgn(s - y) c_v({x, q}, {y, s})
// (zero when {x,q} or {y,s} is not a string, or the determinant lies above
// the excitation cut).  The vv|vv part of the alpha-beta class is
//   S[(p, r)][(x, y, v)] = sum_{q,s virtual} (pq|rs) T[(q, s)][(x, y, v)]
// combined over the four spectator roles of a target determinant exactly
// as in the gathered kernel (T'[x][p][y][r] = S[x][p][y][r] - S[p][x][y][r]
// - S[x][p][r][y] + S[p][x][r][y]).  The unfold kernel writes T once per
// call (columns: spectator block pair, slots, four vectors), so the
// product reads contiguous 16-column operand rows instead of scattered CI
// elements, and the four vectors of a pass share every integral chunk.
//
// Rows (q, s) of T: (q - 2) * ks + (s - 2), s padded to whole blocks of
// four (padding rows are zero).  Column groups: spectator block pair (C, D)
// with (C virtual) + (D virtual) <= L - 2; the occupied block has two
// slots, a virtual block four; a group has slots(C) * slots(D) * 4 columns.
#include <hip/hip_runtime.h>

#include "isci_device.h"
#include "isci_internal.h"

namespace isci {

typedef double v4d_vv __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void k_vv_unfold(SigmaArgs A, int nv, const double *__restrict__ c, int64_t ldc)
{
    const int col = blockIdx.x * 256 + threadIdx.x;
    if (col >= A.vv_ncol) return;
    const int kq = blockIdx.y;
    const int norb = A.norb;
    const int q = 2 + kq / A.vv_ks, s = 2 + kq % A.vv_ks;
    const int d = A.vv_col[col];
    const int x = d & 0xff, y = (d >> 8) & 0xff, v = d >> 16;
    double val = 0.0;
    if (s < norb && x != 255 && y != 255 && x != q && y != s && v < nv) {
        const long long base = A.arow_base[x * norb + q];
        const int len = A.arow_len[x * norb + q];
        const int jb = A.bpidx[y * norb + s];
        if (base >= 0 && jb >= 0 && jb < len) {
            const double cv = c[(int64_t)v * ldc + base + jb];
            val = ((q > x) == (s > y)) ? cv : -cv;
        }
    }
    A.vv_T[(size_t)kq * A.vv_ncol + col] = val;
}

__device__ __forceinline__ int vv_orbital(int B, int i, int norb)
{
    if (B == 0) return i < 2 ? i : -1;
    const int o = 2 + 4 * (B - 1) + i;
    return o < norb ? o : -1;
}

__device__ __forceinline__ int vv_slots(int B) { return B == 0 ? 2 : 4; }

// One workgroup per target tile (X, P, Y, R), P and R virtual blocks; wave
// w computes spectator role w: rows = the 16 active pairs of its row block,
// columns = its spectator group (1, 2 or 4 N tiles), K = the vv|vv chunks
// of the row block (4 columns (q, s) each).  Roles are combined in LDS.
__global__ __launch_bounds__(256) void k_ab_vv(SigmaArgs A, int nv, double *__restrict__ sg, int64_t lds)
{
    __shared__ double tile[4][16][65];
    const uchar4 qd = A.vv_quads[blockIdx.x];
    const int X = qd.x, P = qd.y, Y = qd.z, R = qd.w;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const bool sameA = X == P, sameB = Y == R;
    const int norb = A.norb, nb = A.nblk, ncol = A.vv_ncol;
    int Ab, Bb, Cb, Db;
    bool active;
    if (wave == 0) { Ab = P; Bb = R; Cb = X; Db = Y; active = true; }
    else if (wave == 1) { Ab = X; Bb = R; Cb = P; Db = Y; active = !sameA; }
    else if (wave == 2) { Ab = P; Bb = Y; Cb = X; Db = R; active = !sameB; }
    else { Ab = X; Bb = Y; Cb = P; Db = R; active = !sameA && !sameB; }
    active = active && Ab != 0 && Bb != 0;
    const int g0 = A.vv_gofs[Cb * nb + Db];
    active = active && g0 >= 0;
    const int ntile = vv_slots(Cb) * vv_slots(Db) / 4;   // 16-column tiles of the group
    v4d_vv acc[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t] = v4d_vv{0.0, 0.0, 0.0, 0.0};
    if (active) {
        const int row = Ab * nb + Bb;
        const int e0 = A.chunk_off[row] + A.chunk_cls[row * 3] + A.chunk_cls[row * 3 + 1];
        const int e1 = A.chunk_off[row + 1];
        const int k = lane >> 4, n = lane & 15;
        const double *Tb = A.vv_T + g0 + n;
        auto krow = [&](int e) {
            const int2 dsc = A.chunk_desc[e];
            return (size_t)((dsc.x - 2) * A.vv_ks + 4 * (dsc.y - 1) + k) * ncol;
        };
        double a_c = 0.0, b_c[4] = {0.0, 0.0, 0.0, 0.0};
        if (e0 < e1) {
            const size_t r0 = krow(e0);
            a_c = A.chunk_val[(size_t)e0 * 64 + lane];
#pragma unroll
            for (int t = 0; t < 4; ++t)
                if (t < ntile) b_c[t] = Tb[r0 + 16 * t];
        }
        for (int e = e0; e < e1; ++e) {
            double a_n = 0.0, b_n[4] = {0.0, 0.0, 0.0, 0.0};
            if (e + 1 < e1) {
                const size_t r1 = krow(e + 1);
                a_n = A.chunk_val[(size_t)(e + 1) * 64 + lane];
#pragma unroll
                for (int t = 0; t < 4; ++t)
                    if (t < ntile) b_n[t] = Tb[r1 + 16 * t];
            }
#pragma unroll
            for (int t = 0; t < 4; ++t)
                if (t < ntile) acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a_c, b_c[t], acc[t], 0, 0, 0);
            a_c = a_n;
#pragma unroll
            for (int t = 0; t < 4; ++t) b_c[t] = b_n[t];
        }
    }
    // 16x16x4 f64 result: element g of lane l is D[4 g + l / 16][l % 16]
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int g = 0; g < 4; ++g) tile[wave][4 * g + (lane >> 4)][16 * t + (lane & 15)] = acc[t][g];
    __syncthreads();
    // combine the roles: target slots (ix, ip, iy, ir) and vector v
    const int t1 = sameA ? 0 : 1, t2 = sameB ? 0 : 2;
    const int t3 = (sameA && sameB) ? 0 : sameA ? 2 : sameB ? 1 : 3;
    const int wX = vv_slots(X), wP = vv_slots(P), wY = vv_slots(Y), wR = vv_slots(R);
    for (int t = threadIdx.x; t < 1024; t += 256) {
        const int v = t & 3, ir = (t >> 2) & 3, iy = (t >> 4) & 3, ip = (t >> 6) & 3, ix = t >> 8;
        if (v >= nv || ix >= wX || ip >= wP || iy >= wY || ir >= wR) continue;
        const int x = vv_orbital(X, ix, norb), p = vv_orbital(P, ip, norb);
        const int y = vv_orbital(Y, iy, norb), r = vv_orbital(R, ir, norb);
        if (x < 0 || p < 0 || y < 0 || r < 0 || x >= p || y >= r) continue;
        const long long tb = A.arow_base[x * norb + p];
        const int tl = A.arow_len[x * norb + p];
        const int jb = A.bpidx[y * norb + r];
        if (tb < 0 || jb < 0 || jb >= tl) continue;
        // row = (alpha active slot) * 4 + beta active slot; column =
        // ((alpha spectator slot) * slots(beta spectator block) + beta spectator slot) * 4 + v
        const double s0 = tile[0][ip * 4 + ir][(ix * wY + iy) * 4 + v];
        const double s1 = tile[t1][ix * 4 + ir][(ip * wY + iy) * 4 + v];
        const double s2 = tile[t2][ip * 4 + iy][(ix * wR + ir) * 4 + v];
        const double s3 = tile[t3][ix * 4 + iy][(ip * wR + ir) * 4 + v];
        sg[(int64_t)v * lds + tb + jb] += s0 - s1 - s2 + s3;
    }
}

isci_status launch_ab_vv(const isci_ctx *cx, int nv, const double *c, int64_t ldc, double *s, int64_t lds,
                         hipStream_t st)
{
    if (!cx->have_vv || cx->nvvquad == 0) return ISCI_OK;
    const SigmaArgs A = sigma_args(cx);
    k_vv_unfold<<<dim3((unsigned)((cx->vv_ncol + 255) / 256), (unsigned)cx->vv_krows), 256, 0, st>>>(A, nv, c, ldc);
    k_ab_vv<<<(unsigned)cx->nvvquad, 256, 0, st>>>(A, nv, s, lds);
    ISCI_HIP(hipGetLastError());
    return ISCI_OK;
}

}  // namespace isci
