// Alpha-beta units with all four orbitals virtual (the vv|vv ladder of the
// alpha-beta class; two electrons per spin) as a block-sparse product on
// FP64 matrix cores.
//
// For spectators x (alpha) and y (beta) and virtual q, s
//   T[(q, s)][(x, y, v)] = sgn(q - x) sgn(s - y) c_v({x, q}, {y, s})
// (zero when {x,q} or {y,s} is not a string, or the determinant lies above
// the excitation cut).  The vv|vv part of the alpha-beta class is
//   S[(p, r)][(x, y, v)] = sum_{q,s virtual} (pq|rs) T[(q, s)][(x, y, v)]
// combined over the four spectator roles of a target determinant
// (T'[x][p][y][r] = S[x][p][y][r] - S[p][x][y][r] - S[x][p][r][y]
// + S[p][x][r][y], S indexed [alpha spectator][alpha active][beta
// spectator][beta active]).  The unfold kernel writes T once per
// call (columns: spectator block pair, slots, four vectors), so the
// product reads contiguous 16-column operand rows instead of scattered CI
// elements, and the four vectors of a pass share every integral chunk.
// The product writes S for every virtual row block pair and column (a
// balanced block-sparse GEMM), then a fold adds the four role readings of
// each target determinant into sigma.
//
// Rows (q, s) of T: (q - 2) * ks + (s - 2), s padded to whole blocks of
// four (padding rows are zero).  Column groups: spectator block pair (C, D)
// with (C virtual) + (D virtual) <= L - 2; the occupied block has two
// slots, a virtual block four; a group has slots(C) * slots(D) * 4 columns.
// Zero columns pad the total to a multiple of 64 (one wave's slab).
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

// S = W T for one virtual row block pair (P, R) (16 rows (p, r)) and 256
// columns (blockIdx.y): wave w takes four 16-column N tiles; K runs over the
// vv|vv chunks of the row block.  S rows are (p - 2) * ks + (r - 2) like T's.
__global__ __launch_bounds__(256) void k_vv_gemm(SigmaArgs A)
{
    const int nb = A.nblk, ncol = A.vv_ncol, ks = A.vv_ks;
    const int P = 1 + blockIdx.x / (nb - 1), R = 1 + blockIdx.x % (nb - 1);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int c0 = blockIdx.y * 256 + wave * 64;
    if (c0 >= ncol) return;
    const int row = P * nb + R;
    const int e0 = A.chunk_off[row] + A.chunk_cls[row * 3] + A.chunk_cls[row * 3 + 1];
    const int e1 = A.chunk_off[row + 1];
    const int k = lane >> 4, n = lane & 15;
    const double *Tb = A.vv_T + (size_t)k * ncol + c0 + n;
    v4d_vv acc[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t] = v4d_vv{0.0, 0.0, 0.0, 0.0};
    // two stages of two chunks each, ping-ponged so that the loads of one
    // stage are in flight while the MFMAs of the other issue (no register
    // copies, which would wait for the loads)
    double ax[2], bx[2][4], ay[2], by[2][4];
    // loads are unconditional (clamped chunk index, zero selected past the
    // end), so waiting for one stage never waits for the other
    auto load2 = [&](int e, double *a, double (*b)[4]) {
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int eu = min(e + u, e1 - 1);
            const double *src = Tb + (size_t)A.vv_trow[eu] * ncol;
            const double av = A.chunk_val[(size_t)eu * 64 + lane];
            a[u] = e + u < e1 ? av : 0.0;
#pragma unroll
            for (int t = 0; t < 4; ++t) b[u][t] = src[16 * t];
        }
    };
    auto mma2 = [&](const double *a, const double (*b)[4]) {
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
            for (int t = 0; t < 4; ++t) acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u], b[u][t], acc[t], 0, 0, 0);
    };
    if (e0 < e1) load2(e0, ax, bx);
    for (int e = e0; e < e1; e += 4) {
        load2(e + 2, ay, by);
        mma2(ax, bx);
        load2(e + 4, ax, bx);
        mma2(ay, by);
    }
    // element g of lane l is row 4 g + l / 16 = (p slot g, r slot l / 16), column l % 16
    double *Sb = A.vv_S + ((size_t)(4 * (P - 1)) * ks + 4 * (R - 1) + k) * ncol + c0 + n;
#pragma unroll
    for (int g = 0; g < 4; ++g)
#pragma unroll
        for (int t = 0; t < 4; ++t) Sb[(size_t)g * ks * ncol + 16 * t] = acc[t][g];
}

// sigma({a < b}, {c < d}) += the vv|vv part, from S: every way of reading
// the target as (alpha spectator, alpha active virtual) x (beta spectator,
// beta active virtual) with the spectator pair in a column group,
// sign + for (a, b) / (c, d) spectator-first, - per swapped spin.
__global__ __launch_bounds__(256) void k_vv_fold(SigmaArgs A, int nv, double *__restrict__ sg, int64_t lds)
{
    const int ia = blockIdx.x;
    const int jb = blockIdx.y * 256 + threadIdx.x;
    const int L = A.L;
    const int len = A.sb.le[L - A.alev[ia]];
    if (jb >= len) return;
    const int norb = A.norb, nb = A.nblk, ncol = A.vv_ncol, ks = A.vv_ks;
    const uint32_t as = A.astr[ia], bs = A.bstr[jb];
    const int a0 = as & 0xff, a1 = (as >> 8) & 0xff, b0 = bs & 0xff, b1 = (bs >> 8) & 0xff;
    if (a1 < 2 || b1 < 2) return;   // no virtual active orbital on one spin
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    bool any = false;
#pragma unroll
    for (int ra = 0; ra < 2; ++ra) {
        const int xs = ra ? a1 : a0, xa = ra ? a0 : a1;   // alpha spectator, active
        if (xa < 2) continue;
        const int C = xs < 2 ? 0 : 1 + (xs - 2) / 4, ic = xs < 2 ? xs : (xs - 2) % 4;
#pragma unroll
        for (int rb = 0; rb < 2; ++rb) {
            const int ys = rb ? b1 : b0, ya = rb ? b0 : b1;
            if (ya < 2) continue;
            const int D = ys < 2 ? 0 : 1 + (ys - 2) / 4, id = ys < 2 ? ys : (ys - 2) % 4;
            const int g = A.vv_gofs[C * nb + D];
            if (g < 0) continue;
            const int wD = D == 0 ? 2 : 4;
            const double *src = A.vv_S + (size_t)((xa - 2) * ks + (ya - 2)) * ncol + g + (ic * wD + id) * 4;
            const double f = (ra ^ rb) ? -1.0 : 1.0;
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[v] += f * src[v];
            any = true;
        }
    }
    if (!any) return;
    double *dst = sg + A.rowstart[ia] + jb;
#pragma unroll
    for (int v = 0; v < 4; ++v)
        if (v < nv) dst[(int64_t)v * lds] += acc[v];
}

isci_status launch_ab_vv(const isci_ctx *cx, int nv, const double *c, int64_t ldc, double *s, int64_t lds,
                         hipStream_t st)
{
    if (!cx->have_vv) return ISCI_OK;
    const SigmaArgs A = sigma_args(cx);
    const int nb = cx->nblk;
    k_vv_unfold<<<dim3((unsigned)((cx->vv_ncol + 255) / 256), (unsigned)cx->vv_krows), 256, 0, st>>>(A, nv, c, ldc);
    k_vv_gemm<<<dim3((unsigned)((nb - 1) * (nb - 1)), (unsigned)((cx->vv_ncol + 255) / 256)), 256, 0, st>>>(A);
    k_vv_fold<<<dim3((unsigned)cx->sa.nstr, (unsigned)((cx->max_rowlen + 255) / 256)), 256, 0, st>>>(A, nv, s, lds);
    ISCI_HIP(hipGetLastError());
    return ISCI_OK;
}

}  // namespace isci
