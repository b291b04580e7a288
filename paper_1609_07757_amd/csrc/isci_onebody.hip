// One-body sigma classes for two electrons per spin on FP64 matrix cores.
//
// With two electrons of a spin, the part of the CI vector that belongs to
// one string of the other spin is an antisymmetric orbital matrix
//   T[k][d] = c({k, d}) for k < d,  -c({k, d}) for k > d,  0 on the diagonal,
// zero where {k, d} lies above the excitation cut.  The one-body operator
// sum_pq h_pq E_pq maps T to T' = h T + T h (h symmetric), and
//   sigma({a < b}) += T'[a][b] = U[a][b] - U[b][a],   U = h T.
// U is a dense product (K = norb) that runs on v_mfma_f64_16x16x4; the
// screened units |h_pq| <= tau are zeros of h, so the product adds exactly
// the kept terms (the diagonal units h_pp included).
//
// The cut splits both classes by the level of the other spin's string:
//  * beta class, alpha rows whose beta strings reach level 2: T of the row
//    is built in LDS and U = h T is formed whole;
//  * beta class, rows whose beta strings stop at level 1: only the columns
//    U[:, o] of the two occupied orbitals o are needed (a product over many
//    rows at once), plus two units per target taken directly;
//  * alpha class, beta columns where every alpha pair exists: a workgroup
//    holds the pair values of a few columns in LDS and forms the whole U of
//    each column;
//  * alpha class, columns where only the pairs {0,1}, {o, v} exist: U[:, o]
//    for the two occupied o over 64 columns at once (rows staged in LDS),
//    plus the two-term U[o][v];
//  * alpha class, columns where only {0,1} exists: (h_00 + h_11) c.
// Every sigma element is written by one workgroup of one launch.
//
// Everything adds into sigma.  16x16x4 f64 operand layouts: lane l holds
// A[l % 16][l / 16] and B[l / 16][l % 16]; result element g of lane l is
// D[4 g + l / 16][l % 16].
#include <hip/hip_runtime.h>

#include "isci_device.h"
#include "isci_internal.h"

namespace isci {

typedef double v4d_ob __attribute__((ext_vector_type(4)));

__device__ __forceinline__ v4d_ob mfma16(double a, double b, v4d_ob c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// A operand column of the screened h (symmetric, canonical) for all K
// steps: ah[ks] = h[a][q] with q = 4 ks + kq, from the zero-padded copy
// hp (kObMaxNorb x kObMaxNorb), so the loads carry no conditions and are
// issued together.
template <int NK>
__device__ __forceinline__ void load_hcol(const double *__restrict__ hp, int a, int kq, double *ah)
{
#pragma unroll
    for (int ks = 0; ks < NK; ++ks) ah[ks] = hp[(4 * ks + kq) * kObMaxNorb + a];
}

// global loads per thread issued together in the staging loops below
constexpr int kObBatch = 8;

// start of the row of alpha string ia, from the level structure alone (no
// table load): rows run level by level in string order, a row of level l
// holding the beta strings of level <= L - l; two electrons: levels <= 2
__device__ __forceinline__ int64_t row_start_n2(const SigmaArgs &A, int ia)
{
    int64_t r = 0;
#pragma unroll
    for (int l = 0; l <= 2; ++l) {
        const int lo = A.sa.lev_off[l], hi = A.sa.lev_off[l + 1];
        const int64_t len = A.sb.le[max(A.L - l, 0)];
        if (ia < hi) return r + (int64_t)(ia - lo) * len;
        r += (int64_t)(hi - lo) * len;
    }
    return r;
}

// Beta class on alpha rows [row0, row0 + gridDim.x) whose beta strings reach
// level 2; one workgroup per (row, vector), NT waves, one M tile per wave.
template <int NT>
__global__ __launch_bounds__(64 * NT) void k_ob_beta_full(SigmaArgs A, const double *__restrict__ c, int64_t ldc,
                                                          double *__restrict__ sg, int64_t lds,
                                                          const double *__restrict__ hs, const double *__restrict__ hp, int row0,
                                                          int ovw)
{
    constexpr int NP = 16 * NT, SP = NP + 1, NK = NP / 4, NTH = 64 * NT;   // odd row stride: no bank conflicts
    __shared__ double T[NP * SP];
    const int ia = row0 + blockIdx.x;
    const int v = blockIdx.y;
    const int norb = A.norb;
    const int len = A.sb.le[A.L - A.alev[ia]];
    const double *cr = c + (int64_t)v * ldc + A.rowstart[ia];
    double *sr = sg + (int64_t)v * lds + A.rowstart[ia];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int am = 16 * w + (lane & 15), kq = lane >> 4;
    double ah[NK];
    load_hcol<NK>(hp, am, kq, ah);
    for (int t = threadIdx.x; t < NP * SP; t += NTH) T[t] = 0.0;
    __syncthreads();
    for (int jb = threadIdx.x; jb < len; jb += kObBatch * NTH) {
        uint32_t bs[kObBatch];
        double val[kObBatch];
#pragma unroll
        for (int u = 0; u < kObBatch; ++u) {
            const int j = min(jb + u * NTH, len - 1);
            bs[u] = A.bstr[j];
            val[u] = cr[j];
        }
#pragma unroll
        for (int u = 0; u < kObBatch; ++u)
            if (jb + u * NTH < len) {
                const int y = bs[u] & 0xff, s = (bs[u] >> 8) & 0xff;
                T[y * SP + s] = val[u];
                T[s * SP + y] = -val[u];
            }
    }
    __syncthreads();
    v4d_ob acc[NT];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) acc[nt] = v4d_ob{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int ks = 0; ks < NK; ++ks) {
        const int k = 4 * ks + kq;
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) acc[nt] = mfma16(ah[ks], T[k * SP + 16 * nt + (lane & 15)], acc[nt]);
    }
    __syncthreads();
#pragma unroll
    for (int nt = 0; nt < NT; ++nt)
#pragma unroll
        for (int g = 0; g < 4; ++g) T[(16 * w + 4 * g + kq) * SP + 16 * nt + (lane & 15)] = acc[nt][g];
    __syncthreads();
    for (int jb = threadIdx.x; jb < len; jb += kObBatch * NTH) {
        uint32_t bs[kObBatch];
        double old[kObBatch];
#pragma unroll
        for (int u = 0; u < kObBatch; ++u) {
            const int j = min(jb + u * NTH, len - 1);
            bs[u] = A.bstr[j];
            old[u] = ovw ? 0.0 : sr[j];
        }
#pragma unroll
        for (int u = 0; u < kObBatch; ++u)
            if (jb + u * NTH < len) {
                const int y = bs[u] & 0xff, s = (bs[u] >> 8) & 0xff;
                sr[jb + u * NTH] = old[u] + (T[y * SP + s] - T[s * SP + y]);
            }
    }
}

// Beta class on alpha rows [row0, row0 + nrows) whose beta strings stop at
// level 1 ({0,1} and {o, v}) or level 0 ({0,1} only).  Columns are
// (row, o) for the two occupied orbitals; a workgroup stages 16 consecutive
// rows of one vector in LDS (they are contiguous in memory) and forms 32
// columns.
//   V_o[b] = (h T[:, o])[b] = U[b][o]
//   sigma({o, b}), b virtual: h_oo c({o,b}) + h_oo' c({o',b}) - V_o[b]
//   sigma({0, 1})           : V_1[0] - V_0[1]
template <int NT>
__global__ __launch_bounds__(64 * NT) void k_ob_beta_cap1(SigmaArgs A, const double *__restrict__ c, int64_t ldc,
                                                          double *__restrict__ sg, int64_t lds,
                                                          const double *__restrict__ hs, const double *__restrict__ hp, int row0,
                                                          int nrows, int ovw)
{
    constexpr int NP = 16 * NT, SP = NP + 1, NR = 16, NC = 2 * NR, NK = NP / 4, NTH = 64 * NT;
    constexpr int RMAX = 1 + 2 * (kObMaxNorb - 2);   // longest row of level <= 1 strings
    __shared__ double U[NC * SP];   // U[col][b]
    __shared__ double R[NR * RMAX];
    __shared__ int ro[NR + 1];      // row offsets within R
    const int r0 = blockIdx.x * NR;
    const int v = blockIdx.y;
    const int norb = A.norb;
    const int lo1 = A.sb.lev_off[1];
    const int nr = min(NR, nrows - r0);
    const int64_t base0 = A.rowstart[row0 + r0];
    const int tot = (int)(A.rowstart[row0 + r0 + nr] - base0);
    const double *cv = c + (int64_t)v * ldc + base0;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int am = 16 * w + (lane & 15), kq = lane >> 4;
    double ah[NK];
    load_hcol<NK>(hp, am, kq, ah);
    if (threadIdx.x <= NR) ro[threadIdx.x] = (int)(A.rowstart[row0 + r0 + min((int)threadIdx.x, nr)] - base0);
    for (int tb = threadIdx.x; tb < tot; tb += kObBatch * NTH) {
        double val[kObBatch];
#pragma unroll
        for (int u = 0; u < kObBatch; ++u) val[u] = cv[min(tb + u * NTH, tot - 1)];
#pragma unroll
        for (int u = 0; u < kObBatch; ++u)
            if (tb + u * NTH < tot) R[tb + u * NTH] = val[u];
    }
    __syncthreads();
    int co[2], coff[2], clen[2];
#pragma unroll
    for (int nt = 0; nt < 2; ++nt) {
        const int col = 16 * nt + (lane & 15);
        const int rl = col / 2;   // < NR
        co[nt] = col & 1;
        coff[nt] = ro[rl];
        clen[nt] = ro[rl + 1] - ro[rl];   // 0 past the last row
    }
    v4d_ob acc[2];
#pragma unroll
    for (int nt = 0; nt < 2; ++nt) acc[nt] = v4d_ob{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int ks = 0; ks < NK; ++ks) {
        const int k = 4 * ks + kq;
#pragma unroll
        for (int nt = 0; nt < 2; ++nt) {
            const int o = co[nt];
            // T[k][o]: {k, o} is {0,1} (k occupied) or {o, k} (level 1); the
            // LDS read is clamped into the row and selected afterwards
            const int idx = k < 2 ? 0 : lo1 + 2 * (k - 2) + o;
            const bool ok = k < norb && k != o && idx < clen[nt];
            const double val = R[coff[nt] + (ok ? idx : 0)];
            acc[nt] = mfma16(ah[ks], ok ? (k < o ? val : -val) : 0.0, acc[nt]);
        }
    }
#pragma unroll
    for (int nt = 0; nt < 2; ++nt)
#pragma unroll
        for (int g = 0; g < 4; ++g) U[(16 * nt + (lane & 15)) * SP + 16 * w + 4 * g + kq] = acc[nt][g];
    __syncthreads();
    const double h00 = hs[0], h01 = hs[1], h11 = hs[norb + 1];
    double *sv = sg + (int64_t)v * lds + base0;
    for (int tb = threadIdx.x; tb < tot; tb += kObBatch * NTH) {
        double old[kObBatch];
#pragma unroll
        for (int u = 0; u < kObBatch; ++u) old[u] = ovw ? 0.0 : sv[min(tb + u * NTH, tot - 1)];
#pragma unroll
        for (int u = 0; u < kObBatch; ++u) {
            const int t = tb + u * NTH;
            if (t >= tot) break;
            // row of element t (rows are short and few: scan of the offsets)
            int rl = 0;
            while (rl + 1 < nr && ro[rl + 1] <= t) ++rl;
            const int j = t - ro[rl];
            const double *Ur = U + (2 * rl) * SP;   // column (rl, o = 0); (rl, 1) follows at +SP
            double add;
            if (j < lo1) {
                add = Ur[SP + 0] - Ur[1];
            } else {
                const int o = (j - lo1) & 1, bv = 2 + (j - lo1) / 2;
                const int jo = o ? t - 1 : t + 1;   // {o', b}
                add = (o ? h11 : h00) * R[t] + h01 * R[jo] - Ur[o * SP + bv];
            }
            sv[t] = old[u] + add;
        }
    }
}

// Alpha class on the beta columns [0, jd) where every alpha pair exists
// (beta level <= L - 2).  A workgroup takes NC consecutive columns of one
// vector (consecutive column blocks run on one XCD: they share cache
// lines) and holds their pair values P[col][ia] in LDS, ia the alpha string
// of the pair, with the table pcode[q][b] = +-(ia + 1) of the ordered pair
// (q, b) (sign: q < b; 0: q == b or padding).  Wave w forms the rows
// [16 w, 16 w + 16) of U = h T for every column; the pair differences
// U[a][b] - U[b][a] are gathered back into P (upper entries stored, then
// lower ones subtracted) and added to sigma row by row.
constexpr int kObDenseBatch = 16;

template <int NT, int NC>
__global__ __launch_bounds__(64 * NT) void k_ob_alpha_dense(SigmaArgs A, const double *__restrict__ c, int64_t ldc,
                                                            double *__restrict__ sg, int64_t lds,
                                                            const double *__restrict__ hp, int jd, int ncb_per_xcd)
{
    constexpr int NP = 16 * NT, NK = NP / 4, NTH = 64 * NT;
    extern __shared__ double ob_smem[];
    const int npair = A.sa.nstr;
    double *P = ob_smem;                                      // [NC][npair]
    short *pcode = (short *)(ob_smem + (size_t)NC * npair);   // [NP][NP]
    const int cb = (blockIdx.x & 7) * ncb_per_xcd + (blockIdx.x >> 3);
    const int j0 = cb * NC;
    if (j0 >= jd) return;
    const int v = blockIdx.y;
    const int norb = A.norb;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int n = lane & 15, kq = lane >> 4;
    double ah[NK];
    load_hcol<NK>(hp, 16 * w + n, kq, ah);
    {
        // NP * NP = 4 NT * NTH entries: one batch of table loads
        int ia[4 * NT];
#pragma unroll
        for (int i = 0; i < 4 * NT; ++i) {
            const int t = threadIdx.x + i * NTH, q = t / NP, b = t % NP;
            ia[i] = A.apidx[min(q, norb - 1) * norb + min(b, norb - 1)];
        }
#pragma unroll
        for (int i = 0; i < 4 * NT; ++i) {
            const int t = threadIdx.x + i * NTH, q = t / NP, b = t % NP;
            const bool ok = q < norb && b < norb && q != b && ia[i] >= 0;
            pcode[t] = (short)(ok ? (q < b ? ia[i] + 1 : -(ia[i] + 1)) : 0);
        }
    }
    const double *cv = c + (int64_t)v * ldc;
    const int ne = NC * npair;
    for (int eb = threadIdx.x; eb < ne; eb += kObDenseBatch * NTH) {
        double val[kObDenseBatch];
#pragma unroll
        for (int u = 0; u < kObDenseBatch; ++u) {
            const int e = min(eb + u * NTH, ne - 1), col = e % NC;
            val[u] = cv[row_start_n2(A, e / NC) + min(j0 + col, jd - 1)];
        }
#pragma unroll
        for (int u = 0; u < kObDenseBatch; ++u) {
            const int e = eb + u * NTH;
            if (e < ne) P[(e % NC) * npair + e / NC] = j0 + e % NC < jd ? val[u] : 0.0;
        }
    }
    __syncthreads();
    v4d_ob acc[NC][NT];
#pragma unroll
    for (int col = 0; col < NC; ++col)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) acc[col][nt] = v4d_ob{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int ks = 0; ks < NK; ++ks)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
            // B[q][b] = T[q][b] with q = 4 ks + kq, b = 16 nt + n
            const int code = pcode[(4 * ks + kq) * NP + 16 * nt + n];
            const int idx = (code > 0 ? code : -code) - 1;
            const int ic = idx < 0 ? 0 : idx;
#pragma unroll
            for (int col = 0; col < NC; ++col) {
                const double t = P[col * npair + ic];
                acc[col][nt] = mfma16(ah[ks], code > 0 ? t : (code < 0 ? -t : 0.0), acc[col][nt]);
            }
        }
    __syncthreads();   // P is reused for the pair differences
#pragma unroll
    for (int nt = 0; nt < NT; ++nt)
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            const int code = pcode[(16 * w + 4 * g + kq) * NP + 16 * nt + n];
            if (code > 0)
#pragma unroll
                for (int col = 0; col < NC; ++col) P[col * npair + code - 1] = acc[col][nt][g];
        }
    __syncthreads();
#pragma unroll
    for (int nt = 0; nt < NT; ++nt)
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            const int code = pcode[(16 * w + 4 * g + kq) * NP + 16 * nt + n];
            if (code < 0)
#pragma unroll
                for (int col = 0; col < NC; ++col) P[col * npair - code - 1] -= acc[col][nt][g];
        }
    __syncthreads();
    double *sv = sg + (int64_t)v * lds;
    for (int eb = threadIdx.x; eb < ne; eb += kObDenseBatch * NTH) {
        double old[kObDenseBatch];
#pragma unroll
        for (int u = 0; u < kObDenseBatch; ++u) {
            const int e = min(eb + u * NTH, ne - 1), col = e % NC;
            old[u] = sv[row_start_n2(A, e / NC) + min(j0 + col, jd - 1)];
        }
#pragma unroll
        for (int u = 0; u < kObDenseBatch; ++u) {
            const int e = eb + u * NTH;
            if (e < ne && j0 + e % NC < jd)
                sv[row_start_n2(A, e / NC) + j0 + e % NC] = old[u] + P[(e % NC) * npair + e / NC];
        }
    }
}

// Alpha class on the beta columns [j0c, jc) where the alpha pairs {0,1} and
// {o, v} exist and no {v, w} (beta level L - 1).  A workgroup takes 64
// columns of one vector and stages the signed rows
//   B_o[q][j] = T_j[q][o] = +-c({q, o}, j)
// of both occupied o in LDS; wave w forms U[a][o] for a in [16 w, 16 w + 16)
// (K = q).  Then, for a virtual v,
//   sigma({o, v}) += U[o][v] - U[v][o],  U[o][v] = h_o0 T[0][v] + h_o1 T[1][v]
// (T[q][v] vanishes for virtual q here), and sigma({0,1}) += U[0][1] - U[1][0].
template <int NT>
__global__ __launch_bounds__(64 * NT) void k_ob_alpha_cross(SigmaArgs A, const double *__restrict__ c, int64_t ldc,
                                                            double *__restrict__ sg, int64_t lds,
                                                            const double *__restrict__ hs, const double *__restrict__ hp, int j0c,
                                                            int jc)
{
    constexpr int NP = 16 * NT, NK = NP / 4, NTH = 64 * NT, NRT = 2 * NP / NT;
    __shared__ double B[2 * NP * 64];   // [o][q][jj]
    __shared__ long long rbase[2 * NP];  // row {q, o} of staged row (o, q); -1: none
    const int j0 = j0c + blockIdx.x * 64;
    const int v = blockIdx.y;
    const int norb = A.norb;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int n = lane & 15, kq = lane >> 4;
    double ah[NK];
    load_hcol<NK>(hp, 16 * w + n, kq, ah);
    for (int t = threadIdx.x; t < 2 * NP; t += NTH) {
        const int o = t / NP, q = t % NP;
        rbase[t] = q < norb ? A.arow_base[o * norb + q] : -1;
    }
    __syncthreads();
    const double *cv = c + (int64_t)v * ldc;
    // staged row (o, q) = w + NT i of the 2 NP rows, column lane; rows {q, o}
    // span [0, jc) (none for q = o)
    const int jl = j0 + lane, jcl = min(jl, jc - 1);
    {
        double val[NRT];
#pragma unroll
        for (int i = 0; i < NRT; ++i) {
            const long long base = rbase[w + NT * i];
            val[i] = cv[(base >= 0 ? base : 0) + jcl];
        }
#pragma unroll
        for (int i = 0; i < NRT; ++i) {
            const int r = w + NT * i, o = r / NP, q = r % NP;
            const bool ok = rbase[r] >= 0 && jl < jc;
            B[r * 64 + lane] = ok ? (q < o ? val[i] : -val[i]) : 0.0;
        }
    }
    __syncthreads();
    v4d_ob acc[2][4];
#pragma unroll
    for (int o = 0; o < 2; ++o)
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) acc[o][nt] = v4d_ob{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int ks = 0; ks < NK; ++ks)
#pragma unroll
        for (int o = 0; o < 2; ++o)
#pragma unroll
            for (int nt = 0; nt < 4; ++nt)
                acc[o][nt] = mfma16(ah[ks], B[(o * NP + 4 * ks + kq) * 64 + 16 * nt + n], acc[o][nt]);
    // epilogue per staged row (o, a) of this thread, column lane: first the
    // two-term U[o][a] from the staged operands, then U[a][o] from the
    // products through LDS (over the operands), then one batch of sigma
    // updates (coalesced rows)
    const double h00 = hs[0], h01 = hs[1], h11 = hs[norb + 1];
    double add[NRT];
#pragma unroll
    for (int i = 0; i < NRT; ++i) {
        const int r = w + NT * i, o = r / NP, a = r % NP;
        const double ho0 = o ? h01 : h00, ho1 = o ? h11 : h01;
        // T[0][a] = -B_0[a][jj], T[1][a] = -B_1[a][jj] (zero for a < 2)
        add[i] = a >= 2 ? -(ho0 * B[a * 64 + lane] + ho1 * B[(NP + a) * 64 + lane]) : 0.0;
    }
    __syncthreads();   // B is overwritten with the products U[a][o] below
#pragma unroll
    for (int o = 0; o < 2; ++o)
#pragma unroll
        for (int nt = 0; nt < 4; ++nt)
#pragma unroll
            for (int g = 0; g < 4; ++g) B[(o * NP + 16 * w + 4 * g + kq) * 64 + 16 * nt + n] = acc[o][nt][g];
    __syncthreads();
    double *sv = sg + (int64_t)v * lds;
    const long long b01 = rbase[1];   // row {0, 1} (staged row o = 0, q = 1)
    double old[NRT];
#pragma unroll
    for (int i = 0; i < NRT; ++i) {
        const long long base = rbase[w + NT * i];
        old[i] = sv[(base >= 0 ? base : b01) + jcl];
    }
#pragma unroll
    for (int i = 0; i < NRT; ++i) {
        const int r = w + NT * i, o = r / NP, a = r % NP;
        if (jl >= jc || a >= norb) continue;
        if (a >= 2) {
            // sigma({o, a}) += U[o][a] - U[a][o]
            sv[rbase[r] + jl] = old[i] + (add[i] - B[r * 64 + lane]);
        } else if (o == 1 && a == 0) {
            // sigma({0, 1}) += U[0][1] - U[1][0]
            sv[b01 + jl] = old[i] + (B[(NP + 0) * 64 + lane] - B[1 * 64 + lane]);
        }
    }
}

// Alpha class on the beta columns [j0, j1) where only the alpha pair {0,1}
// exists: U[0][1] - U[1][0] = (h_00 + h_11) c({0,1}).
__global__ __launch_bounds__(256) void k_ob_alpha_occ(SigmaArgs A, const double *__restrict__ c, int64_t ldc,
                                                      double *__restrict__ sg, int64_t lds,
                                                      const double *__restrict__ hs, int j0, int j1)
{
    const int j = j0 + blockIdx.x * 256 + threadIdx.x, v = blockIdx.y;
    if (j >= j1) return;
    const long long base = A.arow_base[1];   // row {0, 1}
    sg[(int64_t)v * lds + base + j] += (hs[0] + hs[A.norb + 1]) * c[(int64_t)v * ldc + base + j];
}

template <int NT>
static isci_status launch_ob_beta(const isci_ctx *cx, const SigmaArgs &A, int nv, const double *c, int64_t ldc,
                                  double *s, int64_t lds, int ovw, hipStream_t st)
{
    const double *hs = cx->d.hscreen, *hp = cx->d.hpad;
    const int L = cx->L;
    // alpha rows by level: beta strings up to level 2 for level <= L - 2
    const int full_end = L >= 2 ? cx->sa.le[L - 2] : 0;
    if (full_end > 0)
        k_ob_beta_full<NT><<<dim3((unsigned)full_end, (unsigned)nv), 64 * NT, 0, st>>>(A, c, ldc, s, lds, hs, hp, 0,
                                                                                      ovw);
    const int ncap1 = cx->sa.nstr - full_end;   // rows whose beta strings stop at level 1 or 0
    if (ncap1 > 0)
        k_ob_beta_cap1<NT><<<dim3((unsigned)((ncap1 + 15) / 16), (unsigned)nv), 64 * NT, 0, st>>>(
            A, c, ldc, s, lds, hs, hp, full_end, ncap1, ovw);
    return ISCI_OK;
}

static int max_lds_bytes(const isci_ctx *cx)
{
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, cx->device) != hipSuccess) v = 65536;
    return v;
}

// The dense block of the first jd beta columns (every alpha row holds
// them) moved to and from a [j][i] layout, row j being column j of c over
// all na alpha rows, through 32 x 32 LDS tiles (coalesced both ways):
//   add = 0: dst[j * na + i]  = src[rowstart[i] + j]
//   add = 1: dst[rowstart[i] + j] += src[j * na + i]
// for vector blockIdx.z (src and dst advanced by lsrc and ldst).
__global__ __launch_bounds__(256) void k_sub_transpose(const int64_t *__restrict__ rowstart, int na, int jd,
                                                       const double *__restrict__ src, int64_t lsrc,
                                                       double *__restrict__ dst, int64_t ldst, int add)
{
    __shared__ double tile[32][33];
    const int j0 = blockIdx.x * 32, i0 = blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    src += (int64_t)blockIdx.z * lsrc;
    dst += (int64_t)blockIdx.z * ldst;
    if (!add) {
        for (int r = ty; r < 32; r += 8) {
            const int i = i0 + r, j = j0 + tx;
            tile[r][tx] = (i < na && j < jd) ? src[rowstart[i] + j] : 0.0;
        }
        __syncthreads();
        for (int r = ty; r < 32; r += 8) {
            const int j = j0 + r, i = i0 + tx;
            if (j < jd && i < na) dst[(int64_t)j * na + i] = tile[tx][r];
        }
    } else {
        for (int r = ty; r < 32; r += 8) {
            const int j = j0 + r, i = i0 + tx;
            tile[r][tx] = (j < jd && i < na) ? src[(int64_t)j * na + i] : 0.0;
        }
        __syncthreads();
        for (int r = ty; r < 32; r += 8) {
            const int i = i0 + r, j = j0 + tx;
            if (i < na && j < jd) dst[rowstart[i] + j] += tile[tx][r];
        }
    }
}

template <int NT, int NC>
static isci_status launch_ob_dense(const isci_ctx *cx, const SigmaArgs &A, int nv, const double *c, int64_t ldc,
                                   double *s, int64_t lds, int jd, size_t shm, hipStream_t st)
{
    const int ncb = (jd + NC - 1) / NC, per = (ncb + 7) / 8;
    if (shm > 65536)
        ISCI_HIP(hipFuncSetAttribute((const void *)k_ob_alpha_dense<NT, NC>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm));
    k_ob_alpha_dense<NT, NC><<<dim3((unsigned)(8 * per), (unsigned)nv), 64 * NT, shm, st>>>(
        A, c, ldc, s, lds, cx->d.hpad, jd, per);
    return ISCI_OK;
}

// block transpose of up to four vectors (defined with k_det_transpose):
// dst = src^T (add = 0) or dst += src^T (add = 1), both in the layout of
// the space (two electrons per spin, alpha and beta string tables equal)
static void launch_block_transpose(const isci_ctx *cx, const SigmaArgs &A, const double *src, int64_t lsrc,
                                   double *dst, int64_t ldst, int add, int nv, hipStream_t st);

template <int NT>
static isci_status launch_ob_alpha(const isci_ctx *cx, const SigmaArgs &A, int nv, const double *c, int64_t ldc,
                                   double *s, int64_t lds, hipStream_t st)
{
    // the spectator form (rows {q, x} as B operands, no transposes) at any size
    if (cx->ob_kernel == ISCI_ONEBODY_SPECTATOR) return launch_onebody_alpha_large(cx, nv, c, ldc, s, lds, st);
    if (cx->ob_kernel == ISCI_ONEBODY_TRANSPOSED && cx->d.obT_c && cx->d.obT_s &&
        cx->sb.le[cx->L >= 2 ? cx->L - 2 : 0] == cx->sb.nstr && cx->sa.nstr == cx->sb.nstr) {
        // every beta column holds every alpha pair (full CI with two
        // electrons per spin): the alpha class is the beta class of the
        // transposed block, whose rows are contiguous; beta kernel there,
        // then added back through a second transpose
        const int64_t dim = cx->dim;
        const int step = cx->obT_nv;   // vectors the transposed scratch holds
        for (int u0 = 0; u0 < nv; u0 += step) {
            const int nu = nv - u0 < step ? nv - u0 : step;
            launch_block_transpose(cx, A, c + (int64_t)u0 * ldc, ldc, cx->d.obT_c, dim, 0, nu, st);
            k_ob_beta_full<NT><<<dim3((unsigned)cx->sa.nstr, (unsigned)nu), 64 * NT, 0, st>>>(
                A, cx->d.obT_c, dim, cx->d.obT_s, dim, cx->d.hscreen, cx->d.hpad, 0, 1);
            launch_block_transpose(cx, A, cx->d.obT_s, dim, s + (int64_t)u0 * lds, lds, 1, nu, st);
        }
        ISCI_HIP(hipGetLastError());
        return ISCI_OK;
    }
    const double *hs = cx->d.hscreen;
    const int L = cx->L;
    // beta columns by level: every alpha pair up to level L - 2, the pairs
    // {0,1} and {o, v} at level L - 1, {0,1} alone at level L
    const int *le_b = cx->sb.le;
    const int jd = L >= 2 ? le_b[L - 2] : 0;
    const int jc = L >= 1 ? le_b[L - 1] : 0;
    const int jall = le_b[L];
    if (jd > 0 && cx->ob_kernel == ISCI_ONEBODY_TRANSPOSED && cx->d.obS_c) {
        // the columns that hold every alpha pair as rows of their own block
        // (alpha and beta string tables coincide): the beta kernel there,
        // then added back; up to 8 vectors a pass
        const int na = cx->sa.nstr;
        const int64_t blk = (int64_t)jd * na;
        SigmaArgs B = A;
        B.rowstart = cx->d.obS_rs;
        const dim3 tg((unsigned)((jd + 31) / 32), (unsigned)((na + 31) / 32));
        for (int u0 = 0; u0 < nv; u0 += 8) {
            const int nu = nv - u0 < 8 ? nv - u0 : 8;
            k_sub_transpose<<<dim3(tg.x, tg.y, (unsigned)nu), 256, 0, st>>>(A.rowstart, na, jd, c + (int64_t)u0 * ldc,
                                                                              ldc, cx->d.obS_c, blk, 0);
            k_ob_beta_full<NT><<<dim3((unsigned)jd, (unsigned)nu), 64 * NT, 0, st>>>(
                B, cx->d.obS_c, blk, cx->d.obS_s, blk, cx->d.hscreen, cx->d.hpad, 0, 1);
            k_sub_transpose<<<dim3(tg.x, tg.y, (unsigned)nu), 256, 0, st>>>(A.rowstart, na, jd, cx->d.obS_s, blk,
                                                                              s + (int64_t)u0 * lds, lds, 1);
        }
        ISCI_HIP(hipGetLastError());
    } else if (jd > 0) {
        // two columns per workgroup: the pair block of 80 orbitals still
        // fits 64 KB of LDS, and two or three workgroups share a CU
        constexpr int NP = 16 * NT;
        const size_t shm = 2 * (size_t)cx->sa.nstr * sizeof(double) + NP * NP * sizeof(short);
        if (shm > (size_t)max_lds_bytes(cx)) {
            set_error("one-body matrix-core path: alpha pair block exceeds LDS");
            return ISCI_E_UNSUPPORTED;
        }
        ISCI_CHECK((launch_ob_dense<NT, 2>(cx, A, nv, c, ldc, s, lds, jd, shm, st)));
    }
    if (jc > jd)
        k_ob_alpha_cross<NT><<<dim3((unsigned)((jc - jd + 63) / 64), (unsigned)nv), 64 * NT, 0, st>>>(
            A, c, ldc, s, lds, hs, cx->d.hpad, jd, jc);
    if (jall > jc)
        k_ob_alpha_occ<<<dim3((unsigned)((jall - jc + 255) / 256), (unsigned)nv), 256, 0, st>>>(A, c, ldc, s, lds,
                                                                                                 hs, jc, jall);
    return ISCI_OK;
}

// ---------------------------------------------------------------------------
// Alpha class above 80 orbitals, where the pair blocks of the kernels above
// no longer fit LDS: spectator x = x0 + blockIdx.x, beta columns blockIdx.y * 64
// + [0, 64) (four 16-column N tiles), vector blockIdx.z / NG and target
// group blockIdx.z % NG (NG groups of four 16-target tiles: four-wave
// workgroups whatever norb); wave w forms the targets a in [16 mt, 16 mt +
// 16), mt = 4 group + w, with a > x (up = 1) or a < x (up = 0),
//   U[a][x][j] = sum_q h_aq T_j[q][x],
// with the B operand read straight from the rows {q, x} (coalesced).  One
// side of x per launch, so each sigma row is written by one workgroup per
// launch.  Columns run to jlim(x): for x virtual the rows {q, x} with q
// virtual stop at the level-2 row length; the columns above reach only
// {0,x} and {1,x} (k_ob_alpha_tail).  K steps without a row holding the
// column block are skipped (64-bit step mask, up to 256 orbitals); the
// operands of the next K step are in flight while the MFMAs of the current
// one issue.
template <int NT>
__global__ __launch_bounds__(256) void k_ob_alpha_spec(SigmaArgs A, const double *__restrict__ c, int64_t ldc,
                                                           double *__restrict__ sg, int64_t lds,
                                                           const double *__restrict__ hs,
                                                           const unsigned long long *__restrict__ hkm, int up,
                                                           int jlim_occ, int jlim_virt, int x0)
{
    constexpr int NP = 16 * NT, NG = (NT + 3) / 4;
    const int x = x0 + blockIdx.x, v = blockIdx.z / NG, grp = blockIdx.z % NG;
    const int norb = A.norb;
    const int jlim = x < 2 ? jlim_occ : jlim_virt;
    const int j0 = blockIdx.y * 64;
    if (j0 >= jlim) return;
    // row starts and lengths of {o, x} in LDS: the operand loads below then
    // depend on no other global load
    __shared__ long long rb[NP];
    __shared__ int rl[NP];
    for (int t = threadIdx.x; t < NP; t += 256) {
        rb[t] = t < norb ? A.arow_base[x * norb + t] : -1;
        rl[t] = t < norb ? A.arow_len[x * norb + t] : 0;
    }
    __syncthreads();
    const int mt = 4 * grp + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    // this wave's targets {a, x} on the requested side of x that hold a
    // column of the block, and the K steps whose sources {q, x} hold one
    const int at = 16 * mt + (lane & 15);
    const bool tok = lane < 16 && at < norb && at != x && ((at > x) == (up != 0)) && rl[at] > j0;
    if (__ballot(tok) == 0) return;
    unsigned long long km = 0;
#pragma unroll
    for (int r = 0; r < (NP + 63) / 64; ++r) {
        const int q = lane + 64 * r;
        const bool sq = q < NP && q < norb && q != x && rl[q] > j0;
        const unsigned long long sm = __ballot(sq);
#pragma unroll
        for (int kk = 0; kk < 16; ++kk)
            if (16 * r + kk < NP / 4 && ((sm >> (4 * kk)) & 0xfull)) km |= 1ull << (16 * r + kk);
    }
    // and whose h operands are not all screened away for this tile's
    // targets (a skipped step would only add zero products)
    km &= hkm[mt];
    const int n = lane & 15, kq = lane >> 4;
    const double *cv = c + (int64_t)v * ldc;
    auto next_ks = [&]() {
        if (!km) return -1;
        const int k = __ffsll((long long)km) - 1;
        km &= km - 1;
        return k;
    };
    // every lane loads from a valid address whatever the step; the loaded
    // values stay raw until their MFMAs, where invalid operands are zeroed,
    // so waiting for one stage's loads never precedes the other stage's
    // products (scheduling barriers keep the order)
    struct Stage {
        double a, b[4];
        double f;       // sign of the source rows, 0 for an invalid step or row
        bool aok;
        int bmask;      // columns inside the source row
    };
    auto load = [&](int ks, Stage &S) {
        const int q = 4 * max(ks, 0) + kq;
        const int qc = min(q, norb - 1), ac = min(16 * mt + n, norb - 1);
        S.a = hs[qc * norb + ac];
        S.aok = ks >= 0 && q < norb && 16 * mt + n < norb;
        const long long base = rb[qc];
        const int len = min(rl[qc], jlim);
        const bool rowok = ks >= 0 && q < norb && q != x && base >= 0;
        S.f = rowok ? (q < x ? 1.0 : -1.0) : 0.0;
        int bm = 0;
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            const int j = j0 + 16 * nt + n;
            const bool ok = rowok && j < len;
            bm |= ok ? 1 << nt : 0;
            S.b[nt] = cv[ok ? base + j : 0];
        }
        S.bmask = bm;
    };
    v4d_ob acc[4];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) acc[nt] = v4d_ob{0.0, 0.0, 0.0, 0.0};
    auto mma = [&](const Stage &S) {
        const double a = S.aok ? S.a : 0.0;
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) acc[nt] = mfma16(a, (S.bmask >> nt) & 1 ? S.f * S.b[nt] : 0.0, acc[nt]);
    };
    // two K steps in flight: stages x and y ping-pong over a counted loop
    // with no exit between the halves (an odd count ends with a step of
    // zero operands), so the stages keep their own registers
    const int nk = __popcll(km);
    Stage sx, sy;
    load(next_ks(), sx);
    __builtin_amdgcn_sched_barrier(0);
    for (int e = 0; e < nk; e += 2) {
        load(next_ks(), sy);
        __builtin_amdgcn_sched_barrier(0);
        mma(sx);
        __builtin_amdgcn_sched_barrier(0);
        load(next_ks(), sx);
        __builtin_amdgcn_sched_barrier(0);
        mma(sy);
        __builtin_amdgcn_sched_barrier(0);
    }
    double *sv = sg + (int64_t)v * lds;
#pragma unroll
    for (int g = 0; g < 4; ++g) {
        const int a = 16 * mt + 4 * g + kq;
        if (a >= norb || a == x || ((a > x) != (up != 0))) continue;
        const long long base = rb[a];
        if (base < 0) continue;
        const int len = min(rl[a], jlim);
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            const int j = j0 + 16 * nt + n;
            if (j < len) sv[base + j] += a < x ? acc[nt][g] : -acc[nt][g];
        }
    }
}

// Alpha class, the columns j in [j0, j1) of a virtual spectator x that only
// the rows {0, x} and {1, x} hold:
//   sigma({o, x}, j) += h_o0 c({0, x}, j) + h_o1 c({1, x}, j),  o = 0, 1.
__global__ __launch_bounds__(256) void k_ob_alpha_tail(SigmaArgs A, const double *__restrict__ c, int64_t ldc,
                                                       double *__restrict__ sg, int64_t lds,
                                                       const double *__restrict__ hs, int j0, int j1)
{
    const int x = 2 + blockIdx.x, v = blockIdx.z;
    const int j = j0 + blockIdx.y * 256 + threadIdx.x;
    const int norb = A.norb;
    const long long b0 = A.arow_base[x * norb + 0], b1 = A.arow_base[x * norb + 1];
    const int l0 = A.arow_len[x * norb + 0], l1 = A.arow_len[x * norb + 1];
    if (j >= j1 || b0 < 0 || b1 < 0) return;
    const double *cv = c + (int64_t)v * ldc;
    double *sv = sg + (int64_t)v * lds;
    const double c0 = j < l0 ? cv[b0 + j] : 0.0, c1 = j < l1 ? cv[b1 + j] : 0.0;
    if (j < l0) sv[b0 + j] += hs[0] * c0 + hs[1] * c1;
    if (j < l1) sv[b1 + j] += hs[norb] * c0 + hs[norb + 1] * c1;
}

// Alpha class, the columns j in [j0, j1) of the reference row {0, 1} past
// the rows of level one (only the reference row reaches them; both
// spectators x = 0, 1 map it onto itself):
//   sigma({0,1}, j) += (h_00 + h_11) c({0,1}, j).
__global__ __launch_bounds__(256) void k_ob_alpha_reftail(SigmaArgs A, const double *__restrict__ c, int64_t ldc,
                                                          double *__restrict__ sg, int64_t lds,
                                                          const double *__restrict__ hs, int j0, int j1)
{
    const int j = j0 + blockIdx.x * 256 + threadIdx.x, v = blockIdx.y;
    const int norb = A.norb;
    const long long b = A.arow_base[1];   // row {0, 1} (spectator 0, active 1)
    const int l = A.arow_len[1];
    if (j >= j1 || j >= l || b < 0) return;
    sg[(int64_t)v * lds + b + j] += (hs[0] + hs[norb + 1]) * c[(int64_t)v * ldc + b + j];
}

// Alpha class for virtual spectators whose rows hold at most kObNarrow
// columns (CISD: the reference beta string only), where a 64-column
// matrix-core tile would be almost all padding.  Workgroup (x, vector):
// T[q][j] = sgn(q - x) c({q,x}, j) for all q staged in LDS, then thread a
// forms U[a][j] = sum_q h_qa T[q][j] and adds sgn(a - x) U[a][j] to
// sigma({a,x}, j) for the targets on one side of x (up: a > x), so each
// row is written by one workgroup per launch.
constexpr int kObNarrow = 8;
__global__ __launch_bounds__(256) void k_ob_alpha_narrow(SigmaArgs A, const double *__restrict__ c, int64_t ldc,
                                                         double *__restrict__ sg, int64_t lds,
                                                         const double *__restrict__ hs, int up, int jlim, int x0)
{
    const int x = x0 + blockIdx.x, v = blockIdx.y;
    const int norb = A.norb;
    __shared__ double tq[256 * kObNarrow];
    const double *cv = c + (int64_t)v * ldc;
    for (int t = threadIdx.x; t < norb * kObNarrow; t += blockDim.x) {
        const int q = t / kObNarrow, j = t % kObNarrow;
        const long long base = A.arow_base[x * norb + q];
        const int len = min(A.arow_len[x * norb + q], jlim);
        tq[t] = (q != x && base >= 0 && j < len) ? (q < x ? 1.0 : -1.0) * cv[base + j] : 0.0;
    }
    __syncthreads();
    double *sv = sg + (int64_t)v * lds;
    for (int a = threadIdx.x; a < norb; a += blockDim.x) {
        if (a == x || (a > x) != (up != 0)) continue;
        const long long base = A.arow_base[x * norb + a];
        if (base < 0) continue;
        const int len = min(A.arow_len[x * norb + a], jlim);
        double u[kObNarrow];
#pragma unroll
        for (int j = 0; j < kObNarrow; ++j) u[j] = 0.0;
        for (int q = 0; q < norb; ++q) {
            const double hv = hs[q * norb + a];
#pragma unroll
            for (int j = 0; j < kObNarrow; ++j) u[j] += hv * tq[q * kObNarrow + j];
        }
#pragma unroll
        for (int j = 0; j < kObNarrow; ++j)
            if (j < len) sv[base + j] += a < x ? u[j] : -u[j];
    }
}

template <int NT>
static void launch_ob_alpha_spec(const isci_ctx *cx, const SigmaArgs &A, int nv, const double *c, int64_t ldc,
                                 double *s, int64_t lds, hipStream_t st)
{
    const double *hs = cx->d.hscreen;
    const int L = cx->L;
    // rows {q, x} hold beta strings up to level L - level({q, x}): for x
    // occupied the columns past the level-1 row length only reach the
    // reference row (k_ob_alpha_reftail), for x virtual the columns past
    // the level-2 row length only reach {0,x}, {1,x} (k_ob_alpha_tail)
    const int *le_b = cx->sb.le;
    const int jlim_occ = L >= 1 ? le_b[L - 1] : le_b[L];
    const int jref = le_b[L];
    const int jlim_virt = L >= 2 ? le_b[L - 2] : 0;
    const int jtail = L >= 1 ? le_b[L - 1] : 0;
    // occupied spectators (x < 2) span jlim_occ columns, virtual ones only
    // jlim_virt: one grid each, so no workgroup is launched past its row
    const int nocc = std::min(2, cx->norb);
    const unsigned ng = (NT + 3) / 4;
    const dim3 go((unsigned)nocc, (unsigned)((jlim_occ + 63) / 64), (unsigned)nv * ng);
    const dim3 gv((unsigned)(cx->norb - nocc), (unsigned)((jlim_virt + 63) / 64), (unsigned)nv * ng);
    const unsigned long long *hkm = cx->d.hkmask;
    for (int up = 1; up >= 0; --up) {
        k_ob_alpha_spec<NT><<<go, 256, 0, st>>>(A, c, ldc, s, lds, hs, hkm, up, jlim_occ, jlim_virt, 0);
        if (gv.x > 0 && gv.y > 0) {
            if (jlim_virt <= kObNarrow)
                k_ob_alpha_narrow<<<dim3(gv.x, (unsigned)nv), 256, 0, st>>>(A, c, ldc, s, lds, hs, up, jlim_virt,
                                                                           nocc);
            else
                k_ob_alpha_spec<NT><<<gv, 256, 0, st>>>(A, c, ldc, s, lds, hs, hkm, up, jlim_occ, jlim_virt, nocc);
        }
    }
    if (jref > jlim_occ && cx->norb >= 2)
        k_ob_alpha_reftail<<<dim3((unsigned)((jref - jlim_occ + 255) / 256), (unsigned)nv), 256, 0, st>>>(
            A, c, ldc, s, lds, hs, jlim_occ, jref);
    if (jtail > jlim_virt && cx->norb > 2)
        k_ob_alpha_tail<<<dim3((unsigned)(cx->norb - 2), (unsigned)((jtail - jlim_virt + 255) / 256), (unsigned)nv), 256,
                          0, st>>>(A, c, ldc, s, lds, hs, jlim_virt, jtail);
}

isci_status launch_onebody_alpha_large(const isci_ctx *cx, int nv, const double *c, int64_t ldc, double *s,
                                       int64_t lds, hipStream_t st)
{
    if (!(cx->d.hscreen && cx->d.hkmask && cx->na == 2 && cx->nb == 2 && cx->d.arow_base && cx->d.arow_len) ||
        cx->norb > 256) {
        set_error("alpha one-body spectator path: needs two electrons per spin and at most 256 orbitals");
        return ISCI_E_UNSUPPORTED;
    }
    const SigmaArgs A = sigma_args(cx);
    const int nt = std::max(6, (cx->norb + 15) / 16);
#define ISCI_OBS_CASE(N)                                         \
    case N: launch_ob_alpha_spec<N>(cx, A, nv, c, ldc, s, lds, st); break;
    switch (nt) {
        ISCI_OBS_CASE(6)
        ISCI_OBS_CASE(7)
        ISCI_OBS_CASE(8)
        ISCI_OBS_CASE(9)
        ISCI_OBS_CASE(10)
        ISCI_OBS_CASE(11)
        ISCI_OBS_CASE(12)
        ISCI_OBS_CASE(13)
        ISCI_OBS_CASE(14)
        ISCI_OBS_CASE(15)
        ISCI_OBS_CASE(16)
    default: set_error("alpha one-body spectator path: norb too large"); return ISCI_E_UNSUPPORTED;
    }
#undef ISCI_OBS_CASE
    ISCI_HIP(hipGetLastError());
    return ISCI_OK;
}

// With two electrons of each spin the alpha and beta string sets, their
// order and the row layout coincide, so the beta class of c is the alpha
// class of its transpose c^T[j][i] = c[i][j] (row = beta string, column =
// alpha string), with the same row tables.  Row i holds the columns
// j < len(i), and len does not grow with i, so a 32 x 32 tile of the
// (row, column) square is empty when its first column lies past its first
// row's length.  A workgroup moves one tile through LDS
// for every vector (coalesced on both sides):
//   add = 0: dst[row a][col b]  = src[row b][col a]
//   add = 1: dst[row a][col b] += src[row b][col a]
// for src rows b in [32 (bt0 + blockIdx.y), +32), columns a in
// [32 blockIdx.x, +32).
__global__ __launch_bounds__(256) void k_det_transpose(SigmaArgs A, const double *__restrict__ src, int64_t lsrc,
                                                       double *__restrict__ dst, int64_t ldst, int add, int bt0,
                                                       int nv)
{
    const int b0 = (bt0 + blockIdx.y) * 32, a0 = blockIdx.x * 32;
    const int n = A.sa.nstr, L = A.L;
    // tile rows of src are b, columns a: empty when a0 >= len(b0)
    if (b0 >= n || a0 >= A.sb.le[L - A.alev[b0]]) return;
    // vectors [4 blockIdx.z, 4 blockIdx.z + 4) of the nv
    src += (int64_t)(4 * blockIdx.z) * lsrc;
    dst += (int64_t)(4 * blockIdx.z) * ldst;
    nv -= 4 * (int)blockIdx.z;
    __shared__ double tile[4][32][33];
    // row starts and lengths of the tile's 32 source rows b and 32 target
    // rows a, read once: the element loads then depend on LDS only
    __shared__ long long rsb[32], rsa[32];
    __shared__ int lnb[32], lna[32];
    if (threadIdx.x < 64) {
        const int t = threadIdx.x & 31, r = (threadIdx.x < 32 ? b0 : a0) + t;
        const long long rs = r < n ? A.rowstart[r] : 0;
        const int ln = r < n ? A.sb.le[L - A.alev[r]] : 0;
        if (threadIdx.x < 32) { rsb[t] = rs; lnb[t] = ln; } else { rsa[t] = rs; lna[t] = ln; }
    }
    __syncthreads();
    const int cx = threadIdx.x & 31, ry = threadIdx.x >> 5;
    // all vectors' loads before the LDS writes
    double val[4][4];
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int r = ry + 8 * i, a = a0 + cx;
            const bool ok = v < nv && a < lnb[r];
            val[v][i] = ok ? src[(int64_t)v * lsrc + rsb[r] + a] : 0.0;
        }
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
        for (int i = 0; i < 4; ++i) tile[v][ry + 8 * i][cx] = val[v][i];
    __syncthreads();
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        if (v >= nv) break;
        double *d = dst + (int64_t)v * ldst;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int r = ry + 8 * i, b = b0 + cx;
            if (b < lna[r]) {
                double *o = d + rsa[r] + b;
                *o = add ? *o + tile[v][cx][r] : tile[v][cx][r];
            }
        }
    }
}

__global__ __launch_bounds__(256) void k_fill_zero(double *__restrict__ p, int64_t n)
{
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
        p[t] = 0.0;
}

// ---------------------------------------------------------------------------
// Beta class above kObMaxNorb on the rows themselves (no transposes), for the
// excitation hierarchy (orbitals 0 and 1 occupied), where a row whose beta
// strings reach level 2 (it then holds every beta pair) fits LDS.  The rank
// of the pair {y < s} in the (level, colex) string order:
//   {0,1}: 0;   {o, v}, o < 2 <= v: lo1 + 2 (v - 2) + o;
//   {v, w}, 2 <= v < w: lo2 + (v - 2) + (w - 2)(w - 3) / 2.
__device__ __forceinline__ int pair_rank_hier(int y, int s, int lo1, int lo2)
{
    return s < 2 ? 0 : (y < 2 ? lo1 + 2 * (s - 2) + y : lo2 + (y - 2) + ((s - 2) * (s - 3)) / 2);
}

// Sum over the K steps of mask km (bit ks: step ks kept) of the products
// of opa(ks) and opb(ks), added to acc: the kept steps are taken eight at a
// time, the operands of a batch loaded together (one memory latency per
// batch), then its products issued into two accumulator chains.  opa and
// opb return zero for ks < 0 (the padding of the last batch).
template <class OpA, class OpB>
__device__ __forceinline__ v4d_ob ob_masked_product(unsigned long long km, OpA opa, OpB opb, v4d_ob acc)
{
    v4d_ob acc2 = v4d_ob{0.0, 0.0, 0.0, 0.0};
    while (km) {
        int ks[8];
#pragma unroll
        for (int g = 0; g < 8; ++g) {
            ks[g] = km ? __ffsll((long long)km) - 1 : -1;
            km &= km - 1;
        }
        double a[8], b[8];
#pragma unroll
        for (int g = 0; g < 8; ++g) {
            a[g] = opa(ks[g]);
            b[g] = opb(ks[g]);
        }
#pragma unroll
        for (int g = 0; g < 8; g += 2) {
            acc = mfma16(a[g], b[g], acc);
            acc2 = mfma16(a[g + 1], b[g + 1], acc2);
        }
    }
    return acc + acc2;
}

// Rows whose beta strings reach level 2: one workgroup per (row, vector)
// stages the row (pair rank -> value) in LDS; the image of the row's
// antisymmetric pair matrix T under the one-body operator is
//   T'[a][x] = (h T)[a][x] + (T h)[a][x],   sigma({a < x}) += T'[a][x]
// (h symmetric, T antisymmetric).  Each wave takes 16 x 16 tile pairs
// (I <= J) of the orbital square and forms both products of its tile on
// matrix cores: the T operands gathered from LDS by pair rank, the h
// operands read from the screened h (coalesced), K steps whose h operands
// are all screened for the tile skipped.  Once every wave has read the
// row, the results replace it in LDS and the row is added to sigma.
constexpr int kObRowWaves = 16;
constexpr int kObRowTpw = 9;   // tile pairs per wave: 16 tiles give 136 pairs

// TAB: the T operands through a table of signed pair codes in LDS beside
// the row (pcode[f][q] = +-(rank of {f, q} + 1), + for q > f, 0 on the
// diagonal and past norb; P x P with P = 16 nt) and the h operands from the
// copy of h zero-padded to P x P, so no operand needs a bounds test or a
// rank formula.
template <bool TAB>
__global__ __launch_bounds__(64 * kObRowWaves) void k_ob_beta_rows(SigmaArgs A, const double *__restrict__ c,
                                                                  int64_t ldc, double *__restrict__ sg, int64_t lds,
                                                                  const double *__restrict__ hs,
                                                                  const double *__restrict__ hp,
                                                                  const unsigned long long *__restrict__ hkm)
{
    constexpr int NTH = 64 * kObRowWaves;
    extern __shared__ double rrow[];
    const int ia = blockIdx.x, v = blockIdx.y;
    const int norb = A.norb, nt = (norb + 15) >> 4;
    const int len = A.sb.le[A.L - A.alev[ia]];
    const int64_t rs = A.rowstart[ia];
    const double *cr = c + (int64_t)v * ldc + rs;
    double *sr = sg + (int64_t)v * lds + rs;
    for (int tb = threadIdx.x; tb < len; tb += kObBatch * NTH) {
        double val[kObBatch];
#pragma unroll
        for (int u = 0; u < kObBatch; ++u) val[u] = cr[min(tb + u * NTH, len - 1)];
#pragma unroll
        for (int u = 0; u < kObBatch; ++u)
            if (tb + u * NTH < len) rrow[tb + u * NTH] = val[u];
    }
    const int lo1 = A.sb.lev_off[1], lo2 = A.sb.lev_off[2];
    const int P = 16 * nt;
    short *pcode = (short *)(rrow + A.sb.nstr);
    if (TAB)
        for (int t = threadIdx.x; t < P * P; t += NTH) {
            const int f = t / P, q = t - f * P;
            const bool ok = f < norb && q < norb && f != q;
            const int r = pair_rank_hier(min(f, q), max(f, q), lo1, lo2) + 1;
            pcode[t] = (short)(ok ? (q > f ? r : -r) : 0);
        }
    __syncthreads();
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int n = lane & 15, kq = lane >> 4;
    const int npairs = nt * (nt + 1) / 2;
    // T[q][x] from the staged row; zero on the diagonal and past norb
    auto tget = [&](int q, int x) -> double {
        if (TAB) {
            const int code = pcode[q * P + x];
            const double r = rrow[max(abs(code) - 1, 0)];
            return code > 0 ? r : (code < 0 ? -r : 0.0);
        }
        const int lo = min(q, x), hi = max(q, x);
        const bool ok = q != x && hi < norb;
        const double r = rrow[ok ? pair_rank_hier(lo, hi, lo1, lo2) : 0];
        return ok ? (q < x ? r : -r) : 0.0;
    };
    // h_aq of the screened h (symmetric), zero past norb
    auto hget = [&](int a, int q) -> double {
        if (TAB) return hp[q * P + a];
        const double h = hs[(size_t)min(q, norb - 1) * norb + min(a, norb - 1)];
        return (a < norb && q < norb) ? h : 0.0;
    };
    v4d_ob acc[kObRowTpw];
    int tI[kObRowTpw], tJ[kObRowTpw];
#pragma unroll
    for (int i = 0; i < kObRowTpw; ++i) {
        acc[i] = v4d_ob{0.0, 0.0, 0.0, 0.0};
        tI[i] = -1;
        tJ[i] = -1;
        const int tp = wave + i * kObRowWaves;
        if (tp >= npairs) continue;   // uniform over the wave
        int I = 0, rem = tp;
        while (rem >= nt - I) { rem -= nt - I; ++I; }
        const int J = I + rem;
        tI[i] = I;
        tJ[i] = J;
        v4d_ob acc2 = v4d_ob{0.0, 0.0, 0.0, 0.0};
        // (h T) of the tile: A = h[16 I + n][q], B = T[q][16 J + n], q = 4 ks + kq;
        // then (T h): A = T[16 I + n][q], B = h[q][16 J + n].  The operands
        // of the next two steps load while the current two steps' products
        // issue.
#pragma unroll
        for (int term = 0; term < 2; ++term) {
            unsigned long long km = hkm[term == 0 ? I : J];
            auto next_ks = [&]() {
                if (!km) return -1;
                const int k = __ffsll((long long)km) - 1;
                km &= km - 1;
                return k;
            };
            auto opa = [&](int ks) {
                const int q = 4 * max(ks, 0) + kq;
                const double a = term == 0 ? hget(16 * I + n, q) : tget(16 * I + n, q);
                return ks >= 0 ? a : 0.0;
            };
            auto opb = [&](int ks) {
                const int q = 4 * max(ks, 0) + kq;
                const double b = term == 0 ? tget(q, 16 * J + n) : hget(16 * J + n, q);
                return ks >= 0 ? b : 0.0;
            };
            // steps taken two at a time into two accumulators (two
            // independent product chains); a missing second step has zero
            // operands
            int k0 = next_ks(), k1 = next_ks();
            double a0 = opa(k0), b0 = opb(k0), a1 = opa(k1), b1 = opb(k1);
            while (k0 >= 0) {
                const int k2 = next_ks(), k3 = next_ks();
                const double a2 = opa(k2), b2 = opb(k2), a3 = opa(k3), b3 = opb(k3);
                acc[i] = mfma16(a0, b0, acc[i]);
                acc2 = mfma16(a1, b1, acc2);
                k0 = k2;
                k1 = k3;
                a0 = a2;
                b0 = b2;
                a1 = a3;
                b1 = b3;
            }
        }
        acc[i] += acc2;
    }
    __syncthreads();   // every wave has read the row
#pragma unroll
    for (int i = 0; i < kObRowTpw; ++i) {
        if (tI[i] < 0) continue;
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            // element g of the lane: a = 16 I + 4 g + kq, x = 16 J + n
            const int a = 16 * tI[i] + 4 * g + kq, x = 16 * tJ[i] + n;
            if (a < x && x < norb) rrow[pair_rank_hier(a, x, lo1, lo2)] = acc[i][g];
        }
    }
    __syncthreads();
    for (int tb = threadIdx.x; tb < len; tb += kObBatch * NTH) {
        double old[kObBatch];
#pragma unroll
        for (int u = 0; u < kObBatch; ++u) old[u] = sr[min(tb + u * NTH, len - 1)];
#pragma unroll
        for (int u = 0; u < kObBatch; ++u)
            if (tb + u * NTH < len) sr[tb + u * NTH] = old[u] + rrow[tb + u * NTH];
    }
}

// Rows whose beta strings stop at level 1 ({0,1} and {o, v}) or level 0,
// above kObMaxNorb: the scheme of k_ob_beta_cap1 (columns (row, o) for the
// two occupied o, V_o[b] = (h T[:, o])[b] on matrix cores) with kObShortRows
// rows per workgroup, eight waves looping over the 16-orbital target tiles,
// the h operands read from the copy of h zero-padded to whole 16-orbital
// tiles with the per-tile K-step masks,
// and LDS sized by norb (dynamic):
//   sigma({o, b}), b virtual: h_oo c({o,b}) + h_oo' c({o',b}) - V_o[b]
//   sigma({0, 1})           : V_1[0] - V_0[1]
constexpr int kObShortRows = 8, kObShortWaves = 8;

__global__ __launch_bounds__(64 * kObShortWaves) void k_ob_beta_short(SigmaArgs A, const double *__restrict__ c, int64_t ldc,
                                                       double *__restrict__ sg, int64_t lds,
                                                       const double *__restrict__ hs, const double *__restrict__ hp,
                                                       const unsigned long long *__restrict__ hkm, int row0, int nrows)
{
    constexpr int NR = kObShortRows, NTH = 64 * kObShortWaves;
    extern __shared__ double ssm[];
    const int norb = A.norb, nt = (norb + 15) >> 4, rmax = 2 * norb - 3;
    double *R = ssm;              // the workgroup's rows, contiguous (at most NR * rmax values)
    double *U = ssm + NR * rmax;  // U[col][b], col = 2 (row) + o
    __shared__ int ro[NR + 1];    // row offsets within R
    const int r0 = blockIdx.x * NR;
    const int v = blockIdx.y;
    const int lo1 = A.sb.lev_off[1];
    const int nr = min(NR, nrows - r0);
    const int64_t base0 = A.rowstart[row0 + r0];
    const int tot = (int)(A.rowstart[row0 + r0 + nr] - base0);
    const double *cv = c + (int64_t)v * ldc + base0;
    if (threadIdx.x <= NR) ro[threadIdx.x] = (int)(A.rowstart[row0 + r0 + min((int)threadIdx.x, nr)] - base0);
    for (int tb = threadIdx.x; tb < tot; tb += kObBatch * NTH) {
        double val[kObBatch];
#pragma unroll
        for (int u = 0; u < kObBatch; ++u) val[u] = cv[min(tb + u * NTH, tot - 1)];
#pragma unroll
        for (int u = 0; u < kObBatch; ++u)
            if (tb + u * NTH < tot) R[tb + u * NTH] = val[u];
    }
    __syncthreads();
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int n = lane & 15, kq = lane >> 4;
    // the lane's column (row rl, occupied o): one 16-column N tile
    const int rl = n >> 1, o = n & 1;
    const int coff = ro[rl], clen = ro[rl + 1] - ro[rl];   // 0 past the last row
    for (int mt = wave; mt < nt; mt += kObShortWaves) {
        const unsigned long long km = hkm[mt];
        // A = h[16 mt + n][k], B = T[k][o] of the column's row: {k, o} is
        // {0,1} (k occupied) or {o, k} (k virtual, level 1); the LDS read is
        // clamped into the row and selected afterwards
        // h from its copy zero-padded to whole 16-orbital tiles (P = 16 nt)
        auto opa = [&](int ks) {
            const int k = 4 * max(ks, 0) + kq, a = 16 * mt + n;
            const double h = hp[k * (16 * nt) + a];
            return ks >= 0 ? h : 0.0;
        };
        auto opb = [&](int ks) {
            const int k = 4 * max(ks, 0) + kq;
            const int idx = k < 2 ? 0 : lo1 + 2 * (k - 2) + o;
            const bool ok = ks >= 0 && k < norb && k != o && idx < clen;
            const double val = R[coff + (ok ? idx : 0)];
            return ok ? (k < o ? val : -val) : 0.0;
        };
        const v4d_ob acc = ob_masked_product(km, opa, opb, v4d_ob{0.0, 0.0, 0.0, 0.0});
        // element g: target b = 16 mt + 4 g + kq, column n
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            const int b = 16 * mt + 4 * g + kq;
            if (b < norb) U[n * norb + b] = acc[g];
        }
    }
    __syncthreads();
    const double h00 = hs[0], h01 = hs[1], h11 = hs[norb + 1];
    double *sv = sg + (int64_t)v * lds + base0;
    for (int tb = threadIdx.x; tb < tot; tb += kObBatch * NTH) {
        double old[kObBatch];
#pragma unroll
        for (int u = 0; u < kObBatch; ++u) old[u] = sv[min(tb + u * NTH, tot - 1)];
#pragma unroll
        for (int u = 0; u < kObBatch; ++u) {
            const int t = tb + u * NTH;
            if (t >= tot) break;
            // row of element t (a scan of the few offsets)
            int r = 0;
            while (r + 1 < nr && ro[r + 1] <= t) ++r;
            const int j = t - ro[r];
            const double *Ur = U + (size_t)(2 * r) * norb;   // column (r, o = 0); (r, 1) follows at +norb
            double add;
            if (j < lo1) {
                add = Ur[norb + 0] - Ur[1];
            } else {
                const int oo = (j - lo1) & 1, bv = 2 + (j - lo1) / 2;
                const int jo = oo ? t - 1 : t + 1;   // {o', b}
                add = (oo ? h11 : h00) * R[t] + h01 * R[jo] - Ur[oo * norb + bv];
            }
            sv[t] = old[u] + add;
        }
    }
}

bool onebody_beta_rows_ok(const isci_ctx *cx)
{
    return cx->d.hscreen && cx->d.hkmask && cx->na == 2 && cx->nb == 2 && cx->norb > kObMaxNorb &&
           cx->d.hpadT && cx->norb <= 256 && cx->sa.nocc == 2 && cx->sb.nocc == 2 && cx->sa.nstr == cx->sb.nstr &&
           (size_t)cx->sb.nstr * sizeof(double) <= (size_t)max_lds_bytes(cx) &&
           ((cx->norb + 15) / 16) * ((cx->norb + 15) / 16 + 1) / 2 <= kObRowWaves * kObRowTpw;
}

static isci_status launch_onebody_beta_rows(const isci_ctx *cx, int nv, const double *c, int64_t ldc, double *s,
                                            int64_t lds, hipStream_t st)
{
    const SigmaArgs A = sigma_args(cx);
    const int L = cx->L, norb = cx->norb;
    // alpha rows by level: every beta pair for level <= L - 2, beta strings
    // up to level 1 (or 0) past those
    const int nfull = L >= 2 ? cx->sa.le[L - 2] : 0;
    if (nfull > 0) {
        // the pair-code table beside the row where both fit LDS
        const int P = 16 * ((norb + 15) / 16);
        const size_t row = sizeof(double) * (size_t)cx->sb.nstr, tab = sizeof(short) * (size_t)P * P;
        const bool use_tab = cx->d.hpadT && row + tab <= (size_t)max_lds_bytes(cx);
        const size_t shm = use_tab ? row + tab : row;
        const void *fn = use_tab ? (const void *)k_ob_beta_rows<true> : (const void *)k_ob_beta_rows<false>;
        if (shm > 65536) ISCI_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm));
        const dim3 grid((unsigned)nfull, (unsigned)nv);
        if (use_tab)
            k_ob_beta_rows<true><<<grid, 64 * kObRowWaves, shm, st>>>(A, c, ldc, s, lds, cx->d.hscreen, cx->d.hpadT,
                                                                    cx->d.hkmask);
        else
            k_ob_beta_rows<false><<<grid, 64 * kObRowWaves, shm, st>>>(A, c, ldc, s, lds, cx->d.hscreen, cx->d.hpadT,
                                                                     cx->d.hkmask);
    }
    const int nshort = cx->sa.nstr - nfull;
    if (nshort > 0) {
        const size_t shm = sizeof(double) * ((size_t)kObShortRows * (2 * norb - 3) + 2 * kObShortRows * (size_t)norb);
        if (shm > 65536)
            ISCI_HIP(hipFuncSetAttribute((const void *)k_ob_beta_short, hipFuncAttributeMaxDynamicSharedMemorySize,
                                         (int)shm));
        k_ob_beta_short<<<dim3((unsigned)((nshort + kObShortRows - 1) / kObShortRows), (unsigned)nv), 64 * kObShortWaves,
                          shm, st>>>(
            A, c, ldc, s, lds, cx->d.hscreen, cx->d.hpadT, cx->d.hkmask, nfull, nshort);
    }
    ISCI_HIP(hipGetLastError());
    return ISCI_OK;
}

isci_status launch_onebody_beta_large(const isci_ctx *cx, int nv, const double *c, int64_t ldc, double *s,
                                      int64_t lds, hipStream_t st)
{
    if (cx->ob_kernel == ISCI_ONEBODY_ROWS) {
        if (!onebody_beta_rows_ok(cx)) {
            set_error("beta one-body row path: not available for this handle");
            return ISCI_E_UNSUPPORTED;
        }
        return launch_onebody_beta_rows(cx, nv, c, ldc, s, lds, st);
    }
    if (!cx->d.obT_c || !cx->d.obT_s || nv > 4 || cx->sa.nstr != cx->sb.nstr) {
        set_error("beta one-body transposed path: scratch missing or more than 4 vectors");
        return ISCI_E_UNSUPPORTED;
    }
    const SigmaArgs A = sigma_args(cx);
    const int64_t dim = cx->dim;
    launch_block_transpose(cx, A, c, ldc, cx->d.obT_c, dim, 0, nv, st);
    k_fill_zero<<<(unsigned)std::min<int64_t>(4096, (dim * nv + 255) / 256), 256, 0, st>>>(cx->d.obT_s, dim * nv);
    ISCI_HIP(hipGetLastError());
    ISCI_CHECK(launch_onebody_alpha_large(cx, nv, cx->d.obT_c, dim, cx->d.obT_s, dim, st));
    launch_block_transpose(cx, A, cx->d.obT_s, dim, s, lds, 1, nv, st);
    ISCI_HIP(hipGetLastError());
    return ISCI_OK;
}

// row tiles grouped by the length of their first row (one value per
// level): each group launches only the column tiles that row reaches
static void launch_block_transpose(const isci_ctx *cx, const SigmaArgs &A, const double *src, int64_t lsrc,
                                   double *dst, int64_t ldst, int add, int nv, hipStream_t st)
{
    const int n = cx->sa.nstr, nt = (n + 31) / 32;
    for (int t0 = 0; t0 < nt;) {
        const int len0 = cx->sb.le[cx->L - cx->h_alev[32 * t0]];
        int t1 = t0 + 1;
        while (t1 < nt && cx->sb.le[cx->L - cx->h_alev[32 * t1]] == len0) ++t1;
        k_det_transpose<<<dim3((unsigned)((len0 + 31) / 32), (unsigned)(t1 - t0), (unsigned)((nv + 3) / 4)), 256, 0,
                          st>>>(A, src, lsrc, dst, ldst, add, t0, nv);
        t0 = t1;
    }
}

bool onebody_mfma_ok(const isci_ctx *cx)
{
    return cx->d.hscreen && cx->na == 2 && cx->nb == 2 && cx->norb >= 3 && cx->norb <= kObMaxNorb &&
           cx->d.arow_base && cx->d.arow_len && cx->d.apidx && cx->d.hpad;
}

isci_status launch_onebody_mfma(const isci_ctx *cx, int nv, const double *c, int64_t ldc, double *s, int64_t lds,
                                hipStream_t st, bool first)
{
    const int ovw = first ? 1 : 0;
    const SigmaArgs A = sigma_args(cx);
    const int nt = (cx->norb + 15) / 16;
#define ISCI_OB_CASE(N)                                                      \
    case N:                                                                  \
        ISCI_CHECK(launch_ob_beta<N>(cx, A, nv, c, ldc, s, lds, ovw, st));   \
        ISCI_CHECK(launch_ob_alpha<N>(cx, A, nv, c, ldc, s, lds, st));       \
        break;
    switch (nt) {
        ISCI_OB_CASE(1)
        ISCI_OB_CASE(2)
        ISCI_OB_CASE(3)
        ISCI_OB_CASE(4)
        ISCI_OB_CASE(5)
    default: set_error("one-body matrix-core path: norb too large"); return ISCI_E_UNSUPPORTED;
    }
#undef ISCI_OB_CASE
    ISCI_HIP(hipGetLastError());
    return ISCI_OK;
}

}  // namespace isci
