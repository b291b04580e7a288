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
//  * beta class, alpha rows whose beta strings reach level 2: T of the row
//    is built in LDS and U = h T is formed whole;
//  * beta class, rows whose beta strings stop at level 1: only the columns
//    U[:, o] of the two occupied orbitals o are needed (a product over many
//    rows at once), plus two units per target taken directly;
//  * alpha class: for a spectator x the rows {q, x} of all q hold, for each
//    beta column j, the column T_j[:, x]; U_j[:, x] = h T_j[:, x] is a
//    product with K = q and the beta columns as N, read straight from the
//    rows (coalesced).  Target rows {a, x} are split by a < x / a > x over
//    two launches so that one workgroup writes each sigma element per launch.
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

// screened h (symmetric, canonical) with zero padding
__device__ __forceinline__ double hpad(const double *__restrict__ hs, int norb, int p, int q)
{
    return (p < norb && q < norb) ? hs[q * norb + p] : 0.0;
}

// Beta class on alpha rows [row0, row0 + gridDim.x) whose beta strings reach
// level 2; one workgroup per (row, vector), NT waves, one M tile per wave.
template <int NT>
__global__ __launch_bounds__(64 * NT) void k_ob_beta_full(SigmaArgs A, const double *__restrict__ c, int64_t ldc,
                                                          double *__restrict__ sg, int64_t lds,
                                                          const double *__restrict__ hs, int row0)
{
    constexpr int NP = 16 * NT, SP = NP + 1;   // odd row stride: no bank conflicts on U[y][s]
    __shared__ double T[NP * SP];
    const int ia = row0 + blockIdx.x;
    const int v = blockIdx.y;
    const int norb = A.norb;
    const int len = A.sb.le[A.L - A.alev[ia]];
    const double *cr = c + (int64_t)v * ldc + A.rowstart[ia];
    double *sr = sg + (int64_t)v * lds + A.rowstart[ia];
    for (int t = threadIdx.x; t < NP * SP; t += 64 * NT) T[t] = 0.0;
    __syncthreads();
    for (int j = threadIdx.x; j < len; j += 64 * NT) {
        const uint32_t bs = A.bstr[j];
        const int y = bs & 0xff, s = (bs >> 8) & 0xff;
        const double val = cr[j];
        T[y * SP + s] = val;
        T[s * SP + y] = -val;
    }
    __syncthreads();
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int am = 16 * w + (lane & 15), kq = lane >> 4;
    v4d_ob acc[NT];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) acc[nt] = v4d_ob{0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
    for (int ks = 0; ks < NP / 4; ++ks) {
        const int k = 4 * ks + kq;
        const double a = hpad(hs, norb, am, k);
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) acc[nt] = mfma16(a, T[k * SP + 16 * nt + (lane & 15)], acc[nt]);
    }
    __syncthreads();
#pragma unroll
    for (int nt = 0; nt < NT; ++nt)
#pragma unroll
        for (int g = 0; g < 4; ++g) T[(16 * w + 4 * g + kq) * SP + 16 * nt + (lane & 15)] = acc[nt][g];
    __syncthreads();
    for (int j = threadIdx.x; j < len; j += 64 * NT) {
        const uint32_t bs = A.bstr[j];
        const int y = bs & 0xff, s = (bs >> 8) & 0xff;
        sr[j] += T[y * SP + s] - T[s * SP + y];
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
                                                          const double *__restrict__ hs, int row0, int nrows)
{
    constexpr int NP = 16 * NT, SP = NP + 1, NR = 16, NC = 2 * NR;
    constexpr int RMAX = 1 + 2 * (kObMaxNorb - 2);   // longest row of level <= 1 strings
    __shared__ double U[NC * SP];   // U[col][b]
    __shared__ double R[NR * RMAX];
    const int r0 = blockIdx.x * NR;
    const int v = blockIdx.y;
    const int norb = A.norb;
    const int lo1 = A.sb.lev_off[1];
    const int nr = min(NR, nrows - r0);
    const int64_t base0 = A.rowstart[row0 + r0];
    const int tot = (int)(A.rowstart[row0 + r0 + nr] - base0);
    const double *cv = c + (int64_t)v * ldc;
    for (int t = threadIdx.x; t < tot; t += 64 * NT) R[t] = cv[base0 + t];
    __syncthreads();
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int am = 16 * w + (lane & 15), kq = lane >> 4;
    int co[2], coff[2], clen[2];
#pragma unroll
    for (int nt = 0; nt < 2; ++nt) {
        const int col = 16 * nt + (lane & 15);
        const int rl = col / 2;
        co[nt] = col & 1;
        coff[nt] = rl < nr ? (int)(A.rowstart[row0 + r0 + rl] - base0) : 0;
        clen[nt] = rl < nr ? (int)(A.rowstart[row0 + r0 + rl + 1] - base0) - coff[nt] : 0;
    }
    v4d_ob acc[2];
#pragma unroll
    for (int nt = 0; nt < 2; ++nt) acc[nt] = v4d_ob{0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
    for (int ks = 0; ks < NP / 4; ++ks) {
        const int k = 4 * ks + kq;
        const double a = hpad(hs, norb, am, k);
#pragma unroll
        for (int nt = 0; nt < 2; ++nt) {
            const int o = co[nt];
            // T[k][o]: {k, o} is {0,1} (k occupied) or {o, k} (level 1)
            const int idx = k < 2 ? 0 : lo1 + 2 * (k - 2) + o;
            double b = 0.0;
            if (k < norb && k != o && idx < clen[nt]) {
                const double val = R[coff[nt] + idx];
                b = k < o ? val : -val;
            }
            acc[nt] = mfma16(a, b, acc[nt]);
        }
    }
#pragma unroll
    for (int nt = 0; nt < 2; ++nt)
#pragma unroll
        for (int g = 0; g < 4; ++g) U[(16 * nt + (lane & 15)) * SP + 16 * w + 4 * g + kq] = acc[nt][g];
    __syncthreads();
    const double h00 = hs[0], h01 = hs[1], h11 = hs[norb + 1];
    double *sv = sg + (int64_t)v * lds + base0;
    for (int t = threadIdx.x; t < tot; t += 64 * NT) {
        // row of element t (rows are short and few: linear scan)
        int rl = 0;
        while (rl + 1 < nr && A.rowstart[row0 + r0 + rl + 1] - base0 <= t) ++rl;
        const int off = (int)(A.rowstart[row0 + r0 + rl] - base0);
        const int j = t - off;
        const double *Ur = U + (2 * rl) * SP;   // column (rl, o = 0); (rl, 1) follows at +SP
        double add;
        if (j < lo1) {
            add = Ur[SP + 0] - Ur[1];
        } else {
            const int o = (j - lo1) & 1, bv = 2 + (j - lo1) / 2;
            const int jo = o ? t - 1 : t + 1;   // {o', b}
            add = (o ? h11 : h00) * R[t] + h01 * R[jo] - Ur[o * SP + bv];
        }
        sv[t] += add;
    }
}

// Alpha class, spectator x = blockIdx.x, beta columns blockIdx.y * 64 +
// [0, 64) (four 16-column N tiles), vector blockIdx.z; wave w computes the
// targets a in [16 w, 16 w + 16) with a > x (up = 1) or a < x (up = 0).
// Columns run to jlim(x): for x virtual the rows {q, x} with q virtual stop
// at the level-2 row length, the columns above reach only {0,x} and {1,x}
// (the two-term tail below).  The operands of the next K step are in
// flight while the MFMAs of the current one issue.
template <int NT>
__global__ __launch_bounds__(64 * NT) void k_ob_alpha(SigmaArgs A, const double *__restrict__ c, int64_t ldc,
                                                      double *__restrict__ sg, int64_t lds,
                                                      const double *__restrict__ hs, int up, int jlim_occ,
                                                      int jlim_virt)
{
    constexpr int NP = 16 * NT;
    const int x = blockIdx.x, v = blockIdx.z;
    const int norb = A.norb;
    const int jlim = x < 2 ? jlim_occ : jlim_virt;
    const int j0 = blockIdx.y * 64;
    if (j0 >= jlim) return;
    // row starts and lengths of {o, x} in LDS: the operand loads below then
    // depend on no other global load
    __shared__ long long rb[NP];
    __shared__ int rl[NP];
    for (int t = threadIdx.x; t < NP; t += 64 * NT) {
        rb[t] = t < norb ? A.arow_base[x * norb + t] : -1;
        rl[t] = t < norb ? A.arow_len[x * norb + t] : 0;
    }
    __syncthreads();
    const int mt = threadIdx.x >> 6, lane = threadIdx.x & 63;
    // this wave's targets {a, x} on the requested side of x that hold a
    // column of the block, and the sources {q, x} that hold one
    const int at = 16 * mt + (lane & 15);
    const bool tok = lane < 16 && at < norb && at != x && ((at > x) == (up != 0)) && rl[at] > j0;
    if (__ballot(tok) == 0) return;
    const int o1 = lane, o2 = lane + 64;
    const bool s1 = o1 < norb && o1 != x && rl[o1] > j0;
    const bool s2 = o2 < NP && o2 < norb && o2 != x && rl[o2] > j0;
    const unsigned long long sm0 = __ballot(s1), sm1 = __ballot(s2);
    unsigned km = 0;
#pragma unroll
    for (int ks = 0; ks < NP / 4; ++ks) {
        const unsigned long long sm = ks < 16 ? sm0 >> (4 * ks) : sm1 >> (4 * (ks - 16));
        if (sm & 0xfull) km |= 1u << ks;
    }
    const int n = lane & 15, kq = lane >> 4;
    const double *cv = c + (int64_t)v * ldc;
    auto next_ks = [&]() {
        if (!km) return -1;
        const int k = __ffs(km) - 1;
        km &= km - 1;
        return k;
    };
    // every lane loads from a valid address whatever the step (invalid
    // operands are selected to zero afterwards): with no loads under
    // branches the compiler can wait for one stage's loads only
    auto load = [&](int ks, double &a, double *b) {
        const int q = 4 * max(ks, 0) + kq;
        const int qc = min(q, norb - 1), ac = min(16 * mt + n, norb - 1);
        const double hv = hs[qc * norb + ac];
        a = (ks >= 0 && q < norb && 16 * mt + n < norb) ? hv : 0.0;
        const long long base = rb[qc];
        const int len = min(rl[qc], jlim);
        const bool rowok = ks >= 0 && q < norb && q != x && base >= 0;
        const double f = q < x ? 1.0 : -1.0;
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            const int j = j0 + 16 * nt + n;
            const bool ok = rowok && j < len;
            const double val = cv[ok ? base + j : 0];
            b[nt] = ok ? f * val : 0.0;
        }
    };
    v4d_ob acc[4];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) acc[nt] = v4d_ob{0.0, 0.0, 0.0, 0.0};
    // two K steps in flight: stages x and y ping-pong (no register copies)
    double ax, bx[4], ay, by[4];
    int kx = next_ks();
    load(kx, ax, bx);
    while (kx >= 0) {
        const int ky = next_ks();
        load(ky, ay, by);
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) acc[nt] = mfma16(ax, bx[nt], acc[nt]);
        if (ky < 0) break;
        kx = next_ks();
        load(kx, ax, bx);
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) acc[nt] = mfma16(ay, by[nt], acc[nt]);
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

template <int NT>
static void launch_ob_beta(const isci_ctx *cx, const SigmaArgs &A, int nv, const double *c, int64_t ldc, double *s,
                           int64_t lds, hipStream_t st)
{
    const double *hs = cx->d.hscreen;
    const int L = cx->L;
    // alpha rows by level: beta strings up to level 2 for level <= L - 2
    const int full_end = L >= 2 ? cx->sa.le[L - 2] : 0;
    if (full_end > 0)
        k_ob_beta_full<NT><<<dim3((unsigned)full_end, (unsigned)nv), 64 * NT, 0, st>>>(A, c, ldc, s, lds, hs, 0);
    const int ncap1 = cx->sa.nstr - full_end;   // rows whose beta strings stop at level 1 or 0
    if (ncap1 > 0)
        k_ob_beta_cap1<NT><<<dim3((unsigned)((ncap1 + 15) / 16), (unsigned)nv), 64 * NT, 0, st>>>(
            A, c, ldc, s, lds, hs, full_end, ncap1);
}

template <int NT>
static void launch_ob_alpha(const isci_ctx *cx, const SigmaArgs &A, int nv, const double *c, int64_t ldc, double *s,
                            int64_t lds, hipStream_t st)
{
    const double *hs = cx->d.hscreen;
    const int L = cx->L;
    // rows {q, x} hold beta strings up to level L - level({q, x}); for x
    // occupied every column reaches some row of level <= 1, for x virtual
    // the columns above the level-2 row length only reach {0,x}, {1,x}
    const int *le_b = cx->sb.le;
    const int jlim_occ = le_b[L];
    const int jlim_virt = L >= 2 ? le_b[L - 2] : 0;
    const int jtail = L >= 1 ? le_b[L - 1] : 0;
    const dim3 ga((unsigned)cx->norb, (unsigned)((jlim_occ + 63) / 64), (unsigned)nv);
    for (int up = 1; up >= 0; --up)
        k_ob_alpha<NT><<<ga, 64 * NT, 0, st>>>(A, c, ldc, s, lds, hs, up, jlim_occ, jlim_virt);
    if (jtail > jlim_virt && cx->norb > 2)
        k_ob_alpha_tail<<<dim3((unsigned)(cx->norb - 2), (unsigned)((jtail - jlim_virt + 255) / 256), (unsigned)nv), 256,
                          0, st>>>(A, c, ldc, s, lds, hs, jlim_virt, jtail);
}

bool onebody_mfma_ok(const isci_ctx *cx)
{
    return cx->d.hscreen && cx->na == 2 && cx->nb == 2 && cx->norb >= 3 && cx->norb <= kObMaxNorb &&
           cx->d.arow_base && cx->d.arow_len;
}

isci_status launch_onebody_mfma(const isci_ctx *cx, int nv, const double *c, int64_t ldc, double *s, int64_t lds,
                                hipStream_t st)
{
    const SigmaArgs A = sigma_args(cx);
    const int nt = (cx->norb + 15) / 16;
#define ISCI_OB_CASE(N)                                               \
    case N:                                                           \
        launch_ob_beta<N>(cx, A, nv, c, ldc, s, lds, st);             \
        launch_ob_alpha<N>(cx, A, nv, c, ldc, s, lds, st);            \
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
