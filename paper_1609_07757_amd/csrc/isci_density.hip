// One-body density matrices by spin (the paper's density-matrix subsection,
// Eq. d1): d[v][s][p][q] = <c_v| a+_{p s} a_{q s} |c_v>.
//
// The paper's density loop is the Hamiltonian's class loop with the
// integral fetch replaced by a product of two coefficients.  Here the
// replacement q -> p of one spin is read through its spectators: for a set
// S of the other n - 1 electrons, source S + q and target S + p, with sign
// (-1)^(members of S strictly between p and q) = s_S(p) s_S(q), s_S(x) =
// (-1)^(members of S below x).  For alpha the beta string is kept, so a
// connected pair contributes the dot product of the two alpha rows over the
// beta prefix both rows hold, and
//   D[p][q] = sum_S sum_b R_S[p][b] R_S[q][b],  R_S[x] = s_S(x) c(S + x, .)
// is a Gram matrix of the set's signed rows per spectator set (k_d1_gram),
// each row read once per set it belongs to.  For beta the same kernel runs
// on the vectors transposed into the spin-swapped layout (rows = beta
// strings, each holding the alpha strings of level <= L - its level, again
// a prefix), with the two spin tables exchanged; a beta replacement passes
// the alpha creators as an even pair and adds no sign.  Sets are split over
// a fixed number of groups whose partial sums k_d1_reduce adds in order, so
// the result is the same on every run.  Row starts follow from the level
// tables (rows of one level are contiguous and equally long).
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include <algorithm>
#include <vector>

#include "isci_device.h"
#include "isci_internal.h"

namespace isci {

namespace {

typedef double v4d_d2 __attribute__((ext_vector_type(4)));

constexpr int kD1Chunk = 8;       // vectors per pass (the handle keeps kD1Chunk * dim doubles for the transposed copy)
constexpr int kD2MaxNorb = 128;   // two-body densities: 8 norb^4 bytes per scratch buffer
constexpr int kD1MaxInner = 16;   // level boundary (inner orbitals) the one-body Gram form handles
constexpr int kGramGroups = 64;   // partial slabs (set groups x piece streams) summed in order by k_d1_reduce

// Fixed-order sum over the 64 lanes of a wave (butterfly).
__device__ inline double wave_sum(double x)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
}

// Start of row i of the layout whose rows are the strings of R (level
// order), the row of a level-k string holding the first C.le[L - k]
// strings of C: rows of one level are contiguous and equally long.
__device__ inline int64_t row_start(const SpinTab &R, const SpinTab &C, int L, int i, int k)
{
    int64_t base = 0;
    for (int l = 0; l < k; ++l) base += (int64_t)(R.lev_off[l + 1] - R.lev_off[l]) * C.le[L - l];
    return base + (int64_t)(i - R.lev_off[k]) * C.le[L - k];
}

// C(x, k) for 0 <= k <= 4 and x <= 255 in closed form: every product fits
// 32 unsigned bits (255 * 254 * 253 * 252 < 2^32) and the divisors are
// constants, so no integer division routine runs.
__device__ inline uint32_t binom_small(int x, int k)
{
    if (k < 0 || x < k) return 0u;
    const uint32_t u = (uint32_t)x;
    switch (k) {
    case 0: return 1u;
    case 1: return u;
    case 2: return u * (u - 1u) / 2u;
    case 3: return u * (u - 1u) * (u - 2u) / 6u;
    default: return u * (u - 1u) * (u - 2u) * (u - 3u) / 24u;
    }
}

// Index of an ascending string in (level, colex) order: the same rank as
// the library's string tables, with the closed-form binomials.
__device__ inline int rank_small(const int *o, const SpinTab &T)
{
    const int n = T.n, b = T.nocc;
    int ip = 0, io = 0;
    uint32_t rp = 0, ro = 0;
    for (int i = 0; i < n; ++i) {
        const int x = o[i];
        if (x >= b) { ++ip; rp += binom_small(x - b, ip); }
        else        { ++io; ro += binom_small(x, io); }
    }
    return T.lev_off[ip] + (int)(rp * (uint32_t)T.occ_mult[ip] + ro);
}

// Spectator set number s (colex) of k orbitals out of norb, ascending.
__device__ inline void unrank_set(uint32_t s, int k, int norb, int *S)
{
    for (int i = k; i >= 1; --i) {
        int x = i - 1;
        while (x + 1 < norb && binom_small(x + 1, i) <= s) ++x;
        S[i - 1] = x;
        s -= binom_small(x, i);
    }
}

// Gram form of the density: for a set S of n - 1 orbitals of the spin whose
// strings index the rows of A (A.sa), the rows R[q] = (-1)^{#S below q}
// c(S + q, .) (zero when S + q is not a string of the space) give
// D[p][q] += sum_b R[p][b] R[q][b] over the prefix both rows hold.  The rows
// of one set have two lengths only (S + q one level higher for q at or above
// the level boundary b), so phase 1 takes every row over the shorter length
// and phase 2 the pairs of the longer rows (q < b: rows 0..b-1 of tile 0;
// b = n <= 4 for the excitation hierarchy, b <= kD1MaxInner for a GAS
// boundary) over the rest.
// Workgroup (tile pair, g * P + p, vector v) sums its tile of the output over
// the sets g, g + G, ... and, of each, the phase-1 column pieces p, p + P, ...
// of W columns (phase 2 with piece stream p = 0), so that long row sets are
// shared out; it writes the tile to part[g * P + p][v] (norb x norb).
constexpr int kGT = 64;   // output tile edge (rows)
constexpr int kGK = 32;   // K step staged in LDS
constexpr int kGramPiece = kGK;   // phase-1 columns per piece

__global__ __launch_bounds__(256) void k_d1_gram(SigmaArgs A, const double *__restrict__ c, int64_t ldc, int nv,
                                                 int nsets, int G, int P, int W, int ntile, double *__restrict__ part)
{
    __shared__ double As[kGT][kGK + 1], Bs[kGT][kGK + 1];
    __shared__ int64_t roff[2][kGT];
    __shared__ double rsg[2][kGT];
    __shared__ int rlen[2][kGT];
    __shared__ int kmin_s, kmax_s;
    __shared__ double ph2[kD1MaxInner][kD1MaxInner];
    const int norb = A.norb, n = A.sa.n, tid = threadIdx.x;
    // tile pair number blockIdx.x of the upper triangle tp <= tq (row-major);
    // each set's Gram matrix is symmetric, so the lower tiles are not formed
    int tp = 0, rem = blockIdx.x;
    while (rem >= ntile - tp) { rem -= ntile - tp; ++tp; }
    const int tq = tp + rem;
    const int P0 = tp * kGT, Q0 = tq * kGT;
    const bool same = (tp == tq);
    const int gp = blockIdx.y, g = gp / P, pc = gp - g * P, v = blockIdx.z;
    const double *cv = c + (int64_t)v * ldc;
    // products on FP64 matrix cores: wave w forms output rows
    // [16 w, 16 w + 16) x 64 columns as four 16 x 16 tiles; element e of
    // lane l of tile nt is row 16 w + 4 e + l / 16, column 16 nt + l % 16
    const int w = tid >> 6, lane = tid & 63;
    v4d_d2 acc[4];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) acc[nt] = v4d_d2{0.0, 0.0, 0.0, 0.0};

    for (int set = g; set < nsets; set += G) {
        int S[ISCI_MAXN];
        unrank_set((uint32_t)set, n - 1, norb, S);
        if (tid == 0) { kmin_s = 0x7fffffff; kmax_s = 0; }
        __syncthreads();
        if (tid < 2 * kGT) {   // row tables of the two tiles
            const int side = tid / kGT, r = tid - side * kGT;
            const int q = (side ? Q0 : P0) + r;
            double sg = 0.0;
            int64_t off = 0;
            int len = 0;
            bool in = (q >= norb);
            int below = 0;
            for (int i = 0; i < n - 1; ++i) { in |= (S[i] == q); below += (S[i] < q); }
            if (!in) {
                int str[ISCI_MAXN], a = 0;
                bool put = false;
                for (int i = 0; i < n - 1; ++i) {
                    if (!put && q < S[i]) { str[a++] = q; put = true; }
                    str[a++] = S[i];
                }
                if (!put) str[a++] = q;
                const int lev = str_level(str, n, A.sa.nocc);
                if (lev <= A.sa.maxlev) {
                    len = A.sb.le[A.L - lev];
                    off = row_start(A.sa, A.sb, A.L, rank_small(str, A.sa), lev);
                    sg = (below & 1) ? -1.0 : 1.0;
                    atomicMin(&kmin_s, len);
                    atomicMax(&kmax_s, len);
                }
            }
            roff[side][r] = off;
            rsg[side][r] = sg;
            rlen[side][r] = len;
        }
        __syncthreads();
        const int K1 = (kmax_s == 0) ? 0 : kmin_s, K2 = kmax_s;
        // phase 1: every row over this workgroup's pieces of [0, K1)
        for (int kb = pc * W; kb < K1; kb += P * W)
        for (int k0 = kb, ke = min(kb + W, K1); k0 < ke; k0 += kGK) {
            for (int e = tid; e < kGT * kGK; e += 256) {
                const int r = e >> 5, kk = e & (kGK - 1), k = k0 + kk;
                const double sa = rsg[0][r];
                As[r][kk] = (sa != 0.0 && k < ke) ? sa * cv[roff[0][r] + k] : 0.0;
                if (!same) {
                    const double sb = rsg[1][r];
                    Bs[r][kk] = (sb != 0.0 && k < ke) ? sb * cv[roff[1][r] + k] : 0.0;
                }
            }
            __syncthreads();
            const double (*Bt)[kGK + 1] = same ? As : Bs;
#pragma unroll
            for (int ks = 0; ks < kGK / 4; ++ks) {
                const double a = As[16 * w + (lane & 15)][4 * ks + (lane >> 4)];
#pragma unroll
                for (int nt = 0; nt < 4; ++nt)
                    acc[nt] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, Bt[16 * nt + (lane & 15)][4 * ks + (lane >> 4)],
                                                                   acc[nt], 0, 0, 0);
            }
            __syncthreads();
        }
        // phase 2: pairs of the longer rows over [K1, min of their lengths)
        if (K2 > K1 && P0 == 0 && Q0 == 0 && pc == 0) {
            const int w = tid >> 6, lane = tid & 63;
            const int nl = max(4, A.sa.nocc);   // rows that may be long (<= kD1MaxInner)
            for (int pairi = w; pairi < nl * nl; pairi += 4) {
                const int i = pairi / nl, j = pairi - i * nl;
                const int le = min(rlen[0][i], rlen[1][j]);
                double part2 = 0.0;
                if (rsg[0][i] != 0.0 && rsg[1][j] != 0.0)
                    for (int k = K1 + lane; k < le; k += 64) part2 = fma(cv[roff[0][i] + k], cv[roff[1][j] + k], part2);
                part2 = wave_sum(part2) * rsg[0][i] * rsg[1][j];
                if (lane == 0) ph2[i][j] = part2;
            }
            __syncthreads();
            // rows and columns 0..nl-1 of the tile: wave 0, tile 0, element
            // e of lane l is row 4 e + l / 16, column l % 16
            if (w == 0)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int i = 4 * e + (lane >> 4), j = lane & 15;
                    if (i < nl && j < nl) acc[0][e] += ph2[i][j];
                }
        }
        __syncthreads();
    }
    double *out = part + ((int64_t)gp * nv + v) * norb * norb;
#pragma unroll
    for (int nt = 0; nt < 4; ++nt)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int p = P0 + 16 * w + 4 * e + (lane >> 4), q = Q0 + 16 * nt + (lane & 15);
            if (p < norb && q < norb) out[(int64_t)p * norb + q] = acc[nt][e];
        }
}

// d1[v0 + v][slot] = sum over g (in order) of part[g][v]; G = 0 writes zeros.
// Elements whose row tile lies below their column tile were not formed:
// they are read at the mirrored position (the sums are symmetric).
__global__ __launch_bounds__(256) void k_d1_reduce(const double *__restrict__ part, int G, int nv, int norb,
                                                   double *__restrict__ d1, int slot, int v0)
{
    const int64_t nn = (int64_t)norb * norb;
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= nv * nn) return;
    const int v = (int)(t / nn);
    const int64_t pq = t - v * nn;
    const int p = (int)(pq / norb), q = (int)(pq - (int64_t)p * norb);
    const int64_t src = (p / kGT > q / kGT) ? (int64_t)q * norb + p : pq;
    double s = 0.0;
    for (int g = 0; g < G; ++g) s += part[((int64_t)g * nv + v) * nn + src];
    d1[((int64_t)(v0 + v) * 2 + slot) * nn + pq] = s;
}

// Vectors v < nv of c into the spin-swapped layout (row = beta string j,
// position = alpha string ia; leading dimension dim).  The determinants of
// one (alpha level ka, beta level kb) pair form a dense block in both
// layouts: in c, row ia starts at baseA + (ia - first) * le_b[L - ka]; in
// cT, row j starts at baseB + (j - first) * le_a[L - kb].  Each workgroup
// moves one 32 x 32 tile of one block through LDS, reading along beta and
// writing along alpha, so both sides are coalesced.  Workgroups are
// numbered block by block (ka outer, kb inner), tile rows outer.
__global__ __launch_bounds__(256) void k_d1_transpose(SigmaArgs A, const double *__restrict__ c, int64_t ldc, int nv,
                                                      int64_t dim, double *__restrict__ cT)
{
    __shared__ double tile[32][33];
    int b = blockIdx.x, ka = 0, kb = 0, ntj = 1;
    for (ka = 0; ka <= A.sa.maxlev; ++ka) {
        bool found = false;
        for (kb = 0; kb <= min(A.L - ka, A.sb.maxlev); ++kb) {
            const int na = A.sa.lev_off[ka + 1] - A.sa.lev_off[ka], nb = A.sb.lev_off[kb + 1] - A.sb.lev_off[kb];
            ntj = (nb + 31) >> 5;
            const int nt = ((na + 31) >> 5) * ntj;
            if (b < nt) { found = true; break; }
            b -= nt;
        }
        if (found) break;
    }
    if (ka > A.sa.maxlev) return;   // beyond the last tile (not launched)
    const int a0 = A.sa.lev_off[ka], a1 = A.sa.lev_off[ka + 1];
    const int j0 = A.sb.lev_off[kb], j1 = A.sb.lev_off[kb + 1];
    const int ia0 = a0 + (b / ntj) * 32, jb0 = j0 + (b % ntj) * 32;
    const int64_t baseA = row_start(A.sa, A.sb, A.L, a0, ka), strideA = A.sb.le[A.L - ka];
    const int64_t baseB = row_start(A.sb, A.sa, A.L, j0, kb), strideB = A.sa.le[A.L - kb];
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    for (int v = 0; v < nv; ++v) {
        const double *cv = c + (int64_t)v * ldc;
        double *tv = cT + (int64_t)v * dim;
        for (int r = ty; r < 32; r += 8) {
            const int ia = ia0 + r, j = jb0 + tx;
            if (ia < a1 && j < j1) tile[r][tx] = cv[baseA + (int64_t)(ia - a0) * strideA + j];
        }
        __syncthreads();
        for (int r = ty; r < 32; r += 8) {
            const int j = jb0 + r, ia = ia0 + tx;
            if (ia < a1 && j < j1) tv[baseB + (int64_t)(j - j0) * strideB + ia] = tile[tx][r];
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------- two-body
// Two-body density matrices (Eq. d2) for two electrons of each spin, from
// Gram matrices of rows of the CI vector:
//  * same spin: a+_p a+_r a_s a_q maps the string {q, s} to {p, r}, so
//    D2ss[p][q][r][s] = eps(p, r) eps(q, s) G[{p,r}][{q,s}] with
//    eps(a, b) = +1 for a < b, -1 for a > b (0 for a == b), and G the Gram
//    matrix of the rows of the string's spin (each row zero beyond its
//    length, so a pair of rows meets over their common prefix): rows of c
//    for alpha, rows of the spin-swapped copy for beta (a beta word passes
//    the alpha creators with four operators: no sign);
//  * alpha-beta: a+_{p a} a+_{r b} a_{s b} a_{q a} = E^a_pq E^b_rs, so with
//    the pair tensor M[(p, r)][(x, y)] = sgn(p - x) sgn(r - y) c({x, p},
//    {y, r}) (zero where x == p, y == r or the determinant is outside the
//    space), D2ab[p][q][r][s] = sum_{x, y} M[(p, r)][(x, y)] M[(q, s)][(x, y)],
//    the Gram matrix of the rows of M.

constexpr int kG2T = 64;   // Gram output tile edge
constexpr int kG2K = 16;   // K step staged in LDS

// G[i][j] = sum_k R_i[k] R_j[k] for rows R_i = src[rstart[i] + k], k <
// rlen[i] (zero beyond), i, j < nrow, on FP64 matrix cores: workgroup =
// one 64 x 64 tile of the upper triangle (tile pairs ti <= tj), wave w the
// 16 rows [16 w, 16 w + 16) x 64 columns; K in steps of 16 through LDS; both
// G[i][j] and G[j][i] written (the same sum in the same order).
__global__ __launch_bounds__(256) void k_gram_rows(const double *__restrict__ src, const int64_t *__restrict__ rstart,
                                                   const int *__restrict__ rlen, int nrow, int ntile,
                                                   double *__restrict__ G, int64_t ldg)
{
    __shared__ double As[kG2T][kG2K + 1], Bs[kG2T][kG2K + 1];
    __shared__ int kmax_s;
    int ti = 0, rem = blockIdx.x;
    while (rem >= ntile - ti) { rem -= ntile - ti; ++ti; }
    const int tj = ti + rem;
    const int I0 = ti * kG2T, J0 = tj * kG2T;
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    if (tid == 0) kmax_s = 0;
    __syncthreads();
    if (tid < 2 * kG2T) {
        const int r = (tid < kG2T ? I0 : J0) + (tid & (kG2T - 1));
        if (r < nrow) atomicMax(&kmax_s, rlen[r]);
    }
    __syncthreads();
    const int kmax = kmax_s;
    v4d_d2 acc[4];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) acc[nt] = v4d_d2{0.0, 0.0, 0.0, 0.0};
    // 2 x 64 x 16 elements per K step, eight per thread (16 consecutive k
    // of a row); the next step's elements are loaded into registers while
    // the current step's products run
    long long rs8[8];
    int rl8[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        const int e = tid + 256 * u;           // < 2048
        const int side = e >> 10, r = (e >> 4) & 63;
        const int row = (side ? J0 : I0) + r;
        rs8[u] = row < nrow ? rstart[row] : 0;
        rl8[u] = row < nrow ? rlen[row] : 0;
    }
    double pre[8];
    auto fetch = [&](int k0) {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int k = k0 + ((tid + 256 * u) & 15);
            pre[u] = k < rl8[u] ? src[rs8[u] + k] : 0.0;
        }
    };
    fetch(0);
    for (int k0 = 0; k0 < kmax; k0 += kG2K) {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = tid + 256 * u;
            const int side = e >> 10, r = (e >> 4) & 63, kk = e & 15;
            if (side) Bs[r][kk] = pre[u]; else As[r][kk] = pre[u];
        }
        __syncthreads();
        if (k0 + kG2K < kmax) fetch(k0 + kG2K);
#pragma unroll
        for (int ks = 0; ks < kG2K / 4; ++ks) {
            const double a = As[16 * w + (lane & 15)][4 * ks + (lane >> 4)];
#pragma unroll
            for (int nt = 0; nt < 4; ++nt)
                acc[nt] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, Bs[16 * nt + (lane & 15)][4 * ks + (lane >> 4)],
                                                               acc[nt], 0, 0, 0);
        }
        __syncthreads();
    }
    // element g of lane l: row 4 g + l / 16, column l % 16 of the 16 x 16 tile
#pragma unroll
    for (int nt = 0; nt < 4; ++nt)
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            const int i = I0 + 16 * w + 4 * g + (lane >> 4), j = J0 + 16 * nt + (lane & 15);
            if (i < nrow && j < nrow) {
                G[(int64_t)i * ldg + j] = acc[nt][g];
                G[(int64_t)j * ldg + i] = acc[nt][g];
            }
        }
}

// M[(p * n + r) * n * n + x * n + y] = sgn(p - x) sgn(r - y) c({x, p}, {y, r})
// for every determinant of the space (one thread per determinant writes its
// four role entries; M was zeroed before)
__global__ __launch_bounds__(256) void k_d2_pair_tensor(const uint32_t *__restrict__ astr,
                                                        const uint32_t *__restrict__ bstr,
                                                        const int64_t *__restrict__ rowstart, int nstr_a,
                                                        const double *__restrict__ c, int64_t dim, int n,
                                                        double *__restrict__ M)
{
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= dim) return;
    // row of determinant t: binary search of the row starts
    int lo = 0, hi = nstr_a;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (rowstart[mid] <= t) lo = mid; else hi = mid;
    }
    const int ia = lo, jb = (int)(t - rowstart[ia]);
    const uint32_t as = astr[ia], bs = bstr[jb];
    const int a0 = as & 0xff, a1 = (as >> 8) & 0xff, b0 = bs & 0xff, b1 = (bs >> 8) & 0xff;
    const double v = c[t];
    const int64_t nn = (int64_t)n * n;
#pragma unroll
    for (int ra = 0; ra < 2; ++ra) {
        const int x = ra ? a1 : a0, p = ra ? a0 : a1;   // spectator, active
#pragma unroll
        for (int rb = 0; rb < 2; ++rb) {
            const int y = rb ? b1 : b0, r = rb ? b0 : b1;
            const double f = (ra ^ rb) ? -1.0 : 1.0;    // sgn(p - x) sgn(r - y)
            M[((int64_t)p * n + r) * nn + (int64_t)x * n + y] = f * v;
        }
    }
}

// d2 block of one vector from a same-spin Gram matrix G (ldg = nstr):
// D[p][q][r][s] = eps(p, r) eps(q, s) G[pidx(p, r)][pidx(q, s)]
__global__ __launch_bounds__(256) void k_d2_expand_same(const double *__restrict__ G, int64_t ldg,
                                                        const int *__restrict__ pidx, int n,
                                                        double *__restrict__ D)
{
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t nn = (int64_t)n * n;
    if (t >= nn * nn) return;
    const int p = (int)(t / (nn * n)), q = (int)((t / nn) % n), r = (int)((t / n) % n), s = (int)(t % n);
    double v = 0.0;
    if (p != r && q != s) {
        const int I = pidx[p * n + r], J = pidx[q * n + s];
        if (I >= 0 && J >= 0) {
            const double e = ((p < r) == (q < s)) ? 1.0 : -1.0;
            v = e * G[(int64_t)I * ldg + J];
        }
    }
    D[t] = v;
}

// alpha-beta block of one vector: D[p][q][r][s] = G[(p, r)][(q, s)]
__global__ __launch_bounds__(256) void k_d2_expand_ab(const double *__restrict__ G, int n, double *__restrict__ D)
{
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t nn = (int64_t)n * n;
    if (t >= nn * nn) return;
    const int p = (int)(t / (nn * n)), q = (int)((t / nn) % n), r = (int)((t / n) % n), s = (int)(t % n);
    D[t] = G[((int64_t)p * n + r) * nn + (int64_t)q * n + s];
}

__global__ __launch_bounds__(256) void k_d2_zero(double *__restrict__ p, int64_t n)
{
    for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < n; t += (int64_t)gridDim.x * 256) p[t] = 0.0;
}

}  // namespace

}  // namespace isci

namespace isci {
namespace {

// Workgroups of k_d1_transpose: 32 x 32 tiles of every (alpha level, beta
// level) block of the space.
unsigned transpose_tiles(const isci_ctx *h)
{
    unsigned n = 0;
    for (int ka = 0; ka <= h->sa.maxlev; ++ka)
        for (int kb = 0; kb <= std::min(h->L - ka, h->sb.maxlev); ++kb) {
            const int na = h->sa.lev_off[ka + 1] - h->sa.lev_off[ka], nb = h->sb.lev_off[kb + 1] - h->sb.lev_off[kb];
            n += (unsigned)(((na + 31) / 32) * ((nb + 31) / 32));
        }
    return n;
}

// One spin block of vectors v0 .. v0 + nv - 1 (nv <= kD1Chunk): the Gram
// kernel over the spectator sets of A's row spin, then the ordered sum of
// its set groups into slot `slot` of d1.  A spin without electrons has no
// sets and gets zeros (c is not read).
isci_status gram_pass(const SigmaArgs &A, const double *c, int64_t ldc, int nv, double *part, double *d1, int slot,
                      int v0, hipStream_t s)
{
    const int norb = A.norb, n = A.sa.n;
    const long long nsets = (n >= 1) ? binom(norb, n - 1) : 0;
    // set groups G and column-piece streams P with G * P <= kGramGroups slabs
    const int G = (int)std::min<long long>(nsets, 16);
    const int P = G > 0 ? kGramGroups / G : 0;
    const int ntile = (norb + kGT - 1) / kGT;
    if (G > 0) {
        k_d1_gram<<<dim3((unsigned)(ntile * (ntile + 1) / 2), (unsigned)(G * P), (unsigned)nv), 256, 0, s>>>(
            A, c, ldc, nv, (int)nsets, G, P, kGramPiece, ntile, part);
        ISCI_HIP(hipGetLastError());
    }
    const int64_t tot = (int64_t)nv * norb * norb;
    k_d1_reduce<<<(unsigned)((tot + 255) / 256), 256, 0, s>>>(part, G * P, nv, norb, d1, slot, v0);
    ISCI_HIP(hipGetLastError());
    return ISCI_OK;
}

}  // namespace
}  // namespace isci

using namespace isci;

// Scratch of isci_density1_noalloc: a file-scope device array that the code
// object brings along (each GPU holds its own copy until the process ends).
// Host code never uses its name as an address: the per-device address comes
// from hipGetSymbolAddress, taken once per device with that device current.
constexpr size_t kScratchBytes = (size_t)64 << 20;
constexpr size_t kScratchDoubles = kScratchBytes / sizeof(double);
static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {

constexpr int kScratchMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[kScratchMaxDevices] = {};

// device address of `scratch` on device dev (the current device)
isci_status scratch_address(int dev, double **out)
{
    if (dev < 0 || dev >= kScratchMaxDevices) { set_error("device index out of range"); return ISCI_E_UNSUPPORTED; }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        double *p = nullptr;
        const hipError_t e = hipGetSymbolAddress((void **)&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return ISCI_OK;
}

// common argument checks of both density entry points
isci_status density_args(isci_handle h, int nvec, const double *c, int64_t ldc, const double *d1)
{
    if (!h || !c || !d1) { set_error("NULL argument"); return ISCI_E_INVALID; }
    if (nvec < 1 || nvec > 65535) { set_error("nvec outside 1..65535"); return ISCI_E_INVALID; }
    if (ldc < h->dim) { set_error("leading dimension < dim"); return ISCI_E_INVALID; }
    const int64_t nd = (int64_t)nvec * 2 * h->norb * h->norb;
    const char *c0 = (const char *)c, *c1 = (const char *)(c + (int64_t)(nvec - 1) * ldc + h->dim);
    const char *d0 = (const char *)d1, *e1 = (const char *)(d1 + nd);
    if (c0 < e1 && d0 < c1) { set_error("density overlaps c"); return ISCI_E_INVALID; }
    if (h->sa.nocc > kD1MaxInner || h->sb.nocc > kD1MaxInner) {
        // the Gram form's second phase holds the pairs of a spectator set's
        // inner rows (those below the level boundary) in a 16 x 16 block
        set_error("isci_density1: a GAS boundary above 16 orbitals is not supported");
        return ISCI_E_UNSUPPORTED;
    }
    if (h->nb > 0) {
        // the spin-swapped layout (rows = beta strings) holds every determinant
        int64_t tot = 0;
        for (int j = 0; j < h->sb.nstr; ++j) tot += h->sa.le[h->L - h->h_blev[j]];
        if (tot != h->dim) { set_error("isci_density1: transposed layout size mismatch"); return ISCI_E_INVALID; }
    }
    return ISCI_OK;
}

// vectors [0, nvec) in passes of nvc: both spin blocks, partial slabs in
// part, the transposed copy in cT
isci_status density_passes(isci_handle h, int nvec, const double *c, int64_t ldc, double *d1, int nvc, double *part,
                           double *cT, hipStream_t stream)
{
    const SigmaArgs A = sigma_args(h);
    SigmaArgs T = A;   // the spin-swapped layout: beta strings index the rows
    T.sa = A.sb;
    T.sb = A.sa;
    T.astr = A.bstr;
    T.bstr = A.astr;
    T.alev = A.blev;
    T.blev = A.alev;
    for (int v0 = 0; v0 < nvec; v0 += nvc) {
        const int nv = std::min(nvc, nvec - v0);
        ISCI_CHECK(gram_pass(A, c + (int64_t)v0 * ldc, ldc, nv, part, d1, 0, v0, stream));
        if (h->nb > 0) {
            k_d1_transpose<<<transpose_tiles(h), 256, 0, stream>>>(A, c + (int64_t)v0 * ldc, ldc, nv, h->dim, cT);
            ISCI_HIP(hipGetLastError());
        }
        ISCI_CHECK(gram_pass(T, cT, h->dim, nv, part, d1, 1, v0, stream));
    }
    return ISCI_OK;
}

}  // namespace

extern "C" {

isci_status isci_density1(isci_handle h, int nvec, const double *c, int64_t ldc, double *d1, hipStream_t stream)
{
    ISCI_CHECK(density_args(h, nvec, c, ldc, d1));
    if (!h->d.d1part) {
        h->d.d1part = (double *)dev_alloc(h, sizeof(double) * kGramGroups * kD1Chunk * (size_t)h->norb * h->norb);
        if (!h->d.d1part) { set_error("isci_density1: out of device memory"); return ISCI_E_OOM; }
    }
    if (h->nb > 0 && !h->d.d1T) {
        double *buf = (double *)dev_alloc(h, sizeof(double) * kD1Chunk * (size_t)h->dim);
        if (!buf) { set_error("isci_density1: out of device memory"); return ISCI_E_OOM; }
        h->d.d1T = buf;
    }
    return density_passes(h, nvec, c, ldc, d1, kD1Chunk, h->d.d1part, h->d.d1T, stream);
}

isci_status isci_density1_noalloc(isci_handle h, int nvec, const double *c, int64_t ldc, double *d1,
                                  hipStream_t stream)
{
    ISCI_CHECK(density_args(h, nvec, c, ldc, d1));
    int dev = -1;
    ISCI_HIP(hipGetDevice(&dev));
    if (dev != h->device) {
        set_error("isci_density1_noalloc: the current device is not the handle's device");
        return ISCI_E_INVALID;
    }
    // vectors per pass: partial slabs (64 norb^2 doubles) and the transposed
    // copy (dim doubles, with beta electrons) of each must fit the scratch
    const size_t per_vec = (size_t)kGramGroups * h->norb * h->norb + (h->nb > 0 ? (size_t)h->dim : 0);
    const size_t fit = kScratchDoubles / per_vec;
    if (fit < 1) {
        set_error("isci_density1_noalloc: one vector needs " + std::to_string(per_vec * sizeof(double)) +
                  " bytes of scratch; the static scratch holds " + std::to_string(kScratchBytes) +
                  " (use isci_density1)");
        return ISCI_E_UNSUPPORTED;
    }
    const int nvc = (int)std::min<size_t>(kD1Chunk, fit);
    double *sp = nullptr;
    ISCI_CHECK(scratch_address(dev, &sp));
    double *part = sp;
    double *cT = sp + (size_t)kGramGroups * nvc * h->norb * h->norb;
    return density_passes(h, nvec, c, ldc, d1, nvc, part, cT, stream);
}

isci_status isci_density2(isci_handle h, int nvec, const double *c, int64_t ldc, double *d2, hipStream_t stream)
{
    if (!h || !c || !d2) { set_error("NULL argument"); return ISCI_E_INVALID; }
    if (nvec < 1 || nvec > 65535) { set_error("nvec outside 1..65535"); return ISCI_E_INVALID; }
    if (ldc < h->dim) { set_error("leading dimension < dim"); return ISCI_E_INVALID; }
    const int n = h->norb;
    const int64_t n4 = (int64_t)n * n * n * n;
    {
        const char *c0 = (const char *)c, *c1 = (const char *)(c + (int64_t)(nvec - 1) * ldc + h->dim);
        const char *d0 = (const char *)d2, *e1 = (const char *)(d2 + (int64_t)nvec * 3 * n4);
        if (c0 < e1 && d0 < c1) { set_error("density overlaps c"); return ISCI_E_INVALID; }
    }
    if (h->na != 2 || h->nb != 2) {
        set_error("isci_density2: two electrons of each spin only");
        return ISCI_E_UNSUPPORTED;
    }
    if (n > kD2MaxNorb) {
        set_error("isci_density2: at most 128 orbitals (the pair tensor and Gram matrix take 8 norb^4 bytes each)");
        return ISCI_E_UNSUPPORTED;
    }
    const int na = h->sa.nstr, nb = h->sb.nstr, nn = n * n;
    if (!h->d.d2G) {
        // spin-swapped layout: rows = beta strings holding alpha prefixes
        std::vector<int64_t> rs((size_t)na + nb + nn);
        std::vector<int> rl(rs.size());
        for (int i = 0; i < na; ++i) {
            rs[i] = h->h_rowstart[i];
            rl[i] = (int)(h->h_rowstart[i + 1] - h->h_rowstart[i]);
        }
        int64_t acc = 0;
        for (int j = 0; j < nb; ++j) {
            rs[na + j] = acc;
            rl[na + j] = h->sa.le[h->L - h->h_blev[j]];
            acc += rl[na + j];
        }
        if (acc != h->dim) { set_error("isci_density2: transposed layout size mismatch"); return ISCI_E_INVALID; }
        for (int t = 0; t < nn; ++t) {
            rs[na + nb + t] = (int64_t)t * nn;
            rl[na + nb + t] = nn;
        }
        const int64_t gsz = std::max<int64_t>(std::max<int64_t>((int64_t)na * na, (int64_t)nb * nb), n4);
        h->d.d2G = (double *)dev_alloc(h, sizeof(double) * (size_t)gsz);
        h->d.d2M = (double *)dev_alloc(h, sizeof(double) * (size_t)n4);
        h->d.d2cT = (double *)dev_alloc(h, sizeof(double) * (size_t)h->dim);
        int64_t *drs = (int64_t *)dev_alloc(h, sizeof(int64_t) * rs.size());
        int *drl = (int *)dev_alloc(h, sizeof(int) * rl.size());
        if (!h->d.d2G || !h->d.d2M || !h->d.d2cT || !drs || !drl) {
            set_error("isci_density2: out of device memory");
            return ISCI_E_OOM;
        }
        ISCI_HIP(hipMemcpyAsync(drs, rs.data(), sizeof(int64_t) * rs.size(), hipMemcpyHostToDevice, stream));
        ISCI_HIP(hipMemcpyAsync(drl, rl.data(), sizeof(int) * rl.size(), hipMemcpyHostToDevice, stream));
        ISCI_HIP(hipStreamSynchronize(stream));   // the host tables die here
        h->d.d2rs = drs;
        h->d.d2rl = drl;
    }
    const SigmaArgs A = sigma_args(h);
    double *G = h->d.d2G, *M = h->d.d2M;
    auto gram = [&](const double *src, int roff, int nrow, hipStream_t st) {
        const int nt = (nrow + kG2T - 1) / kG2T;
        k_gram_rows<<<(unsigned)(nt * (nt + 1) / 2), 256, 0, st>>>(src, h->d.d2rs + roff, h->d.d2rl + roff, nrow, nt, G,
                                                                   nrow);
    };
    const unsigned ge = (unsigned)((n4 + 255) / 256);
    for (int v = 0; v < nvec; ++v) {
        const double *cv = c + (int64_t)v * ldc;
        double *dv = d2 + (int64_t)v * 3 * n4;
        // alpha-alpha: Gram of the rows of c
        gram(cv, 0, na, stream);
        k_d2_expand_same<<<ge, 256, 0, stream>>>(G, na, h->d.apidx, n, dv);
        // beta-beta: Gram of the rows of the spin-swapped copy
        k_d1_transpose<<<transpose_tiles(h), 256, 0, stream>>>(A, cv, ldc, 1, h->dim, h->d.d2cT);
        gram(h->d.d2cT, na, nb, stream);
        k_d2_expand_same<<<ge, 256, 0, stream>>>(G, nb, h->d.bpidx, n, dv + 2 * n4);
        // alpha-beta: Gram of the rows of the pair tensor
        k_d2_zero<<<(unsigned)std::min<int64_t>(4096, (n4 + 255) / 256), 256, 0, stream>>>(M, n4);
        k_d2_pair_tensor<<<(unsigned)((h->dim + 255) / 256), 256, 0, stream>>>(A.astr, A.bstr, A.rowstart, na, cv, h->dim,
                                                                               n, M);
        gram(M, na + nb, nn, stream);
        k_d2_expand_ab<<<ge, 256, 0, stream>>>(G, n, dv + n4);
        ISCI_HIP(hipGetLastError());
    }
    return ISCI_OK;
}

}  // extern "C"
