// libisci sigma kernels (Eq. sigma), FP64.
//
// Owner-computes: a workgroup owns one alpha row (one alpha target string
// Ia) and a chunk of its beta targets Ib, one thread per target
// determinant.  Every contribution to sigma(Ia, Ib) is accumulated in that
// thread's registers and written once, so the result is deterministic and
// needs no atomics.
//
// Each class loops over kept integral units first and over vector
// elements inside (the integral-outer order of the paper's second part,
// section "The ISCI Algorithm"); screened units never enter the loops.
// The string algebra of Eqs. four..last is done on the fly:
//   E_pq |X u {q}> = eps(X,q) eps(X,p) |X u {p}>,  eps(X,o) = (-1)^#{x in X : x < o}
// (a creator moved past the smaller spectators), so the alpha-beta phase
// factorises into an alpha and a beta phase (the separability of
// Eq. final), and the same-spin unit [(pq|rs) - (ps|rq)] carries
// eta(Y,p,r) eta(Y,q,s) with eta(Y,q,s) = eps(Y,q) eps(Y,s).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "isci_device.h"
#include "isci_internal.h"

namespace isci {

// phase (-1)^#{x in o, x not at positions i or j, x < p}
__device__ inline int phase_below2(const int *o, int n, int i, int j, int p)
{
    int c = 0;
    for (int k = 0; k < n; ++k) c += (k != i) & (k != j) & (o[k] < p);
    return (c & 1) ? -1 : 1;
}

// Y = o without positions i, j; insert q > s; returns false on a clash
__device__ inline bool replace_two(const int *o, int n, int i, int j, int q, int s, int *out)
{
    int k = 0;
    bool ps = false, pq = false;
    for (int t = 0; t < n; ++t) {
        if (t == i || t == j) continue;
        int x = o[t];
        if (x == q || x == s) return false;
        if (!ps && s < x) { out[k++] = s; ps = true; }
        if (!pq && q < x) { out[k++] = q; pq = true; }
        out[k++] = x;
    }
    if (!ps) out[k++] = s;
    if (!pq) out[k++] = q;
    return true;
}

// sigma for the target determinant (ia, ib) of one instance, vectors v < nv
template <int NV>
__device__ __forceinline__ void sigma_target(const SigmaArgs &A, int ia, int ib, int nv,
                                             const double *__restrict__ c, int64_t ldc,
                                             double *__restrict__ sg, int64_t lds)
{
    const int la = A.alev[ia];
    const int L = A.L;
    const int rlen = A.sb.le[L - la];
    if (ib >= rlen) return;
    const int na = A.sa.n, nb = A.sb.n, norb = A.norb;
    int ao[ISCI_MAXN], bo[ISCI_MAXN], jo[ISCI_MAXN];
    unpack_str(A.astr[ia], na, ao);
    unpack_str(A.bstr[ib], nb, bo);
    const int lb = A.blev[ib];
    const int64_t myrow = A.rowstart[ia];

    double acc[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[v] = 0.0;

    // ---------------- one-body alpha: sum_q h_pq E^a_pq, p in Ia
    for (int i = 0; i < na; ++i) {
        const int p = ao[i];
        const int sp = phase_below(ao, na, i, p);
        for (int e = A.h_off[p]; e < A.h_off[p + 1]; ++e) {
            const int q = A.h_q[e];
            if (!replace_one(ao, na, i, q, jo)) continue;
            const int lj = str_level(jo, na, A.sa.nocc);
            if (lj + lb > L) continue;
            const int ja = str_index(jo, A.sa);
            const double f = (sp * phase_below(ao, na, i, q)) * A.h_v[e];
            const double *src = c + A.rowstart[ja] + ib;
#pragma unroll
            for (int v = 0; v < NV; ++v)
                if (v < nv) acc[v] += f * src[v * ldc];
        }
    }
    // ---------------- same-spin alpha: pairs p > r in Ia
    for (int i = 0; i < na; ++i)
        for (int j = i + 1; j < na; ++j) {
            const int r = ao[i], p = ao[j];
            const int eta_pr = phase_below2(ao, na, i, j, p) * phase_below2(ao, na, i, j, r);
            const int P = p * (p - 1) / 2 + r;
            for (int e = A.ss_off[P]; e < A.ss_off[P + 1]; ++e) {
                const int q = A.ss_qs[e] >> 8, s = A.ss_qs[e] & 0xff;
                if (!replace_two(ao, na, i, j, q, s, jo)) continue;
                const int lj = str_level(jo, na, A.sa.nocc);
                if (lj + lb > L) continue;
                const int ja = str_index(jo, A.sa);
                const int eta_qs = phase_below2(ao, na, i, j, q) * phase_below2(ao, na, i, j, s);
                const double f = (eta_pr * eta_qs) * A.ss_v[e];
                const double *src = c + A.rowstart[ja] + ib;
#pragma unroll
                for (int v = 0; v < NV; ++v)
                    if (v < nv) acc[v] += f * src[v * ldc];
            }
        }
    // ---------------- one-body beta
    const int bmax = A.sb.le[L - la];
    for (int i = 0; i < nb; ++i) {
        const int r = bo[i];
        const int sr = phase_below(bo, nb, i, r);
        for (int e = A.h_off[r]; e < A.h_off[r + 1]; ++e) {
            const int s = A.h_q[e];
            if (!replace_one(bo, nb, i, s, jo)) continue;
            const int jb = str_index(jo, A.sb);
            if (jb >= bmax) continue;
            const double f = (sr * phase_below(bo, nb, i, s)) * A.h_v[e];
            const double *src = c + myrow + jb;
#pragma unroll
            for (int v = 0; v < NV; ++v)
                if (v < nv) acc[v] += f * src[v * ldc];
        }
    }
    // ---------------- same-spin beta
    for (int i = 0; i < nb; ++i)
        for (int j = i + 1; j < nb; ++j) {
            const int r = bo[i], p = bo[j];
            const int eta_pr = phase_below2(bo, nb, i, j, p) * phase_below2(bo, nb, i, j, r);
            const int P = p * (p - 1) / 2 + r;
            for (int e = A.ss_off[P]; e < A.ss_off[P + 1]; ++e) {
                const int q = A.ss_qs[e] >> 8, s = A.ss_qs[e] & 0xff;
                if (!replace_two(bo, nb, i, j, q, s, jo)) continue;
                const int jb = str_index(jo, A.sb);
                if (jb >= bmax) continue;
                const int eta_qs = phase_below2(bo, nb, i, j, q) * phase_below2(bo, nb, i, j, s);
                const double f = (eta_pr * eta_qs) * A.ss_v[e];
                const double *src = c + myrow + jb;
#pragma unroll
                for (int v = 0; v < NV; ++v)
                    if (v < nv) acc[v] += f * src[v * ldc];
            }
        }
    // ---------------- alpha-beta: sum (pq|rs) E^a_pq E^b_rs
    int jb_o[ISCI_MAXN];
    for (int i = 0; i < na; ++i) {
        const int p = ao[i];
        const int sp = phase_below(ao, na, i, p);
        for (int e1 = A.pq_off[p]; e1 < A.pq_off[p + 1]; ++e1) {
            const int q = A.pq_q[e1];
            if (!replace_one(ao, na, i, q, jo)) continue;
            const int lj = str_level(jo, na, A.sa.nocc);
            if (lj > L) continue;
            const int ja = str_index(jo, A.sa);
            const int lenJ = A.sb.le[L - lj];
            const int sa = sp * phase_below(ao, na, i, q);
            const double *rowJ = c + A.rowstart[ja];
            const long long base = ((long long)p * norb + q) * norb;
            for (int k = 0; k < nb; ++k) {
                const int r = bo[k];
                const int sr = sa * phase_below(bo, nb, k, r);
                const long long e0 = A.ab_off[base + r], e1e = A.ab_off[base + r + 1];
                for (long long e = e0; e < e1e; ++e) {
                    const int s = A.ab_s[e];
                    if (!replace_one(bo, nb, k, s, jb_o)) continue;
                    const int jb = str_index(jb_o, A.sb);
                    if (jb >= lenJ) continue;
                    const double f = (sr * phase_below(bo, nb, k, s)) * A.ab_v[e];
                    const double *src = rowJ + jb;
#pragma unroll
                    for (int v = 0; v < NV; ++v)
                        if (v < nv) acc[v] += f * src[v * ldc];
                }
            }
        }
    }
    double *dst = sg + myrow + ib;
#pragma unroll
    for (int v = 0; v < NV; ++v)
        if (v < nv) dst[v * lds] = acc[v];
}


// Two electrons of each spin.  Strings are orbital pairs; E_pq takes
// {x, q} to {x, p} with phase sgn(p - x) sgn(q - x) (x the spectator), and
// the same-spin unit maps {s < q} to {r < p} with phase +1.  String
// indices come from the pair tables, so no string algebra remains in the
// loops.
__device__ __forceinline__ int sgn2(int a, int b) { return (a > b) ? 1 : -1; }   // sgn(a - b), a != b

template <int NV>
__device__ __forceinline__ void sigma_target_n2(const SigmaArgs &A, int ia, int ib, int nv,
                                                const double *__restrict__ c, int64_t ldc,
                                                double *__restrict__ sg, int64_t lds)
{
    const int la = A.alev[ia];
    const int L = A.L;
    const int rlen = A.sb.le[L - la];
    if (ib >= rlen) return;
    const int norb = A.norb;
    const uint32_t as = A.astr[ia], bs = A.bstr[ib];
    const int a0 = as & 0xff, a1 = (as >> 8) & 0xff;
    const int b0 = bs & 0xff, b1 = (bs >> 8) & 0xff;
    const int lb = A.blev[ib];
    const int64_t myrow = A.rowstart[ia];
    const int *__restrict__ apx = A.apidx;
    const int *__restrict__ bpx = A.bpidx;

    double acc[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[v] = 0.0;

    const bool do1 = A.classes & 1, doss = A.classes & 2, doab = A.classes & 4;
    // one-body alpha
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const int p = i ? a1 : a0, x = i ? a0 : a1;
        const int sp = sgn2(p, x);
        for (int e = do1 ? A.h_off[p] : 0; e < (do1 ? A.h_off[p + 1] : 0); ++e) {
            const int q = A.h_q[e];
            if (q == x) continue;
            const int ja = apx[x * norb + q];
            if (ja < 0 || A.alev[ja] + lb > L) continue;
            const double f = (double)(sp * sgn2(q, x)) * A.h_v[e];
            const double *src = c + A.rowstart[ja] + ib;
#pragma unroll
            for (int v = 0; v < NV; ++v)
                if (v < nv) acc[v] += f * src[v * ldc];
        }
    }
    // same-spin alpha: {s < q} -> {a0 < a1}
    if (doss) {
        const int P = a1 * (a1 - 1) / 2 + a0;
        for (int e = A.ss_off[P]; e < A.ss_off[P + 1]; ++e) {
            const int q = A.ss_qs[e] >> 8, s2 = A.ss_qs[e] & 0xff;
            const int ja = apx[q * norb + s2];
            if (ja < 0 || A.alev[ja] + lb > L) continue;
            const double f = A.ss_v[e];
            const double *src = c + A.rowstart[ja] + ib;
#pragma unroll
            for (int v = 0; v < NV; ++v)
                if (v < nv) acc[v] += f * src[v * ldc];
        }
    }
    const int bmax = rlen;
    // one-body beta
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const int r = i ? b1 : b0, y = i ? b0 : b1;
        const int sr = sgn2(r, y);
        for (int e = do1 ? A.h_off[r] : 0; e < (do1 ? A.h_off[r + 1] : 0); ++e) {
            const int s2 = A.h_q[e];
            if (s2 == y) continue;
            const int jb = bpx[y * norb + s2];
            if (jb < 0 || jb >= bmax) continue;
            const double f = (double)(sr * sgn2(s2, y)) * A.h_v[e];
            const double *src = c + myrow + jb;
#pragma unroll
            for (int v = 0; v < NV; ++v)
                if (v < nv) acc[v] += f * src[v * ldc];
        }
    }
    // same-spin beta
    if (doss) {
        const int P = b1 * (b1 - 1) / 2 + b0;
        for (int e = A.ss_off[P]; e < A.ss_off[P + 1]; ++e) {
            const int q = A.ss_qs[e] >> 8, s2 = A.ss_qs[e] & 0xff;
            const int jb = bpx[q * norb + s2];
            if (jb < 0 || jb >= bmax) continue;
            const double f = A.ss_v[e];
            const double *src = c + myrow + jb;
#pragma unroll
            for (int v = 0; v < NV; ++v)
                if (v < nv) acc[v] += f * src[v * ldc];
        }
    }
    // alpha-beta
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const int p = i ? a1 : a0, x = i ? a0 : a1;
        const int sp = sgn2(p, x);
        for (int e1 = doab ? A.pq_off[p] : 0; e1 < (doab ? A.pq_off[p + 1] : 0); ++e1) {
            const int q = A.pq_q[e1];
            if (q == x) continue;
            const int ja = apx[x * norb + q];
            if (ja < 0) continue;
            const int lj = A.alev[ja];
            if (lj > L) continue;
            const int lenJ = A.sb.le[L - lj];
            const int sa = sp * sgn2(q, x);
            const double *rowJ = c + A.rowstart[ja];
            const long long base = ((long long)p * norb + q) * norb;
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                const int r = k ? b1 : b0, y = k ? b0 : b1;
                const int sr = sa * sgn2(r, y);
                const int *__restrict__ yrow = bpx + y * norb;
                const long long e0 = A.ab_off[base + r], e1e = A.ab_off[base + r + 1];
                for (long long e = e0; e < e1e; ++e) {
                    const int s2 = A.ab_s[e];
                    if (s2 == y) continue;
                    const int jb = yrow[s2];
                    if (jb < 0 || jb >= lenJ) continue;
                    const double f = (double)(sr * sgn2(s2, y)) * A.ab_v[e];
                    const double *src = rowJ + jb;
#pragma unroll
                    for (int v = 0; v < NV; ++v)
                        if (v < nv) acc[v] += f * src[v * ldc];
                }
            }
        }
    }
    double *dst = sg + myrow + ib;
    if (A.accumulate) {
#pragma unroll
        for (int v = 0; v < NV; ++v)
            if (v < nv) dst[v * lds] += acc[v];
    } else {
#pragma unroll
        for (int v = 0; v < NV; ++v)
            if (v < nv) dst[v * lds] = acc[v];
    }
}

// ---------------------------------------------------------------------------
// Alpha-beta class on FP64 matrix cores (two electrons per spin).
//
// With T[x][q][y][s] = sgn(q-x) sgn(s-y) c({x,q},{y,s}) (the CI vector as an
// antisymmetric pair tensor in each spin), the alpha-beta class is
//   T'[x][p][y][r] = S[x][p][y][r] - S[p][x][y][r] - S[x][p][r][y] + S[p][x][r][y],
//   S[x][p][y][r]  = sum_{q,s} (pq|rs) T[x][q][y][s],
// i.e. for fixed spectators (x, y) a product with the screened matrix
// W[(p,r),(q,s)] = (pq|rs) (the alpha-beta ladder of Eqs. h200ca..h200ab
// when all four indices are virtual).  Orbitals are grouped in blocks of
// four (inner / outer pure); a workgroup owns the sigma tile {x,p} x {y,r} with x in
// block X, p in P, y in Y, r in R and computes the four role products
// (which of x/p and y/r is the spectator) on four waves, one
// 16 x 16 x 4 MFMA per (column chunk, vector): rows = the 16 active pairs,
// columns = the 16 spectator pairs, K = 4 columns (q, s) of a chunk.  The
// roles are combined through LDS and sigma is written once (no atomics).
typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int kTabMax = 128;   // orbitals covered by the LDS lookup tables

// B operand of one chunk for this lane: sign * c(v, {x,q}, {y,s}) or 0.
// Table reads and loads are unconditional (clamped indices, invalid
// operands selected to zero), so the compiler can overlap chunks.
template <int NV, bool TAB>
__device__ __forceinline__ void gather_b(const SigmaArgs &A, const double *__restrict__ c, int64_t ldc, int nv,
                                         int x, int y, int ic, int id, int q, int s, int norb,
                                         const long long *rb, const int *rl, const int *bi, double *b)
{
    const bool idx_ok = x >= 0 && y >= 0 && s >= 0 && x != q && y != s;
    const int xc = max(x, 0), yc = max(y, 0), sc = max(s, 0);
    long long base;
    int len, jb;
    if (TAB) {
        base = rb[ic * kTabMax + q];
        len = rl[ic * kTabMax + q];
        jb = bi[id * kTabMax + sc];
    } else {
        base = A.arow_base[xc * norb + q];
        len = A.arow_len[xc * norb + q];
        jb = A.bpidx[yc * norb + sc];
    }
    const bool ok = idx_ok && base >= 0 && jb >= 0 && jb < len;
    const double f = ((q > x) == (s > y)) ? 1.0 : -1.0;
    const double *src = c + (ok ? base + jb : 0);
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        const double val = src[(int64_t)min(v, nv - 1) * ldc];
        b[v] = (ok && v < nv) ? f * val : 0.0;
    }
}

// ---------------------------------------------------------------------------
// Alpha-beta class on FP64 matrix cores (two electrons per spin).
//
// With T[x][q][y][s] = sgn(q-x) sgn(s-y) c({x,q},{y,s}) (the CI vector as an
// antisymmetric pair tensor in each spin), the alpha-beta class is
//   T'[x][p][y][r] = S[x][p][y][r] - S[p][x][y][r] - S[x][p][r][y] + S[p][x][r][y],
//   S[x][p][y][r]  = sum_{q,s} (pq|rs) T[x][q][y][s],
// i.e. for fixed spectators (x, y) a product with the screened matrix
// W[(p,r),(q,s)] = (pq|rs) (the alpha-beta ladder of Eqs. h200ca..h200ab
// when all four indices are virtual).  Orbitals are grouped in blocks of
// four (inner / outer pure); a workgroup owns the sigma tile {x,p} x {y,r} with x in
// block X, p in P, y in Y, r in R and computes the four role products
// (which of x/p and y/r is the spectator) on four waves, one
// 16 x 16 x 4 MFMA per (column chunk, vector): rows = the 16 active pairs,
// columns = the 16 spectator pairs, K = 4 columns (q, s) of a chunk.  The
// chunks of a row block are stored by source level class, so the chunks a
// role may use (source level <= L) are a prefix.  Row starts and beta
// indices of the wave's spectators are staged in LDS (TAB), and four
// chunks are loaded before their MFMAs issue.  The roles are combined
// through LDS and sigma is written once (no atomics).
template <int NV, bool TAB>
__global__ __launch_bounds__(256) void k_sigma_ab_mfma(SigmaArgs A, int nv, const double *__restrict__ c,
                                                       int64_t ldc, double *__restrict__ sg, int64_t lds)
{
    constexpr size_t kTileBytes = sizeof(double) * 4 * NV * 16 * 17;
    constexpr size_t kTabBytes = TAB ? (size_t)4 * 4 * kTabMax * (sizeof(long long) + 2 * sizeof(int)) : 16;
    __shared__ __attribute__((aligned(16))) char smem[kTileBytes > kTabBytes ? kTileBytes : kTabBytes];
    double(*tile)[NV][16][17] = reinterpret_cast<double(*)[NV][16][17]>(smem);
    long long *rb_all = reinterpret_cast<long long *>(smem);
    int *rl_all = reinterpret_cast<int *>(smem + (size_t)4 * 4 * kTabMax * sizeof(long long));
    int *bi_all = rl_all + 4 * 4 * kTabMax;

    const uchar4 qd = A.quads[blockIdx.x];
    const int X = qd.x, P = qd.y, Y = qd.z, R = qd.w;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const bool sameA = X == P, sameB = Y == R;
    const int norb = A.norb, L = A.L, nb = A.nblk;
    int Ab, Bb, Cb, Db;
    bool active;
    if (wave == 0) { Ab = P; Bb = R; Cb = X; Db = Y; active = true; }
    else if (wave == 1) { Ab = X; Bb = R; Cb = P; Db = Y; active = !sameA; }
    else if (wave == 2) { Ab = P; Bb = Y; Cb = X; Db = R; active = !sameB; }
    else { Ab = X; Bb = Y; Cb = P; Db = R; active = !sameA && !sameB; }
    long long *rb = rb_all + wave * 4 * kTabMax;
    int *rl = rl_all + wave * 4 * kTabMax;
    int *bi = bi_all + wave * 4 * kTabMax;
    if (TAB && active)
        for (int t = lane; t < 4 * norb; t += 64) {
            const int i = t / norb, o = t % norb;
            const int xx = ab_orbital(A, Cb, i), yy = ab_orbital(A, Db, i);
            rb[i * kTabMax + o] = xx >= 0 ? A.arow_base[xx * norb + o] : -1;
            rl[i * kTabMax + o] = xx >= 0 ? A.arow_len[xx * norb + o] : 0;
            bi[i * kTabMax + o] = yy >= 0 ? A.bpidx[yy * norb + o] : -1;
        }
    __syncthreads();
    v4d acc[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[v] = v4d{0.0, 0.0, 0.0, 0.0};
    if (active) {
        const int n = lane & 15, k = lane >> 4;
        const int ic = n >> 2, id = n & 3;
        const int x = ab_orbital(A, Cb, ic), y = ab_orbital(A, Db, id);
        const int espec = ab_outer(A, Cb) + ab_outer(A, Db);
        const int row = Ab * nb + Bb;
        const int e0 = A.chunk_off[row];
        int e1 = e0;
        for (int l = 0; l < 3; ++l)
            if (espec + l <= L) e1 += A.chunk_cls[row * 3 + l];
        int e = e0;
        for (; e + 4 <= e1; e += 4) {
            double a[4], b[4][NV];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int2 d = A.chunk_desc[e + u];
                a[u] = A.chunk_val[(size_t)(e + u) * 64 + lane];
                gather_b<NV, TAB>(A, c, ldc, nv, x, y, ic, id, d.x, ab_orbital(A, d.y, k), norb, rb, rl, bi, b[u]);
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int v = 0; v < NV; ++v) acc[v] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u], b[u][v], acc[v], 0, 0, 0);
        }
        for (; e < e1; ++e) {
            double b[NV];
            const int2 d = A.chunk_desc[e];
            const double a = A.chunk_val[(size_t)e * 64 + lane];
            gather_b<NV, TAB>(A, c, ldc, nv, x, y, ic, id, d.x, ab_orbital(A, d.y, k), norb, rb, rl, bi, b);
#pragma unroll
            for (int v = 0; v < NV; ++v) acc[v] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b[v], acc[v], 0, 0, 0);
        }
    }
    __syncthreads();   // the lookup tables share LDS with the role tiles
    if (active) {
        // 16x16x4 f64 result layout: element g of lane l is D[4 g + l / 16][l % 16]
#pragma unroll
        for (int v = 0; v < NV; ++v)
#pragma unroll
            for (int g = 0; g < 4; ++g) tile[wave][v][4 * g + (lane >> 4)][lane & 15] = acc[v][g];
    }
    __syncthreads();
    const int t = threadIdx.x;
    const int ix = (t >> 6) & 3, ip = (t >> 4) & 3, iy = (t >> 2) & 3, ir = t & 3;
    const int x = ab_orbital(A, X, ix), p = ab_orbital(A, P, ip);
    const int y = ab_orbital(A, Y, iy), r = ab_orbital(A, R, ir);
    if (x < 0 || p < 0 || y < 0 || r < 0 || x >= p || y >= r) return;
    const long long tb = A.arow_base[x * norb + p];
    const int tl = A.arow_len[x * norb + p];
    const int jb = A.bpidx[y * norb + r];
    if (tb < 0 || jb < 0 || jb >= tl) return;
    const int t1 = sameA ? 0 : 1, t2 = sameB ? 0 : 2;
    const int t3 = (sameA && sameB) ? 0 : sameA ? 2 : sameB ? 1 : 3;
    double *dst = sg + tb + jb;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        if (v >= nv) break;
        const double val = tile[0][v][ip * 4 + ir][ix * 4 + iy] - tile[t1][v][ix * 4 + ir][ip * 4 + iy]
                         - tile[t2][v][ip * 4 + iy][ix * 4 + ir] + tile[t3][v][ix * 4 + iy][ip * 4 + ir];
        dst[v * lds] = val;
    }
}

template <int NV>
__global__ __launch_bounds__(256) void k_sigma_n2(SigmaArgs A, int nv, const double *__restrict__ c,
                                                  int64_t ldc, double *__restrict__ sg, int64_t lds)
{
    int ia, j0, len;
    row_block(A, blockIdx.x, ia, j0, len);
    sigma_target_n2<NV>(A, ia, j0 + threadIdx.x, nv, c, ldc, sg, lds);
}

template <int NV>
__global__ __launch_bounds__(256) void k_sigma_generic(SigmaArgs A, int nv, const double *__restrict__ c,
                                                       int64_t ldc, double *__restrict__ sg, int64_t lds)
{
    int ia, j0, len;
    row_block(A, blockIdx.x, ia, j0, len);
    sigma_target<NV>(A, ia, j0 + threadIdx.x, nv, c, ldc, sg, lds);
}

// Fused sigma over many instances: a persistent grid walks the global
// work-item range; item g belongs to the job whose range holds it (jobs
// are few, so a linear search over their start offsets is cheap and
// uniform across the workgroup).
template <int NV>
__global__ __launch_bounds__(256) void k_sigma_batched(const SigmaArgs *__restrict__ args,
                                                       const BatchVec *__restrict__ vecs, int njobs, int nitems)
{
    int job = 0;
    for (int g = blockIdx.x; g < nitems; g += gridDim.x) {
        while (job + 1 < njobs && vecs[job + 1].item0 <= g) ++job;
        const BatchVec &bv = vecs[job];
        const int2 w = bv.plan[g - bv.item0];
        const SigmaArgs &A = args[bv.inst];
        if (A.variant >= 2)
            sigma_target_n2<NV>(A, w.x, w.y + threadIdx.x, bv.nv, bv.c, bv.ldc, bv.s, bv.lds);
        else
            sigma_target<NV>(A, w.x, w.y + threadIdx.x, bv.nv, bv.c, bv.ldc, bv.s, bv.lds);
    }
}

// diagonal of H_tau: kept diagonal units
__global__ __launch_bounds__(256) void k_diag(SigmaArgs A, double *__restrict__ out)
{
    int ia, j0, rlen;
    row_block(A, blockIdx.x, ia, j0, rlen);
    const int ib = j0 + threadIdx.x;
    if (ib >= rlen) return;
    const int na = A.sa.n, nb = A.sb.n, n = A.norb;
    int ao[ISCI_MAXN], bo[ISCI_MAXN];
    unpack_str(A.astr[ia], na, ao);
    unpack_str(A.bstr[ib], nb, bo);
    const double tau = A.tau;
    double acc = 0.0;
    for (int i = 0; i < na; ++i) { double u = A.hd[ao[i]]; if (fabs(u) > tau) acc += u; }
    for (int i = 0; i < nb; ++i) { double u = A.hd[bo[i]]; if (fabs(u) > tau) acc += u; }
    for (int i = 0; i < na; ++i)
        for (int j = i + 1; j < na; ++j) { double u = A.ssd[ao[i] * n + ao[j]]; if (fabs(u) > tau) acc += u; }
    for (int i = 0; i < nb; ++i)
        for (int j = i + 1; j < nb; ++j) { double u = A.ssd[bo[i] * n + bo[j]]; if (fabs(u) > tau) acc += u; }
    for (int i = 0; i < na; ++i)
        for (int j = 0; j < nb; ++j) { double u = A.jj[ao[i] * n + bo[j]]; if (fabs(u) > tau) acc += u; }
    out[A.rowstart[ia] + ib] = acc;
}

isci_status launch_sigma(const isci_ctx *c, int nvec, const double *cv, int64_t ldc, double *sv, int64_t lds,
                         hipStream_t s, bool side)
{
    const SigmaArgs A = sigma_args(c);
    const dim3 grid((unsigned)c->nplan);
    for (int v0 = 0; v0 < nvec; v0 += 8) {
        const int nv = nvec - v0 < 8 ? nvec - v0 : 8;
        const double *cc = cv + (int64_t)v0 * ldc;
        double *ss = sv + (int64_t)v0 * lds;
        if (A.variant == 3) {
            // Matrix-core path: the alpha-beta class writes sigma (as the
            // unfold / block-sparse product / fold path when its operands
            // fit, else with the gathered tile kernel), then the one-body
            // (unless the tiles carry it) and same-spin classes add.
            if (c->ob_stream && !c->ab_gather && c->d.hscreen && !c->onebody_in_tiles) {
                // the one-body classes (beta writes sigma, alpha adds) run on
                // the side stream while the unfolds and products of both
                // 4-vector passes run here (into two S buffers); the folds
                // wait for them and add
                side = side && c->ob_side;
                const hipStream_t os = side ? c->ob_stream : s;
                if (side) {
                    ISCI_HIP(hipEventRecord(c->ob_fork, s));
                    ISCI_HIP(hipStreamWaitEvent(c->ob_stream, c->ob_fork, 0));
                }
                ISCI_CHECK(prof_mark(c, ISCI_KERNEL_ONEBODY, true, os));
                ISCI_CHECK(launch_onebody_mfma(c, nv, cc, ldc, ss, lds, os, true));
                ISCI_CHECK(prof_mark(c, ISCI_KERNEL_ONEBODY, false, os));
                if (side) ISCI_HIP(hipEventRecord(c->ob_join, c->ob_stream));
                for (int u0 = 0; u0 < nv; u0 += 4)
                    ISCI_CHECK(launch_ab_unfold_gemm(c, nv - u0 < 4 ? nv - u0 : 4, cc + (int64_t)u0 * ldc, ldc,
                                                     u0 ? c->d.abx_S2 : c->d.abx_S, s));
                if (side) ISCI_HIP(hipStreamWaitEvent(s, c->ob_join, 0));
                for (int u0 = 0; u0 < nv; u0 += 4)
                    ISCI_CHECK(launch_ab_fold(c, nv - u0 < 4 ? nv - u0 : 4, u0 ? c->d.abx_S2 : c->d.abx_S,
                                              ss + (int64_t)u0 * lds, lds, true, s));
                if (c->stats.kept_total - c->nkept_h - c->nkept_ab == 0) continue;   // no same-spin units
            } else {
                for (int u0 = 0; u0 < nv; u0 += 4) {
                    const int nu = nv - u0 < 4 ? nv - u0 : 4;
                    if (c->have_abx && !c->ab_gather) {
                        ISCI_CHECK(launch_ab_product(c, nu, cc + (int64_t)u0 * ldc, ldc, ss + (int64_t)u0 * lds, lds, s));
                    } else if (c->nquad > 0) {
                        ISCI_CHECK(prof_mark(c, ISCI_KERNEL_AB_MFMA, true, s));
                        if (c->norb <= kTabMax)
                            k_sigma_ab_mfma<4, true><<<c->nquad, 256, 0, s>>>(A, nu, cc + (int64_t)u0 * ldc, ldc,
                                                                               ss + (int64_t)u0 * lds, lds);
                        else
                            k_sigma_ab_mfma<4, false><<<c->nquad, 256, 0, s>>>(A, nu, cc + (int64_t)u0 * ldc, ldc,
                                                                                ss + (int64_t)u0 * lds, lds);
                        ISCI_CHECK(prof_mark(c, ISCI_KERNEL_AB_MFMA, false, s));
                    }
                }
                if (c->d.hscreen && !c->onebody_in_tiles) {
                    // one-body classes on matrix cores (above 80 orbitals alpha in
                    // the spectator form, two launches by spectator side, and
                    // beta as the alpha class of the transposed block), then
                    // same-spin if any; with dense integrals the tiles carry
                    // the one-body units instead
                    ISCI_CHECK(prof_mark(c, ISCI_KERNEL_ONEBODY, true, s));
                    if (onebody_mfma_ok(c)) {
                        ISCI_CHECK(launch_onebody_mfma(c, nv, cc, ldc, ss, lds, s));
                    } else {
                        ISCI_CHECK(launch_onebody_alpha_large(c, nv, cc, ldc, ss, lds, s));
                        for (int u0 = 0; u0 < nv; u0 += 4)
                            ISCI_CHECK(launch_onebody_beta_large(c, nv - u0 < 4 ? nv - u0 : 4, cc + (int64_t)u0 * ldc,
                                                                 ldc, ss + (int64_t)u0 * lds, lds, s));
                        ISCI_HIP(hipGetLastError());
                    }
                    ISCI_CHECK(prof_mark(c, ISCI_KERNEL_ONEBODY, false, s));
                }
                if (c->d.hscreen && c->stats.kept_total - c->nkept_h - c->nkept_ab == 0) continue;   // no same-spin units
            }
            ISCI_CHECK(prof_mark(c, ISCI_KERNEL_PAIR_REST, true, s));
            SigmaArgs B = A;
            B.classes = c->d.hscreen ? 2 : 3;
            B.accumulate = 1;
            if (nv == 1)
                k_sigma_n2<1><<<grid, 256, 0, s>>>(B, nv, cc, ldc, ss, lds);
            else if (nv == 2)
                k_sigma_n2<2><<<grid, 256, 0, s>>>(B, nv, cc, ldc, ss, lds);
            else if (nv <= 4)
                k_sigma_n2<4><<<grid, 256, 0, s>>>(B, nv, cc, ldc, ss, lds);
            else
                k_sigma_n2<8><<<grid, 256, 0, s>>>(B, nv, cc, ldc, ss, lds);
            ISCI_HIP(hipGetLastError());
            ISCI_CHECK(prof_mark(c, ISCI_KERNEL_PAIR_REST, false, s));
            continue;
        }
        const bool n2 = A.variant == 2;
        const int kid = n2 ? ISCI_KERNEL_PAIR : ISCI_KERNEL_GENERAL;
        ISCI_CHECK(prof_mark(c, kid, true, s));
        if (n2) {
            if (nv == 1)
                k_sigma_n2<1><<<grid, 256, 0, s>>>(A, nv, cc, ldc, ss, lds);
            else if (nv == 2)
                k_sigma_n2<2><<<grid, 256, 0, s>>>(A, nv, cc, ldc, ss, lds);
            else if (nv <= 4)
                k_sigma_n2<4><<<grid, 256, 0, s>>>(A, nv, cc, ldc, ss, lds);
            else
                k_sigma_n2<8><<<grid, 256, 0, s>>>(A, nv, cc, ldc, ss, lds);
        } else if (nv == 1)
            k_sigma_generic<1><<<grid, 256, 0, s>>>(A, nv, cc, ldc, ss, lds);
        else if (nv == 2)
            k_sigma_generic<2><<<grid, 256, 0, s>>>(A, nv, cc, ldc, ss, lds);
        else if (nv <= 4)
            k_sigma_generic<4><<<grid, 256, 0, s>>>(A, nv, cc, ldc, ss, lds);
        else
            k_sigma_generic<8><<<grid, 256, 0, s>>>(A, nv, cc, ldc, ss, lds);
        ISCI_HIP(hipGetLastError());
        ISCI_CHECK(prof_mark(c, kid, false, s));
    }
    return ISCI_OK;
}

isci_status launch_sigma_batched(const SigmaArgs *args_dev, const BatchVec *vecs_dev, int njobs, int nitems,
                                 int nvmax, int grid, hipStream_t s)
{
    if (nitems <= 0 || njobs <= 0) return ISCI_OK;
    grid = grid > 0 ? std::min(grid, nitems) : nitems;
    if (nvmax <= 1)
        k_sigma_batched<1><<<grid, 256, 0, s>>>(args_dev, vecs_dev, njobs, nitems);
    else if (nvmax <= 2)
        k_sigma_batched<2><<<grid, 256, 0, s>>>(args_dev, vecs_dev, njobs, nitems);
    else if (nvmax <= 4)
        k_sigma_batched<4><<<grid, 256, 0, s>>>(args_dev, vecs_dev, njobs, nitems);
    else
        k_sigma_batched<8><<<grid, 256, 0, s>>>(args_dev, vecs_dev, njobs, nitems);
    ISCI_HIP(hipGetLastError());
    return ISCI_OK;
}

isci_status launch_diag(const isci_ctx *c, double *diag, hipStream_t s)
{
    const SigmaArgs A = sigma_args(c);
    const dim3 grid((unsigned)c->nplan);
    k_diag<<<grid, 256, 0, s>>>(A, diag);
    ISCI_HIP(hipGetLastError());
    return ISCI_OK;
}

}  // namespace isci

using namespace isci;

extern "C" {

isci_status isci_sigma(isci_handle c, int nvec, const double *cv, int64_t ldc, double *sv, int64_t lds,
                       hipStream_t stream)
{
    if (!c || !cv || !sv) { set_error("NULL argument"); return ISCI_E_INVALID; }
    if (nvec < 1) { set_error("nvec < 1"); return ISCI_E_INVALID; }
    if (ldc < c->dim || lds < c->dim) { set_error("leading dimension < dim"); return ISCI_E_INVALID; }
    const char *c0 = (const char *)cv, *c1 = (const char *)(cv + (int64_t)(nvec - 1) * ldc + c->dim);
    const char *s0 = (const char *)sv, *s1 = (const char *)(sv + (int64_t)(nvec - 1) * lds + c->dim);
    if (c0 < s1 && s0 < c1) { set_error("sigma overlaps c"); return ISCI_E_INVALID; }
    return launch_sigma(c, nvec, cv, ldc, sv, lds, stream);
}

struct isci_graph_s {
    hipGraph_t g = nullptr;
    hipGraphExec_t x = nullptr;
};

void isci_graph_destroy(isci_graph g)
{
    if (!g) return;
    if (g->x) (void)hipGraphExecDestroy(g->x);
    if (g->g) (void)hipGraphDestroy(g->g);
    delete g;
}

isci_status isci_sigma_graph_create(isci_handle c, int nvec, const double *cv, int64_t ldc, double *sv, int64_t lds,
                                    isci_graph *out)
{
    if (!out) { set_error("NULL argument"); return ISCI_E_INVALID; }
    *out = nullptr;
    if (!c || !cv || !sv) { set_error("NULL argument"); return ISCI_E_INVALID; }
    if (nvec < 1) { set_error("nvec < 1"); return ISCI_E_INVALID; }
    if (ldc < c->dim || lds < c->dim) { set_error("leading dimension < dim"); return ISCI_E_INVALID; }
    const char *c0 = (const char *)cv, *c1 = (const char *)(cv + (int64_t)(nvec - 1) * ldc + c->dim);
    const char *s0 = (const char *)sv, *s1 = (const char *)(sv + (int64_t)(nvec - 1) * lds + c->dim);
    if (c0 < s1 && s0 < c1) { set_error("sigma overlaps c"); return ISCI_E_INVALID; }
    if (c->profile) { set_error("kernel profiling is enabled on this handle"); return ISCI_E_INVALID; }
    hipStream_t cs = nullptr;
    ISCI_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    isci_graph g = new isci_graph_s;
    isci_status st = ISCI_OK;
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        st = launch_sigma(c, nvec, cv, ldc, sv, lds, cs);
        // the capture is ended in every case, so the streams leave capture mode
        const hipError_t e2 = hipStreamEndCapture(cs, &g->g);
        if (st == ISCI_OK && e2 != hipSuccess) st = hip_fail(e2, "hipStreamEndCapture");
        if (st == ISCI_OK) {
            e = hipGraphInstantiate(&g->x, g->g, nullptr, nullptr, 0);
            if (e != hipSuccess) st = hip_fail(e, "hipGraphInstantiate");
        }
    } else {
        st = hip_fail(e, "hipStreamBeginCapture");
    }
    (void)hipStreamDestroy(cs);
    if (st != ISCI_OK) { isci_graph_destroy(g); return st; }
    *out = g;
    return ISCI_OK;
}

isci_status isci_graph_launch(isci_graph g, hipStream_t stream)
{
    if (!g || !g->x) { set_error("NULL argument"); return ISCI_E_INVALID; }
    ISCI_HIP(hipGraphLaunch(g->x, stream));
    return ISCI_OK;
}

isci_status isci_diag(isci_handle c, double *diag, hipStream_t stream)
{
    if (!c || !diag) { set_error("NULL argument"); return ISCI_E_INVALID; }
    return launch_diag(c, diag, stream);
}

}  // extern "C"
