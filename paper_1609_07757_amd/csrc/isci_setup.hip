// libisci setup: argument checks, string enumeration and row layout,
// the on-device screened-integral list builder, screening statistics and
// the small entry points of the ABI.
//
// The list builder is one pass over h and the canonical elements of eri.
// Every elementary unit of the paper's index-restricted Hamiltonian
// (Eq. index_re) is formed once and kept iff |unit| > tau (Eqs. sigma_int,
// sigma_split):
//   one-body   h_pq                          CSR over p        -> (q, h_pq)
//   same-spin  (pq|rs) - (ps|rq), p>r, q>s   CSR over pair(p,r) -> (q, s, value)
//   alpha-beta (pq|rs)                       CSR over (p,q,r)  -> (s, value)
// These lists are the "integral loops" of the sigma kernels: the kernels
// iterate over kept units only, so screened integrals cost nothing there.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "isci_device.h"
#include "isci_internal.h"

namespace isci {

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }

isci_status hip_fail(hipError_t e, const char *what)
{
    set_error(std::string(what) + ": " + hipGetErrorString(e));
    return e == hipErrorOutOfMemory ? ISCI_E_OOM : ISCI_E_HIP;
}

void *dev_alloc(isci_ctx *c, size_t bytes)
{
    void *p = nullptr;
    if (bytes == 0) bytes = 8;
    if (c->allocator.alloc) {
        p = c->allocator.alloc(bytes, c->alloc_stream, c->allocator.ctx);
        if (!p) return nullptr;
    } else if (hipMalloc(&p, bytes) != hipSuccess) {
        return nullptr;
    }
    c->allocs.push_back(p);
    c->stats.device_bytes += (int64_t)bytes;
    return p;
}

// ------------------------------------------------------------------ host tables

// b: level boundary (n for the excitation hierarchy, n <= b <= norb)
static void spin_table(SpinTab &T, int norb, int n, int L, int b)
{
    memset(&T, 0, sizeof(T));
    T.n = n;
    T.nocc = b;
    T.nvirt = norb - b;
    T.maxlev = std::min(std::min(n, norb - b), L);
    int acc = 0;
    for (int k = 0; k <= T.maxlev; ++k) {
        T.lev_off[k] = acc;
        T.occ_mult[k] = (int)binom(b, n - k);
        acc += (int)(binom(b, n - k) * binom(norb - b, k));
    }
    for (int k = T.maxlev + 1; k <= ISCI_MAXLEV + 1; ++k) T.lev_off[k] = acc;
    T.nstr = acc;
    for (int l = 0; l <= ISCI_MAXLEV + 1; ++l) T.le[l] = T.lev_off[std::min(l, T.maxlev) + 1];
}

// enumerate all strings of a spin and place each at its rank; checks that
// the rank is a bijection onto 0..nstr-1
static bool enumerate(const SpinTab &T, int norb, std::vector<int32_t> &orb,
                      std::vector<int32_t> &lev, std::vector<uint32_t> &packed)
{
    const int n = T.n;
    orb.assign((size_t)T.nstr * std::max(n, 1), 0);
    lev.assign(T.nstr, -1);
    packed.assign(T.nstr, 0);
    int idx[ISCI_MAXN];
    for (int i = 0; i < n; ++i) idx[i] = i;
    for (;;) {
        int l = str_level(idx, n, T.nocc);
        if (l <= T.maxlev) {
            int r = str_index(idx, T);
            if (r < 0 || r >= T.nstr || lev[r] >= 0) return false;
            lev[r] = l;
            packed[r] = pack_str(idx, n);
            for (int i = 0; i < n; ++i) orb[(size_t)r * n + i] = idx[i];
        }
        int i = n - 1;
        while (i >= 0 && idx[i] == norb - n + i) --i;
        if (i < 0) break;
        idx[i]++;
        for (int j = i + 1; j < n; ++j) idx[j] = idx[j - 1] + 1;
    }
    for (int r = 0; r < T.nstr; ++r)
        if (lev[r] < 0) return false;
    return true;
}

// ------------------------------------------------------------------ scan

template <typename T>
__global__ void k_scan_block(const T *in, T *out, T *bsum, int64_t N)
{
    __shared__ T s[1024];
    const int tid = threadIdx.x;
    const int64_t i = (int64_t)blockIdx.x * 1024 + tid;
    const T v = i < N ? in[i] : 0;
    s[tid] = v;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        T t = tid >= off ? s[tid - off] : 0;
        __syncthreads();
        s[tid] += t;
        __syncthreads();
    }
    if (i < N) out[i] = s[tid] - v;
    if (tid == 1023) bsum[blockIdx.x] = s[1023];
}

template <typename T>
__global__ void k_scan_add(T *out, const T *boff, int64_t N)
{
    const int64_t i = (int64_t)blockIdx.x * 1024 + threadIdx.x;
    if (i < N) out[i] += boff[blockIdx.x];
}

// exclusive scan in place of a[0..N-1] on stream s
template <typename T>
static isci_status scan_inplace(T *a, int64_t N, hipStream_t s)
{
    const int64_t nb = (N + 1023) / 1024;
    T *bs = nullptr;
    ISCI_HIP(hipMallocAsync((void **)&bs, sizeof(T) * (size_t)(nb + 1), s));
    k_scan_block<T><<<(unsigned)nb, 1024, 0, s>>>(a, a, bs, N);
    ISCI_HIP(hipGetLastError());
    if (nb > 1) {
        isci_status st = scan_inplace<T>(bs, nb, s);
        if (st != ISCI_OK) return st;
        k_scan_add<T><<<(unsigned)nb, 1024, 0, s>>>(a, bs, N);
        ISCI_HIP(hipGetLastError());
    }
    ISCI_HIP(hipFreeAsync(bs, s));
    return ISCI_OK;
}

// ------------------------------------------------------------------ term counting

// number of m-subsets (spectators) of the orbitals outside a set that
// holds o_ex occupied and v_ex virtual orbitals of this spin, at level l
__device__ inline long long nsub(const SpinTab &T, int m, int l, int o_ex, int v_ex)
{
    if (m < 0 || l < 0 || l > m) return 0;
    return binom(T.nocc - o_ex, m - l) * binom(T.nvirt - v_ex, l);
}

__device__ inline int isv(const SpinTab &T, int x) { return x >= T.nocc; }

// strings of the other spin with level <= l (0 if l < 0)
__device__ inline long long le_of(const SpinTab &T, int l)
{
    if (l < 0) return 0;
    return T.le[l > ISCI_MAXLEV + 1 ? ISCI_MAXLEV + 1 : l];
}

// sigma terms of one-body unit h_pq acting in spin T (other spin U)
__device__ long long terms_1b(const SpinTab &T, const SpinTab &U, int L, int p, int q)
{
    if (T.n < 1) return 0;
    int o = (p < T.nocc) + (q != p && q < T.nocc);
    int v = (p >= T.nocc) + (q != p && q >= T.nocc);
    int em = max(isv(T, p), isv(T, q));
    long long t = 0;
    for (int l = 0; l <= T.n - 1; ++l) t += nsub(T, T.n - 1, l, o, v) * le_of(U, L - l - em);
    return t;
}

// sigma terms of same-spin unit (p>r, q>s) acting in spin T
__device__ long long terms_ss(const SpinTab &T, const SpinTab &U, int L, int p, int r, int q, int s)
{
    if (T.n < 2) return 0;
    int e[4] = {p, r, q, s};
    int o = 0, v = 0;
    for (int i = 0; i < 4; ++i) {
        bool dup = false;
        for (int j = 0; j < i; ++j) dup |= (e[j] == e[i]);
        if (dup) continue;
        if (e[i] < T.nocc) ++o; else ++v;
    }
    int em = max(isv(T, p) + isv(T, r), isv(T, q) + isv(T, s));
    long long t = 0;
    for (int l = 0; l <= T.n - 2; ++l) t += nsub(T, T.n - 2, l, o, v) * le_of(U, L - l - em);
    return t;
}

// sigma terms of alpha-beta unit (pq|rs), alpha q->p, beta s->r
__device__ long long terms_ab(const SpinTab &A, const SpinTab &B, int L, int p, int q, int r, int s)
{
    if (A.n < 1 || B.n < 1) return 0;
    int oa = (p < A.nocc) + (q != p && q < A.nocc), va = (p >= A.nocc) + (q != p && q >= A.nocc);
    int ob = (r < B.nocc) + (s != r && s < B.nocc), vb = (r >= B.nocc) + (s != r && s >= B.nocc);
    int T = L - max(isv(A, q) + isv(B, s), isv(A, p) + isv(B, r));
    long long t = 0;
    for (int la = 0; la <= A.n - 1; ++la) {
        long long na = nsub(A, A.n - 1, la, oa, va);
        if (!na) continue;
        for (int lb = 0; lb <= B.n - 1 && la + lb <= T; ++lb) t += na * nsub(B, B.n - 1, lb, ob, vb);
    }
    return t;
}

// ------------------------------------------------------------------ list builder kernels

__global__ void k_h_count(const double *h, int n, double tau, int *cnt)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    int c = 0;
    for (int q = 0; q < n; ++q) c += fabs(gh(h, n, p, q)) > tau;
    cnt[p] = c;
}

__global__ void k_h_fill(const double *h, int n, double tau, const int *off, uint8_t *hq, double *hv,
                         SpinTab sa, SpinTab sb, int L, unsigned long long *ctr)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    int k = off[p];
    for (int q = 0; q < n; ++q) {
        double v = gh(h, n, p, q);
        if (!(fabs(v) > tau)) continue;
        hq[k] = (uint8_t)q;
        hv[k] = v;
        ++k;
        int ba = 2 * isv(sa, p) + isv(sa, q), bb = 4 + 2 * isv(sb, p) + isv(sb, q);
        if (sa.n > 0) {
            atomicAdd(&ctr[ba], 1ull);
            atomicAdd(&ctr[ISCI_NBUCKET + ba], (unsigned long long)terms_1b(sa, sb, L, p, q));
        }
        if (sb.n > 0) {
            atomicAdd(&ctr[bb], 1ull);
            atomicAdd(&ctr[ISCI_NBUCKET + bb], (unsigned long long)terms_1b(sb, sa, L, p, q));
        }
    }
}

__device__ inline void pair_of(int P, int &p, int &r)
{
    // P = p(p-1)/2 + r, p > r >= 0
    int x = (int)((1.0 + sqrt(1.0 + 8.0 * (double)P)) * 0.5);
    while (x * (x - 1) / 2 > P) --x;
    while ((x + 1) * x / 2 <= P) ++x;
    p = x;
    r = P - x * (x - 1) / 2;
}

// same-spin unit (pq|rs) - (ps|rq), or 0 when both integrals are surely
// below tau/2 (1 - 1e-6): then the difference, rounded, is below tau and
// would be screened anyway
__device__ inline double ss_unit(const EriSrc &E, int p, int q, int r, int s, double tau)
{
    const double t2 = 0.5 * tau * (1.0 - 1e-6);
    if (eri_negligible(E, p, q, r, s, t2) && eri_negligible(E, p, s, r, q, t2)) return 0.0;
    return eri_value(E, p, q, r, s) - eri_value(E, p, s, r, q);
}

__global__ void k_ss_count(EriSrc E, double tau, int *cnt)
{
    const int n = E.n;
    const int np = n * (n - 1) / 2;
    const int P = blockIdx.x * blockDim.x + threadIdx.x;
    if (P >= np) return;
    int p, r;
    pair_of(P, p, r);
    int c = 0;
    for (int q = 1; q < n; ++q)
        for (int s = 0; s < q; ++s) {
            const double v = ss_unit(E, p, q, r, s, tau);
            c += fabs(v) > tau;
        }
    cnt[P] = c;
}

__global__ void k_ss_fill(EriSrc E, double tau, const int *off, uint16_t *qs,
                          double *val, SpinTab sa, SpinTab sb, int L, unsigned long long *ctr)
{
    const int n = E.n;
    const int np = n * (n - 1) / 2;
    const int P = blockIdx.x * blockDim.x + threadIdx.x;
    if (P >= np) return;
    int p, r;
    pair_of(P, p, r);
    int k = off[P];
    for (int q = 1; q < n; ++q)
        for (int s = 0; s < q; ++s) {
            const double v = ss_unit(E, p, q, r, s, tau);
            if (!(fabs(v) > tau)) continue;
            qs[k] = (uint16_t)((q << 8) | s);
            val[k] = v;
            ++k;
            for (int spin = 0; spin < 2; ++spin) {
                const SpinTab &T = spin ? sb : sa;
                const SpinTab &U = spin ? sa : sb;
                if (T.n < 2) continue;
                int b = 8 + 9 * spin + 3 * (isv(T, p) + isv(T, r)) + isv(T, q) + isv(T, s);
                atomicAdd(&ctr[b], 1ull);
                atomicAdd(&ctr[ISCI_NBUCKET + b], (unsigned long long)terms_ss(T, U, L, p, r, q, s));
            }
        }
}

// Input check: *bad = 1 if any element the builders read (the canonical
// element of every (pq|rs), the lower triangle of h) is NaN or infinite.
// Such a unit would fail |unit| > tau and be screened out silently, so the
// handle would apply a corrupted H; isci_create refuses it instead.
__global__ void k_check_finite(const double *h, const double *eri, int n, int *bad)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t n3 = (int64_t)n * n * n;
    if (t >= n3) return;
    const int p = (int)(t / ((int64_t)n * n)), q = (int)((t / n) % n), r = (int)(t % n);
    bool ok = true;
    for (int s = 0; s < n; ++s) ok &= isfinite(geri(eri, n, p, q, r, s));
    if (t < (int64_t)n * n) ok &= isfinite(gh(h, n, (int)(t / n), (int)(t % n)));
    if (!ok) atomicOr(bad, 1);
}

// distance screening of h: hm[p][q] = h[p][q], or 0 when d(p, q) > dmax
__global__ void k_mask_h(const double *h, const double *dist, double dmax, int n, double *hm)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n * n) hm[t] = dist[t] > dmax ? 0.0 : h[t];
}

// The factored form of the input check, h part: *bad = 1 if an element of
// the lower triangle of h is not finite (the factors are checked through
// their norms in k_factor_prep).
__global__ void k_check_finite_h(const double *h, int n, int *bad)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n * n && !isfinite(gh(h, n, t / n, t % n))) atomicOr(bad, 1);
}

// Lt[pq][K] = L[K][pq] for the canonical pairs p >= q (the ones read), and
// nrm[pq] = nrm[qp] = (1 + 1e-12) sqrt(sum_K L[K][pq]^2) for all pairs; the
// factor makes it an upper bound of the exact norm.  *bad = 1 when a norm
// is not finite (a NaN or infinite factor entry) or its square overflows
// (then a sum of products could).
__global__ void k_factor_prep(const double *L, int n, int naux, double *Lt, double *nrm, int *bad)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * n) return;
    const int p = t / n, q = t % n;
    if (p < q) return;
    double ss = 0.0;
    for (int K = 0; K < naux; ++K) {
        const double v = L[(size_t)K * n * n + t];
        Lt[(size_t)t * naux + K] = v;
        ss = fma(v, v, ss);
    }
    const double b = sqrt(ss) * (1.0 + 1e-12);
    nrm[t] = b;
    nrm[q * n + p] = b;
    if (!isfinite(b) || !isfinite(b * b)) atomicOr(bad, 1);
}

__global__ void k_ab_count(EriSrc E, double tau, long long *cnt)
{
    const int n = E.n;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t n3 = (int64_t)n * n * n;
    if (t >= n3) return;
    const int p = (int)(t / ((int64_t)n * n)), q = (int)((t / n) % n), r = (int)(t % n);
    int c = 0;
    for (int s = 0; s < n; ++s)
        if (!eri_negligible(E, p, q, r, s, tau)) c += fabs(eri_value(E, p, q, r, s)) > tau;
    cnt[t] = c;
}

__global__ void k_ab_fill(EriSrc E, double tau, const long long *off, uint8_t *ss, double *val,
                          SpinTab sa, SpinTab sb, int L, unsigned long long *ctr)
{
    const int n = E.n;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t n3 = (int64_t)n * n * n;
    if (t >= n3) return;
    const int p = (int)(t / ((int64_t)n * n)), q = (int)((t / n) % n), r = (int)(t % n);
    long long k = off[t];
    unsigned long long kept[16] = {0}, terms[16] = {0};
    for (int s = 0; s < n; ++s) {
        if (eri_negligible(E, p, q, r, s, tau)) continue;
        const double v = eri_value(E, p, q, r, s);
        if (!(fabs(v) > tau)) continue;
        ss[k] = (uint8_t)s;
        val[k] = v;
        ++k;
        int b = 8 * isv(sa, p) + 4 * isv(sa, q) + 2 * isv(sb, r) + isv(sb, s);
        kept[b] += 1;
        terms[b] += (unsigned long long)terms_ab(sa, sb, L, p, q, r, s);
    }
    if (sa.n > 0 && sb.n > 0)
        for (int b = 0; b < 16; ++b)
            if (kept[b]) {
                atomicAdd(&ctr[26 + b], kept[b]);
                atomicAdd(&ctr[ISCI_NBUCKET + 26 + b], terms[b]);
            }
}

// number of active q (non-empty (p,q,*) alpha-beta lists) per p
__global__ void k_pq_count(const long long *ab_off, int n, int *cnt)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    int c = 0;
    for (int q = 0; q < n; ++q) {
        int64_t b = ((int64_t)p * n + q) * n;
        c += ab_off[b + n] > ab_off[b];
    }
    cnt[p] = c;
}

__global__ void k_pq_fill(const long long *ab_off, int n, const int *off, uint8_t *pq)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    int k = off[p];
    for (int q = 0; q < n; ++q) {
        int64_t b = ((int64_t)p * n + q) * n;
        if (ab_off[b + n] > ab_off[b]) pq[k++] = (uint8_t)q;
    }
}

// h with every screened unit zeroed (dense, for the one-body row kernels)
__global__ void k_hscreen(const double *h, int n, double tau, double *hs)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * n) return;
    const double v = gh(h, n, t / n, t % n);
    hs[t] = fabs(v) > tau ? v : 0.0;
}

// K-step masks of the screened h for the spectator-form one-body kernel:
// one thread per 16-orbital target tile mt (n <= 256, so at most 16 tiles
// and 64 steps of four orbitals)
__global__ void k_hkmask(const double *hs, int n, unsigned long long *mask)
{
    const int mt = threadIdx.x;
    if (mt >= 16) return;
    unsigned long long m = 0;
    for (int ks = 0; 4 * ks < n; ++ks) {
        bool any = false;
        for (int q = 4 * ks; q < 4 * ks + 4 && q < n; ++q)
            for (int a = 16 * mt; a < 16 * mt + 16 && a < n; ++a) any |= hs[(size_t)q * n + a] != 0.0;
        if (any) m |= 1ull << ks;
    }
    mask[mt] = m;
}

// hs (n x n) into the top-left corner of a zeroed P x P array
__global__ void k_hpad(const double *hs, int n, int P, double *hp)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= P * P) return;
    const int p = t / P, q = t % P;
    hp[t] = (p < n && q < n) ? hs[p * n + q] : 0.0;
}

// diagonal units: h_pp, (pp|qq), and (pp|qq) - (pq|qp) formed with the
// smaller index first
__global__ void k_diag_units(const double *h, EriSrc E, double *hd, double *jj, double *ssd)
{
    const int n = E.n;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * n) return;
    const int p = t / n, q = t % n;
    if (q == 0) hd[p] = gh(h, n, p, p);
    jj[t] = eri_value(E, p, p, q, q);
    const int a = min(p, q), b = max(p, q);
    ssd[t] = eri_value(E, a, a, b, b) - eri_value(E, a, b, b, a);
}

static inline unsigned nblk(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

SigmaArgs sigma_args(const isci_ctx *c)
{
    SigmaArgs A;
    A.norb = c->norb; A.L = c->L; A.tau = c->tau;
    A.sa = c->sa; A.sb = c->sb;
    A.astr = c->d.astr; A.bstr = c->d.bstr; A.alev = c->d.alev; A.blev = c->d.blev;
    A.rowstart = c->d.rowstart;
    A.h_off = c->d.h_off; A.h_q = c->d.h_q; A.h_v = c->d.h_v;
    A.ss_off = c->d.ss_off; A.ss_qs = c->d.ss_qs; A.ss_v = c->d.ss_v;
    A.ab_off = c->d.ab_off; A.ab_s = c->d.ab_s; A.ab_v = c->d.ab_v;
    A.pq_off = c->d.pq_off; A.pq_q = c->d.pq_q;
    A.hd = c->d.hd; A.jj = c->d.jj; A.ssd = c->d.ssd;
    A.apidx = c->d.apidx; A.bpidx = c->d.bpidx;
    const bool pair_ok = c->sa.n == 2 && c->sb.n == 2;
    A.variant = (c->sigma_variant == ISCI_SIGMA_GENERAL || !pair_ok) ? 1 : 2;
    // automatic choice: the matrix-core path whenever it is built (two
    // electrons per spin); it is faster than the pair kernel from the
    // smallest spaces on (20 orbitals CISD: 0.057 vs 0.197 ms per sigma)
    const bool auto_mfma = c->sigma_variant == ISCI_SIGMA_AUTO;
    if (pair_ok && c->have_tiles && (c->sigma_variant == ISCI_SIGMA_MFMA || auto_mfma)) A.variant = 3;
    A.classes = 7;
    A.accumulate = 0;
    A.nblk = c->nblk;
    A.ab_b = c->ab_b;
    A.ab_nib = c->ab_nib;
    A.blk_orb = c->d.blk_orb;
    A.chunk_off = c->d.chunk_off;
    A.chunk_desc = c->d.chunk_desc;
    A.chunk_val = c->d.chunk_val;
    A.quads = c->d.quads;
    A.arow_base = c->d.arow_base;
    A.arow_len = c->d.arow_len;
    A.chunk_cls = c->d.chunk_cls;
    A.abx_gofs = c->d.abx_gofs;
    A.abx_col = c->d.abx_col;
    A.abx_trow = c->d.abx_trow;
    A.abx_tq = c->d.abx_tq;
    A.abx_chunk = c->d.abx_chunk;
    A.abx_rows = c->d.abx_rows;
    A.abx_soff = c->d.abx_soff;
    A.abx_blk = c->d.abx_blk;
    A.abx_ctof = c->d.abx_ctof;
    A.abx_pchunk = c->d.abx_pchunk;
    A.pchunk_val = c->d.pchunk_val;
    A.abx_pblk = c->d.abx_pblk;
    A.nchunk = c->nchunk;
    A.abx_T = c->d.abx_T;
    A.abx_S = c->d.abx_S;
    for (int k = 0; k < 3; ++k) A.abx_pcols[k] = c->abx_pcols[k];
    A.abx_vs = 4;
    return A;
}


// ------------------------------------------------------------------ alpha-beta MFMA tiles

// mark column chunk ((A*nb + B)*norb + q)*nb + S of every kept (pq|rs)
__global__ void k_chunk_mark(const long long *ab_off, const uint8_t *ab_s, int n, const int *orb_blk, int nb,
                             unsigned *bits)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)n * n * n) return;
    const int p = (int)(t / ((int64_t)n * n)), q = (int)((t / n) % n), r = (int)(t % n);
    for (long long e = ab_off[t]; e < ab_off[t + 1]; ++e) {
        const int s = ab_s[e];
        const long long key = (((long long)orb_blk[p] * nb + orb_blk[r]) * n + q) * nb + orb_blk[s];
        atomicOr(&bits[key >> 5], 1u << (key & 31));
    }
}

// With two electrons of each spin, N_beta = sum_r E^beta_rr is 2 on the
// whole space (and likewise for alpha), so the kept one-body units are
// alpha-beta units as well:
//   h_pq E^alpha_pq = sum_r (h_pq / 2) E^alpha_pq E^beta_rr,
//   h_rs E^beta_rs  = sum_p (h_rs / 2) E^alpha_pp E^beta_rs.
// Their chunks are marked here and their values added in k_chunk_fill, so
// the alpha-beta product forms the one-body classes too.  Thread (p, q):
// the alpha image of h_pq over every r, and the beta image of h_pq (as
// h_rs with r = p, s = q) over every alpha diagonal orbital.
__global__ void k_chunk_mark_1b(const double *hs, int n, const int *orb_blk, int nb, unsigned *bits)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * n) return;
    const int p = t / n, q = t % n;
    if (hs[t] == 0.0) return;
    for (int o = 0; o < n; ++o) {
        const long long ka = (((long long)orb_blk[p] * nb + orb_blk[o]) * n + q) * nb + orb_blk[o];
        atomicOr(&bits[ka >> 5], 1u << (ka & 31));
        const long long kb = (((long long)orb_blk[o] * nb + orb_blk[p]) * n + o) * nb + orb_blk[q];
        atomicOr(&bits[kb >> 5], 1u << (kb & 31));
    }
}

// one workgroup per row block pair g: marked chunks among its n * nb keys
__global__ __launch_bounds__(256) void k_chunk_count(const unsigned *bits, int n, int nb, int *cnt)
{
    const int g = blockIdx.x;
    const long long k0 = (long long)g * n * nb;
    const int nk = n * nb;
    int c = 0;
    for (int key = threadIdx.x; key < nk; key += blockDim.x) {
        const long long k = k0 + key;
        c += (bits[k >> 5] >> (k & 31)) & 1u;
    }
    for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off, 64);
    __shared__ int ws[4];
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) cnt[g] = ws[0] + ws[1] + ws[2] + ws[3];
}

// Chunks of a row block pair are written in order of their source level
// class (outer q) + (outer S-block), so the chunks a role may use form
// a prefix; cls[g*3 + l] counts the chunks of class l.  One workgroup per
// row block pair g: for each class, block-wide scans over batches of 256
// (q, S) keys (in q, S order) place the marked chunks, then 64-lane groups
// fill the 64 values of each chunk placed in the batch.
__global__ __launch_bounds__(256) void k_chunk_fill(const unsigned *bits, EriSrc E, const double *hs, int n,
                                                    int nb, int bnd, int nib, double tau, const int16_t *blk_orb,
                                                    const int *off, int2 *desc, double *val, int *cls)
{
    const int g = blockIdx.x;
    const int Ab = g / nb, Bb = g % nb;
    const long long k0 = (long long)g * n * nb;
    const int nk = n * nb;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    __shared__ int ws[4];
    __shared__ int sel[256];
    int w = off[g];
    for (int lc = 0; lc < 3; ++lc) {
        int cnt = 0;
        for (int base = 0; base < nk; base += 256) {
            const int key = base + (int)threadIdx.x;
            const int q = key / nb, S = key % nb;
            bool f = false;
            if (key < nk) {
                const long long k = k0 + key;
                f = ((bits[k >> 5] >> (k & 31)) & 1u) && (q >= bnd) + (S >= nib) == lc;
            }
            const unsigned long long bal = __ballot(f);
            const int pre = __popcll(bal & ((1ull << lane) - 1ull));
            if (lane == 0) ws[wv] = __popcll(bal);
            __syncthreads();
            int woff = 0;
            for (int i = 0; i < wv; ++i) woff += ws[i];
            const int tot = ws[0] + ws[1] + ws[2] + ws[3];
            if (f) {
                sel[woff + pre] = key;
                desc[w + woff + pre] = make_int2(q, S);
            }
            __syncthreads();
            for (int c = wv; c < tot; c += 4) {
                const int kq = sel[c] / nb, kS = sel[c] % nb;
                const int i = lane & 15, kk = lane >> 4;
                const int p = blk_orb[Ab * 4 + (i >> 2)], r = blk_orb[Bb * 4 + (i & 3)], s = blk_orb[kS * 4 + kk];
                double v = 0.0;
                if (p >= 0 && r >= 0 && s >= 0) {
                    v = eri_value(E, p, kq, r, s);
                    if (!(fabs(v) > tau)) v = 0.0;
                    // one-body units in alpha-beta form (hs holds the kept h)
                    if (hs && r == s) v += 0.5 * hs[p * n + kq];
                    if (hs && p == kq) v += 0.5 * hs[r * n + s];
                }
                val[(size_t)(w + c) * 64 + lane] = v;
            }
            w += tot;
            cnt += tot;
            __syncthreads();   // ws and sel are reused by the next batch
        }
        if (threadIdx.x == 0) cls[g * 3 + lc] = cnt;
    }
}

// spaces up to this many determinants take the one-body units into the
// tiles by default (fewer launches; measured faster up to about 10^5)
static constexpr int64_t kObTilesMaxDim = 65536;

// blocks of four orbitals, inner / outer pure (split at the level boundary;
// for the excitation hierarchy the occupied block is {0, 1, -, -}); target
// tiles with level <= L; column chunks
static isci_status build_tiles(isci_ctx *c, const EriSrc &E, hipStream_t s)
{
    const int n = c->norb;
    // orbitals of each block slot, -1 for padding (16 bits: up to 255
    // orbitals): the inner orbitals 0..b-1 in blocks of four (the last one
    // short), then the outer ones in blocks of four from b
    const int bnd = std::min(c->sa.nocc, n);
    std::vector<int16_t> bo;
    for (int v = 0; v < bnd; v += 4)
        for (int k = 0; k < 4; ++k) bo.push_back((int16_t)(v + k < bnd ? v + k : -1));
    const int nib = (int)bo.size() / 4;
    for (int v = bnd; v < n; v += 4)
        for (int k = 0; k < 4; ++k) bo.push_back((int16_t)(v + k < n ? v + k : -1));
    const int nb = (int)bo.size() / 4;
    c->ab_b = bnd;
    c->ab_nib = nib;
    std::vector<int> ob(n, 0);
    for (int b = 0; b < nb; ++b)
        for (int k = 0; k < 4; ++k)
            if (bo[b * 4 + k] >= 0) ob[bo[b * 4 + k]] = b;
    std::vector<uchar4> quads;
    for (int X = 0; X < nb; ++X)
        for (int P = X; P < nb; ++P)
            for (int Y = 0; Y < nb; ++Y)
                for (int R = Y; R < nb; ++R) {
                    const int lev = (X >= nib) + (P >= nib) + (Y >= nib) + (R >= nib);
                    if (lev > c->L) continue;
                    quads.push_back(make_uchar4((unsigned char)X, (unsigned char)P, (unsigned char)Y, (unsigned char)R));
                }
    c->nblk = nb;
    c->nquad = (int)quads.size();
    DevTabs &d = c->d;
    d.blk_orb = (int16_t *)dev_alloc(c, sizeof(int16_t) * bo.size());
    d.quads = (uchar4 *)dev_alloc(c, sizeof(uchar4) * std::max<size_t>(1, quads.size()));
    int *dob = (int *)dev_alloc(c, sizeof(int) * n);
    const long long nkeys = (long long)nb * nb * n * nb;
    unsigned *bits = nullptr;
    ISCI_HIP(hipMallocAsync((void **)&bits, sizeof(unsigned) * (size_t)((nkeys + 31) / 32 + 1), s));
    d.chunk_off = (int *)dev_alloc(c, sizeof(int) * (nb * nb + 1));
    if (!d.blk_orb || !d.quads || !dob || !d.chunk_off) { set_error("device allocation failed (tiles)"); return ISCI_E_OOM; }
    ISCI_HIP(hipMemcpyAsync(d.blk_orb, bo.data(), sizeof(int16_t) * bo.size(), hipMemcpyHostToDevice, s));
    if (!quads.empty())
        ISCI_HIP(hipMemcpyAsync(d.quads, quads.data(), sizeof(uchar4) * quads.size(), hipMemcpyHostToDevice, s));
    ISCI_HIP(hipMemcpyAsync(dob, ob.data(), sizeof(int) * n, hipMemcpyHostToDevice, s));
    ISCI_HIP(hipMemsetAsync(bits, 0, sizeof(unsigned) * (size_t)((nkeys + 31) / 32 + 1), s));
    ISCI_HIP(hipMemsetAsync(d.chunk_off, 0, sizeof(int) * (nb * nb + 1), s));
    const int64_t n3 = (int64_t)n * n * n;
    const size_t nbits = sizeof(unsigned) * (size_t)((nkeys + 31) / 32 + 1);
    k_chunk_mark<<<(unsigned)((n3 + 255) / 256), 256, 0, s>>>(d.ab_off, d.ab_s, n, dob, nb, bits);
    ISCI_HIP(hipGetLastError());
    // chunk count of a mark set (offsets left in chunk_off)
    auto count_chunks = [&](const unsigned *b, int *tot) -> isci_status {
        ISCI_HIP(hipMemsetAsync(d.chunk_off, 0, sizeof(int) * (nb * nb + 1), s));
        k_chunk_count<<<nb * nb, 256, 0, s>>>(b, n, nb, d.chunk_off);
        ISCI_HIP(hipGetLastError());
        isci_status st = scan_inplace<int>(d.chunk_off, nb * nb + 1, s);
        if (st != ISCI_OK) return st;
        ISCI_HIP(hipMemcpyAsync(tot, d.chunk_off + nb * nb, sizeof(int), hipMemcpyDeviceToHost, s));
        ISCI_HIP(hipStreamSynchronize(s));   // also keeps the host tables above alive until copied
        return ISCI_OK;
    };
    int tot = 0;
    isci_status st = count_chunks(bits, &tot);
    if (st != ISCI_OK) return st;
    // the one-body units join the tiles when asked to, or by default when
    // that adds at most one chunk in eight (dense integrals: their chunks
    // are mostly there already) or the space is small (launch latency
    // outweighs the extra tiles); else they keep their own kernels
    bool merged = false;
    // below three orbitals (no virtual orbital) the one-body kernels do not
    // apply: the tiles always carry the units there
    // (a GAS-restricted handle always: the one-body kernels take orbitals 0
    // and 1 as the occupied ones)
    if (d.hscreen && (c->ob_place != ISCI_OB_SEPARATE || n < 3 || c->gas_bnd)) {
        unsigned *bits1 = nullptr;
        ISCI_HIP(hipMallocAsync((void **)&bits1, nbits, s));
        ISCI_HIP(hipMemcpyAsync(bits1, bits, nbits, hipMemcpyDeviceToDevice, s));
        k_chunk_mark_1b<<<(unsigned)((n * n + 255) / 256), 256, 0, s>>>(d.hscreen, n, dob, nb, bits1);
        ISCI_HIP(hipGetLastError());
        int tot1 = 0;
        st = count_chunks(bits1, &tot1);
        if (st != ISCI_OK) return st;
        if (c->ob_place == ISCI_OB_TILES || n < 3 || c->gas_bnd || (long long)tot1 * 8 <= (long long)tot * 9 ||
            c->dim <= kObTilesMaxDim) {
            merged = true;
            std::swap(bits, bits1);
            tot = tot1;
        } else {
            st = count_chunks(bits, &tot);
            if (st != ISCI_OK) return st;
        }
        ISCI_HIP(hipFreeAsync(bits1, s));
    }
    d.chunk_desc = (int2 *)dev_alloc(c, sizeof(int2) * std::max(1, tot));
    // one more chunk, all zero: the product kernels point past-the-end
    // loads at it instead of selecting zeros
    d.chunk_val = (double *)dev_alloc(c, sizeof(double) * 64 * ((size_t)std::max(1, tot) + 1));
    d.chunk_cls = (int *)dev_alloc(c, sizeof(int) * 3 * nb * nb);
    if (!d.chunk_desc || !d.chunk_val || !d.chunk_cls) { set_error("device allocation failed (chunks)"); return ISCI_E_OOM; }
    ISCI_HIP(hipMemsetAsync(d.chunk_val + (size_t)64 * tot, 0, sizeof(double) * 64, s));
    k_chunk_fill<<<nb * nb, 256, 0, s>>>(bits, E, merged ? d.hscreen : nullptr, n, nb, bnd, nib, c->tau, d.blk_orb,
                                          d.chunk_off, d.chunk_desc, d.chunk_val, d.chunk_cls);
    ISCI_HIP(hipGetLastError());
    ISCI_HIP(hipFreeAsync(bits, s));
    ISCI_HIP(hipStreamSynchronize(s));
    c->nchunk = tot;
    c->have_tiles = true;
    c->onebody_in_tiles = merged;
    return ISCI_OK;
}

// alpha-beta product path (unfold -> block-sparse GEMM -> fold); its
// per-call operands T and S are bounded (four vectors per pass)
static constexpr size_t kAbxMaxBytes = (size_t)2 << 30;

static isci_status build_abx(isci_ctx *c, hipStream_t s)
{
    const int n = c->norb, nb = c->nblk, L = c->L, nib = c->ab_nib, bnd = c->ab_b;
    if (nb < 1 || c->nchunk == 0) return ISCI_OK;
    // slots of block B, its orbital i, its level (1: outer)
    auto width = [&](int B) { return B < nib ? std::min(4, bnd - 4 * B) : 4; };
    auto orbital = [&](int B, int i) { return B < nib ? 4 * B + i : bnd + 4 * (B - nib) + i; };
    auto outer = [&](int B) { return B >= nib ? 1 : 0; };
    // chunk lists from the device
    std::vector<int> off(nb * nb + 1), cls(3 * nb * nb);
    std::vector<int2> desc(c->nchunk);
    ISCI_HIP(hipMemcpyAsync(off.data(), c->d.chunk_off, sizeof(int) * off.size(), hipMemcpyDeviceToHost, s));
    ISCI_HIP(hipMemcpyAsync(cls.data(), c->d.chunk_cls, sizeof(int) * cls.size(), hipMemcpyDeviceToHost, s));
    ISCI_HIP(hipMemcpyAsync(desc.data(), c->d.chunk_desc, sizeof(int2) * c->nchunk, hipMemcpyDeviceToHost, s));
    ISCI_HIP(hipStreamSynchronize(s));
    // The operand layout for VS vector slots per spectator pair (four for the
    // passes of a sigma call, one for single-vector calls): column groups
    // level by level (each level padded to 64 columns), the valid prefix of
    // each class, the T rows (4 per (q, S) that opens a chunk whose class
    // admits some spectator) and the S blocks (row block pairs holding chunks)
    struct Layout {
        std::vector<int> gofs, col, rows;
        int pcols[3] = {0, 0, 0};
        std::vector<int> krow_of;
        std::vector<int4> trow;
        std::vector<int2> chunk;
        std::vector<long long> soff;
        size_t tsize = 0, ssize = 0;
        bool fits = true;
    };
    auto layout = [&](int VS, Layout &Y) {
        Y.gofs.assign((size_t)nb * nb, -1);
        int plev[3] = {0, 0, 0};
        for (int lev = 0; lev <= 2; ++lev) {
            if (lev <= L)
                for (int C = 0; C < nb; ++C)
                    for (int D = 0; D < nb; ++D) {
                        if (outer(C) + outer(D) != lev) continue;
                        Y.gofs[(size_t)C * nb + D] = (int)Y.col.size();
                        for (int ic = 0; ic < width(C); ++ic)
                            for (int id = 0; id < width(D); ++id) {
                                const int x = orbital(C, ic);
                                const int y = orbital(D, id);
                                for (int v = 0; v < VS; ++v)
                                    Y.col.push_back((x < n ? x : 255) | ((y < n ? y : 255) << 8) | (v << 16));
                            }
                    }
            while (Y.col.size() % 64) Y.col.push_back(255 | (255 << 8));
            plev[lev] = (int)Y.col.size();
        }
        for (int k = 0; k < 3; ++k) Y.pcols[k] = L - k < 0 ? 0 : plev[std::min(2, L - k)];
        Y.krow_of.assign((size_t)n * nb, -1);
        Y.chunk.assign(c->nchunk, make_int2(0, 0));
        for (int g = 0; g < nb * nb; ++g) {
            int e = off[g];
            for (int l = 0; l < 3; ++l)
                for (int i = 0; i < cls[3 * g + l]; ++i, ++e) {
                    if (Y.pcols[l] == 0) continue;
                    const int q = desc[e].x, S = desc[e].y;
                    int &kr = Y.krow_of[(size_t)q * nb + S];
                    if (kr < 0) {
                        kr = (int)Y.trow.size();
                        Y.trow.push_back(make_int4(q, S, (int)0, Y.pcols[l]));
                        if (Y.tsize + (size_t)4 * Y.pcols[l] > (size_t)INT32_MAX) { Y.fits = false; return; }   // offsets stay int
                        Y.trow.back().z = (int)Y.tsize;
                        Y.tsize += (size_t)4 * Y.pcols[l];
                    }
                    Y.chunk[e] = make_int2(Y.trow[kr].z, Y.trow[kr].w);
                }
        }
        Y.soff.assign((size_t)nb * nb, -1);
        for (int g = 0; g < nb * nb; ++g) {
            const int m = outer(g / nb) + outer(g % nb);
            if (off[g + 1] == off[g] || Y.pcols[m] == 0) continue;
            Y.soff[g] = (long long)Y.ssize;
            Y.rows.push_back(g);
            Y.ssize += (size_t)16 * Y.pcols[m];
        }
    };
    Layout Y4;
    layout(4, Y4);
    if (!Y4.fits) return ISCI_OK;
    const size_t tbytes = sizeof(double) * std::max<size_t>(1, Y4.tsize);
    const size_t sbytes = sizeof(double) * std::max<size_t>(1, Y4.ssize);
    if (tbytes + sbytes > kAbxMaxBytes) return ISCI_OK;   // gathered kernel instead
    // product tiles column slab by column slab (all row block pairs of a
    // slab of kAbSlabCols columns together: the slab of T they read, a few
    // MB, stays in one XCD's L2), the kAbTile-column tiles of one row block
    // pair in a slab next to each other (their chunk values are read from
    // memory once and then from L2), cost ~ chunks applied + 1, cut into
    // eight contiguous runs of about equal cost (one per XCD); for the chunk
    // lists given by (offsets, class counts) and a layout's columns
    auto make_tiles = [&](const std::vector<int> &loff, const std::vector<int> &lcls, const Layout &Y, int &xmax_out) {
        const int *pcols = Y.pcols;
        std::vector<int2> tiles;
        std::vector<double> cost;
        const int nslab = (std::max(pcols[0], std::max(pcols[1], pcols[2])) + kAbTile - 1) / kAbTile;
        constexpr int sgrp = kAbSlabCols / kAbTile;
        for (int sg = 0; sg < nslab; sg += sgrp)
            for (int g : Y.rows)
                for (int sl = sg; sl < std::min(sg + sgrp, nslab); ++sl) {
                    const int m = outer(g / nb) + outer(g % nb);
                    if (sl * kAbTile >= pcols[m]) continue;
                    int ne = 0;
                    for (int l = 0; l < 3; ++l)
                        if (sl * kAbTile < pcols[std::max(l, m)]) ne += lcls[3 * g + l];
                    tiles.push_back(make_int2(g, sl));
                    cost.push_back(1.0 + ne);
                }
        double total = 0.0;
        for (double w : cost) total += w;
        std::vector<int> xrun(9, 0);
        {
            double acc = 0.0;
            int r = 1;
            for (size_t t = 0; t < tiles.size() && r < 8; ++t) {
                acc += cost[t];
                while (r < 8 && acc >= total * r / 8.0) xrun[r++] = (int)t + 1;
            }
            while (r < 8) xrun[r++] = (int)tiles.size();
            xrun[8] = (int)tiles.size();
        }
        int xmax = 0;
        for (int r = 0; r < 8; ++r) xmax = std::max(xmax, xrun[r + 1] - xrun[r]);
        // workgroup b runs on XCD b % 8 and takes tile b / 8 of that XCD's run
        std::vector<AbBlk> blk((size_t)8 * std::max(xmax, 1));
        for (size_t b = 0; b < blk.size(); ++b) {
            AbBlk &e = blk[b];
            e = AbBlk{-1, 0, 0, 0, {0, 0, 0}, 0};
            const int r = (int)(b % 8), t = xrun[r] + (int)(b / 8);
            if (t >= xrun[r + 1]) continue;
            const int g = tiles[t].x;
            e.g = g;
            e.c0 = tiles[t].y * kAbTile;
            e.eb = loff[g];
            int acc = loff[g];
            for (int l = 0; l < 3; ++l) e.end[l] = (acc += lcls[3 * g + l]);
        }
        xmax_out = xmax;
        return blk;
    };
    int xmax = 0;
    const std::vector<AbBlk> blk = make_tiles(off, cls, Y4, xmax);
    // packed chunks: the columns (q, s) of a row block pair's chunks of one
    // class that hold a kept value, four per chunk in list order (a short
    // last chunk of a class is filled with zero columns reading a valid row);
    // psel keeps each packed column's (chunk, column k) so the row offsets of
    // another layout follow from the same selection
    std::vector<double> cval((size_t)64 * c->nchunk);
    ISCI_HIP(hipMemcpyAsync(cval.data(), c->d.chunk_val, sizeof(double) * cval.size(), hipMemcpyDeviceToHost, s));
    ISCI_HIP(hipStreamSynchronize(s));
    std::vector<int> poff(nb * nb + 1, 0), pcls(3 * nb * nb, 0);
    std::vector<int2> psel;
    std::vector<double> pval;
    for (int g = 0; g < nb * nb; ++g) {
        poff[g] = (int)(psel.size() / 4);
        int e = off[g];
        for (int l = 0; l < 3; ++l) {
            std::vector<int2> cols;   // (chunk, column k)
            for (int i = 0; i < cls[3 * g + l]; ++i, ++e) {
                if (Y4.pcols[l] == 0) continue;
                for (int k = 0; k < 4; ++k) {
                    bool any = false;
                    for (int r = 0; r < 16; ++r) any |= cval[(size_t)e * 64 + 16 * k + r] != 0.0;
                    if (any) cols.push_back(make_int2(e, k));
                }
            }
            const int npc = (int)(cols.size() + 3) / 4;
            for (int pc = 0; pc < npc; ++pc) {
                const size_t base = pval.size();
                pval.resize(base + 64, 0.0);
                for (int k = 0; k < 4; ++k) {
                    const size_t ci = (size_t)pc * 4 + k;
                    const int2 ck = cols[ci < cols.size() ? ci : (size_t)pc * 4];
                    psel.push_back(ck);
                    if (ci < cols.size())
                        for (int r = 0; r < 16; ++r) pval[base + 16 * k + r] = cval[(size_t)ck.x * 64 + 16 * ck.y + r];
                }
            }
            pcls[3 * g + l] = npc;
        }
    }
    poff[nb * nb] = (int)(psel.size() / 4);
    auto pchunk_of = [&](const Layout &Y) {
        std::vector<int4> pc(psel.size() / 4);
        for (size_t i = 0; i < pc.size(); ++i) {
            int rowk[4];
            for (int k = 0; k < 4; ++k) {
                const int2 ck = psel[4 * i + k];
                rowk[k] = Y.chunk[ck.x].x + ck.y * Y.chunk[ck.x].y;
            }
            pc[i] = make_int4(rowk[0], rowk[1], rowk[2], rowk[3]);
        }
        return pc;
    };
    const std::vector<int4> pchunk = pchunk_of(Y4);
    int pxmax = 0;
    const std::vector<AbBlk> pblk = make_tiles(poff, pcls, Y4, pxmax);
    // the narrow layouts (packed product only) for passes of one and two
    // vectors: their own column groups, T rows and S blocks over the same
    // chunks, and their own T, whose entries that no determinant fills must
    // stay zero (S is shared)
    Layout YN[2];
    int pxmaxn[2] = {0, 0};
    std::vector<int4> pchunkn[2];
    std::vector<AbBlk> pblkn[2];
    for (int w = 0; w < 2; ++w) {
        layout(w + 1, YN[w]);
        if (YN[w].fits && YN[w].ssize <= Y4.ssize && !pchunk.empty()) {
            pchunkn[w] = pchunk_of(YN[w]);
            pblkn[w] = make_tiles(poff, pcls, YN[w], pxmaxn[w]);
        }
    }
    auto tq_of = [&](const Layout &Y) {
        std::vector<int2> t((size_t)n * nb, make_int2(0, 0));
        for (size_t i = 0; i < t.size(); ++i)
            if (Y.krow_of[i] >= 0) t[i] = make_int2(Y.trow[Y.krow_of[i]].z, Y.trow[Y.krow_of[i]].w);
        return t;
    };
    const std::vector<int2> tq = tq_of(Y4);
    DevTabs &d = c->d;
    d.abx_gofs = (int *)dev_alloc(c, sizeof(int) * Y4.gofs.size());
    d.abx_col = (int *)dev_alloc(c, sizeof(int) * Y4.col.size());
    d.abx_trow = (int4 *)dev_alloc(c, sizeof(int4) * std::max<size_t>(1, Y4.trow.size()));
    d.abx_tq = (int2 *)dev_alloc(c, sizeof(int2) * (size_t)n * nb);
    d.abx_chunk = (int2 *)dev_alloc(c, sizeof(int2) * Y4.chunk.size());
    d.abx_ctof = (int *)dev_alloc(c, sizeof(int) * (Y4.chunk.size() + 8));
    d.abx_rows = (int *)dev_alloc(c, sizeof(int) * std::max<size_t>(1, Y4.rows.size()));
    d.abx_soff = (long long *)dev_alloc(c, sizeof(long long) * Y4.soff.size());
    d.abx_blk = (AbBlk *)dev_alloc(c, sizeof(AbBlk) * blk.size());
    d.abx_pchunk = (int4 *)dev_alloc(c, sizeof(int4) * std::max<size_t>(1, pchunk.size()));
    d.pchunk_val = (double *)dev_alloc(c, sizeof(double) * std::max<size_t>(64, pval.size()));
    d.abx_pblk = (AbBlk *)dev_alloc(c, sizeof(AbBlk) * pblk.size());
    d.abx_T = (double *)dev_alloc(c, tbytes);
    d.abx_S = (double *)dev_alloc(c, sbytes);
    if (!d.abx_gofs || !d.abx_col || !d.abx_trow || !d.abx_tq || !d.abx_chunk || !d.abx_ctof || !d.abx_rows || !d.abx_soff || !d.abx_blk ||
        !d.abx_pchunk || !d.pchunk_val || !d.abx_pblk || !d.abx_T || !d.abx_S) {
        set_error("device allocation failed (alpha-beta product)");
        return ISCI_E_OOM;
    }
    ISCI_HIP(hipMemcpyAsync(d.abx_gofs, Y4.gofs.data(), sizeof(int) * Y4.gofs.size(), hipMemcpyHostToDevice, s));
    ISCI_HIP(hipMemcpyAsync(d.abx_col, Y4.col.data(), sizeof(int) * Y4.col.size(), hipMemcpyHostToDevice, s));
    if (!Y4.trow.empty())
        ISCI_HIP(hipMemcpyAsync(d.abx_trow, Y4.trow.data(), sizeof(int4) * Y4.trow.size(), hipMemcpyHostToDevice, s));
    ISCI_HIP(hipMemcpyAsync(d.abx_tq, tq.data(), sizeof(int2) * tq.size(), hipMemcpyHostToDevice, s));
    // entries of T that no determinant of the space fills stay zero; the
    // scatter unfold writes the others every call
    ISCI_HIP(hipMemsetAsync(d.abx_T, 0, tbytes, s));
    ISCI_HIP(hipMemcpyAsync(d.abx_chunk, Y4.chunk.data(), sizeof(int2) * Y4.chunk.size(), hipMemcpyHostToDevice, s));
    std::vector<int> ctof(Y4.chunk.size() + 8, 0);
    for (size_t e = 0; e < Y4.chunk.size(); ++e) ctof[e] = Y4.chunk[e].x;
    ISCI_HIP(hipMemcpyAsync(d.abx_ctof, ctof.data(), sizeof(int) * ctof.size(), hipMemcpyHostToDevice, s));
    if (!Y4.rows.empty())
        ISCI_HIP(hipMemcpyAsync(d.abx_rows, Y4.rows.data(), sizeof(int) * Y4.rows.size(), hipMemcpyHostToDevice, s));
    ISCI_HIP(hipMemcpyAsync(d.abx_soff, Y4.soff.data(), sizeof(long long) * Y4.soff.size(), hipMemcpyHostToDevice, s));
    ISCI_HIP(hipMemcpyAsync(d.abx_blk, blk.data(), sizeof(AbBlk) * blk.size(), hipMemcpyHostToDevice, s));
    if (!pchunk.empty()) {
        ISCI_HIP(hipMemcpyAsync(d.abx_pchunk, pchunk.data(), sizeof(int4) * pchunk.size(), hipMemcpyHostToDevice, s));
        ISCI_HIP(hipMemcpyAsync(d.pchunk_val, pval.data(), sizeof(double) * pval.size(), hipMemcpyHostToDevice, s));
    }
    ISCI_HIP(hipMemcpyAsync(d.abx_pblk, pblk.data(), sizeof(AbBlk) * pblk.size(), hipMemcpyHostToDevice, s));
    for (int w = 0; w < 2; ++w) {
        if (pblkn[w].empty()) continue;
        const Layout &Y = YN[w];
        const std::vector<int2> tqn = tq_of(Y);
        const size_t tb = sizeof(double) * std::max<size_t>(1, Y.tsize);
        auto &x = d.abxn[w];
        x.gofs = (int *)dev_alloc(c, sizeof(int) * Y.gofs.size());
        x.tq = (int2 *)dev_alloc(c, sizeof(int2) * tqn.size());
        x.soff = (long long *)dev_alloc(c, sizeof(long long) * Y.soff.size());
        x.pchunk = (int4 *)dev_alloc(c, sizeof(int4) * pchunkn[w].size());
        x.pblk = (AbBlk *)dev_alloc(c, sizeof(AbBlk) * pblkn[w].size());
        x.T = (double *)dev_alloc(c, tb);
        if (!x.gofs || !x.tq || !x.soff || !x.pchunk || !x.pblk || !x.T) {
            set_error("device allocation failed (narrow alpha-beta product layout)");
            return ISCI_E_OOM;
        }
        ISCI_HIP(hipMemcpyAsync(x.gofs, Y.gofs.data(), sizeof(int) * Y.gofs.size(), hipMemcpyHostToDevice, s));
        ISCI_HIP(hipMemcpyAsync(x.tq, tqn.data(), sizeof(int2) * tqn.size(), hipMemcpyHostToDevice, s));
        ISCI_HIP(hipMemcpyAsync(x.soff, Y.soff.data(), sizeof(long long) * Y.soff.size(), hipMemcpyHostToDevice, s));
        ISCI_HIP(hipMemcpyAsync(x.pchunk, pchunkn[w].data(), sizeof(int4) * pchunkn[w].size(), hipMemcpyHostToDevice, s));
        ISCI_HIP(hipMemcpyAsync(x.pblk, pblkn[w].data(), sizeof(AbBlk) * pblkn[w].size(), hipMemcpyHostToDevice, s));
        ISCI_HIP(hipMemsetAsync(x.T, 0, tb, s));
        ISCI_HIP(hipStreamSynchronize(s));   // tqn dies here
        for (int k = 0; k < 3; ++k) c->abxn_pcols[w][k] = Y.pcols[k];
        c->abxn_pxmax[w] = pxmaxn[w];
        c->have_abxn[w] = true;
    }
    ISCI_HIP(hipStreamSynchronize(s));   // host tables above are freed on return
    c->abx_ntrow = (int)Y4.trow.size();
    c->abx_nrows = (int)Y4.rows.size();
    c->abx_sbytes = sbytes;
    c->abx_xmax = xmax;
    c->abx_pxmax = pxmax;
    c->npchunk = (int)pchunk.size();
    for (int k = 0; k < 3; ++k) c->abx_pcols[k] = Y4.pcols[k];
    c->have_abx = true;
    return ISCI_OK;
}

// Scratch of the transposed-block one-body routes: the beta class above
// kObMaxNorb as the alpha class of the transposed block (where the beta
// rows do not fit LDS, or on request), and the full-CI alpha class up to
// kObMaxNorb as the beta class of the transposed block.  A block of vectors
// and its image: eight vectors (one pass per sigma block) for full CI up to
// 80 orbitals and 4 Mi determinants, else four.
static isci_status alloc_onebody_scratch(isci_ctx *c)
{
    if (c->d.obT_c && c->d.obT_s) return ISCI_OK;
    c->obT_nv = (c->norb <= kObMaxNorb && c->dim <= ((int64_t)1 << 22)) ? 8 : 4;
    c->d.obT_c = (double *)dev_alloc(c, sizeof(double) * c->obT_nv * (size_t)c->dim);
    c->d.obT_s = (double *)dev_alloc(c, sizeof(double) * c->obT_nv * (size_t)c->dim);
    if (!c->d.obT_c || !c->d.obT_s) {
        set_error("device allocation failed (one-body scratch)");
        return ISCI_E_OOM;
    }
    return ISCI_OK;
}

static isci_status build_hscreen(isci_ctx *c, const double *h, hipStream_t s)
{
    const int n = c->norb;
    c->d.hscreen = (double *)dev_alloc(c, sizeof(double) * n * n);
    if (!c->d.hscreen) { set_error("device allocation failed (h)"); return ISCI_E_OOM; }
    k_hscreen<<<(n * n + 255) / 256, 256, 0, s>>>(h, n, c->tau, c->d.hscreen);
    ISCI_HIP(hipGetLastError());
    if (n <= 256) {
        c->d.hkmask = (unsigned long long *)dev_alloc(c, sizeof(unsigned long long) * 16);
        if (!c->d.hkmask) { set_error("device allocation failed (h masks)"); return ISCI_E_OOM; }
        k_hkmask<<<1, 64, 0, s>>>(c->d.hscreen, n, c->d.hkmask);
        ISCI_HIP(hipGetLastError());
    }
    if (n > kObMaxNorb && n <= 256) {
        // zero-padded copy to whole 16-orbital tiles for the beta row kernel
        const int P = 16 * ((n + 15) / 16);
        c->d.hpadT = (double *)dev_alloc(c, sizeof(double) * P * P);
        if (!c->d.hpadT) { set_error("device allocation failed (h)"); return ISCI_E_OOM; }
        k_hpad<<<(P * P + 255) / 256, 256, 0, s>>>(c->d.hscreen, n, P, c->d.hpadT);
        ISCI_HIP(hipGetLastError());
    }
    if (n <= kObMaxNorb) {
        // zero-padded copy: the matrix-core one-body kernels load their h
        // operands with no bounds conditions
        constexpr int P = kObMaxNorb;
        c->d.hpad = (double *)dev_alloc(c, sizeof(double) * P * P);
        if (!c->d.hpad) { set_error("device allocation failed (h)"); return ISCI_E_OOM; }
        k_hpad<<<(P * P + 255) / 256, 256, 0, s>>>(c->d.hscreen, n, P, c->d.hpad);
        ISCI_HIP(hipGetLastError());
    }
    return ISCI_OK;
}

static isci_status build_lists(isci_ctx *c, const double *h, const EriSrc &E, hipStream_t s)
{
    const int n = c->norb;
    const int64_t n3 = (int64_t)n * n * n;
    const int np = n * (n - 1) / 2;
    DevTabs &d = c->d;
    d.h_off = (int *)dev_alloc(c, sizeof(int) * (n + 1));
    d.ss_off = (int *)dev_alloc(c, sizeof(int) * (np + 1));
    d.ab_off = (long long *)dev_alloc(c, sizeof(long long) * (n3 + 1));
    d.pq_off = (int *)dev_alloc(c, sizeof(int) * (n + 1));
    d.counters = (unsigned long long *)dev_alloc(c, sizeof(unsigned long long) * 2 * ISCI_NBUCKET);
    d.hd = (double *)dev_alloc(c, sizeof(double) * n);
    d.jj = (double *)dev_alloc(c, sizeof(double) * n * n);
    d.ssd = (double *)dev_alloc(c, sizeof(double) * n * n);
    if (!d.h_off || !d.ss_off || !d.ab_off || !d.pq_off || !d.counters || !d.hd || !d.jj || !d.ssd) {
        set_error("device allocation failed (list offsets)");
        return ISCI_E_OOM;
    }
    ISCI_HIP(hipMemsetAsync(d.counters, 0, sizeof(unsigned long long) * 2 * ISCI_NBUCKET, s));
    ISCI_HIP(hipMemsetAsync(d.h_off, 0, sizeof(int) * (n + 1), s));
    ISCI_HIP(hipMemsetAsync(d.ss_off, 0, sizeof(int) * (np + 1), s));
    ISCI_HIP(hipMemsetAsync(d.ab_off, 0, sizeof(long long) * (n3 + 1), s));
    ISCI_HIP(hipMemsetAsync(d.pq_off, 0, sizeof(int) * (n + 1), s));

    k_h_count<<<nblk(n, 64), 64, 0, s>>>(h, n, c->tau, d.h_off);
    if (np > 0) k_ss_count<<<nblk(np, 64), 64, 0, s>>>(E, c->tau, d.ss_off);
    k_ab_count<<<nblk(n3, 256), 256, 0, s>>>(E, c->tau, d.ab_off);
    k_diag_units<<<nblk((int64_t)n * n, 256), 256, 0, s>>>(h, E, d.hd, d.jj, d.ssd);
    ISCI_HIP(hipGetLastError());
    isci_status st;
    if ((st = scan_inplace<int>(d.h_off, n + 1, s)) != ISCI_OK) return st;
    if ((st = scan_inplace<int>(d.ss_off, np + 1, s)) != ISCI_OK) return st;
    if ((st = scan_inplace<long long>(d.ab_off, n3 + 1, s)) != ISCI_OK) return st;
    k_pq_count<<<nblk(n, 64), 64, 0, s>>>(d.ab_off, n, d.pq_off);
    ISCI_HIP(hipGetLastError());
    if ((st = scan_inplace<int>(d.pq_off, n + 1, s)) != ISCI_OK) return st;

    int tot[4];
    long long tot_ab = 0;
    ISCI_HIP(hipMemcpyAsync(&tot[0], d.h_off + n, sizeof(int), hipMemcpyDeviceToHost, s));
    ISCI_HIP(hipMemcpyAsync(&tot[1], d.ss_off + np, sizeof(int), hipMemcpyDeviceToHost, s));
    ISCI_HIP(hipMemcpyAsync(&tot_ab, d.ab_off + n3, sizeof(long long), hipMemcpyDeviceToHost, s));
    ISCI_HIP(hipMemcpyAsync(&tot[3], d.pq_off + n, sizeof(int), hipMemcpyDeviceToHost, s));
    ISCI_HIP(hipStreamSynchronize(s));

    d.h_q = (uint8_t *)dev_alloc(c, tot[0]);
    d.h_v = (double *)dev_alloc(c, sizeof(double) * tot[0]);
    d.ss_qs = (uint16_t *)dev_alloc(c, sizeof(uint16_t) * tot[1]);
    d.ss_v = (double *)dev_alloc(c, sizeof(double) * tot[1]);
    d.ab_s = (uint8_t *)dev_alloc(c, (size_t)tot_ab);
    d.ab_v = (double *)dev_alloc(c, sizeof(double) * (size_t)tot_ab);
    d.pq_q = (uint8_t *)dev_alloc(c, tot[3]);
    if (!d.h_q || !d.h_v || !d.ss_qs || !d.ss_v || !d.ab_s || !d.ab_v || !d.pq_q) {
        set_error("device allocation failed (lists)");
        return ISCI_E_OOM;
    }
    k_h_fill<<<nblk(n, 64), 64, 0, s>>>(h, n, c->tau, d.h_off, d.h_q, d.h_v, c->sa, c->sb, c->L, d.counters);
    if (np > 0)
        k_ss_fill<<<nblk(np, 64), 64, 0, s>>>(E, c->tau, d.ss_off, d.ss_qs, d.ss_v, c->sa, c->sb, c->L,
                                               d.counters);
    k_ab_fill<<<nblk(n3, 256), 256, 0, s>>>(E, c->tau, d.ab_off, d.ab_s, d.ab_v, c->sa, c->sb, c->L,
                                             d.counters);
    k_pq_fill<<<nblk(n, 64), 64, 0, s>>>(d.ab_off, n, d.pq_off, d.pq_q);
    ISCI_HIP(hipGetLastError());
    unsigned long long ctr[2 * ISCI_NBUCKET];
    ISCI_HIP(hipMemcpyAsync(ctr, d.counters, sizeof(ctr), hipMemcpyDeviceToHost, s));
    ISCI_HIP(hipStreamSynchronize(s));
    c->stats.kept_total = 0;
    c->stats.terms_total = 0;
    for (int b = 0; b < ISCI_NBUCKET; ++b) {
        c->stats.kept[b] = (int64_t)ctr[b];
        c->stats.terms[b] = (int64_t)ctr[ISCI_NBUCKET + b];
        c->stats.terms_total += c->stats.terms[b];
    }
    // distinct kept integral units: one-body counted once, same-spin once, alpha-beta once
    c->stats.kept_total = (int64_t)tot[0] + tot[1] + tot_ab;
    c->nkept_h = tot[0];
    c->nkept_ab = tot_ab;
    return ISCI_OK;
}

isci_status prof_mark(const isci_ctx *cc, int k, bool begin, hipStream_t s)
{
    if (!cc->profile) return ISCI_OK;
    isci_ctx *c = const_cast<isci_ctx *>(cc);
    hipEvent_t ev;
    ISCI_HIP(hipEventCreate(&ev));
    ISCI_HIP(hipEventRecord(ev, s));
    (void)begin;
    c->prof_ev[k].push_back(ev);
    return ISCI_OK;
}

static void prof_clear(isci_ctx *c)
{
    for (int k = 0; k < ISCI_NKERNEL_IDS; ++k) {
        for (hipEvent_t e : c->prof_ev[k]) (void)hipEventDestroy(e);
        c->prof_ev[k].clear();
    }
}

static void destroy(isci_ctx *c)
{
    if (!c) return;
    prof_clear(c);
    if (c->ob_stream) {
        (void)hipStreamSynchronize(c->ob_stream);
        (void)hipStreamDestroy(c->ob_stream);
    }
    if (c->ob_fork) (void)hipEventDestroy(c->ob_fork);
    if (c->ob_join) (void)hipEventDestroy(c->ob_join);
    if (c->allocator.free) {
        // the provider may hand the blocks to other work at once: let every
        // launch that reads them finish first, on whichever stream it ran
        (void)hipDeviceSynchronize();
        for (void *p : c->allocs) c->allocator.free(p, c->alloc_stream, c->allocator.ctx);
    } else {
        for (void *p : c->allocs) (void)hipFree(p);
    }
    for (void *p : c->work) (void)hipFree(p);
    delete c;
}

}  // namespace isci

using namespace isci;

extern "C" {

const char *isci_last_error(void) { return g_last_error.c_str(); }

const char *isci_status_string(isci_status s)
{
    switch (s) {
    case ISCI_OK: return "ok";
    case ISCI_E_INVALID: return "invalid argument";
    case ISCI_E_OOM: return "out of device memory";
    case ISCI_E_HIP: return "HIP runtime error";
    case ISCI_E_NOT_CONVERGED: return "not converged";
    case ISCI_E_UNSUPPORTED: return "unsupported by this build";
    }
    return "unknown status";
}

isci_status isci_create(isci_handle *out, const double *h, const double *eri, int norb, int nalpha,
                        int nbeta, int max_excitation, double tau, hipStream_t stream)
{
    return isci_create_ex(out, h, eri, norb, nalpha, nbeta, max_excitation, tau, nullptr, stream);
}

// Shared body of isci_create_ex (dense eri) and isci_create_factored
// (factors Lfac [naux][norb][norb], eri == nullptr).
static isci_status create_impl(isci_handle *out, const double *h, const double *eri, const double *Lfac, int naux,
                               int norb, int nalpha, int nbeta, int max_excitation, double tau,
                               const isci_create_opts *opts, hipStream_t stream)
{
    if (!out) { set_error("out is NULL"); return ISCI_E_INVALID; }
    *out = nullptr;
    const int ob_place = opts ? opts->onebody : ISCI_OB_AUTO;
    if (ob_place != ISCI_OB_AUTO && ob_place != ISCI_OB_SEPARATE && ob_place != ISCI_OB_TILES) {
        set_error("isci_create_opts.onebody must be ISCI_OB_AUTO, ISCI_OB_SEPARATE or ISCI_OB_TILES");
        return ISCI_E_INVALID;
    }
    *out = nullptr;
    const isci_allocator *al = opts ? opts->allocator : nullptr;
    if (al && (!al->alloc || !al->free)) {
        set_error("isci_create_opts.allocator needs both alloc and free");
        return ISCI_E_INVALID;
    }
    if (!h || (!eri && !Lfac)) { set_error("h or the two-electron integrals are NULL"); return ISCI_E_INVALID; }
    if (Lfac && naux < 1) { set_error("naux < 1"); return ISCI_E_INVALID; }
    if (norb < 1) { set_error("norb < 1"); return ISCI_E_INVALID; }
    if (nalpha < 0 || nbeta < 0 || nalpha > norb || nbeta > norb) {
        set_error("electron counts outside [0, norb]");
        return ISCI_E_INVALID;
    }
    if (max_excitation < 0) { set_error("max_excitation < 0"); return ISCI_E_INVALID; }
    if (!(tau >= 0.0) || std::isinf(tau)) { set_error("tau must be finite and >= 0"); return ISCI_E_INVALID; }
    if (norb > ISCI_MAXNORB) { set_error("norb > 255 is not supported"); return ISCI_E_UNSUPPORTED; }
    if (nalpha > ISCI_MAXN || nbeta > ISCI_MAXN) {
        set_error("more than 4 electrons per spin is not supported");
        return ISCI_E_UNSUPPORTED;
    }
    const int gas_bnd = opts ? opts->gas_boundary : 0;
    if (gas_bnd != 0 && (gas_bnd < nalpha || gas_bnd < nbeta || gas_bnd > norb)) {
        set_error("isci_create_opts.gas_boundary must be 0 or within [max(nalpha, nbeta), norb]");
        return ISCI_E_INVALID;
    }
    if (nalpha == 2 && nbeta == 2 && norb > kPairMaxNorb) {
        set_error("two electrons per spin: at most 200 orbitals (the verified range of the large-orbital one-body kernels)");
        return ISCI_E_UNSUPPORTED;
    }
    isci_ctx *c = new (std::nothrow) isci_ctx();
    if (!c) { set_error("host allocation failed"); return ISCI_E_OOM; }
    c->norb = norb; c->na = nalpha; c->nb = nbeta; c->tau = tau;
    c->ob_place = ob_place;
    c->gas_bnd = gas_bnd;
    if (al) c->allocator = *al;
    c->alloc_stream = stream;
    // level boundary per spin: n (excitation hierarchy) or the GAS boundary
    const int ba = c->gas_bnd ? c->gas_bnd : nalpha, bb = c->gas_bnd ? c->gas_bnd : nbeta;
    const int lmax = std::min(nalpha, norb - ba) + std::min(nbeta, norb - bb);
    c->L = std::min(max_excitation, lmax);
    spin_table(c->sa, norb, nalpha, c->L, ba);
    spin_table(c->sb, norb, nbeta, c->L, bb);
    if (hipGetDevice(&c->device) != hipSuccess) { destroy(c); set_error("hipGetDevice failed"); return ISCI_E_HIP; }

    std::vector<uint32_t> pa, pb;
    if (!enumerate(c->sa, norb, c->h_aorb, c->h_alev, pa) || !enumerate(c->sb, norb, c->h_borb, c->h_blev, pb)) {
        destroy(c);
        set_error("internal: string rank is not a bijection");
        return ISCI_E_HIP;
    }
    // rows: alpha strings; row of level k holds beta strings of level <= L - k
    c->h_rowstart.assign((size_t)c->sa.nstr + 1, 0);
    int64_t acc = 0;
    for (int i = 0; i < c->sa.nstr; ++i) {
        c->h_rowstart[i] = acc;
        int64_t len = c->sb.le[c->L - c->h_alev[i]];
        c->max_rowlen = std::max<int>(c->max_rowlen, (int)len);
        acc += len;
    }
    c->h_rowstart[c->sa.nstr] = acc;
    c->dim = acc;
    // work plan of one sigma job: (alpha row, first beta target) per block of
    // 256 targets, rows in layout order
    std::vector<int2> plan;
    for (int i = 0; i < c->sa.nstr; ++i) {
        const int len = (int)(c->h_rowstart[i + 1] - c->h_rowstart[i]);
        for (int b0 = 0; b0 < len; b0 += 256) plan.push_back(make_int2(i, b0));
    }
    c->nplan = (int)plan.size();
    if (acc >= ((int64_t)1 << 62)) { destroy(c); set_error("dimension too large"); return ISCI_E_UNSUPPORTED; }
    c->stats.dim = acc;
    c->stats.nstr_alpha = c->sa.nstr;
    c->stats.nstr_beta = c->sb.nstr;

    // upload string tables
    std::vector<int8_t> la(c->sa.nstr), lb(c->sb.nstr);
    for (int i = 0; i < c->sa.nstr; ++i) la[i] = (int8_t)c->h_alev[i];
    for (int i = 0; i < c->sb.nstr; ++i) lb[i] = (int8_t)c->h_blev[i];
    c->d.astr = (uint32_t *)dev_alloc(c, sizeof(uint32_t) * c->sa.nstr);
    c->d.bstr = (uint32_t *)dev_alloc(c, sizeof(uint32_t) * c->sb.nstr);
    c->d.alev = (int8_t *)dev_alloc(c, c->sa.nstr);
    c->d.blev = (int8_t *)dev_alloc(c, c->sb.nstr);
    c->d.rowstart = (int64_t *)dev_alloc(c, sizeof(int64_t) * (c->sa.nstr + 1));
    c->d.plan = (int2 *)dev_alloc(c, sizeof(int2) * plan.size());
    if (!c->d.astr || !c->d.bstr || !c->d.alev || !c->d.blev || !c->d.rowstart || !c->d.plan) {
        destroy(c);
        set_error("device allocation failed (strings)");
        return ISCI_E_OOM;
    }
    hipError_t e = hipSuccess;
    e = e ? e : hipMemcpyAsync(c->d.astr, pa.data(), sizeof(uint32_t) * pa.size(), hipMemcpyHostToDevice, stream);
    e = e ? e : hipMemcpyAsync(c->d.bstr, pb.data(), sizeof(uint32_t) * pb.size(), hipMemcpyHostToDevice, stream);
    e = e ? e : hipMemcpyAsync(c->d.alev, la.data(), la.size(), hipMemcpyHostToDevice, stream);
    e = e ? e : hipMemcpyAsync(c->d.blev, lb.data(), lb.size(), hipMemcpyHostToDevice, stream);
    e = e ? e : hipMemcpyAsync(c->d.rowstart, c->h_rowstart.data(), sizeof(int64_t) * c->h_rowstart.size(),
                               hipMemcpyHostToDevice, stream);
    e = e ? e : hipMemcpyAsync(c->d.plan, plan.data(), sizeof(int2) * plan.size(), hipMemcpyHostToDevice, stream);
    if (e != hipSuccess) { destroy(c); return hip_fail(e, "upload string tables"); }
    // pair-index tables for two-electron spins
    for (int spin = 0; spin < 2; ++spin) {
        const SpinTab &T = spin ? c->sb : c->sa;
        if (T.n != 2) continue;
        std::vector<int> pidx((size_t)norb * norb, -1);
        for (int a = 0; a < norb; ++a)
            for (int b = 0; b < norb; ++b) {
                if (a == b) continue;
                int o[2] = {std::min(a, b), std::max(a, b)};
                if (str_level(o, 2, T.nocc) > T.maxlev) continue;
                pidx[(size_t)a * norb + b] = str_index(o, T);
            }
        int *dp = (int *)dev_alloc(c, sizeof(int) * pidx.size());
        if (!dp) { destroy(c); set_error("device allocation failed (pair index)"); return ISCI_E_OOM; }
        hipError_t e2 = hipMemcpyAsync(dp, pidx.data(), sizeof(int) * pidx.size(), hipMemcpyHostToDevice, stream);
        if (e2 != hipSuccess) { destroy(c); return hip_fail(e2, "upload pair index"); }
        // the host vector dies here: wait for the copy
        e2 = hipStreamSynchronize(stream);
        if (e2 != hipSuccess) { destroy(c); return hip_fail(e2, "upload pair index"); }
        (spin ? c->d.bpidx : c->d.apidx) = dp;
        if (spin == 0) {
            // alpha row (start, length) of every ordered pair (x, q)
            std::vector<long long> base((size_t)norb * norb, -1);
            std::vector<int> len((size_t)norb * norb, 0);
            for (size_t k = 0; k < pidx.size(); ++k)
                if (pidx[k] >= 0) {
                    base[k] = c->h_rowstart[pidx[k]];
                    len[k] = (int)(c->h_rowstart[pidx[k] + 1] - c->h_rowstart[pidx[k]]);
                }
            c->d.arow_base = (long long *)dev_alloc(c, sizeof(long long) * base.size());
            c->d.arow_len = (int *)dev_alloc(c, sizeof(int) * len.size());
            if (!c->d.arow_base || !c->d.arow_len) { destroy(c); set_error("device allocation failed (row tables)"); return ISCI_E_OOM; }
            e2 = hipMemcpyAsync(c->d.arow_base, base.data(), sizeof(long long) * base.size(), hipMemcpyHostToDevice, stream);
            if (e2 == hipSuccess)
                e2 = hipMemcpyAsync(c->d.arow_len, len.data(), sizeof(int) * len.size(), hipMemcpyHostToDevice, stream);
            if (e2 == hipSuccess) e2 = hipStreamSynchronize(stream);
            if (e2 != hipSuccess) { destroy(c); return hip_fail(e2, "upload row tables"); }
        }
    }
    // integral source; for factors, their transposed copy and norm bounds
    // live for this call only
    EriSrc E{eri, nullptr, nullptr, norb, 0, nullptr, 0.0};
    double *Lt = nullptr, *nrm = nullptr, *dist = nullptr, *hm = nullptr;
    auto free_factors = [&]() {
        if (Lt) (void)hipFreeAsync(Lt, stream);
        if (nrm) (void)hipFreeAsync(nrm, stream);
        if (dist) (void)hipFreeAsync(dist, stream);
        if (hm) (void)hipFreeAsync(hm, stream);
        Lt = nrm = dist = hm = nullptr;
    };
    const bool by_dist = opts && opts->orb_dist && opts->max_dist > 0.0;
    if (opts && opts->orb_dist && !(opts->max_dist >= 0.0)) {
        destroy(c);
        set_error("max_dist is NaN or negative");
        return ISCI_E_INVALID;
    }
    if (by_dist) {
        // the pair distance is the larger of d(p, q) and d(q, p), so that
        // the mask does not depend on the order in which a unit is named
        std::vector<double> dsym((size_t)norb * norb);
        for (int p = 0; p < norb; ++p)
            for (int q = 0; q < norb; ++q) {
                const double a = opts->orb_dist[(size_t)p * norb + q], b = opts->orb_dist[(size_t)q * norb + p];
                if (!std::isfinite(a) || a < 0.0) {
                    destroy(c);
                    set_error("orb_dist holds a NaN, infinite or negative distance");
                    return ISCI_E_INVALID;
                }
                dsym[(size_t)p * norb + q] = std::max(a, b);
            }
        // distance screening: the distances on the device, and h with the
        // elements of distant pairs set to zero (read by every builder)
        hipError_t ed = hipMallocAsync((void **)&dist, sizeof(double) * (size_t)norb * norb, stream);
        if (ed == hipSuccess) ed = hipMallocAsync((void **)&hm, sizeof(double) * (size_t)norb * norb, stream);
        if (ed == hipSuccess)
            ed = hipMemcpyAsync(dist, dsym.data(), sizeof(double) * (size_t)norb * norb, hipMemcpyHostToDevice, stream);
        if (ed == hipSuccess) {
            k_mask_h<<<nblk((int64_t)norb * norb, 256), 256, 0, stream>>>(h, dist, opts->max_dist, norb, hm);
            ed = hipGetLastError();
        }
        if (ed == hipSuccess) ed = hipStreamSynchronize(stream);   // dsym is read
        if (ed != hipSuccess) { free_factors(); (void)hipStreamSynchronize(stream); destroy(c); return hip_fail(ed, "distance screening"); }
        h = hm;
    }
    {
        // refuse non-finite integrals before any list is built
        int *bad = nullptr, hbad = 0;
        const int64_t n3 = (int64_t)norb * norb * norb;
        hipError_t e3 = hipMallocAsync((void **)&bad, sizeof(int), stream);
        if (e3 == hipSuccess) e3 = hipMemsetAsync(bad, 0, sizeof(int), stream);
        if (e3 == hipSuccess && Lfac) {
            e3 = hipMallocAsync((void **)&Lt, sizeof(double) * (size_t)naux * norb * norb, stream);
            if (e3 == hipSuccess) e3 = hipMallocAsync((void **)&nrm, sizeof(double) * (size_t)norb * norb, stream);
            if (e3 == hipSuccess) {
                k_check_finite_h<<<nblk((int64_t)norb * norb, 256), 256, 0, stream>>>(h, norb, bad);
                k_factor_prep<<<nblk((int64_t)norb * norb, 256), 256, 0, stream>>>(Lfac, norb, naux, Lt, nrm, bad);
                e3 = hipGetLastError();
            }
            E = EriSrc{nullptr, Lt, nrm, norb, naux, nullptr, 0.0};
        } else if (e3 == hipSuccess) {
            k_check_finite<<<nblk(n3, 256), 256, 0, stream>>>(h, eri, norb, bad);
            e3 = hipGetLastError();
        }
        if (e3 == hipSuccess) e3 = hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, stream);
        if (bad) (void)hipFreeAsync(bad, stream);
        if (e3 == hipSuccess) e3 = hipStreamSynchronize(stream);
        if (e3 != hipSuccess) { free_factors(); (void)hipStreamSynchronize(stream); destroy(c); return hip_fail(e3, "integral check"); }
        if (hbad) {
            free_factors();
            (void)hipStreamSynchronize(stream);
            destroy(c);
            set_error(Lfac ? "h or the factors hold a NaN or infinite value in a position that is read, or a factor norm overflows"
                           : "h or eri holds a NaN or infinite value in a position that is read");
            return ISCI_E_INVALID;
        }
    }
    if (by_dist) {
        E.dist = dist;
        E.dmax = opts->max_dist;
    }
    isci_status st = build_lists(c, h, E, stream);
    if (st != ISCI_OK) { free_factors(); (void)hipStreamSynchronize(stream); destroy(c); return st; }
    // the matrix-core path for two electrons per spin (orbital blocks split
    // at the level boundary: the two occupied orbitals, or a GAS boundary)
    if (c->sa.n == 2 && c->sb.n == 2 && norb >= 2) {
        st = build_hscreen(c, h, stream);
        if (st == ISCI_OK) st = build_tiles(c, E, stream);
        free_factors();
        if (st == ISCI_OK) st = build_abx(c, stream);
        const bool full_pairs = c->L >= 2 && c->sb.le[c->L - 2] == c->sb.nstr && c->sa.nstr == c->sb.nstr;
        // above kObMaxNorb the beta class runs on the rows where it can
        const bool beta_rows = st == ISCI_OK && norb > kObMaxNorb && onebody_beta_rows_ok(c);
        if (beta_rows) c->ob_kernel = ISCI_ONEBODY_ROWS;
        if (st == ISCI_OK && c->have_tiles && !c->onebody_in_tiles &&
            (norb > kObMaxNorb ? !beta_rows : full_pairs))
            st = alloc_onebody_scratch(c);
        if (st == ISCI_OK && c->have_tiles && !c->onebody_in_tiles && norb <= kObMaxNorb && !full_pairs && c->L >= 2 &&
            c->sa.nstr == c->sb.nstr && c->sb.le[c->L - 2] > 0) {
            // the alpha class on the beta columns that hold every alpha pair,
            // as the beta class of that block transposed: its scratch
            const int64_t jd = c->sb.le[c->L - 2], na = c->sa.nstr;
            c->d.obS_c = (double *)dev_alloc(c, sizeof(double) * 8 * (size_t)(jd * na));
            c->d.obS_s = (double *)dev_alloc(c, sizeof(double) * 8 * (size_t)(jd * na));
            c->d.obS_rs = (int64_t *)dev_alloc(c, sizeof(int64_t) * (size_t)(jd + 1));
            if (!c->d.obS_c || !c->d.obS_s || !c->d.obS_rs) {
                set_error("device allocation failed (one-body scratch)");
                st = ISCI_E_OOM;
            } else {
                std::vector<int64_t> rs((size_t)jd + 1);
                for (int64_t j = 0; j <= jd; ++j) rs[(size_t)j] = j * na;
                hipError_t e5 = hipMemcpyAsync(c->d.obS_rs, rs.data(), sizeof(int64_t) * rs.size(), hipMemcpyHostToDevice,
                                               stream);
                if (e5 == hipSuccess) e5 = hipStreamSynchronize(stream);   // rs dies here
                if (e5 != hipSuccess) st = hip_fail(e5, "one-body block row starts");
            }
        }
        if (st == ISCI_OK && c->have_abx && !c->onebody_in_tiles && onebody_mfma_ok(c)) {
            // side stream (default priority) for the one-body classes and a
            // second S buffer, so both 4-vector products run before the
            // folds; without the buffer sigma runs the classes in turn
            c->d.abx_S2 = (double *)dev_alloc(c, c->abx_sbytes);
            if (c->d.abx_S2) {
                hipError_t e = hipStreamCreateWithFlags(&c->ob_stream, hipStreamNonBlocking);
                if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ob_fork, hipEventDisableTiming);
                if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ob_join, hipEventDisableTiming);
                if (e != hipSuccess) st = hip_fail(e, "one-body side stream");
            }
        }
        if (st == ISCI_OK && hipStreamSynchronize(stream) != hipSuccess) st = ISCI_E_HIP;
        if (st != ISCI_OK) { (void)hipStreamSynchronize(stream); destroy(c); return st; }
    }
    free_factors();
    if (hipStreamSynchronize(stream) != hipSuccess) { destroy(c); set_error("stream synchronisation failed"); return ISCI_E_HIP; }
    *out = c;
    return ISCI_OK;
}

isci_status isci_create_ex(isci_handle *out, const double *h, const double *eri, int norb, int nalpha,
                           int nbeta, int max_excitation, double tau, const isci_create_opts *opts,
                           hipStream_t stream)
{
    if (out) *out = nullptr;
    if (!eri) { set_error("eri is NULL"); return ISCI_E_INVALID; }
    return create_impl(out, h, eri, nullptr, 0, norb, nalpha, nbeta, max_excitation, tau, opts, stream);
}

isci_status isci_create_factored(isci_handle *out, const double *h, const double *Lfac, int naux, int norb,
                                 int nalpha, int nbeta, int max_excitation, double tau,
                                 const isci_create_opts *opts, hipStream_t stream)
{
    if (out) *out = nullptr;
    if (!Lfac) { set_error("Lfac is NULL"); return ISCI_E_INVALID; }
    return create_impl(out, h, nullptr, Lfac, naux, norb, nalpha, nbeta, max_excitation, tau, opts, stream);
}

isci_status isci_dim(isci_handle c, int64_t *dim)
{
    if (!c || !dim) { set_error("NULL argument"); return ISCI_E_INVALID; }
    *dim = c->dim;
    return ISCI_OK;
}

isci_status isci_get_stats(isci_handle c, isci_stats *s)
{
    if (!c || !s) { set_error("NULL argument"); return ISCI_E_INVALID; }
    *s = c->stats;
    return ISCI_OK;
}

isci_status isci_strings(isci_handle c, int spin, int32_t *orbitals, int32_t *level, int64_t *nstr)
{
    if (!c || (spin != 0 && spin != 1)) { set_error("bad handle or spin"); return ISCI_E_INVALID; }
    const SpinTab &T = spin ? c->sb : c->sa;
    const std::vector<int32_t> &o = spin ? c->h_borb : c->h_aorb;
    const std::vector<int32_t> &l = spin ? c->h_blev : c->h_alev;
    if (nstr) *nstr = T.nstr;
    if (orbitals && T.n > 0)
        for (int i = 0; i < T.nstr; ++i)
            for (int j = 0; j < T.n; ++j) orbitals[(size_t)i * T.n + j] = o[(size_t)i * T.n + j];
    if (level) std::copy(l.begin(), l.end(), level);
    return ISCI_OK;
}

isci_status isci_rowstart(isci_handle c, int64_t *rowstart)
{
    if (!c || !rowstart) { set_error("NULL argument"); return ISCI_E_INVALID; }
    std::copy(c->h_rowstart.begin(), c->h_rowstart.end(), rowstart);
    return ISCI_OK;
}

isci_status isci_set_option(isci_handle c, int option, int value)
{
    if (!c) { set_error("NULL handle"); return ISCI_E_INVALID; }
    switch (option) {
    case ISCI_OPT_SIGMA_KERNEL:
        if (value < ISCI_SIGMA_AUTO || value > ISCI_SIGMA_MFMA) { set_error("bad sigma kernel"); return ISCI_E_INVALID; }
        if ((value == ISCI_SIGMA_PAIR || value == ISCI_SIGMA_MFMA) && !(c->sa.n == 2 && c->sb.n == 2)) {
            set_error("pair kernel needs two electrons of each spin");
            return ISCI_E_UNSUPPORTED;
        }
        if (value == ISCI_SIGMA_MFMA && !c->have_tiles) {
            set_error("matrix-core kernel: its tiles were not built for this handle");
            return ISCI_E_UNSUPPORTED;
        }
        c->sigma_variant = value;
        return ISCI_OK;
    case ISCI_OPT_AB_PRODUCT:
        if (value != ISCI_AB_PLAIN && value != ISCI_AB_PIPE && value != ISCI_AB_WIDE && value != ISCI_AB_PACKED) {
            set_error("bad alpha-beta product kernel");
            return ISCI_E_INVALID;
        }
        c->ab_kernel = value;
        return ISCI_OK;
    case ISCI_OPT_ONEBODY_KERNEL:
        if (value != ISCI_ONEBODY_SINGLE && value != ISCI_ONEBODY_TRANSPOSED && value != ISCI_ONEBODY_SPECTATOR &&
            value != ISCI_ONEBODY_ROWS) {
            set_error("bad one-body kernel");
            return ISCI_E_INVALID;
        }
        if (value == ISCI_ONEBODY_ROWS && !onebody_beta_rows_ok(c)) {
            set_error("beta one-body row path: needs more than 80 orbitals, the excitation hierarchy and a beta row "
                      "that fits LDS");
            return ISCI_E_UNSUPPORTED;
        }
        if (value != ISCI_ONEBODY_ROWS && c->norb > kObMaxNorb && c->have_tiles && !c->onebody_in_tiles &&
            !c->d.obT_c) {
            // the transposed-block beta route of a handle that runs it on the
            // rows by default: its scratch, on the handle's device
            int prev = -1;
            if (hipGetDevice(&prev) != hipSuccess) { set_error("hipGetDevice failed"); return ISCI_E_HIP; }
            if (prev != c->device && hipSetDevice(c->device) != hipSuccess) {
                set_error("hipSetDevice failed");
                return ISCI_E_HIP;
            }
            const isci_status st = alloc_onebody_scratch(c);
            if (prev != c->device) (void)hipSetDevice(prev);
            if (st != ISCI_OK) return st;
        }
        c->ob_kernel = value;
        return ISCI_OK;
    case ISCI_OPT_ONEBODY_STREAM:
        if (value != ISCI_ONEBODY_SIDE && value != ISCI_ONEBODY_INLINE) { set_error("bad one-body stream"); return ISCI_E_INVALID; }
        c->ob_side = value == ISCI_ONEBODY_SIDE;
        return ISCI_OK;
    case ISCI_OPT_AB_PATH:
        if (value != ISCI_AB_AUTO && value != ISCI_AB_GATHER) { set_error("bad alpha-beta path"); return ISCI_E_INVALID; }
        c->ab_gather = value == ISCI_AB_GATHER;
        return ISCI_OK;
    default:
        set_error("unknown option");
        return ISCI_E_INVALID;
    }
}

isci_status isci_profile(isci_handle c, int enable)
{
    if (!c) { set_error("NULL handle"); return ISCI_E_INVALID; }
    c->profile = enable != 0;
    if (!c->profile) prof_clear(c);
    return ISCI_OK;
}

isci_status isci_profile_read(isci_handle c, int kernel, double *total_ms, int64_t *launches)
{
    if (!c || kernel < 0 || kernel >= ISCI_NKERNEL_IDS || !total_ms || !launches) {
        set_error("bad profile query");
        return ISCI_E_INVALID;
    }
    std::vector<hipEvent_t> &ev = c->prof_ev[kernel];
    double tot = 0.0;
    int64_t n = 0;
    for (size_t i = 0; i + 1 < ev.size(); i += 2) {
        ISCI_HIP(hipEventSynchronize(ev[i + 1]));
        float ms = 0.0f;
        ISCI_HIP(hipEventElapsedTime(&ms, ev[i], ev[i + 1]));
        tot += ms;
        ++n;
    }
    for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    ev.clear();
    *total_ms = tot;
    *launches = n;
    return ISCI_OK;
}

void isci_destroy(isci_handle c) { destroy(c); }

}  // extern "C"
