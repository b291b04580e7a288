// One-body density matrices by spin (the paper's density-matrix subsection,
// Eq. d1): d[v][s][p][q] = <c_v| a+_{p s} a_{q s} |c_v>.
//
// The paper's density loop is the Hamiltonian's class loop with the
// integral fetch replaced by a product of two coefficients.  Here the
// element (p, q) of one spin owns a workgroup: it walks the sets of the
// other n - 1 electrons ("spectators", the orbitals other than p and q),
// forms the source string spectators + q and the target string
// spectators + p, and adds sign * c(target) * c(source) over every
// determinant pair the replacement connects.  For alpha the beta string is
// kept, so the pair is a dot product of the two alpha rows over the beta
// prefix both rows hold (coalesced).  For beta the same kernel runs on the
// vectors transposed into the spin-swapped layout (rows = beta strings,
// each holding the alpha strings of level <= L - its level, again a
// prefix), with the two spin tables exchanged.  The sign is
// (-1)^(spectators strictly between p and q); a beta replacement passes
// the alpha creators as an even pair and adds nothing.
// One wave owns an element (four per workgroup); each lane accumulates its own terms and the
// wave sums them in a fixed order, so the result is the same on every run.
// Row starts follow from the level tables (rows of one level are contiguous
// and equally long), so the walk issues no index loads.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "isci_device.h"
#include "isci_internal.h"

namespace isci {

namespace {

constexpr int kD1Threads = 256;  // four waves, one density element each
constexpr int kD1Chunk = 4;   // vectors per transposed batch (the handle keeps kD1Chunk * dim doubles)

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
    const int n = T.n;
    int ip = 0, io = 0;
    uint32_t rp = 0, ro = 0;
    for (int i = 0; i < n; ++i) {
        const int x = o[i];
        if (x >= n) { ++ip; rp += binom_small(x - n, ip); }
        else        { ++io; ro += binom_small(x, io); }
    }
    return T.lev_off[ip] + (int)(rp * (uint32_t)T.occ_mult[ip] + ro);
}

// Spectator walk of one element (p, q) of a spin with n electrons: the
// (n - 1)-subsets of the orbitals other than p and q in colex order,
// advanced by `next`.  Gives the ascending source (spectators + q) and
// target (spectators + p) strings and the replacement sign.
struct SpecWalk {
    int n, m, lo, hi;     // m orbitals to choose from; lo <= hi the skipped ones
    int e[ISCI_MAXN];     // current subset as indices into the m orbitals
    bool more;

    __device__ void init(int n_, int norb, int p, int q)
    {
        n = n_;
        lo = min(p, q);
        hi = max(p, q);
        m = norb - (p == q ? 1 : 2);
        const int k = n - 1;
        more = (n >= 1) && (k <= m);
        for (int i = 0; i < k; ++i) e[i] = i;
    }
    __device__ int orb(int x) const
    {
        if (x >= lo) ++x;
        if (lo != hi && x >= hi) ++x;
        return x;
    }
    __device__ void next()
    {
        const int k = n - 1;
        int i = k - 1;
        while (i >= 0 && e[i] == m - k + i) --i;
        if (i < 0) { more = false; return; }
        ++e[i];
        for (int j = i + 1; j < k; ++j) e[j] = e[j - 1] + 1;
    }
    // strings and sign of the current subset
    __device__ int strings(int p, int q, int *src, int *dst) const
    {
        const int k = n - 1;
        int between = 0, a = 0, b = 0;
        bool qin = false, pin = false;
        for (int i = 0; i < k; ++i) {
            const int o = orb(e[i]);
            between += (o > lo && o < hi);
            if (!qin && q < o) { src[a++] = q; qin = true; }
            if (!pin && p < o) { dst[b++] = p; pin = true; }
            src[a++] = o;
            dst[b++] = o;
        }
        if (!qin) src[a++] = q;
        if (!pin) dst[b++] = p;
        return (between & 1) ? -1 : 1;
    }
};

// Element (p, q) of the spin whose strings index the rows of A (A.sa), for
// vector blockIdx.y of c, written to slot `slot` of vector v0 + blockIdx.y.
__global__ __launch_bounds__(kD1Threads) void k_d1_rows(SigmaArgs A, const double *__restrict__ c, int64_t ldc,
                                                         double *__restrict__ d1, int slot, int v0)
{
    const int norb = A.norb;
    const int lane = threadIdx.x & 63;
    const int pq = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (pq >= norb * norb) return;   // whole wave: no barrier follows
    const int p = pq / norb, q = pq - p * norb;
    const int v = blockIdx.y;
    const double *cv = c + (int64_t)v * ldc;
    double acc = 0.0;
    SpecWalk w;
    w.init(A.sa.n, norb, p, q);
    for (; w.more; w.next()) {
        int src[ISCI_MAXN], dst[ISCI_MAXN];
        const double sg = (double)w.strings(p, q, src, dst);
        const int ls = str_level(src, A.sa.n), lt = str_level(dst, A.sa.n);
        if (ls > A.sa.maxlev || lt > A.sa.maxlev) continue;
        const int len = A.sb.le[A.L - max(ls, lt)];
        const double *rs = cv + row_start(A.sa, A.sb, A.L, rank_small(src, A.sa), ls);
        const double *rt = cv + row_start(A.sa, A.sb, A.L, rank_small(dst, A.sa), lt);
        double p0 = 0.0, p1 = 0.0;
        int b = lane;
        for (; b + 64 < len; b += 128) {
            p0 = fma(rt[b], rs[b], p0);
            p1 = fma(rt[b + 64], rs[b + 64], p1);
        }
        if (b < len) p0 = fma(rt[b], rs[b], p0);
        acc = fma(sg, p0 + p1, acc);
    }
    const double tot = wave_sum(acc);
    if (lane == 0) d1[(((int64_t)(v0 + v) * 2 + slot) * norb + p) * norb + q] = tot;
}

// Vectors v < nv of c into the spin-swapped layout: determinant (ia, j) of
// c (row ia, beta string j) goes to row j, position ia of cT (leading
// dimension dim).  One thread per determinant, workgroups laid out by
// row_block; reads are coalesced along the row, writes are scattered.
__global__ __launch_bounds__(256) void k_d1_transpose(SigmaArgs A, const double *__restrict__ c, int64_t ldc, int nv,
                                                      const int64_t *__restrict__ rowT, int64_t dim,
                                                      double *__restrict__ cT)
{
    int ia, j0, len;
    row_block(A, blockIdx.x, ia, j0, len);
    const int j = j0 + threadIdx.x;
    if (j >= len) return;
    const int64_t src = A.rowstart[ia] + j, dst = rowT[j] + ia;
    for (int v = 0; v < nv; ++v) cT[(int64_t)v * dim + dst] = c[(int64_t)v * ldc + src];
}

}  // namespace

}  // namespace isci

using namespace isci;

extern "C" {

isci_status isci_density1(isci_handle h, int nvec, const double *c, int64_t ldc, double *d1, hipStream_t stream)
{
    if (!h || !c || !d1) { set_error("NULL argument"); return ISCI_E_INVALID; }
    if (nvec < 1 || nvec > 65535) { set_error("nvec outside 1..65535"); return ISCI_E_INVALID; }
    if (ldc < h->dim) { set_error("leading dimension < dim"); return ISCI_E_INVALID; }
    const int64_t nd = (int64_t)nvec * 2 * h->norb * h->norb;
    const char *c0 = (const char *)c, *c1 = (const char *)(c + (int64_t)(nvec - 1) * ldc + h->dim);
    const char *d0 = (const char *)d1, *e1 = (const char *)(d1 + nd);
    if (c0 < e1 && d0 < c1) { set_error("density overlaps c"); return ISCI_E_INVALID; }
    const SigmaArgs A = sigma_args(h);
    const unsigned npq = (unsigned)((h->norb * h->norb + 3) / 4);   // workgroups of four elements
    k_d1_rows<<<dim3(npq, (unsigned)nvec), kD1Threads, 0, stream>>>(A, c, ldc, d1, 0, 0);
    ISCI_HIP(hipGetLastError());
    // beta: the same kernel on the spin-swapped layout, kD1Chunk vectors at a time
    SigmaArgs T = A;
    T.sa = A.sb;
    T.sb = A.sa;
    T.astr = A.bstr;
    T.bstr = A.astr;
    T.alev = A.blev;
    T.blev = A.alev;
    if (h->nb == 0) {   // no beta strings to replace: the kernel writes zeros without reading c
        k_d1_rows<<<dim3(npq, (unsigned)nvec), kD1Threads, 0, stream>>>(T, c, ldc, d1, 1, 0);
        ISCI_HIP(hipGetLastError());
        return ISCI_OK;
    }
    if (!h->d.d1T) {
        const int nsb = h->sb.nstr;
        std::vector<int64_t> rt(nsb + 1);
        rt[0] = 0;
        for (int j = 0; j < nsb; ++j) rt[j + 1] = rt[j] + h->sa.le[h->L - h->h_blev[j]];
        if (rt[nsb] != h->dim) { set_error("isci_density1: transposed layout size mismatch"); return ISCI_E_INVALID; }
        int64_t *rtd = (int64_t *)dev_alloc(h, sizeof(int64_t) * (nsb + 1));
        double *buf = (double *)dev_alloc(h, sizeof(double) * kD1Chunk * (size_t)h->dim);
        if (!rtd || !buf) { set_error("isci_density1: out of device memory"); return ISCI_E_OOM; }
        ISCI_HIP(hipMemcpy(rtd, rt.data(), sizeof(int64_t) * (nsb + 1), hipMemcpyHostToDevice));
        h->d.d1T_rowstart = rtd;
        h->d.d1T = buf;
    }
    T.rowstart = h->d.d1T_rowstart;
    for (int v0 = 0; v0 < nvec; v0 += kD1Chunk) {
        const int nv = std::min(kD1Chunk, nvec - v0);
        k_d1_transpose<<<h->nplan, 256, 0, stream>>>(A, c + (int64_t)v0 * ldc, ldc, nv, h->d.d1T_rowstart, h->dim,
                                                      h->d.d1T);
        ISCI_HIP(hipGetLastError());
        k_d1_rows<<<dim3(npq, (unsigned)nv), kD1Threads, 0, stream>>>(T, h->d.d1T, h->dim, d1, 1, v0);
        ISCI_HIP(hipGetLastError());
    }
    return ISCI_OK;
}

}  // extern "C"
