// Device helpers shared by the libisci kernels: binomials, packed strings,
// string ranks in (level, colex) order, phases, canonical integral reads.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "isci_internal.h"

namespace isci {


// C(x, k) for 0 <= k <= 4 (exact: each partial product is a binomial).
__host__ __device__ inline long long binom(int x, int k)
{
    if (k < 0 || x < k) return 0;
    long long r = 1;
    for (int i = 1; i <= k; ++i) r = r * (x - k + i) / i;
    return r;
}

__host__ __device__ inline void unpack_str(uint32_t s, int n, int *o)
{
#pragma unroll
    for (int i = 0; i < ISCI_MAXN; ++i)
        if (i < n) o[i] = (s >> (8 * i)) & 0xff;
}

__host__ __device__ inline uint32_t pack_str(const int *o, int n)
{
    uint32_t s = 0;
    for (int i = 0; i < n; ++i) s |= (uint32_t)o[i] << (8 * i);
    return s;
}

// level = number of electrons in orbitals >= b (b = n: excitation level;
// a GAS boundary: electrons in the outer space)
__host__ __device__ inline int str_level(const int *o, int n, int b)
{
    int l = 0;
    for (int i = 0; i < n; ++i) l += (o[i] >= b);
    return l;
}

// index of an ascending orbital list in (level, colex) order
__host__ __device__ inline int str_index(const int *o, const SpinTab &T)
{
    const int n = T.n, b = T.nocc;
    int ip = 0, io = 0;
    long long rp = 0, ro = 0;
    for (int i = 0; i < n; ++i) {
        int x = o[i];
        if (x >= b) { ++ip; rp += binom(x - b, ip); }
        else        { ++io; ro += binom(x, io); }
    }
    return T.lev_off[ip] + (int)(rp * T.occ_mult[ip] + ro);
}

// (-1)^{#{x in o, x != o[skip], x < p}}: phase of a+_p acting on the
// string o without element `skip` (skip = -1: none)
__host__ __device__ inline int phase_below(const int *o, int n, int skip, int p)
{
    int c = 0;
    for (int i = 0; i < n; ++i) c += (i != skip) & (o[i] < p);
    return (c & 1) ? -1 : 1;
}

// o without element `skip`, then insert q (kept ascending) -> out; returns
// false if q is already present among the kept elements.
__host__ __device__ inline bool replace_one(const int *o, int n, int skip, int q, int *out)
{
    int k = 0;
    bool placed = false;
    for (int i = 0; i < n; ++i) {
        if (i == skip) continue;
        int x = o[i];
        if (x == q) return false;
        if (!placed && q < x) { out[k++] = q; placed = true; }
        out[k++] = x;
    }
    if (!placed) out[k++] = q;
    return true;
}

// canonical element of (pq|rs): p>=q, r>=s, (p,q) >= (r,s)
__host__ __device__ inline size_t eri_canon(int n, int p, int q, int r, int s)
{
    int t;
    if (p < q) { t = p; p = q; q = t; }
    if (r < s) { t = r; r = s; s = t; }
    if (p < r || (p == r && q < s)) { t = p; p = r; r = t; t = q; q = s; s = t; }
    return (((size_t)p * n + q) * n + r) * n + s;
}

__device__ inline double geri(const double *eri, int n, int p, int q, int r, int s)
{
    return eri[eri_canon(n, p, q, r, s)];
}

// Source of the two-electron integrals read by the list builders: the
// canonical element of a dense tensor, or, for a handle built from factors
// (pq|rs) = sum_K L^K_pq L^K_rs, the sum formed on the fly at the canonical
// indices in a fixed order (K ascending, each product and each partial sum
// rounded once, no fused multiply-add), so every unit is the same double
// whatever builder reads it; the dense tensor is never formed (the
// minimum-integral-calculation idea of the paper's set-up part: each
// integral is computed once, when the screened lists are built, and only
// fetched by the sigma steps).  nrm[pq] >= sqrt(sum_K (L^K_pq)^2) gives the
// Cauchy-Schwarz bound |(pq|rs)| <= nrm[pq] nrm[rs], which lets a builder
// skip a unit it would screen away without forming it.
struct EriSrc {
    const double *eri;   // dense [n^4] ((pq|rs) at ((p n + q) n + r) n + s), or nullptr
    const double *Lt;    // factored: [n * n][naux], L^K_pq at (p n + q) naux + K
    const double *nrm;   // factored: [n * n] bounds of the factor norms
    int n, naux;
    const double *dist;  // distance screening: [n * n] orbital distances, or nullptr
    double dmax;         // units whose orbitals are not all within dmax read as 0
};

// largest pairwise distance among p, q, r, s
__device__ inline double eri_span(const EriSrc &E, int p, int q, int r, int s)
{
    const double *d = E.dist;
    const int n = E.n;
    return fmax(fmax(fmax(d[p * n + q], d[p * n + r]), fmax(d[p * n + s], d[q * n + r])),
                fmax(d[q * n + s], d[r * n + s]));
}

__device__ inline double eri_value(const EriSrc &E, int p, int q, int r, int s)
{
    if (E.dist && eri_span(E, p, q, r, s) > E.dmax) return 0.0;
    if (E.eri) return geri(E.eri, E.n, p, q, r, s);
    int t;
    if (p < q) { t = p; p = q; q = t; }
    if (r < s) { t = r; r = s; s = t; }
    if (p < r || (p == r && q < s)) { t = p; p = r; r = t; t = q; q = s; s = t; }
    const double *a = E.Lt + ((size_t)p * E.n + q) * E.naux;
    const double *b = E.Lt + ((size_t)r * E.n + s) * E.naux;
    double acc = 0.0;
    {
        // product and sum rounded separately (no contraction to an FMA)
#pragma clang fp contract(off)
        for (int K = 0; K < E.naux; ++K) acc = acc + a[K] * b[K];
    }
    return acc;
}

// true when |(pq|rs)| as eri_value forms it is surely <= t (factored
// sources only; the margin covers the rounding of the sums and the norms)
__device__ inline bool eri_negligible(const EriSrc &E, int p, int q, int r, int s, double t)
{
    if (E.dist && eri_span(E, p, q, r, s) > E.dmax) return true;
    if (!E.nrm) return false;
    return E.nrm[p * E.n + q] * E.nrm[r * E.n + s] * (1.0 + 1e-9) <= t;
}

__device__ inline double gh(const double *h, int n, int p, int q)
{
    return p >= q ? h[(size_t)p * n + q] : h[(size_t)q * n + p];
}

}  // namespace isci
