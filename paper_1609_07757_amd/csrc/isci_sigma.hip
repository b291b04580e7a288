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
            const int lj = str_level(jo, na);
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
                const int lj = str_level(jo, na);
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
            const int lj = str_level(jo, na);
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

template <int NV>
__global__ __launch_bounds__(256) void k_sigma_generic(SigmaArgs A, int nv, const double *__restrict__ c,
                                                       int64_t ldc, double *__restrict__ sg, int64_t lds)
{
    sigma_target<NV>(A, blockIdx.x, blockIdx.y * blockDim.x + threadIdx.x, nv, c, ldc, sg, lds);
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
        sigma_target<NV>(args[bv.inst], w.x, w.y + threadIdx.x, bv.nv, bv.c, bv.ldc, bv.s, bv.lds);
    }
}

// diagonal of H_tau: kept diagonal units
__global__ __launch_bounds__(256) void k_diag(SigmaArgs A, double *__restrict__ out)
{
    const int ia = blockIdx.x;
    const int la = A.alev[ia];
    const int rlen = A.sb.le[A.L - la];
    const int ib = blockIdx.y * blockDim.x + threadIdx.x;
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
                         hipStream_t s)
{
    const SigmaArgs A = sigma_args(c);
    const dim3 grid((unsigned)c->sa.nstr, (unsigned)((c->max_rowlen + 255) / 256));
    for (int v0 = 0; v0 < nvec; v0 += 8) {
        const int nv = nvec - v0 < 8 ? nvec - v0 : 8;
        const double *cc = cv + (int64_t)v0 * ldc;
        double *ss = sv + (int64_t)v0 * lds;
        if (nv == 1)
            k_sigma_generic<1><<<grid, 256, 0, s>>>(A, nv, cc, ldc, ss, lds);
        else if (nv == 2)
            k_sigma_generic<2><<<grid, 256, 0, s>>>(A, nv, cc, ldc, ss, lds);
        else if (nv <= 4)
            k_sigma_generic<4><<<grid, 256, 0, s>>>(A, nv, cc, ldc, ss, lds);
        else
            k_sigma_generic<8><<<grid, 256, 0, s>>>(A, nv, cc, ldc, ss, lds);
        ISCI_HIP(hipGetLastError());
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
    const dim3 grid((unsigned)c->sa.nstr, (unsigned)((c->max_rowlen + 255) / 256));
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

isci_status isci_diag(isci_handle c, double *diag, hipStream_t stream)
{
    if (!c || !diag) { set_error("NULL argument"); return ISCI_E_INVALID; }
    return launch_diag(c, diag, stream);
}

}  // extern "C"
