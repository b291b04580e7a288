// Short-iterative Arnoldi-Lanczos (SIAL) propagation of CI vectors under
// H_tau, the optimiser the paper uses for the CI coefficients (propagation
// in imaginary time, in its application section, with the method of its
// references on short-iterative Lanczos propagators), and real-time
// propagation for dynamics; with an optional screening of small CI
// coefficients (its section on the distribution of coefficients proposes
// screening the CI vector as the integrals are screened).
//
// One step of length dt: a Krylov basis V = [v_0 .. v_{m-1}] of H_tau from
// v_0 = u / |u|, each new direction H v_j orthogonalised against v_{j-1},
// v_j and then, once more, against the whole basis (classical
// Gram-Schmidt, Arnoldi form with full reorthogonalisation), the projected matrix
// T = V^T H V (symmetrised), and
//   imaginary time:  u <- |u| V exp(-T dt) e_1, then normalised;
//   real time:       u <- |u| V exp(-i T dt) e_1 for a real u; a complex
//                    vector re + i im is propagated as its two real parts,
//                    each with its own basis, and recombined.
// The basis grows until the residual estimate beta_{m} |[f(T) e_1]_{m-1}|
// falls below tol |u| or reaches the Krylov limit (or an invariant
// subspace is found).  exp of the small T comes from its eigendecomposition
// on the host.  Every sigma runs on the device through the sigma path; the
// vectors never leave it.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "isci_internal.h"

namespace isci {
namespace {

__global__ void k_scale_to(const double *__restrict__ src, double *__restrict__ dst, int64_t n, double f)
{
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
        dst[t] = f * src[t];
}

__global__ void k_scale_inplace(double *__restrict__ x, int64_t n, double f)
{
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
        x[t] *= f;
}

// coefficient screening: zero every element whose modulus (real vector:
// absolute value) is at most thr; *cnt += number zeroed (non-zero before)
__global__ void k_coef_screen(double *__restrict__ re, double *__restrict__ im, int64_t n, double thr,
                              unsigned long long *__restrict__ cnt)
{
    unsigned long long mine = 0;
    const double t2 = thr * thr;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
        const double a = re[t], b = im ? im[t] : 0.0;
        if (a * a + b * b <= t2 && (a != 0.0 || b != 0.0)) {
            re[t] = 0.0;
            if (im) im[t] = 0.0;
            ++mine;
        }
    }
    for (int off = 32; off > 0; off >>= 1) mine += __shfl_xor(mine, off, 64);
    if ((threadIdx.x & 63) == 0 && mine) atomicAdd(cnt, mine);
}

// one Gram-Schmidt pass of each chain ch < nch over basis vectors i0 ..
// i0 + m - 1: the dots h = V^T w just formed (outd[ch][i], i < m) are added
// to column j of the chain's projected matrix (T[ch][i0 + i][j], leading
// dimension mm) and negated into the coefficients of the update w -= V h
__global__ void k_gs_pass(const double *__restrict__ outd, int nch, int mm, int m, int i0, int j,
                          double *__restrict__ T, double *__restrict__ coef)
{
    for (int t = threadIdx.x; t < nch * m; t += blockDim.x) {
        const int ch = t / m, i = t - ch * m;
        const double hv = outd[(size_t)ch * mm + i];
        T[((size_t)ch * mm + i0 + i) * mm + j] += hv;
        coef[(size_t)ch * mm + i] = -hv;
    }
}

unsigned grid_of(int64_t n) { return (unsigned)std::min<int64_t>(4096, std::max<int64_t>(1, (n + 255) / 256)); }

// the symmetric m x m projected matrix from the Arnoldi entries T[i][j]
// (i <= j + 1, leading dimension mm): upper entries as computed, the
// off-diagonal pair (j, j + 1) as the mean of <v_j, H v_{j+1}> and the
// norm that made v_{j+1} (equal for a symmetric H up to rounding)
std::vector<double> projected(const std::vector<double> &T, int mm, int m)
{
    std::vector<double> A((size_t)m * m, 0.0);
    for (int a = 0; a < m; ++a)
        for (int b = a; b < m; ++b) {
            const double x = b == a + 1 ? 0.5 * (T[(size_t)a * mm + b] + T[(size_t)b * mm + a]) : T[(size_t)a * mm + b];
            A[(size_t)a * m + b] = A[(size_t)b * m + a] = x;
        }
    return A;
}

// Krylov basis of one or two chains (the real vectors being propagated);
// the chains' j-th vectors are stored consecutively so one sigma call
// serves them all
struct Krylov {
    int nch = 0, mmax = 0;
    int64_t n = 0;
    double *V = nullptr;      // [mmax + 1][nch][n]
    double *W = nullptr;      // [nch][n]
    double *coef = nullptr;   // [4][mmax + 1] device coefficients (Gram-Schmidt:
                              // [nch][mmax + 1]; real-time recombination: 4 rows)
    double *part = nullptr;   // dot partials
    double *outd = nullptr;   // [nch][mmax + 1] dot results
    double *Td = nullptr;     // [nch][mmax + 1][mmax + 1] projected matrices (Arnoldi entries)
    int nblk = 1;
    double *vec(int j, int ch) const { return V + ((int64_t)j * nch + ch) * n; }
};

}  // namespace
}  // namespace isci

using namespace isci;

extern "C" {

void isci_propagate_defaults(isci_propagate_opts *o)
{
    if (!o) return;
    o->krylov = 16;
    o->imaginary = 1;
    o->tol = 1e-12;
    o->coef_tau = 0.0;
}

isci_status isci_propagate(isci_handle h, double *c_re, double *c_im, double dt, int nsteps,
                           const isci_propagate_opts *opts, isci_propagate_info *info, hipStream_t stream)
{
    if (!h || !c_re) { set_error("NULL argument"); return ISCI_E_INVALID; }
    isci_propagate_opts o;
    isci_propagate_defaults(&o);
    if (opts) o = *opts;
    if (o.krylov < 1 || o.krylov > 128) { set_error("krylov outside 1..128"); return ISCI_E_INVALID; }
    if (!(dt >= 0.0) || std::isinf(dt) || nsteps < 0) { set_error("dt must be finite and >= 0, nsteps >= 0"); return ISCI_E_INVALID; }
    if (!(o.tol >= 0.0) || !(o.coef_tau >= 0.0)) { set_error("tol and coef_tau must be >= 0"); return ISCI_E_INVALID; }
    if (!o.imaginary && !c_im) { set_error("real-time propagation needs the imaginary part c_im"); return ISCI_E_INVALID; }
    if (c_im && c_im == c_re) { set_error("c_re and c_im must be distinct"); return ISCI_E_INVALID; }
    const int64_t n = h->dim;
    Krylov K;
    K.nch = o.imaginary ? 1 : 2;
    K.mmax = o.krylov;
    K.n = n;
    K.nblk = dots_blocks(n);
    const int mm = K.mmax + 1;
    hipError_t e = hipSuccess;
    unsigned long long *dcnt = nullptr;
    e = hipMallocAsync((void **)&K.V, sizeof(double) * (size_t)mm * K.nch * n, stream);
    if (e == hipSuccess) e = hipMallocAsync((void **)&K.W, sizeof(double) * (size_t)K.nch * n, stream);
    if (e == hipSuccess) e = hipMallocAsync((void **)&K.coef, sizeof(double) * (size_t)4 * mm, stream);
    if (e == hipSuccess) e = hipMallocAsync((void **)&K.part, sizeof(double) * (size_t)K.nblk * mm, stream);
    if (e == hipSuccess) e = hipMallocAsync((void **)&K.outd, sizeof(double) * (size_t)K.nch * mm, stream);
    if (e == hipSuccess) e = hipMallocAsync((void **)&K.Td, sizeof(double) * (size_t)K.nch * mm * mm, stream);
    if (e == hipSuccess) e = hipMallocAsync((void **)&dcnt, sizeof(unsigned long long), stream);
    auto release = [&]() {
        for (void *p : {(void *)K.V, (void *)K.W, (void *)K.coef, (void *)K.part, (void *)K.outd, (void *)K.Td, (void *)dcnt})
            if (p) (void)hipFreeAsync(p, stream);
        (void)hipStreamSynchronize(stream);
    };
    if (e != hipSuccess) { release(); set_error("isci_propagate: out of device memory"); return ISCI_E_OOM; }
    // a chain that is zero keeps a zero basis (never written below)
    ISCI_HIP(hipMemsetAsync(K.V, 0, sizeof(double) * (size_t)mm * K.nch * n, stream));
    isci_status st = ISCI_OK;
    int sigma_calls = 0;
    int64_t screened = 0;
    int mlast = 0;
    double *chain[2] = {c_re, o.imaginary ? nullptr : c_im};
    // host copy of dot results of chain ch (count k) after a sync
    std::vector<double> hbuf((size_t)K.nch * mm);
    auto fetch = [&]() -> isci_status {
        ISCI_HIP(hipMemcpyAsync(hbuf.data(), K.outd, sizeof(double) * hbuf.size(), hipMemcpyDeviceToHost, stream));
        ISCI_HIP(hipStreamSynchronize(stream));
        return ISCI_OK;
    };
    for (int step = 0; step < nsteps && st == ISCI_OK; ++step) {
        // |u| per chain, first basis vectors
        double beta0[2] = {0.0, 0.0};
        for (int ch = 0; ch < K.nch; ++ch)
            if ((st = dots(chain[ch], n, 1, chain[ch], n, 1, n, K.outd + (size_t)ch * mm, K.part, K.nblk, stream)) != ISCI_OK) break;
        if (st != ISCI_OK || (st = fetch()) != ISCI_OK) break;
        bool live[2] = {false, false};
        for (int ch = 0; ch < K.nch; ++ch) {
            beta0[ch] = std::sqrt(std::max(0.0, hbuf[(size_t)ch * mm]));
            live[ch] = beta0[ch] > 0.0;
            k_scale_to<<<grid_of(n), 256, 0, stream>>>(chain[ch], K.vec(0, ch), n, live[ch] ? 1.0 / beta0[ch] : 0.0);
        }
        if (!live[0] && !live[1]) break;
        // Arnoldi: T[ch][i][j] = <v_i, H v_j>, i <= j + 1, accumulated on the
        // device pass by pass; one host wait per basis vector brings back
        // the new column and the norm of the remainder for the stopping test
        std::vector<std::vector<double>> T(K.nch, std::vector<double>((size_t)mm * mm, 0.0));
        std::vector<double> Th((size_t)K.nch * mm * mm);
        ISCI_HIP(hipMemsetAsync(K.Td, 0, sizeof(double) * Th.size(), stream));
        int m = 0;
        bool stop = false;
        for (int j = 0; j < K.mmax && !stop; ++j) {
            if ((st = launch_sigma(h, K.nch, K.vec(j, 0), n, K.W, n, stream)) != ISCI_OK) break;
            sigma_calls += K.nch;
            // Gram-Schmidt in two passes: against v_{j-1}, v_j first (the
            // three-term part, which removes the bulk of H v_j), then one
            // classical pass against the whole basis v_0 .. v_j
            auto gs_pass = [&](int i0, int cnt) -> isci_status {
                for (int ch = 0; ch < K.nch; ++ch)
                    ISCI_CHECK(dots(K.vec(i0, ch), (int64_t)K.nch * n, cnt, K.W + (size_t)ch * n, n, 1, n,
                                    K.outd + (size_t)ch * mm, K.part, K.nblk, stream));
                k_gs_pass<<<1, 256, 0, stream>>>(K.outd, K.nch, mm, cnt, i0, j, K.Td, K.coef);
                ISCI_HIP(hipGetLastError());
                for (int ch = 0; ch < K.nch; ++ch)
                    ISCI_CHECK(lincomb(K.vec(i0, ch), (int64_t)K.nch * n, cnt, K.coef + (size_t)ch * mm, 1,
                                       K.W + (size_t)ch * n, n, n, 1.0, stream));
                return ISCI_OK;
            };
            const int i0 = j > 0 ? j - 1 : 0;
            if ((st = gs_pass(i0, j + 1 - i0)) != ISCI_OK || (st = gs_pass(0, j + 1)) != ISCI_OK) break;
            for (int ch = 0; ch < K.nch && st == ISCI_OK; ++ch)
                st = dots(K.W + (size_t)ch * n, n, 1, K.W + (size_t)ch * n, n, 1, n, K.outd + (size_t)ch * mm, K.part,
                          K.nblk, stream);
            if (st != ISCI_OK) break;
            ISCI_HIP(hipMemcpyAsync(Th.data(), K.Td, sizeof(double) * Th.size(), hipMemcpyDeviceToHost, stream));
            if ((st = fetch()) != ISCI_OK) break;   // also waits for Th
            m = j + 1;
            double worst = 0.0;
            bool invariant = true;
            for (int ch = 0; ch < K.nch; ++ch) {
                if (!live[ch]) continue;
                for (int i = 0; i <= j; ++i) T[ch][(size_t)i * mm + j] = Th[((size_t)ch * mm + i) * mm + j];
                const double beta = std::sqrt(std::max(0.0, hbuf[(size_t)ch * mm]));
                T[ch][(size_t)(j + 1) * mm + j] = beta;
                // residual estimate of exp over the current basis
                std::vector<double> A = projected(T[ch], mm, m), w, Z;
                sym_eigh(m, A, w, Z);
                double yr = 0.0, yi = 0.0;   // last component of f(T) e_1
                for (int q = 0; q < m; ++q) {
                    const double zz = Z[(size_t)(m - 1) * m + q] * Z[q];
                    if (o.imaginary) {
                        yr += zz * std::exp(-(w[q] - w[0]) * dt);
                    } else {
                        yr += zz * std::cos(w[q] * dt);
                        yi -= zz * std::sin(w[q] * dt);
                    }
                }
                worst = std::max(worst, beta * std::sqrt(yr * yr + yi * yi));
                const double scale = std::abs(T[ch][0]) + 1.0;
                if (beta > 1e-13 * scale) invariant = false;
                k_scale_to<<<grid_of(n), 256, 0, stream>>>(K.W + (size_t)ch * n, K.vec(j + 1, ch), n,
                                                           beta > 0.0 ? 1.0 / beta : 0.0);
            }
            if (invariant || worst <= o.tol) stop = true;
        }
        if (st != ISCI_OK) break;
        mlast = m;
        // f(T) e_1 per chain and the recombination
        std::vector<double> coef((size_t)K.nch * mm * 2, 0.0);   // [ch][re/im][m]
        for (int ch = 0; ch < K.nch; ++ch) {
            if (!live[ch]) continue;
            std::vector<double> A = projected(T[ch], mm, m), w, Z;
            sym_eigh(m, A, w, Z);
            for (int a = 0; a < m; ++a) {
                double yr = 0.0, yi = 0.0;
                for (int q = 0; q < m; ++q) {
                    const double zz = Z[(size_t)a * m + q] * Z[q];
                    if (o.imaginary) {
                        // shifted by the lowest Ritz value: the vector is
                        // renormalised, so the shift only avoids overflow
                        yr += zz * std::exp(-(w[q] - w[0]) * dt);
                    } else {
                        yr += zz * std::cos(w[q] * dt);
                        yi -= zz * std::sin(w[q] * dt);
                    }
                }
                coef[((size_t)ch * 2 + 0) * mm + a] = beta0[ch] * yr;
                coef[((size_t)ch * 2 + 1) * mm + a] = beta0[ch] * yi;
            }
        }
        // new chains: imaginary u = V y_r; real time
        //   re' = V_re a_re - V_im b_im,  im' = V_re b_re + V_im a_im
        std::vector<double> Y;
        if (o.imaginary) {
            Y.assign(coef.begin(), coef.begin() + m);
        } else {
            // out chain 0 (re'): from basis re with a_re, from basis im with -b_im
            // out chain 1 (im'): from basis re with b_re, from basis im with a_im
            Y.assign((size_t)4 * mm, 0.0);
            for (int a = 0; a < m; ++a) {
                Y[0 * mm + a] = coef[(0 * 2 + 0) * mm + a];    // re basis -> re'
                Y[1 * mm + a] = coef[(0 * 2 + 1) * mm + a];    // re basis -> im'
                Y[2 * mm + a] = -coef[(1 * 2 + 1) * mm + a];   // im basis -> re'
                Y[3 * mm + a] = coef[(1 * 2 + 0) * mm + a];    // im basis -> im'
            }
        }
        ISCI_HIP(hipMemcpyAsync(K.coef, Y.data(), sizeof(double) * Y.size(), hipMemcpyHostToDevice, stream));
        if (o.imaginary) {
            st = lincomb(K.vec(0, 0), (int64_t)K.nch * n, m, K.coef, 1, chain[0], n, n, 0.0, stream);
        } else {
            st = lincomb(K.vec(0, 0), (int64_t)K.nch * n, m, K.coef + 0 * mm, 1, chain[0], n, n, 0.0, stream);
            if (st == ISCI_OK) st = lincomb(K.vec(0, 1), (int64_t)K.nch * n, m, K.coef + 2 * mm, 1, chain[0], n, n, 1.0, stream);
            if (st == ISCI_OK) st = lincomb(K.vec(0, 0), (int64_t)K.nch * n, m, K.coef + 1 * mm, 1, chain[1], n, n, 0.0, stream);
            if (st == ISCI_OK) st = lincomb(K.vec(0, 1), (int64_t)K.nch * n, m, K.coef + 3 * mm, 1, chain[1], n, n, 1.0, stream);
        }
        if (st != ISCI_OK) break;
        ISCI_HIP(hipStreamSynchronize(stream));   // Y is rewritten next step
        if (o.imaginary) {
            if ((st = dots(chain[0], n, 1, chain[0], n, 1, n, K.outd, K.part, K.nblk, stream)) != ISCI_OK) break;
            if ((st = fetch()) != ISCI_OK) break;
            const double nrm = std::sqrt(std::max(0.0, hbuf[0]));
            if (nrm > 0.0) k_scale_inplace<<<grid_of(n), 256, 0, stream>>>(chain[0], n, 1.0 / nrm);
        }
        if (o.coef_tau > 0.0) {
            ISCI_HIP(hipMemsetAsync(dcnt, 0, sizeof(unsigned long long), stream));
            k_coef_screen<<<grid_of(n), 256, 0, stream>>>(chain[0], chain[1], n, o.coef_tau, dcnt);
            unsigned long long hc = 0;
            ISCI_HIP(hipMemcpyAsync(&hc, dcnt, sizeof(hc), hipMemcpyDeviceToHost, stream));
            ISCI_HIP(hipStreamSynchronize(stream));
            screened = (int64_t)hc;
        }
        ISCI_HIP(hipGetLastError());
    }
    // energy <u|H|u> / <u|u> of the final vector (sum over the chains)
    double energy = 0.0, norm2 = 0.0;
    if (st == ISCI_OK && info) {
        for (int ch = 0; ch < K.nch && st == ISCI_OK; ++ch)
            st = launch_sigma(h, 1, chain[ch], n, K.W + (size_t)ch * n, n, stream);
        sigma_calls += K.nch;
        for (int ch = 0; ch < K.nch && st == ISCI_OK; ++ch) {
            st = dots(chain[ch], n, 1, K.W + (size_t)ch * n, n, 1, n, K.outd + (size_t)ch * mm, K.part, K.nblk, stream);
            if (st == ISCI_OK)
                st = dots(chain[ch], n, 1, chain[ch], n, 1, n, K.outd + (size_t)ch * mm + 1, K.part, K.nblk, stream);
        }
        if (st == ISCI_OK) st = fetch();
        for (int ch = 0; ch < K.nch && st == ISCI_OK; ++ch) {
            energy += hbuf[(size_t)ch * mm];
            norm2 += hbuf[(size_t)ch * mm + 1];
        }
    }
    release();
    if (st != ISCI_OK) return st;
    if (info) {
        info->energy = norm2 > 0.0 ? energy / norm2 : 0.0;
        info->norm = std::sqrt(norm2);
        info->sigma_calls = sigma_calls;
        info->krylov_last = mlast;
        info->screened_last = screened;
    }
    return ISCI_OK;
}

}  // extern "C"
