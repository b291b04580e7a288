// libisci eigensolver: block Davidson (Davidson 1975) around the sigma
// step (Eq. sigma; the paper names Davidson and Lanczos as the usual
// optimisers following the sigma step).  FP64 throughout.
//
// Vectors stay on the device.  Per iteration: sigma of the new basis
// vectors, the new columns of the projected matrix G = V^T H V, Ritz
// vectors and residuals, a diagonal (Davidson) preconditioner, and
// classical Gram-Schmidt applied twice (CGS2) to orthonormalise the
// corrections.  The small symmetric eigenproblem of G is solved on the
// host with cyclic Jacobi rotations; this is the only device-to-host
// traffic inside the loop.  The basis is restarted from the current Ritz
// vectors when it would exceed max_subspace.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <vector>

#include "isci_device.h"
#include "isci_internal.h"

namespace isci {

constexpr int kDotBlocks = 512;
constexpr int kTile = 8;

// partial[(blk * m + i) * k + j] = sum_{t in blk's range} A_i[t] B_j[t]
__global__ __launch_bounds__(256) void k_dots(const double *__restrict__ A, int64_t lda, int m,
                                              const double *__restrict__ B, int64_t ldb, int k, int64_t n,
                                              double *__restrict__ partial)
{
    const int i0 = blockIdx.y * kTile, j0 = blockIdx.z * kTile;
    double acc[kTile][kTile];
#pragma unroll
    for (int a = 0; a < kTile; ++a)
#pragma unroll
        for (int b = 0; b < kTile; ++b) acc[a][b] = 0.0;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
        double bv[kTile];
#pragma unroll
        for (int b = 0; b < kTile; ++b) bv[b] = (j0 + b < k) ? B[(int64_t)(j0 + b) * ldb + t] : 0.0;
#pragma unroll
        for (int a = 0; a < kTile; ++a) {
            if (i0 + a >= m) break;
            const double av = A[(int64_t)(i0 + a) * lda + t];
#pragma unroll
            for (int b = 0; b < kTile; ++b) acc[a][b] += av * bv[b];
        }
    }
    __shared__ double red[4][kTile * kTile];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int a = 0; a < kTile; ++a)
#pragma unroll
        for (int b = 0; b < kTile; ++b) {
            double v = acc[a][b];
            for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
            if (lane == 0) red[wave][a * kTile + b] = v;
        }
    __syncthreads();
    if (threadIdx.x < kTile * kTile) {
        const int a = threadIdx.x / kTile, b = threadIdx.x % kTile;
        const double v = red[0][threadIdx.x] + red[1][threadIdx.x] + red[2][threadIdx.x] + red[3][threadIdx.x];
        if (i0 + a < m && j0 + b < k) partial[((int64_t)blockIdx.x * m + i0 + a) * k + j0 + b] = v;
    }
}

__global__ void k_dots_reduce(const double *__restrict__ partial, int nblk, int mk, double *__restrict__ out)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= mk) return;
    double s = 0.0;
    for (int b = 0; b < nblk; ++b) s += partial[(int64_t)b * mk + e];
    out[e] = s;
}

int dots_blocks(int64_t n) { return (int)std::min<int64_t>(kDotBlocks, std::max<int64_t>(1, (n + 255) / 256)); }

isci_status dots(const double *A, int64_t lda, int m, const double *B, int64_t ldb, int k, int64_t n,
                 double *out_dev, double *partial, int nblk, hipStream_t s)
{
    dim3 grid(nblk, (m + kTile - 1) / kTile, (k + kTile - 1) / kTile);
    k_dots<<<grid, 256, 0, s>>>(A, lda, m, B, ldb, k, n, partial);
    k_dots_reduce<<<(m * k + 255) / 256, 256, 0, s>>>(partial, nblk, m * k, out_dev);
    ISCI_HIP(hipGetLastError());
    return ISCI_OK;
}

// out_j[t] = beta out_j[t] + sum_i V_i[t] Y[j*m + i], j < k
__global__ __launch_bounds__(256) void k_lincomb(const double *__restrict__ V, int64_t ldv, int m,
                                                 const double *__restrict__ Y, int k, double *__restrict__ out,
                                                 int64_t ldo, int64_t n, double beta)
{
    const int j0 = blockIdx.y * kTile;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
        double acc[kTile];
#pragma unroll
        for (int b = 0; b < kTile; ++b) acc[b] = 0.0;
        for (int i = 0; i < m; ++i) {
            const double v = V[(int64_t)i * ldv + t];
#pragma unroll
            for (int b = 0; b < kTile; ++b)
                if (j0 + b < k) acc[b] += v * Y[(j0 + b) * m + i];
        }
#pragma unroll
        for (int b = 0; b < kTile; ++b)
            if (j0 + b < k) {
                double *o = out + (int64_t)(j0 + b) * ldo + t;
                *o = (beta == 0.0 ? 0.0 : beta * *o) + acc[b];
            }
    }
}

isci_status lincomb(const double *V, int64_t ldv, int m, const double *Y, int k, double *out, int64_t ldo,
                    int64_t n, double beta, hipStream_t s)
{
    dim3 grid((unsigned)std::min<int64_t>(2048, (n + 255) / 256), (k + kTile - 1) / kTile);
    k_lincomb<<<grid, 256, 0, s>>>(V, ldv, m, Y, k, out, ldo, n, beta);
    ISCI_HIP(hipGetLastError());
    return ISCI_OK;
}

// R_j = WY_j - theta_j X_j (in place in WY), then T_j = R_j / clip(theta_j - D)
__global__ void k_resid_precond(double *__restrict__ WY, const double *__restrict__ X, const double *__restrict__ D,
                                const double *__restrict__ theta, int k, int64_t ld, int64_t n,
                                double *__restrict__ T)
{
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
        const double d = D[t];
        for (int j = 0; j < k; ++j) {
            const double r = WY[(int64_t)j * ld + t] - theta[j] * X[(int64_t)j * ld + t];
            WY[(int64_t)j * ld + t] = r;
            double den = theta[j] - d;
            if (fabs(den) < 1e-8) den = den < 0.0 ? -1e-8 : 1e-8;
            T[(int64_t)j * ld + t] = r / den;
        }
    }
}

__global__ void k_scale(double *__restrict__ x, int64_t n, const double *__restrict__ f)
{
    const double a = *f;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
        x[t] *= a;
}

__global__ void k_unit(double *__restrict__ x, int64_t n, int64_t pos)
{
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
        x[t] = (t == pos) ? 1.0 : 0.0;
}

static unsigned grid1(int64_t n) { return (unsigned)std::min<int64_t>(4096, std::max<int64_t>(1, (n + 255) / 256)); }

// cyclic Jacobi: A (m x m, row major, symmetric) -> eigenvalues w ascending, vectors Z (column j in Z[i*m+j])
static void jacobi_eigh(int m, std::vector<double> A, std::vector<double> &w, std::vector<double> &Z)
{
    Z.assign((size_t)m * m, 0.0);
    for (int i = 0; i < m; ++i) Z[(size_t)i * m + i] = 1.0;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < m; ++j) {
                double a = A[(size_t)i * m + j] * A[(size_t)i * m + j];
                tot += a;
                if (i != j) off += a;
            }
        if (off <= 1e-30 * tot || off == 0.0) break;
        for (int p = 0; p < m; ++p)
            for (int q = p + 1; q < m; ++q) {
                const double apq = A[(size_t)p * m + q];
                if (apq == 0.0) continue;
                const double app = A[(size_t)p * m + p], aqq = A[(size_t)q * m + q];
                const double theta = (aqq - app) / (2.0 * apq);
                const double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                const double cs = 1.0 / sqrt(t * t + 1.0), sn = t * cs;
                for (int k = 0; k < m; ++k) {
                    const double akp = A[(size_t)k * m + p], akq = A[(size_t)k * m + q];
                    A[(size_t)k * m + p] = cs * akp - sn * akq;
                    A[(size_t)k * m + q] = sn * akp + cs * akq;
                }
                for (int k = 0; k < m; ++k) {
                    const double apk = A[(size_t)p * m + k], aqk = A[(size_t)q * m + k];
                    A[(size_t)p * m + k] = cs * apk - sn * aqk;
                    A[(size_t)q * m + k] = sn * apk + cs * aqk;
                }
                for (int k = 0; k < m; ++k) {
                    const double zkp = Z[(size_t)k * m + p], zkq = Z[(size_t)k * m + q];
                    Z[(size_t)k * m + p] = cs * zkp - sn * zkq;
                    Z[(size_t)k * m + q] = sn * zkp + cs * zkq;
                }
            }
    }
    std::vector<int> ord(m);
    std::iota(ord.begin(), ord.end(), 0);
    std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return A[(size_t)a * m + a] < A[(size_t)b * m + b]; });
    w.resize(m);
    std::vector<double> Z2((size_t)m * m);
    for (int j = 0; j < m; ++j) {
        w[j] = A[(size_t)ord[j] * m + ord[j]];
        for (int i = 0; i < m; ++i) Z2[(size_t)i * m + j] = Z[(size_t)i * m + ord[j]];
    }
    Z.swap(Z2);
}

struct DavWork {
    double *V = nullptr, *W = nullptr, *X = nullptr, *R = nullptr, *T = nullptr, *D = nullptr;
    double *small = nullptr, *partial = nullptr;
};

}  // namespace isci

using namespace isci;

extern "C" {

void isci_davidson_defaults(isci_davidson_opts *o)
{
    if (!o) return;
    o->tol_residual = 1e-7;
    o->tol_energy = 1e-11;
    o->max_iter = 200;
    o->max_subspace = 0;
    o->block = 0;
}

isci_status isci_davidson(isci_handle c, int nroots, const isci_davidson_opts *opts, const double *guess,
                          int nguess, double *energies, double *vectors, isci_davidson_info *info,
                          hipStream_t s)
{
    if (!c || !energies) { set_error("NULL argument"); return ISCI_E_INVALID; }
    const int64_t dim = c->dim;
    if (nroots < 1 || nroots > ISCI_MAX_ROOTS || nroots > dim) { set_error("bad nroots"); return ISCI_E_INVALID; }
    if (nguess < 0 || (nguess > 0 && !guess)) { set_error("bad guess"); return ISCI_E_INVALID; }
    isci_davidson_opts o;
    isci_davidson_defaults(&o);
    if (opts) o = *opts;
    if (!(o.tol_residual > 0)) o.tol_residual = 1e-7;
    if (!(o.tol_energy > 0)) o.tol_energy = 1e-11;
    if (o.max_iter <= 0) o.max_iter = 200;
    // Ritz pairs followed: the requested roots plus up to two guard roots,
    // which keeps a nearly degenerate partner of the highest requested root
    // inside the corrected block.
    const int k = nroots;
    const int kk = (int)std::min<int64_t>(dim, (int64_t)k + 2);
    const int block = std::max(1, std::min(o.block > 0 ? o.block : kk, kk));
    int mmax = o.max_subspace > 0 ? o.max_subspace : std::max(32, 6 * kk);
    mmax = (int)std::min<int64_t>(std::max(mmax, kk + block), dim);
    const int keep_max = std::max(kk, std::min(2 * kk + 4, mmax / 2));

    DavWork w;
    const int nblk = dots_blocks(dim);
    std::vector<void *> mine;
    auto alloc = [&](size_t bytes) -> double * {
        void *p = nullptr;
        if (hipMalloc(&p, std::max<size_t>(bytes, 8)) != hipSuccess) return nullptr;
        mine.push_back(p);
        return (double *)p;
    };
    auto cleanup = [&]() { for (void *p : mine) (void)hipFree(p); };
    const int nscr = std::max(kk, keep_max);
    w.V = alloc(sizeof(double) * (size_t)mmax * dim);
    w.W = alloc(sizeof(double) * (size_t)mmax * dim);
    w.X = alloc(sizeof(double) * (size_t)nscr * dim);   // Ritz vectors (also restart scratch)
    w.R = alloc(sizeof(double) * (size_t)kk * dim);     // residuals
    w.T = alloc(sizeof(double) * (size_t)kk * dim);     // preconditioned corrections
    w.D = alloc(sizeof(double) * (size_t)dim);
    w.small = alloc(sizeof(double) * (size_t)(mmax * mmax + 4 * mmax + 64));
    w.partial = alloc(sizeof(double) * (size_t)nblk * mmax * mmax);
    if (!w.V || !w.W || !w.X || !w.R || !w.T || !w.D || !w.small || !w.partial) {
        cleanup();
        set_error("device allocation failed (Davidson)");
        return ISCI_E_OOM;
    }
#define DAV_CHECK(x)                                 \
    do {                                             \
        isci_status _s = (x);                        \
        if (_s != ISCI_OK) { cleanup(); return _s; } \
    } while (0)
#define DAV_HIP(x)                                                     \
    do {                                                               \
        hipError_t _e = (x);                                           \
        if (_e != hipSuccess) { cleanup(); return hip_fail(_e, #x); }  \
    } while (0)

    DAV_CHECK(launch_diag(c, w.D, s));
    int m = 0;
    double *dsmall = w.small;
    std::vector<double> hsmall((size_t)mmax * mmax + 64);

    // CGS2: orthonormalise x (device) against V[0..m) into V[m]; 1 if appended,
    // 0 if it was (numerically) in the span, negative status on failure
    auto append = [&](const double *x) -> int {
        double *dst = w.V + (size_t)m * dim;
        if (dst != x) DAV_HIP(hipMemcpyAsync(dst, x, sizeof(double) * dim, hipMemcpyDeviceToDevice, s));
        double nrm0 = 0.0;
        DAV_CHECK(dots(dst, dim, 1, dst, dim, 1, dim, dsmall, w.partial, nblk, s));
        DAV_HIP(hipMemcpyAsync(&nrm0, dsmall, sizeof(double), hipMemcpyDeviceToHost, s));
        DAV_HIP(hipStreamSynchronize(s));
        nrm0 = sqrt(nrm0);
        if (!(nrm0 > 0.0) || !std::isfinite(nrm0)) return 0;
        for (int pass = 0; pass < 2 && m > 0; ++pass) {
            DAV_CHECK(dots(w.V, dim, m, dst, dim, 1, dim, dsmall, w.partial, nblk, s));
            DAV_HIP(hipMemcpyAsync(hsmall.data(), dsmall, sizeof(double) * m, hipMemcpyDeviceToHost, s));
            DAV_HIP(hipStreamSynchronize(s));
            for (int i = 0; i < m; ++i) hsmall[i] = -hsmall[i];
            DAV_HIP(hipMemcpyAsync(dsmall, hsmall.data(), sizeof(double) * m, hipMemcpyHostToDevice, s));
            DAV_CHECK(lincomb(w.V, dim, m, dsmall, 1, dst, dim, dim, 1.0, s));
        }
        double nrm = 0.0;
        DAV_CHECK(dots(dst, dim, 1, dst, dim, 1, dim, dsmall, w.partial, nblk, s));
        DAV_HIP(hipMemcpyAsync(&nrm, dsmall, sizeof(double), hipMemcpyDeviceToHost, s));
        DAV_HIP(hipStreamSynchronize(s));
        nrm = sqrt(nrm);
        if (!(nrm > 1e-10 * nrm0)) return 0;
        const double inv = 1.0 / nrm;
        DAV_HIP(hipMemcpyAsync(dsmall, &inv, sizeof(double), hipMemcpyHostToDevice, s));
        k_scale<<<grid1(dim), 256, 0, s>>>(dst, dim, dsmall);
        DAV_HIP(hipGetLastError());
        DAV_HIP(hipStreamSynchronize(s));
        ++m;
        return 1;
    };

    // ---- initial basis: caller's guess vectors, then unit vectors on the
    // lowest diagonal entries (ties to the lowest address)
    for (int g = 0; g < nguess && m < kk; ++g)
        if (append(guess + (size_t)g * dim) < 0) return ISCI_E_HIP;
    if (m < kk) {
        std::vector<double> hd(dim);
        DAV_HIP(hipMemcpyAsync(hd.data(), w.D, sizeof(double) * dim, hipMemcpyDeviceToHost, s));
        DAV_HIP(hipStreamSynchronize(s));
        std::vector<int64_t> ord(dim);
        std::iota(ord.begin(), ord.end(), 0);
        const int64_t take = std::min<int64_t>(dim, kk + 64);
        std::partial_sort(ord.begin(), ord.begin() + take, ord.end(), [&](int64_t a, int64_t b) {
            return hd[a] < hd[b] || (hd[a] == hd[b] && a < b);
        });
        for (int64_t u = 0; u < take && m < kk; ++u) {
            k_unit<<<grid1(dim), 256, 0, s>>>(w.T, dim, ord[u]);
            DAV_HIP(hipGetLastError());
            if (append(w.T) < 0) return ISCI_E_HIP;
        }
    }
    if (m == 0) { cleanup(); set_error("empty initial basis"); return ISCI_E_INVALID; }

    std::vector<double> G((size_t)mmax * mmax, 0.0), theta(kk, 0.0), prev(kk, 1e300), rn(kk, 0.0);
    std::vector<double> evals, Z;
    int nsig = 0, mdone = 0, iter = 0;
    bool conv = false;
    for (iter = 1; iter <= o.max_iter; ++iter) {
        // sigma of the new basis vectors
        const int nnew = m - mdone;
        DAV_CHECK(launch_sigma(c, nnew, w.V + (size_t)mdone * dim, dim, w.W + (size_t)mdone * dim, dim, s));
        nsig += nnew;
        // new columns of G = V^T W: (m x nnew)
        DAV_CHECK(dots(w.V, dim, m, w.W + (size_t)mdone * dim, dim, nnew, dim, dsmall, w.partial, nblk, s));
        DAV_HIP(hipMemcpyAsync(hsmall.data(), dsmall, sizeof(double) * m * nnew, hipMemcpyDeviceToHost, s));
        DAV_HIP(hipStreamSynchronize(s));
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < nnew; ++j) {
                const double v = hsmall[(size_t)i * nnew + j];
                G[(size_t)i * mmax + mdone + j] = v;
                if (i < mdone) G[(size_t)(mdone + j) * mmax + i] = v;
            }
        for (int i = mdone; i < m; ++i)   // new-new block: symmetrise
            for (int j = mdone; j < i; ++j) {
                const double a = 0.5 * (G[(size_t)i * mmax + j] + G[(size_t)j * mmax + i]);
                G[(size_t)i * mmax + j] = a;
                G[(size_t)j * mmax + i] = a;
            }
        mdone = m;
        std::vector<double> Gm((size_t)m * m);
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < m; ++j) Gm[(size_t)i * m + j] = G[(size_t)i * mmax + j];
        jacobi_eigh(m, Gm, evals, Z);
        const int kr = std::min(kk, m);
        std::vector<double> Y((size_t)kr * m);   // Y[j*m + i] = Z[i][j]
        for (int j = 0; j < kr; ++j)
            for (int i = 0; i < m; ++i) Y[(size_t)j * m + i] = Z[(size_t)i * m + j];
        for (int j = 0; j < kr; ++j) theta[j] = evals[j];
        double *dY = dsmall, *dth = dsmall + (size_t)kr * m;
        DAV_HIP(hipMemcpyAsync(dY, Y.data(), sizeof(double) * Y.size(), hipMemcpyHostToDevice, s));
        DAV_HIP(hipMemcpyAsync(dth, theta.data(), sizeof(double) * kr, hipMemcpyHostToDevice, s));
        DAV_CHECK(lincomb(w.V, dim, m, dY, kr, w.X, dim, dim, 0.0, s));
        DAV_CHECK(lincomb(w.W, dim, m, dY, kr, w.R, dim, dim, 0.0, s));
        k_resid_precond<<<grid1(dim), 256, 0, s>>>(w.R, w.X, w.D, dth, kr, dim, dim, w.T);
        DAV_HIP(hipGetLastError());
        double *dn = dth + kr;
        DAV_CHECK(dots(w.R, dim, kr, w.R, dim, kr, dim, dn, w.partial, nblk, s));
        std::vector<double> rr((size_t)kr * kr);
        DAV_HIP(hipMemcpyAsync(rr.data(), dn, sizeof(double) * kr * kr, hipMemcpyDeviceToHost, s));
        DAV_HIP(hipStreamSynchronize(s));
        conv = kr >= k;
        for (int j = 0; j < kr; ++j) {
            rn[j] = sqrt(std::max(0.0, rr[(size_t)j * kr + j]));
            if (j < k) conv = conv && rn[j] <= o.tol_residual && fabs(theta[j] - prev[j]) <= o.tol_energy;
        }
        for (int j = 0; j < kr; ++j) prev[j] = theta[j];
        if (conv || iter == o.max_iter) break;
        // corrections of the unconverged Ritz pairs (at most `block`)
        std::vector<int> pick;
        for (int j = 0; j < kr && (int)pick.size() < block; ++j)
            if (rn[j] > o.tol_residual) pick.push_back(j);
        if (pick.empty())
            for (int j = 0; j < kr && (int)pick.size() < block; ++j) pick.push_back(j);
        if (m + (int)pick.size() > mmax) {
            // thick restart: keep the lowest `keep` Ritz vectors of the basis
            const int keep = std::min(m, keep_max);
            std::vector<double> Yk((size_t)keep * m);
            for (int j = 0; j < keep; ++j)
                for (int i = 0; i < m; ++i) Yk[(size_t)j * m + i] = Z[(size_t)i * m + j];
            double *dYk = dsmall + (size_t)kr * m + kr + (size_t)kr * kr;
            if ((size_t)(dYk - dsmall) + Yk.size() > (size_t)(mmax * mmax + 4 * mmax + 64)) dYk = dsmall;
            DAV_HIP(hipMemcpyAsync(dYk, Yk.data(), sizeof(double) * Yk.size(), hipMemcpyHostToDevice, s));
            DAV_CHECK(lincomb(w.V, dim, m, dYk, keep, w.X, dim, dim, 0.0, s));
            DAV_HIP(hipMemcpyAsync(w.V, w.X, sizeof(double) * (size_t)keep * dim, hipMemcpyDeviceToDevice, s));
            DAV_CHECK(lincomb(w.W, dim, m, dYk, keep, w.X, dim, dim, 0.0, s));
            DAV_HIP(hipMemcpyAsync(w.W, w.X, sizeof(double) * (size_t)keep * dim, hipMemcpyDeviceToDevice, s));
            // Ritz vectors of the restarted basis are its first kr vectors
            DAV_HIP(hipMemcpyAsync(w.X, w.V, sizeof(double) * (size_t)kr * dim, hipMemcpyDeviceToDevice, s));
            m = keep;
            mdone = keep;
            std::fill(G.begin(), G.end(), 0.0);
            for (int j = 0; j < keep; ++j) G[(size_t)j * mmax + j] = evals[j];
        }
        int added = 0;
        for (int j : pick) {
            if (m >= mmax) break;
            const int r = append(w.T + (size_t)j * dim);
            if (r < 0) return ISCI_E_HIP;
            added += r;
        }
        if (added == 0) break;
    }
    for (int j = 0; j < k; ++j) energies[j] = theta[j];
    if (vectors) DAV_HIP(hipMemcpyAsync(vectors, w.X, sizeof(double) * (size_t)k * dim, hipMemcpyDeviceToDevice, s));
    DAV_HIP(hipStreamSynchronize(s));
    if (info) {
        info->iterations = std::min(iter, o.max_iter);
        info->converged = conv ? 1 : 0;
        info->sigma_calls = nsig;
        for (int j = 0; j < ISCI_MAX_ROOTS; ++j) info->residual[j] = j < k ? rn[j] : 0.0;
    }
    cleanup();
    return conv ? ISCI_OK : ISCI_E_NOT_CONVERGED;
}

}  // extern "C"
