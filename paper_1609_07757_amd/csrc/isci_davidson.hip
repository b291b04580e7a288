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
#include <atomic>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <functional>
#include <mutex>
#include <numeric>
#include <thread>
#include <vector>

#include "isci_device.h"
#include "isci_internal.h"

namespace isci {

constexpr int kDotBlocks = 256;
constexpr int kTile = 8;
// coefficient matrices of a linear combination staged in LDS up to this
// many basis vectors (the default subspace bound is below it)
constexpr int kLinMaxM = 256;

// vectors are device (global) memory: reading them through global-space
// pointers keeps the loads off the flat path, whose completion the
// compiler must also wait for before LDS reads
typedef __attribute__((address_space(1))) const double gdouble;
typedef __attribute__((address_space(1))) double gdouble_w;
__device__ __forceinline__ const gdouble *gptr(const double *p) { return (const gdouble *)p; }
__device__ __forceinline__ gdouble_w *gptr_w(double *p) { return (gdouble_w *)p; }

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
    // rows past m / k are read clamped and zeroed: no load sits under a branch
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
        double av[kTile], bv[kTile];
#pragma unroll
        for (int b = 0; b < kTile; ++b) {
            const double x = B[(int64_t)min(j0 + b, k - 1) * ldb + t];
            bv[b] = j0 + b < k ? x : 0.0;
        }
#pragma unroll
        for (int a = 0; a < kTile; ++a) {
            const double x = A[(int64_t)min(i0 + a, m - 1) * lda + t];
            av[a] = i0 + a < m ? x : 0.0;
        }
#pragma unroll
        for (int a = 0; a < kTile; ++a)
#pragma unroll
            for (int b = 0; b < kTile; ++b) acc[a][b] += av[a] * bv[b];
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

// one wave per output: lanes stride over the block partials, then a
// shuffle tree (fixed order for a given block count)
__device__ __forceinline__ double wave_sum_partials(const double *__restrict__ partial, int nblk, int mk, int e,
                                                    int lane)
{
    double s = 0.0;
    for (int b = lane; b < nblk; b += 64) s += partial[(int64_t)b * mk + e];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    return s;
}

__global__ __launch_bounds__(256) void k_dots_reduce(const double *__restrict__ partial, int nblk, int mk,
                                                     double *__restrict__ out)
{
    const int e = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (e >= mk) return;
    const double s = wave_sum_partials(partial, nblk, mk, e, lane);
    if (lane == 0) out[e] = s;
}

// partial-sum blocks for a dot product of length n: about 2048 elements
// (8 per thread) per block, at most kDotBlocks
// one element block (summed inside its workgroup, no second kernel) for
// vectors of at most kDotOneBlock elements, else one block per 512 elements
constexpr int64_t kDotOneBlock = 2048;
int dots_blocks(int64_t n)
{
    return n <= kDotOneBlock ? 1 : (int)std::min<int64_t>(kDotBlocks, std::max<int64_t>(1, (n + 511) / 512));
}

isci_status dots(const double *A, int64_t lda, int m, const double *B, int64_t ldb, int k, int64_t n,
                 double *out_dev, double *partial, int nblk, hipStream_t s)
{
    dim3 grid(nblk, (m + kTile - 1) / kTile, (k + kTile - 1) / kTile);
    k_dots<<<grid, 256, 0, s>>>(A, lda, m, B, ldb, k, n, partial);
    k_dots_reduce<<<(m * k + 3) / 4, 256, 0, s>>>(partial, nblk, m * k, out_dev);
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


// Symmetric eigensolver: Householder reduction to tridiagonal form, then the
// implicit symmetric QR iteration with Wilkinson shifts (Golub and Van Loan,
// Matrix Computations, sections 8.3.1 and 8.3.2).  A (m x m, row major,
// symmetric) -> eigenvalues w ascending, vectors Z (column j in Z[i*m+j]).
// Returns false when the QR iteration does not settle (the caller then uses
// the Jacobi solver).
static bool tridiag_eigh(int m, std::vector<double> A, std::vector<double> &w, std::vector<double> &Z)
{
    Z.assign((size_t)m * m, 0.0);
    for (int i = 0; i < m; ++i) Z[(size_t)i * m + i] = 1.0;
    std::vector<double> v(m), p(m), d(m), e(std::max(m, 1), 0.0);
    // (1) A <- H A H with H = I - 2 v v^T zeroing column k below its subdiagonal; Z <- Z H
    for (int k = 0; k + 2 < m; ++k) {
        const int n = m - k - 1;   // trailing size, indices k+1 .. m-1
        double nx = 0.0;
        for (int i = 0; i < n; ++i) nx += A[(size_t)(k + 1 + i) * m + k] * A[(size_t)(k + 1 + i) * m + k];
        nx = sqrt(nx);
        const double x0 = A[(size_t)(k + 1) * m + k];
        const double alpha = x0 >= 0.0 ? -nx : nx;
        for (int i = 0; i < n; ++i) v[i] = A[(size_t)(k + 1 + i) * m + k];
        v[0] -= alpha;
        double nv = 0.0;
        for (int i = 0; i < n; ++i) nv += v[i] * v[i];
        if (nv == 0.0) continue;   // column already reduced
        nv = 1.0 / sqrt(nv);
        for (int i = 0; i < n; ++i) v[i] *= nv;
        double K = 0.0;
        for (int i = 0; i < n; ++i) {
            double s = 0.0;
            const double *row = &A[(size_t)(k + 1 + i) * m + k + 1];
            for (int j = 0; j < n; ++j) s += row[j] * v[j];
            p[i] = s;
            K += v[i] * s;
        }
        for (int i = 0; i < n; ++i) p[i] = 2.0 * (p[i] - K * v[i]);
        for (int i = 0; i < n; ++i) {
            double *row = &A[(size_t)(k + 1 + i) * m + k + 1];
            for (int j = 0; j < n; ++j) row[j] -= v[i] * p[j] + p[i] * v[j];
        }
        A[(size_t)(k + 1) * m + k] = A[(size_t)k * m + k + 1] = alpha;
        for (int i = 1; i < n; ++i) A[(size_t)(k + 1 + i) * m + k] = A[(size_t)k * m + k + 1 + i] = 0.0;
        for (int r = 0; r < m; ++r) {
            double *zr = &Z[(size_t)r * m + k + 1];
            double s = 0.0;
            for (int j = 0; j < n; ++j) s += zr[j] * v[j];
            s *= 2.0;
            for (int j = 0; j < n; ++j) zr[j] -= s * v[j];
        }
    }
    // rotations below act on pairs of columns of Z: keep them as rows of Zt
    std::vector<double> Zt((size_t)m * m);
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < m; ++j) Zt[(size_t)j * m + i] = Z[(size_t)i * m + j];
    for (int i = 0; i < m; ++i) d[i] = A[(size_t)i * m + i];
    for (int i = 0; i + 1 < m; ++i) e[i] = A[(size_t)(i + 1) * m + i];
    // (2) implicit QR steps on the unreduced trailing block [lo, hi]; a
    // subdiagonal entry at rounding level of its neighbours is set to zero
    const double eps = 2.220446049250313e-16;
    int hi = m - 1, steps = 0;
    while (hi > 0) {
        if (fabs(e[hi - 1]) <= eps * (fabs(d[hi - 1]) + fabs(d[hi]))) { e[hi - 1] = 0.0; --hi; continue; }
        if (++steps > 60 * m) return false;
        int lo = hi - 1;
        while (lo > 0 && fabs(e[lo - 1]) > eps * (fabs(d[lo - 1]) + fabs(d[lo]))) --lo;
        if (lo > 0) e[lo - 1] = 0.0;
        // Wilkinson shift: the eigenvalue of the trailing 2 x 2 block nearer d[hi]
        const double dl = 0.5 * (d[hi - 1] - d[hi]), b = e[hi - 1];
        const double mu = d[hi] - b * b / (dl + (dl >= 0.0 ? 1.0 : -1.0) * hypot(dl, b));
        double x = d[lo] - mu, z = e[lo], bulge = 0.0;
        for (int k = lo; k < hi; ++k) {
            if (k > lo) { x = e[k - 1]; z = bulge; }
            const double r = hypot(x, z);
            double c = 1.0, s = 0.0;
            if (r != 0.0) { c = x / r; s = z / r; }
            if (k > lo) e[k - 1] = r;
            const double a = d[k], bb = e[k], cc = d[k + 1];
            d[k] = c * c * a + 2.0 * c * s * bb + s * s * cc;
            d[k + 1] = s * s * a - 2.0 * c * s * bb + c * c * cc;
            e[k] = c * s * (cc - a) + (c * c - s * s) * bb;
            if (k + 1 < hi) { bulge = s * e[k + 1]; e[k + 1] *= c; }
            double *z0 = &Zt[(size_t)k * m], *z1 = z0 + m;
            for (int r2 = 0; r2 < m; ++r2) {
                const double a0 = z0[r2], a1 = z1[r2];
                z0[r2] = c * a0 + s * a1;
                z1[r2] = -s * a0 + c * a1;
            }
        }
    }
    std::vector<int> ord(m);
    std::iota(ord.begin(), ord.end(), 0);
    std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return d[a] < d[b]; });
    w.resize(m);
    for (int j = 0; j < m; ++j) {
        w[j] = d[ord[j]];
        const double *zt = &Zt[(size_t)ord[j] * m];
        for (int i = 0; i < m; ++i) Z[(size_t)i * m + j] = zt[i];
    }
    return true;
}

// symmetric eigensolver for small projected matrices (used by the
// propagator too): tridiagonal QR, cyclic Jacobi when that does not settle
void sym_eigh(int m, const std::vector<double> &A, std::vector<double> &w, std::vector<double> &Z)
{
    if (!tridiag_eigh(m, A, w, Z)) jacobi_eigh(m, A, w, Z);
}

__global__ void k_neg(double *__restrict__ x, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = -x[i];
}

// x *= 1/||x|| when ||x|| > rel ||x0||, else x = 0; fac[0] records the factor
__global__ void k_normalize(double *__restrict__ x, int64_t n, const double *__restrict__ nrm2_0,
                            const double *__restrict__ nrm2, double rel, double *__restrict__ fac)
{
    const double a = sqrt(*nrm2), a0 = sqrt(*nrm2_0);
    const double f = (a > rel * a0 && a > 0.0) ? 1.0 / a : 0.0;
    if (blockIdx.x == 0 && threadIdx.x == 0) *fac = f;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
        x[t] *= f;
}


// ---------------------------------------------------------------- batched block algebra
// One launch serves every slot of an engine: each kernel reads a device
// array of per-slot descriptors and blockIdx.z selects the descriptor.

struct BDot {              // out[i*k + j] = sum_t A[i*lda + t] B[j*ldb + t]
    const double *A, *B;
    double *out, *partial;
    int64_t lda, ldb, n;
    int m, k, nblk;
    const double *skip = nullptr;   // device flag: nonzero skips the job
};

// Sum each of the 64 values v[] over the wave's 64 lanes, halving the
// values per lane at every step: lane L ends with the sum of value L in
// v[0] (63 lane exchanges instead of 6 per value).
template <int O>
__device__ __forceinline__ void transpose_sum_step(double (&v)[64], int lane)
{
    const bool up = (lane & O) != 0;
#pragma unroll
    for (int i = 0; i < O; ++i) {
        const double send = up ? v[i] : v[i + O];
        const double keep = up ? v[i + O] : v[i];
        v[i] = keep + __shfl_xor(send, O, 64);
    }
}

__device__ __forceinline__ void wave_transpose_sum64(double (&v)[64], int lane)
{
    transpose_sum_step<32>(v, lane);
    transpose_sum_step<16>(v, lane);
    transpose_sum_step<8>(v, lane);
    transpose_sum_step<4>(v, lane);
    transpose_sum_step<2>(v, lane);
    transpose_sum_step<1>(v, lane);
}

// Workgroup id -> (tile, block of the element range): the tiles of one
// element block are consecutive ids eight apart, so they run on one XCD
// at about the same time and share the block's rows in its L2.
__global__ __launch_bounds__(256) void k_bdots(const BDot *__restrict__ jobs, int tiles_i, int tiles_j)
{
    const BDot J = jobs[blockIdx.z];
    if (J.skip && *J.skip != 0.0) return;
    const int ntiles = tiles_i * tiles_j;
    const int id = blockIdx.x, rest = id >> 3;
    const int tile = rest % ntiles, blk = (rest / ntiles) * 8 + (id & 7);
    const int ti = tile / tiles_j, tj = tile % tiles_j;
    const int i0 = ti * kTile, j0 = tj * kTile;
    if (blk >= J.nblk || i0 >= J.m || j0 >= J.k) return;
    double acc[kTile][kTile];
#pragma unroll
    for (int a = 0; a < kTile; ++a)
#pragma unroll
        for (int b = 0; b < kTile; ++b) acc[a][b] = 0.0;
    // rows past m / k are skipped; the conditions are uniform over the
    // workgroup (scalar branches), so only valid rows are loaded
    const gdouble *A = gptr(J.A), *B = gptr(J.B);
    const int na = __builtin_amdgcn_readfirstlane(min(kTile, J.m - i0));
    const int nb = __builtin_amdgcn_readfirstlane(min(kTile, J.k - j0));
    for (int64_t t = (int64_t)blk * blockDim.x + threadIdx.x; t < J.n; t += (int64_t)J.nblk * blockDim.x) {
        double av[kTile], bv[kTile];
#pragma unroll
        for (int b = 0; b < kTile; ++b) bv[b] = b < nb ? B[(int64_t)(j0 + b) * J.ldb + t] : 0.0;
#pragma unroll
        for (int a = 0; a < kTile; ++a) av[a] = a < na ? A[(int64_t)(i0 + a) * J.lda + t] : 0.0;
#pragma unroll
        for (int a = 0; a < kTile; ++a)
#pragma unroll
            for (int b = 0; b < kTile; ++b) acc[a][b] += av[a] * bv[b];
    }
    __shared__ double red[4][kTile * kTile];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    static_assert(kTile * kTile == 64, "one accumulator per lane after the transpose sum");
    double v[64];
#pragma unroll
    for (int a = 0; a < kTile; ++a)
#pragma unroll
        for (int b = 0; b < kTile; ++b) v[a * kTile + b] = acc[a][b];
    wave_transpose_sum64(v, lane);
    red[wave][lane] = v[0];
    __syncthreads();
    if (threadIdx.x < kTile * kTile) {
        const int a = threadIdx.x / kTile, b = threadIdx.x % kTile;
        const double r = red[0][threadIdx.x] + red[1][threadIdx.x] + red[2][threadIdx.x] + red[3][threadIdx.x];
        // a job of one element block is complete here
        if (i0 + a < J.m && j0 + b < J.k) {
            if (J.nblk == 1) J.out[(i0 + a) * J.k + j0 + b] = r;
            else J.partial[((int64_t)blk * J.m + i0 + a) * J.k + j0 + b] = r;
        }
    }
}

__global__ __launch_bounds__(256) void k_bdots_reduce(const BDot *__restrict__ jobs)
{
    const BDot J = jobs[blockIdx.z];
    if (J.nblk == 1 || (J.skip && *J.skip != 0.0)) return;
    const int e = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int mk = J.m * J.k;
    if (e >= mk) return;
    const double s = wave_sum_partials(J.partial, J.nblk, mk, e, lane);
    if (lane == 0) J.out[e] = s;
}

struct BLin {              // out_j[t] = beta out_j[t] + sign * sum_i V_i[t] Y[j*m + i]
    const double *V, *Y;
    double *out;
    int64_t ldv, ldo, n;
    int m, k;
    double beta, sign;
    const double *skip = nullptr;   // device flag: nonzero skips the job
};

// Daniel-Gragg-Kaufman-Stewart test after the first projection of a block
// against the basis: when every column kept at least half of its squared
// norm (gm[q][q] >= g0[q][q] / 2), one projection already leaves it
// orthogonal to working precision and the second is skipped.
struct BFlag {
    const double *g0, *gm;
    double *flag;
    int p;
};

__global__ void k_dgks_flag(const BFlag *__restrict__ jobs, int njobs)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= njobs) return;
    const BFlag J = jobs[j];
    bool ok = true;
    for (int q = 0; q < J.p; ++q) ok = ok && J.gm[q * J.p + q] >= 0.5 * J.g0[q * J.p + q];
    *J.flag = ok ? 1.0 : 0.0;
}

__global__ __launch_bounds__(256) void k_blincomb(const BLin *__restrict__ jobs)
{
    const BLin J = jobs[blockIdx.z];
    const int j0 = blockIdx.y * kTile;
    // the grid is sized for the longest job: workgroups past this job's
    // elements leave before staging the coefficients
    if (j0 >= J.k || (int64_t)blockIdx.x * blockDim.x >= J.n || (J.skip && *J.skip != 0.0)) return;
    const int m = J.m, kb = min(kTile, J.k - j0);
    // this block's coefficients Y[(j0 + b) m + i] in LDS as Ys[i][b] (zero
    // for b >= kb and for the eight rows past m), read back as broadcasts
    __shared__ double Ys[(kLinMaxM + 8) * kTile];
    const bool staged = m <= kLinMaxM;
    if (staged)
        for (int e = threadIdx.x; e < (m + 8) * kTile; e += blockDim.x) {
            const int i = e / kTile, b = e % kTile;
            Ys[e] = (b < kb && i < m) ? J.Y[(int64_t)(j0 + b) * m + i] : 0.0;
        }
    __syncthreads();
    const gdouble *__restrict__ V = gptr(J.V);
    const gdouble *__restrict__ Y = gptr(J.Y);
    gdouble_w *__restrict__ out = gptr_w(J.out);
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < J.n; t += (int64_t)gridDim.x * blockDim.x) {
        double acc[kTile];
#pragma unroll
        for (int b = 0; b < kTile; ++b) acc[b] = 0.0;
        if (staged) {
            // eight basis rows per step, loaded together (rows past m
            // clamped; their coefficients are zero)
            for (int i0 = 0; i0 < m; i0 += 8) {
                double v[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) v[u] = V[(int64_t)min(i0 + u, m - 1) * J.ldv + t];
#pragma unroll
                for (int u = 0; u < 8; ++u)
#pragma unroll
                    for (int b = 0; b < kTile; ++b) acc[b] += v[u] * Ys[(i0 + u) * kTile + b];
            }
        } else {
            for (int i = 0; i < m; ++i) {
                const double v = V[(int64_t)i * J.ldv + t];
#pragma unroll
                for (int b = 0; b < kTile; ++b) acc[b] += v * Y[(int64_t)min(j0 + b, J.k - 1) * m + i];
            }
        }
        double old[kTile];
#pragma unroll
        for (int b = 0; b < kTile; ++b) old[b] = 0.0;
        if (J.beta != 0.0)
#pragma unroll
            for (int b = 0; b < kTile; ++b) old[b] = out[(int64_t)(j0 + min(b, kb - 1)) * J.ldo + t];
#pragma unroll
        for (int b = 0; b < kTile; ++b)
            if (b < kb) out[(int64_t)(j0 + b) * J.ldo + t] = J.beta * old[b] + J.sign * acc[b];
    }
}

struct BRes {              // residuals and Davidson corrections of one slot
    double *WY, *T;
    const double *X, *D, *theta;
    int64_t ld, n;
    int k;
};

// Grid-stride element loops below take four elements per step, all loads
// before any store, through restrict pointers: the loads of a step are in
// flight together instead of one latency per element.  Loads past the end
// are masked off, not clamped, so short vectors issue no extra traffic.
__global__ void k_bresid(const BRes *__restrict__ jobs)
{
    const BRes J = jobs[blockIdx.z];
    const int64_t st = (int64_t)gridDim.x * blockDim.x, n = J.n, ld = J.ld;
    const int k = J.k;
    const gdouble *__restrict__ X = gptr(J.X);
    const gdouble *__restrict__ D = gptr(J.D);
    gdouble_w *__restrict__ WY = gptr_w(J.WY);
    gdouble_w *__restrict__ T = gptr_w(J.T);
    for (int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t0 < n; t0 += 4 * st) {
        double d[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) d[u] = t0 + u * st < n ? D[t0 + u * st] : 0.0;
        for (int j = 0; j < k; ++j) {
            const double th = J.theta[j];
            const int64_t o = (int64_t)j * ld;
            double w[4], x[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int64_t t = t0 + u * st;
                w[u] = t < n ? WY[o + t] : 0.0;
                x[u] = t < n ? X[o + t] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int64_t t = t0 + u * st;
                if (t >= n) break;
                const double r = w[u] - th * x[u];
                double den = th - d[u];
                if (fabs(den) < 1e-8) den = den < 0.0 ? -1e-8 : 1e-8;
                WY[o + t] = r;
                T[o + t] = r / den;
            }
        }
    }
}

struct BVecOp {            // copy src -> dst, or normalise dst (see k_bnormalize)
    const double *src;
    double *dst;
    const double *n0, *n1;
    double *fac;
    int64_t n;
};

__global__ void k_bcopy(const BVecOp *__restrict__ jobs)
{
    const BVecOp J = jobs[blockIdx.z];
    const int64_t st = (int64_t)gridDim.x * blockDim.x, n = J.n;
    const gdouble *__restrict__ src = gptr(J.src);
    gdouble_w *__restrict__ dst = gptr_w(J.dst);
    for (int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t0 < n; t0 += 4 * st) {
        double v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = t0 + u * st < n ? src[t0 + u * st] : 0.0;
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (t0 + u * st < n) dst[t0 + u * st] = v[u];
    }
}

__global__ void k_bnormalize(const BVecOp *__restrict__ jobs, double rel)
{
    const BVecOp J = jobs[blockIdx.z];
    const double a = sqrt(*J.n1), a0 = sqrt(*J.n0);
    const double f = (a > rel * a0 && a > 0.0) ? 1.0 / a : 0.0;
    if (blockIdx.x == 0 && threadIdx.x == 0) *J.fac = f;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < J.n; t += (int64_t)gridDim.x * blockDim.x)
        J.dst[t] *= f;
}

// ---------------------------------------------------------------- engine

// Per-solve state.  Device buffers: V, W (mmax x dim), X (nscr x dim), R, T
// (kk x dim), D (dim); small: projected-matrix and coefficient scratch.
struct Slot {
    isci_handle h = nullptr;
    isci_davidson_opts o{};
    int k = 0, kk = 0, block = 0, mmax = 0, keep_max = 0, nscr = 0, nblk = 1;
    int m = 0, mdone = 0, iter = 0, nsig = 0, kr = 0;
    bool done = false, conv = false, failed = false;
    isci_status status = ISCI_OK;
    int64_t dim = 0;
    std::vector<double> G, theta, prev, rn, evals, Z;
    std::vector<int> pick;
    double *V = nullptr, *W = nullptr, *X = nullptr, *R = nullptr, *T = nullptr, *D = nullptr;
    double *small = nullptr, *partial = nullptr, *scal = nullptr;  // scal: per-append scalars
    double *hsmall = nullptr;                                       // pinned host mirror of small
    double *hscal = nullptr;                                        // pinned host mirror of scal
    size_t small_len = 0, scal_len = 0;
    std::vector<void *> mem;
};

static size_t slot_small_len(int mmax) { return (size_t)mmax * mmax + 8 * (size_t)mmax + 64; }

static int64_t slot_bytes(int64_t dim, int k, const isci_davidson_opts &o, int *kk_o, int *mmax_o, int *keep_o)
{
    const int kk = (int)std::min<int64_t>(dim, (int64_t)k + 2);
    const int block = std::max(1, std::min(o.block > 0 ? o.block : kk, kk));
    int mmax = o.max_subspace > 0 ? o.max_subspace : std::max(32, 6 * kk);
    mmax = (int)std::min<int64_t>(std::max(mmax, kk + block), dim);
    const int keep = std::max(kk, std::min(2 * kk + 4, mmax / 2));
    if (kk_o) *kk_o = kk;
    if (mmax_o) *mmax_o = mmax;
    if (keep_o) *keep_o = keep;
    const int nscr = std::max(kk, keep);
    const int nblk = dots_blocks(dim);
    int64_t b = (int64_t)sizeof(double) * dim * (2 * (int64_t)mmax + nscr + 2 * kk + 1);
    b += (int64_t)sizeof(double) * ((int64_t)slot_small_len(mmax) + (int64_t)nblk * mmax * mmax + 3 * (mmax + 8));
    return b;
}

// Host worker threads kept for an engine's life: run(count, f) calls f(j)
// for j in [0, count) on the workers and the calling thread and returns
// when all calls have finished (the per-step projected eigenproblems).
class HostPool {
  public:
    explicit HostPool(int nworkers)
    {
        for (int t = 0; t < nworkers; ++t) th_.emplace_back([this]() { loop(); });
    }
    ~HostPool()
    {
        {
            std::lock_guard<std::mutex> g(mu_);
            stop_ = true;
        }
        cv_.notify_all();
        for (std::thread &t : th_) t.join();
    }
    void run(int count, const std::function<void(int)> &f)
    {
        {
            std::lock_guard<std::mutex> g(mu_);
            fn_ = &f;
            total_ = count;
            next_.store(0);
            left_ = count;
            ++gen_;
        }
        cv_.notify_all();
        work();
        std::unique_lock<std::mutex> g(mu_);
        done_.wait(g, [this]() { return left_ == 0; });
        fn_ = nullptr;
    }

  private:
    void work()
    {
        for (;;) {
            const int j = next_.fetch_add(1);
            if (j >= total_) return;
            (*fn_)(j);
            std::lock_guard<std::mutex> g(mu_);
            if (--left_ == 0) done_.notify_all();
        }
    }
    void loop()
    {
        long seen = 0;
        for (;;) {
            {
                std::unique_lock<std::mutex> g(mu_);
                cv_.wait(g, [&]() { return stop_ || gen_ != seen; });
                if (stop_) return;
                seen = gen_;
            }
            work();
        }
    }
    std::vector<std::thread> th_;
    std::mutex mu_;
    std::condition_variable cv_, done_;
    const std::function<void(int)> *fn_ = nullptr;
    std::atomic<int> next_{0};
    int total_ = 0, left_ = 0;
    long gen_ = 0;
    bool stop_ = false;
};

}  // namespace isci

struct isci_engine_s {
    hipStream_t s = nullptr;
    std::vector<isci::Slot *> slots;   // index = slot id; nullptr when released
    // fused-sigma staging (device and pinned host), grown on demand
    isci::SigmaArgs *d_args = nullptr, *h_args = nullptr;
    isci::BatchVec *d_vecs = nullptr, *h_vecs = nullptr;
    size_t cap_args = 0, cap_vecs = 0;
    int grid = 0;          // persistent grid size for the fused sigma (0: one block per item)
    int order = 1;         // 1: heaviest work items first, 0: natural order
    // per-phase descriptor arena (pinned host -> device) and result arena
    // (device -> pinned host) of the batched block algebra
    char *arena_d = nullptr, *arena_h = nullptr;
    double *res_d = nullptr, *res_h = nullptr;
    size_t arena_cap = 0, res_cap = 0;
    // the last upload from arena_h: the host rewrites the arena only after
    // that copy has run
    hipEvent_t arena_ev = nullptr;
    bool arena_pending = false;
    // side streams for the per-instance matrix-core sigma launches (default
    // priority), forked from and joined back into s with events
    std::vector<hipStream_t> side;
    std::vector<hipEvent_t> side_ev;   // [0]: fork, [1 + i]: join of side[i]
    isci::HostPool *pool = nullptr;    // created on the first step with many slots
};

namespace isci {

static void slot_free(Slot *sl)
{
    if (!sl) return;
    for (void *p : sl->mem) (void)hipFree(p);
    if (sl->hsmall) (void)hipHostFree(sl->hsmall);
    if (sl->hscal) (void)hipHostFree(sl->hscal);
    delete sl;
}

template <typename T>
static bool grow(T *&d, T *&h, size_t &cap, size_t need)
{
    if (need <= cap) return true;
    size_t n = std::max<size_t>(need, 2 * cap + 16);
    if (d) (void)hipFree(d);
    if (h) (void)hipHostFree(h);
    d = nullptr;
    h = nullptr;
    cap = 0;
    if (hipMalloc((void **)&d, sizeof(T) * n) != hipSuccess) return false;
    if (hipHostMalloc((void **)&h, sizeof(T) * n, hipHostMallocDefault) != hipSuccess) return false;
    cap = n;
    return true;
}

#define SLOT_HIP(sl, x)                                                          \
    do {                                                                         \
        hipError_t _e = (x);                                                     \
        if (_e != hipSuccess) { (sl)->failed = true; return hip_fail(_e, #x); }  \
    } while (0)
#define SLOT_CHECK(sl, x)                                              \
    do {                                                               \
        isci_status _s = (x);                                          \
        if (_s != ISCI_OK) { (sl)->failed = true; return _s; }         \
    } while (0)

// Device-side CGS2 of vector T_src into V[m] (no host synchronisation);
// records the normalisation factor in scal[2*slotpos + 1].
static isci_status cgs2_enqueue(Slot *sl, const double *src, int pos, hipStream_t s)
{
    const int64_t dim = sl->dim;
    double *dst = sl->V + (size_t)sl->m * dim;
    double *sc = sl->scal + 3 * pos;
    if (dst != src) SLOT_HIP(sl, hipMemcpyAsync(dst, src, sizeof(double) * dim, hipMemcpyDeviceToDevice, s));
    SLOT_CHECK(sl, dots(dst, dim, 1, dst, dim, 1, dim, sc, sl->partial, sl->nblk, s));
    for (int pass = 0; pass < 2 && sl->m > 0; ++pass) {
        double *coef = sl->small;   // m coefficients
        SLOT_CHECK(sl, dots(sl->V, dim, sl->m, dst, dim, 1, dim, coef, sl->partial, sl->nblk, s));
        k_neg<<<(sl->m + 255) / 256, 256, 0, s>>>(coef, sl->m);
        SLOT_CHECK(sl, lincomb(sl->V, dim, sl->m, coef, 1, dst, dim, dim, 1.0, s));
    }
    SLOT_CHECK(sl, dots(dst, dim, 1, dst, dim, 1, dim, sc + 1, sl->partial, sl->nblk, s));
    k_normalize<<<grid1(dim), 256, 0, s>>>(dst, dim, sc, sc + 1, 1e-10, sc + 2);
    SLOT_HIP(sl, hipGetLastError());
    sl->m += 1;
    return ISCI_OK;
}

// After the enqueued appends of this call (count n, first at basis index
// m0) completed: drop the vectors whose factor is 0 by moving later ones
// into their place.
static isci_status cgs2_finish(Slot *sl, int m0, int n, hipStream_t s)
{
    const int64_t dim = sl->dim;
    int w = m0;
    for (int i = 0; i < n; ++i) {
        const bool keep = sl->hscal[3 * i + 2] != 0.0;
        if (!keep) continue;
        if (w != m0 + i)
            SLOT_HIP(sl, hipMemcpyAsync(sl->V + (size_t)w * dim, sl->V + (size_t)(m0 + i) * dim,
                                        sizeof(double) * dim, hipMemcpyDeviceToDevice, s));
        ++w;
    }
    sl->m = w;
    return ISCI_OK;
}

static isci_status slot_init(isci_engine e, Slot *sl, const double *guess, int nguess)
{
    hipStream_t s = e->s;
    const int64_t dim = sl->dim;
    int64_t bytes = slot_bytes(dim, sl->k, sl->o, &sl->kk, &sl->mmax, &sl->keep_max);
    (void)bytes;
    sl->block = std::max(1, std::min(sl->o.block > 0 ? sl->o.block : sl->kk, sl->kk));
    sl->nscr = std::max(sl->kk, sl->keep_max);
    sl->nblk = dots_blocks(dim);
    sl->small_len = slot_small_len(sl->mmax);
    sl->scal_len = 3 * (size_t)(sl->mmax + 8);
    auto alloc = [&](size_t n) -> double * {
        void *p = nullptr;
        if (hipMalloc(&p, std::max<size_t>(n * sizeof(double), 8)) != hipSuccess) return nullptr;
        sl->mem.push_back(p);
        return (double *)p;
    };
    sl->V = alloc((size_t)sl->mmax * dim);
    sl->W = alloc((size_t)sl->mmax * dim);
    sl->X = alloc((size_t)sl->nscr * dim);
    sl->R = alloc((size_t)sl->kk * dim);
    sl->T = alloc((size_t)sl->kk * dim);
    sl->D = alloc((size_t)dim);
    sl->small = alloc(sl->small_len);
    sl->partial = alloc((size_t)sl->nblk * sl->mmax * sl->mmax);
    sl->scal = alloc(sl->scal_len);
    if (!sl->V || !sl->W || !sl->X || !sl->R || !sl->T || !sl->D || !sl->small || !sl->partial || !sl->scal) {
        set_error("device allocation failed (Davidson subspace)");
        return ISCI_E_OOM;
    }
    if (hipHostMalloc((void **)&sl->hsmall, sizeof(double) * sl->small_len, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void **)&sl->hscal, sizeof(double) * sl->scal_len, hipHostMallocDefault) != hipSuccess) {
        set_error("pinned host allocation failed");
        return ISCI_E_OOM;
    }
    sl->G.assign((size_t)sl->mmax * sl->mmax, 0.0);
    sl->theta.assign(sl->kk, 0.0);
    sl->prev.assign(sl->kk, 1e300);
    sl->rn.assign(sl->kk, 0.0);
    isci_status st = launch_diag(sl->h, sl->D, s);
    if (st != ISCI_OK) return st;
    // initial basis: the caller's guesses, then unit vectors on the lowest
    // diagonal entries (ties to the lowest address)
    std::vector<const double *> cand;
    for (int g = 0; g < nguess; ++g) cand.push_back(guess + (size_t)g * dim);
    int take = 0;
    std::vector<int64_t> ord;
    if (nguess < sl->kk) {
        std::vector<double> hd(dim);
        ISCI_HIP(hipMemcpyAsync(hd.data(), sl->D, sizeof(double) * dim, hipMemcpyDeviceToHost, s));
        ISCI_HIP(hipStreamSynchronize(s));
        ord.resize(dim);
        std::iota(ord.begin(), ord.end(), 0);
        take = (int)std::min<int64_t>(dim, sl->kk + 64);
        std::partial_sort(ord.begin(), ord.begin() + take, ord.end(), [&](int64_t a, int64_t b) {
            return hd[a] < hd[b] || (hd[a] == hd[b] && a < b);
        });
    }
    size_t ci = 0;
    int u = 0;
    while (sl->m < sl->kk && (ci < cand.size() || u < take)) {
        const int m0 = sl->m;
        const int want = std::min(sl->kk - sl->m, sl->mmax - sl->m);
        int n = 0;
        for (; n < want && (ci < cand.size() || u < take); ++n) {
            if (ci < cand.size()) {
                st = cgs2_enqueue(sl, cand[ci++], n, s);
            } else {
                k_unit<<<grid1(dim), 256, 0, s>>>(sl->T, dim, ord[u++]);
                st = cgs2_enqueue(sl, sl->T, n, s);
            }
            if (st != ISCI_OK) return st;
        }
        ISCI_HIP(hipMemcpyAsync(sl->hscal, sl->scal, sizeof(double) * 3 * n, hipMemcpyDeviceToHost, s));
        ISCI_HIP(hipStreamSynchronize(s));
        if ((st = cgs2_finish(sl, m0, n, s)) != ISCI_OK) return st;
    }
    if (sl->m == 0) { set_error("empty initial basis"); return ISCI_E_INVALID; }
    return ISCI_OK;
}

// one fused sigma launch over n (handle, vector block) jobs; jobs are
// ordered by estimated cost (heaviest first) unless configured otherwise
static isci_status fused_sigma(isci_engine e, int n, const isci_handle *hds, const int *nvec,
                               const double *const *cv, const int64_t *ldc, double *const *sv,
                               const int64_t *lds)
{
    std::vector<SigmaArgs> args;
    std::vector<BatchVec> vecs;
    std::vector<double> cost;
    int nvmax = 1;
    for (int i = 0; i < n; ++i) {
        const isci_ctx *c = hds[i];
        const int inst = (int)args.size();
        args.push_back(sigma_args(c));
        for (int v0 = 0; v0 < nvec[i]; v0 += 8) {
            const int nv = std::min(8, nvec[i] - v0);
            nvmax = std::max(nvmax, nv);
            BatchVec bv;
            bv.inst = inst;
            bv.nv = nv;
            bv.c = cv[i] + (size_t)v0 * ldc[i];
            bv.s = sv[i] + (size_t)v0 * lds[i];
            bv.ldc = ldc[i];
            bv.lds = lds[i];
            bv.plan = c->d.plan;
            bv.nitems = c->nplan;
            bv.item0 = 0;
            vecs.push_back(bv);
            cost.push_back((double)c->stats.terms_total * (0.5 + 0.5 * nv / 8.0));
        }
    }
    if (vecs.empty()) return ISCI_OK;
    std::vector<int> ord(vecs.size());
    std::iota(ord.begin(), ord.end(), 0);
    if (e->order) std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return cost[a] > cost[b]; });
    std::vector<BatchVec> sorted;
    int64_t total = 0;
    for (int j : ord) {
        BatchVec bv = vecs[j];
        bv.item0 = (int)total;
        total += bv.nitems;
        sorted.push_back(bv);
    }
    if (total >= (int64_t)1 << 31) { set_error("fused sigma: too many work items"); return ISCI_E_UNSUPPORTED; }
    // the pinned staging of the previous launch may still be in flight
    ISCI_HIP(hipStreamSynchronize(e->s));
    if (!grow(e->d_args, e->h_args, e->cap_args, args.size()) || !grow(e->d_vecs, e->h_vecs, e->cap_vecs, sorted.size())) {
        set_error("allocation failed (fused sigma staging)");
        return ISCI_E_OOM;
    }
    std::copy(args.begin(), args.end(), e->h_args);
    std::copy(sorted.begin(), sorted.end(), e->h_vecs);
    ISCI_HIP(hipMemcpyAsync(e->d_args, e->h_args, sizeof(SigmaArgs) * args.size(), hipMemcpyHostToDevice, e->s));
    ISCI_HIP(hipMemcpyAsync(e->d_vecs, e->h_vecs, sizeof(BatchVec) * sorted.size(), hipMemcpyHostToDevice, e->s));
    return launch_sigma_batched(e->d_args, e->d_vecs, (int)sorted.size(), (int)total, nvmax, e->grid, e->s);
}

// side streams of the per-instance sigma launches
static constexpr int kSideStreams = 4;

static isci_status ensure_side_streams(isci_engine e)
{
    if (!e->side.empty()) return ISCI_OK;
    for (int i = 0; i < kSideStreams; ++i) {
        hipStream_t st;
        ISCI_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
        e->side.push_back(st);
    }
    for (int i = 0; i <= kSideStreams; ++i) {
        hipEvent_t ev;
        ISCI_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
        e->side_ev.push_back(ev);
    }
    return ISCI_OK;
}

// sigma of n (handle, vector block) jobs: handles on the matrix-core path
// run their own launches (overlapping on side streams when there are
// several; jobs sharing a handle share a stream, its product operands being
// per handle), the others share one fused launch on e->s
static isci_status batch_sigma(isci_engine e, int n, const isci_handle *hds, const int *nvec,
                               const double *const *c, const int64_t *ldc, double *const *sg, const int64_t *lds)
{
    std::vector<int> own, rest;
    for (int i = 0; i < n; ++i) (sigma_args(hds[i]).variant == 3 ? own : rest).push_back(i);
    if (own.size() > 1) {
        ISCI_CHECK(ensure_side_streams(e));
        ISCI_HIP(hipEventRecord(e->side_ev[0], e->s));
        for (hipStream_t st : e->side) ISCI_HIP(hipStreamWaitEvent(st, e->side_ev[0], 0));
        // longest work first, each job onto the side stream with the least
        // work so far (work ~ determinants x vectors); jobs of one handle
        // share its stream, its product operands being per handle
        std::vector<int> ord(own);
        std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) {
            return (double)hds[a]->dim * nvec[a] > (double)hds[b]->dim * nvec[b];
        });
        std::vector<double> load(e->side.size(), 0.0);
        std::vector<std::pair<isci_handle, size_t>> placed;
        for (int i : ord) {
            size_t k = 0;
            bool found = false;
            for (const auto &pl : placed)
                if (pl.first == hds[i]) { k = pl.second; found = true; break; }
            if (!found) {
                k = (size_t)(std::min_element(load.begin(), load.end()) - load.begin());
                placed.emplace_back(hds[i], k);
            }
            load[k] += (double)hds[i]->dim * nvec[i];
            // the handles already overlap on the side streams: each runs its
            // one-body kernels in line (same results as with its own side
            // stream, fewer cross-stream waits)
            ISCI_CHECK(launch_sigma(hds[i], nvec[i], c[i], ldc[i], sg[i], lds[i], e->side[k], false));
        }
        for (size_t k = 0; k < e->side.size(); ++k) {
            ISCI_HIP(hipEventRecord(e->side_ev[1 + k], e->side[k]));
            ISCI_HIP(hipStreamWaitEvent(e->s, e->side_ev[1 + k], 0));
        }
    } else if (own.size() == 1) {
        const int i = own[0];
        ISCI_CHECK(launch_sigma(hds[i], nvec[i], c[i], ldc[i], sg[i], lds[i], e->s));
    }
    std::vector<isci_handle> h2;
    std::vector<int> n2;
    std::vector<const double *> c2;
    std::vector<double *> s2;
    std::vector<int64_t> lc2, ls2;
    for (int i : rest) {
        h2.push_back(hds[i]);
        n2.push_back(nvec[i]);
        c2.push_back(c[i]);
        s2.push_back(sg[i]);
        lc2.push_back(ldc[i]);
        ls2.push_back(lds[i]);
    }
    return fused_sigma(e, (int)h2.size(), h2.data(), n2.data(), c2.data(), lc2.data(), s2.data(), ls2.data());
}

// ---- phase A: sigma of the new basis vectors of every active slot
static isci_status phase_sigma(isci_engine e, const std::vector<Slot *> &act)
{
    std::vector<isci_handle> hs;
    std::vector<int> nv;
    std::vector<const double *> cv;
    std::vector<double *> sv;
    std::vector<int64_t> ld;
    for (Slot *sl : act) {
        const int nnew = sl->m - sl->mdone;
        if (nnew <= 0) continue;
        sl->nsig += nnew;
        hs.push_back(sl->h);
        nv.push_back(nnew);
        cv.push_back(sl->V + (size_t)sl->mdone * sl->dim);
        sv.push_back(sl->W + (size_t)sl->mdone * sl->dim);
        ld.push_back(sl->dim);
    }
    return batch_sigma(e, (int)hs.size(), hs.data(), nv.data(), cv.data(), ld.data(), sv.data(), ld.data());
}

// ---- descriptor arena: the host packs one phase's descriptors into
// pinned memory, one copy moves them to the device, kernels read them there
struct ArenaPack {
    isci_engine e;
    size_t used = 0;
    template <typename T>
    size_t push(const std::vector<T> &v)
    {
        const size_t off = (used + 255) & ~(size_t)255;
        used = off + sizeof(T) * v.size();
        return off;
    }
};

// wait for the previous upload, then make room (called before the host
// writes a phase's descriptors)
static bool arena_reserve(isci_engine e, size_t bytes)
{
    if (e->arena_pending) {
        if (hipEventSynchronize(e->arena_ev) != hipSuccess) return false;
        e->arena_pending = false;
    }
    if (bytes <= e->arena_cap) return true;
    size_t n = std::max(bytes, 2 * e->arena_cap + 65536);
    if (e->arena_d) (void)hipFree(e->arena_d);
    if (e->arena_h) (void)hipHostFree(e->arena_h);
    e->arena_d = nullptr;
    e->arena_h = nullptr;
    e->arena_cap = 0;
    if (hipMalloc((void **)&e->arena_d, n) != hipSuccess) return false;
    if (hipHostMalloc((void **)&e->arena_h, n, hipHostMallocDefault) != hipSuccess) return false;
    e->arena_cap = n;
    return true;
}

static bool res_reserve(isci_engine e, size_t ndouble)
{
    if (ndouble <= e->res_cap) return true;
    size_t n = std::max(ndouble, 2 * e->res_cap + 4096);
    if (e->res_d) (void)hipFree(e->res_d);
    if (e->res_h) (void)hipHostFree(e->res_h);
    e->res_d = nullptr;
    e->res_h = nullptr;
    e->res_cap = 0;
    if (hipMalloc((void **)&e->res_d, sizeof(double) * n) != hipSuccess) return false;
    if (hipHostMalloc((void **)&e->res_h, sizeof(double) * n, hipHostMallocDefault) != hipSuccess) return false;
    e->res_cap = n;
    return true;
}

// copy a phase's descriptors to the device on s and mark the arena busy
static isci_status arena_upload(isci_engine e, size_t bytes, hipStream_t s)
{
    ISCI_HIP(hipMemcpyAsync(e->arena_d, e->arena_h, bytes, hipMemcpyHostToDevice, s));
    if (!e->arena_ev) ISCI_HIP(hipEventCreateWithFlags(&e->arena_ev, hipEventDisableTiming));
    ISCI_HIP(hipEventRecord(e->arena_ev, s));
    e->arena_pending = true;
    return ISCI_OK;
}

template <typename T>
static T *arena_put(isci_engine e, size_t off, const std::vector<T> &v)
{
    if (!v.empty()) memcpy(e->arena_h + off, v.data(), sizeof(T) * v.size());
    return (T *)(e->arena_d + off);
}

static isci_status launch_bdots(const BDot *d, const std::vector<BDot> &h, hipStream_t s)
{
    if (h.empty()) return ISCI_OK;
    int gx = 1, ti = 1, tj = 1, mk = 1;
    bool reduce = false;
    for (const BDot &j : h) {
        reduce = reduce || j.nblk > 1;
        gx = std::max(gx, j.nblk);
        ti = std::max(ti, (j.m + kTile - 1) / kTile);
        tj = std::max(tj, (j.k + kTile - 1) / kTile);
        mk = std::max(mk, j.m * j.k);
    }
    k_bdots<<<dim3((unsigned)(((gx + 7) / 8) * 8 * ti * tj), 1, (unsigned)h.size()), 256, 0, s>>>(d, ti, tj);
    if (reduce) k_bdots_reduce<<<dim3((mk + 3) / 4, 1, (unsigned)h.size()), 256, 0, s>>>(d);
    ISCI_HIP(hipGetLastError());
    return ISCI_OK;
}

static isci_status launch_blincomb(const BLin *d, const std::vector<BLin> &h, hipStream_t s)
{
    if (h.empty()) return ISCI_OK;
    int64_t n = 1;
    int k = 1;
    for (const BLin &j : h) { n = std::max(n, j.n); k = std::max(k, j.k); }
    k_blincomb<<<dim3((unsigned)std::min<int64_t>(2048, (n + 255) / 256), (k + kTile - 1) / kTile,
                      (unsigned)h.size()), 256, 0, s>>>(d);
    ISCI_HIP(hipGetLastError());
    return ISCI_OK;
}

template <typename J>
static int64_t max_n(const std::vector<J> &h)
{
    int64_t n = 1;
    for (const J &j : h) n = std::max(n, j.n);
    return n;
}

// Cholesky QR coefficients of a block X of p columns from its Gram matrix G
// (p x p, row major): columns are taken in order, and column i is dropped
// when its norm after removing the kept earlier columns is <= thr[i].
// C receives q x p coefficients (C[j * p + i]: weight of X_i in output j)
// with X C^T orthonormal; returns q.
static int chol_qr_coeffs(int p, const double *G, const double *thr, std::vector<double> &C)
{
    std::vector<double> R((size_t)p * p, 0.0);
    std::vector<int> kept;
    for (int i = 0; i < p; ++i) {
        double d = G[(size_t)i * p + i];
        for (int k : kept) d -= R[(size_t)k * p + i] * R[(size_t)k * p + i];
        if (!(d > thr[i] * thr[i]) || !(d > 0.0)) continue;
        const double rii = sqrt(d);
        R[(size_t)i * p + i] = rii;
        for (int jj = i + 1; jj < p; ++jj) {
            double v = G[(size_t)i * p + jj];
            for (int k : kept) v -= R[(size_t)k * p + i] * R[(size_t)k * p + jj];
            R[(size_t)i * p + jj] = v / rii;
        }
        kept.push_back(i);
    }
    const int q = (int)kept.size();
    C.assign((size_t)q * p, 0.0);
    for (int a = 0; a < q; ++a) {
        const int i = kept[a];
        double *c = &C[(size_t)a * p];
        c[i] = 1.0;
        for (int b = 0; b < a; ++b) {
            const double r = R[(size_t)kept[b] * p + i];
            const double *cb = &C[(size_t)b * p];
            for (int t = 0; t < p; ++t) c[t] -= r * cb[t];
        }
        for (int t = 0; t < p; ++t) c[t] /= R[(size_t)i * p + i];
    }
    return q;
}

// one Davidson iteration for every active slot
static isci_status engine_step(isci_engine e, int *nactive)
{
    hipStream_t s = e->s;
    std::vector<Slot *> act;
    for (Slot *sl : e->slots)
        if (sl && !sl->done) act.push_back(sl);
    if (nactive) *nactive = (int)act.size();
    if (act.empty()) return ISCI_OK;
    isci_status st = phase_sigma(e, act);
    if (st != ISCI_OK) return st;
    const int na = (int)act.size();
    // results needed this step: G columns, residual Gram matrices, CGS2 scalars
    size_t need = 0;
    for (Slot *sl : act) need += (size_t)sl->m * (sl->m - sl->mdone) + (size_t)sl->kk * sl->kk + 3 * (size_t)sl->block * sl->block;
    if (!res_reserve(e, need + 64)) { set_error("allocation failed (engine results)"); return ISCI_E_OOM; }

    // ---- phase B: new columns of G = V^T W_new, all slots in one launch pair
    std::vector<BDot> jb;
    std::vector<size_t> offB(na);
    size_t roff = 0;
    for (int j = 0; j < na; ++j) {
        Slot *sl = act[j];
        const int nnew = sl->m - sl->mdone;
        offB[j] = roff;
        BDot d;
        d.A = sl->V; d.B = sl->W + (size_t)sl->mdone * sl->dim;
        d.out = e->res_d + roff; d.partial = sl->partial;
        d.lda = sl->dim; d.ldb = sl->dim; d.n = sl->dim;
        d.m = sl->m; d.k = nnew; d.nblk = sl->nblk;
        if (nnew > 0) jb.push_back(d);
        roff += (size_t)sl->m * nnew;
    }
    {
        ArenaPack ap{e};
        const size_t o = ap.push(jb);
        if (!arena_reserve(e, ap.used + 256)) { set_error("allocation failed (arena)"); return ISCI_E_OOM; }
        BDot *dd = arena_put(e, o, jb);
        ISCI_CHECK(arena_upload(e, ap.used, s));
        if ((st = launch_bdots(dd, jb, s)) != ISCI_OK) return st;
        ISCI_HIP(hipMemcpyAsync(e->res_h, e->res_d, sizeof(double) * std::max<size_t>(roff, 1), hipMemcpyDeviceToHost, s));
        ISCI_HIP(hipStreamSynchronize(s));
    }
    // ---- host: projected eigenproblems; phase C: Ritz vectors, residuals,
    // corrections and residual norms for all slots
    std::vector<double> params;
    std::vector<size_t> offY(na), offR(na);
    size_t rC = roff;
    // each slot's projected matrix and its eigendecomposition depend on that
    // slot alone: with many slots they are spread over host threads
    auto project = [&](int j) {
        Slot *sl = act[j];
        const int m = sl->m, mdone = sl->mdone, nnew = m - mdone, mmax = sl->mmax;
        const double *col = e->res_h + offB[j];
        for (int i = 0; i < m; ++i)
            for (int q = 0; q < nnew; ++q) {
                const double v = col[(size_t)i * nnew + q];
                sl->G[(size_t)i * mmax + mdone + q] = v;
                if (i < mdone) sl->G[(size_t)(mdone + q) * mmax + i] = v;
            }
        for (int i = mdone; i < m; ++i)
            for (int q = mdone; q < i; ++q) {
                const double a2 = 0.5 * (sl->G[(size_t)i * mmax + q] + sl->G[(size_t)q * mmax + i]);
                sl->G[(size_t)i * mmax + q] = a2;
                sl->G[(size_t)q * mmax + i] = a2;
            }
        sl->mdone = m;
        std::vector<double> Gm((size_t)m * m);
        for (int i = 0; i < m; ++i)
            for (int q = 0; q < m; ++q) Gm[(size_t)i * m + q] = sl->G[(size_t)i * mmax + q];
        if (!tridiag_eigh(m, Gm, sl->evals, sl->Z)) jacobi_eigh(m, Gm, sl->evals, sl->Z);
    };
    if (na >= 8) {
        if (!e->pool) {
            const int hw = (int)std::max(2u, std::thread::hardware_concurrency());
            e->pool = new HostPool(std::min(15, hw - 1));
        }
        e->pool->run(na, project);
    } else {
        for (int j = 0; j < na; ++j) project(j);
    }
    for (int j = 0; j < na; ++j) {
        Slot *sl = act[j];
        const int m = sl->m;
        const int kr = std::min(sl->kk, m);
        sl->kr = kr;
        offY[j] = params.size();
        for (int q = 0; q < kr; ++q)
            for (int i = 0; i < m; ++i) params.push_back(sl->Z[(size_t)i * m + q]);
        for (int q = 0; q < kr; ++q) params.push_back(sl->theta[q] = sl->evals[q]);
        offR[j] = rC;
        rC += (size_t)kr * kr;
    }
    {
        ArenaPack ap{e};
        std::vector<BLin> jl(2 * na);
        std::vector<BRes> jr(na);
        std::vector<BDot> jd(na);
        const size_t op = ap.push(params);
        const size_t ol = ap.push(jl), orr = ap.push(jr), od = ap.push(jd);
        if (!arena_reserve(e, ap.used + 256)) { set_error("allocation failed (arena)"); return ISCI_E_OOM; }
        jl.clear();
        jr.clear();
        jd.clear();
        // the parameters' device addresses are fixed now that the arena is
        const double *pd = (const double *)(e->arena_d + op);
        for (int j = 0; j < na; ++j) {
            Slot *sl = act[j];
            const int m = sl->m, kr = sl->kr;
            const double *Y = pd + offY[j], *th = Y + (size_t)kr * m;
            jl.push_back(BLin{sl->V, Y, sl->X, sl->dim, sl->dim, sl->dim, m, kr, 0.0, 1.0});
            jl.push_back(BLin{sl->W, Y, sl->R, sl->dim, sl->dim, sl->dim, m, kr, 0.0, 1.0});
            jr.push_back(BRes{sl->R, sl->T, sl->X, sl->D, th, sl->dim, sl->dim, kr});
            BDot d;
            d.A = sl->R; d.B = sl->R; d.out = e->res_d + offR[j]; d.partial = sl->partial;
            d.lda = sl->dim; d.ldb = sl->dim; d.n = sl->dim; d.m = kr; d.k = kr; d.nblk = sl->nblk;
            jd.push_back(d);
        }
        arena_put(e, op, params);
        BLin *dl = arena_put(e, ol, jl);
        BRes *dr = arena_put(e, orr, jr);
        BDot *dd = arena_put(e, od, jd);
        ISCI_CHECK(arena_upload(e, ap.used, s));
        if ((st = launch_blincomb(dl, jl, s)) != ISCI_OK) return st;
        k_bresid<<<dim3((unsigned)std::min<int64_t>(4096, (max_n(jr) + 255) / 256), 1, (unsigned)jr.size()), 256, 0, s>>>(dr);
        ISCI_HIP(hipGetLastError());
        if ((st = launch_bdots(dd, jd, s)) != ISCI_OK) return st;
        ISCI_HIP(hipMemcpyAsync(e->res_h + roff, e->res_d + roff, sizeof(double) * std::max<size_t>(rC - roff, 1),
                                hipMemcpyDeviceToHost, s));
        ISCI_HIP(hipStreamSynchronize(s));
    }
    // ---- host: convergence, corrections, thick restarts
    std::vector<Slot *> grow_set;
    // thick restarts of this step: their linear combinations run in the
    // next launch group, batched over the slots, with no host wait
    struct Restart { Slot *sl; int keep, m, kr; size_t off; };
    std::vector<Restart> rst;
    std::vector<double> rpar;
    for (int j = 0; j < na; ++j) {
        Slot *sl = act[j];
        const int m = sl->m, kr = sl->kr, k = sl->k;
        const double *rr = e->res_h + offR[j];
        sl->iter += 1;
        bool conv = kr >= k;
        for (int q = 0; q < kr; ++q) {
            sl->rn[q] = sqrt(std::max(0.0, rr[(size_t)q * kr + q]));
            if (q < k) conv = conv && sl->rn[q] <= sl->o.tol_residual && fabs(sl->theta[q] - sl->prev[q]) <= sl->o.tol_energy;
        }
        for (int q = 0; q < kr; ++q) sl->prev[q] = sl->theta[q];
        sl->conv = conv;
        if (conv || sl->iter >= sl->o.max_iter) {
            sl->done = true;
            sl->status = conv ? ISCI_OK : ISCI_E_NOT_CONVERGED;
            continue;
        }
        sl->pick.clear();
        for (int q = 0; q < kr && (int)sl->pick.size() < sl->block; ++q)
            if (sl->rn[q] > sl->o.tol_residual) sl->pick.push_back(q);
        if (sl->pick.empty())
            for (int q = 0; q < kr && (int)sl->pick.size() < sl->block; ++q) sl->pick.push_back(q);
        if (m + (int)sl->pick.size() > sl->mmax) {
            // thick restart (per slot): keep the lowest `keep` Ritz vectors;
            // V and W become V Z_keep and W Z_keep (launched below)
            const int keep = std::min(m, sl->keep_max);
            rst.push_back(Restart{sl, keep, m, kr, rpar.size()});
            for (int q = 0; q < keep; ++q)
                for (int i = 0; i < m; ++i) rpar.push_back(sl->Z[(size_t)i * m + q]);
            sl->m = keep;
            sl->mdone = keep;
            std::fill(sl->G.begin(), sl->G.end(), 0.0);
            for (int q = 0; q < keep; ++q) sl->G[(size_t)q * sl->mmax + q] = sl->evals[q];
        }
        grow_set.push_back(sl);
    }
    // ---- phase D: the picked corrections of every slot are appended as a
    // block: classical Gram-Schmidt against the basis applied twice (CGS2),
    // then Cholesky QR applied twice inside the block.  A correction whose
    // norm after the projections falls to 1e-10 of its norm before is in
    // the span and dropped.  Every launch serves all slots.
    if (grow_set.empty()) return ISCI_OK;
    const size_t ng = grow_set.size();
    std::vector<int> m0(ng), np(ng);
    std::vector<size_t> offG0(ng), offG1(ng), offG2(ng), offGm(ng), offF(ng);
    size_t rs = rC;
    for (size_t j = 0; j < ng; ++j) {
        Slot *sl = grow_set[j];
        m0[j] = sl->m;
        np[j] = std::max(0, std::min((int)sl->pick.size(), sl->mmax - sl->m));
        const size_t p2 = (size_t)np[j] * np[j];
        offG0[j] = rs; rs += p2;
        offG1[j] = rs; rs += p2;
        offG2[j] = rs; rs += p2;
        offGm[j] = rs; rs += p2;
        offF[j] = rs; rs += 1;
    }
    if (!res_reserve(e, rs + 64)) { set_error("allocation failed (engine results)"); return ISCI_E_OOM; }
    // D1: copy, pre-norm Gram, first projection, its Gram and the DGKS
    // flag, second projection (skipped on the device when the flag says
    // so), Gram of the projected block
    {
        std::vector<BVecOp> cp;
        std::vector<BDot> g0, c1, c2, g1, gm;
        std::vector<BLin> l1, l2;
        std::vector<BFlag> fl;
        for (size_t j = 0; j < ng; ++j) {
            Slot *sl = grow_set[j];
            const int p = np[j], m = m0[j];
            if (p == 0) continue;
            double *X = sl->V + (size_t)m * sl->dim;
            for (int i = 0; i < p; ++i)
                cp.push_back(BVecOp{sl->T + (size_t)sl->pick[i] * sl->dim, X + (size_t)i * sl->dim, nullptr, nullptr,
                                    nullptr, sl->dim});
            BDot d;
            d.partial = sl->partial; d.lda = sl->dim; d.ldb = sl->dim; d.n = sl->dim; d.nblk = sl->nblk;
            d.A = X; d.B = X; d.m = p; d.k = p;
            d.out = e->res_d + offG0[j];
            g0.push_back(d);
            d.out = e->res_d + offG1[j];
            g1.push_back(d);
            if (m > 0) {
                const double *flag = e->res_d + offF[j];
                d.out = e->res_d + offGm[j];
                gm.push_back(d);
                fl.push_back(BFlag{e->res_d + offG0[j], e->res_d + offGm[j], e->res_d + offF[j], p});
                d.A = X; d.B = sl->V; d.m = p; d.k = m; d.out = sl->small;   // Y[q * m + i] = X_q . V_i
                c1.push_back(d);
                d.skip = flag;
                c2.push_back(d);
                l1.push_back(BLin{sl->V, sl->small, X, sl->dim, sl->dim, sl->dim, m, p, 1.0, -1.0});
                l2.push_back(BLin{sl->V, sl->small, X, sl->dim, sl->dim, sl->dim, m, p, 1.0, -1.0, flag});
            }
        }
        // restarts: X = V Z_keep, V = X; X = W Z_keep, W = X; X = V[0, kr)
        // (the Ritz vectors, kept in X for the results)
        std::vector<BLin> rv(rst.size()), rw(rst.size());
        std::vector<BVecOp> rcv, rcw, rcx;
        ArenaPack ap{e};
        const size_t orp = ap.push(rpar), orv = ap.push(rv), orw = ap.push(rw);
        for (size_t r = 0; r < rst.size(); ++r) {
            Slot *sl = rst[r].sl;
            const int64_t dim = sl->dim;
            rcv.push_back(BVecOp{sl->X, sl->V, nullptr, nullptr, nullptr, (int64_t)rst[r].keep * dim});
            rcw.push_back(BVecOp{sl->X, sl->W, nullptr, nullptr, nullptr, (int64_t)rst[r].keep * dim});
            rcx.push_back(BVecOp{sl->V, sl->X, nullptr, nullptr, nullptr, (int64_t)rst[r].kr * dim});
        }
        const size_t orcv = ap.push(rcv), orcw = ap.push(rcw), orcx = ap.push(rcx);
        const size_t ocp = ap.push(cp), og0 = ap.push(g0), oc1 = ap.push(c1), oc2 = ap.push(c2), og1 = ap.push(g1),
                     ol1 = ap.push(l1), ol2 = ap.push(l2), ogm = ap.push(gm), ofl = ap.push(fl);
        if (!arena_reserve(e, ap.used + 256)) { set_error("allocation failed (arena)"); return ISCI_E_OOM; }
        {
            const double *pd = (const double *)(e->arena_d + orp);
            for (size_t r = 0; r < rst.size(); ++r) {
                Slot *sl = rst[r].sl;
                const Restart &q = rst[r];
                rv[r] = BLin{sl->V, pd + q.off, sl->X, sl->dim, sl->dim, sl->dim, q.m, q.keep, 0.0, 1.0};
                rw[r] = BLin{sl->W, pd + q.off, sl->X, sl->dim, sl->dim, sl->dim, q.m, q.keep, 0.0, 1.0};
            }
        }
        arena_put(e, orp, rpar);
        BLin *drv = arena_put(e, orv, rv), *drw = arena_put(e, orw, rw);
        BVecOp *drcv = arena_put(e, orcv, rcv), *drcw = arena_put(e, orcw, rcw), *drcx = arena_put(e, orcx, rcx);
        BVecOp *dcp = arena_put(e, ocp, cp);
        BDot *dg0 = arena_put(e, og0, g0), *dc1 = arena_put(e, oc1, c1), *dc2 = arena_put(e, oc2, c2),
             *dg1 = arena_put(e, og1, g1), *dgm = arena_put(e, ogm, gm);
        BLin *dl1 = arena_put(e, ol1, l1), *dl2 = arena_put(e, ol2, l2);
        BFlag *dfl = arena_put(e, ofl, fl);
        ISCI_CHECK(arena_upload(e, ap.used, s));
        if (!rst.empty()) {
            if ((st = launch_blincomb(drv, rv, s)) != ISCI_OK) return st;
            k_bcopy<<<dim3(grid1(max_n(rcv)), 1, (unsigned)rcv.size()), 256, 0, s>>>(drcv);
            if ((st = launch_blincomb(drw, rw, s)) != ISCI_OK) return st;
            k_bcopy<<<dim3(grid1(max_n(rcw)), 1, (unsigned)rcw.size()), 256, 0, s>>>(drcw);
            k_bcopy<<<dim3(grid1(max_n(rcx)), 1, (unsigned)rcx.size()), 256, 0, s>>>(drcx);
            ISCI_HIP(hipGetLastError());
        }
        if (!cp.empty()) {
            const unsigned gx = (unsigned)std::min<int64_t>(4096, (max_n(cp) + 255) / 256);
            k_bcopy<<<dim3(gx, 1, (unsigned)cp.size()), 256, 0, s>>>(dcp);
            ISCI_HIP(hipGetLastError());
        }
        if ((st = launch_bdots(dg0, g0, s)) != ISCI_OK) return st;
        if ((st = launch_bdots(dc1, c1, s)) != ISCI_OK) return st;
        if ((st = launch_blincomb(dl1, l1, s)) != ISCI_OK) return st;
        if ((st = launch_bdots(dgm, gm, s)) != ISCI_OK) return st;
        if (!fl.empty()) {
            k_dgks_flag<<<(unsigned)((fl.size() + 63) / 64), 64, 0, s>>>(dfl, (int)fl.size());
            ISCI_HIP(hipGetLastError());
        }
        if ((st = launch_bdots(dc2, c2, s)) != ISCI_OK) return st;
        if ((st = launch_blincomb(dl2, l2, s)) != ISCI_OK) return st;
        if ((st = launch_bdots(dg1, g1, s)) != ISCI_OK) return st;
        ISCI_HIP(hipMemcpyAsync(e->res_h + rC, e->res_d + rC, sizeof(double) * std::max<size_t>(rs - rC, 1),
                                hipMemcpyDeviceToHost, s));
        ISCI_HIP(hipStreamSynchronize(s));
    }
    // D2 / D3: Cholesky QR of the projected block (columns in the span
    // dropped), then once more on the result
    std::vector<int> nq(ng, 0);
    for (int pass = 0; pass < 2; ++pass) {
        std::vector<double> params;
        std::vector<size_t> offC(ng);
        std::vector<int> nout(ng, 0);
        for (size_t j = 0; j < ng; ++j) {
            const int p = pass == 0 ? np[j] : nq[j];
            if (p == 0) continue;
            const double *Gp = e->res_h + (pass == 0 ? offG1[j] : offG2[j]);
            std::vector<double> thr(p);
            for (int i = 0; i < p; ++i)
                thr[i] = pass == 0 ? 1e-10 * sqrt(std::max(0.0, e->res_h[offG0[j] + (size_t)i * p + i])) : 1e-8;
            std::vector<double> C;
            nout[j] = chol_qr_coeffs(p, Gp, thr.data(), C);
            offC[j] = params.size();
            params.insert(params.end(), C.begin(), C.end());
        }
        std::vector<BLin> lq;
        std::vector<BDot> g2;
        ArenaPack ap{e};
        const size_t opar = ap.push(params);
        std::vector<BLin> lq_sz(ng);
        std::vector<BDot> g2_sz(ng);
        const size_t olq = ap.push(lq_sz), og2 = ap.push(g2_sz);
        if (!arena_reserve(e, ap.used + 256)) { set_error("allocation failed (arena)"); return ISCI_E_OOM; }
        const double *pd = (const double *)(e->arena_d + opar);
        for (size_t j = 0; j < ng; ++j) {
            Slot *sl = grow_set[j];
            const int p = pass == 0 ? np[j] : nq[j], q = nout[j];
            if (p == 0 || q == 0) continue;
            double *X = sl->V + (size_t)m0[j] * sl->dim;
            // pass 0: X (p columns) -> T (q columns); pass 1: T -> X
            const double *src = pass == 0 ? X : sl->T;
            double *dst = pass == 0 ? sl->T : X;
            lq.push_back(BLin{src, pd + offC[j], dst, sl->dim, sl->dim, sl->dim, p, q, 0.0, 1.0});
            if (pass == 0) {
                BDot d;
                d.partial = sl->partial; d.lda = sl->dim; d.ldb = sl->dim; d.n = sl->dim; d.nblk = sl->nblk;
                d.A = sl->T; d.B = sl->T; d.m = q; d.k = q; d.out = e->res_d + offG2[j];
                g2.push_back(d);
            }
        }
        arena_put(e, opar, params);
        BLin *dlq = arena_put(e, olq, lq);
        BDot *dg2 = arena_put(e, og2, g2);
        ISCI_CHECK(arena_upload(e, ap.used, s));
        if ((st = launch_blincomb(dlq, lq, s)) != ISCI_OK) return st;
        if (pass == 0) {
            if ((st = launch_bdots(dg2, g2, s)) != ISCI_OK) return st;
            ISCI_HIP(hipMemcpyAsync(e->res_h + rC, e->res_d + rC, sizeof(double) * std::max<size_t>(rs - rC, 1),
                                    hipMemcpyDeviceToHost, s));
            ISCI_HIP(hipStreamSynchronize(s));
        }
        for (size_t j = 0; j < ng; ++j) nq[j] = nout[j];
    }
    for (size_t j = 0; j < ng; ++j) {
        Slot *sl = grow_set[j];
        sl->m = m0[j] + nq[j];
        if (nq[j] == 0) {   // stagnation: no new direction
            sl->done = true;
            sl->status = sl->conv ? ISCI_OK : ISCI_E_NOT_CONVERGED;
        }
    }
    return ISCI_OK;
}

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

static isci_davidson_opts normalized_opts(const isci_davidson_opts *opts)
{
    isci_davidson_opts o;
    isci_davidson_defaults(&o);
    if (opts) o = *opts;
    if (!(o.tol_residual > 0)) o.tol_residual = 1e-7;
    if (!(o.tol_energy > 0)) o.tol_energy = 1e-11;
    if (o.max_iter <= 0) o.max_iter = 200;
    return o;
}

int64_t isci_davidson_footprint(isci_handle h, int nroots, const isci_davidson_opts *opts)
{
    if (!h || nroots < 1 || nroots > h->dim) return -1;
    isci_davidson_opts o = normalized_opts(opts);
    return slot_bytes(h->dim, nroots, o, nullptr, nullptr, nullptr);
}

isci_status isci_engine_create(isci_engine *out, hipStream_t stream)
{
    if (!out) { set_error("out is NULL"); return ISCI_E_INVALID; }
    isci_engine e = new (std::nothrow) isci_engine_s();
    if (!e) { set_error("host allocation failed"); return ISCI_E_OOM; }
    e->s = stream;
    *out = e;
    return ISCI_OK;
}

isci_status isci_engine_config(isci_engine e, int grid, int heaviest_first)
{
    if (!e || grid < 0) { set_error("bad engine config"); return ISCI_E_INVALID; }
    e->grid = grid;
    e->order = heaviest_first ? 1 : 0;
    return ISCI_OK;
}

isci_status isci_engine_add(isci_engine e, isci_handle h, int nroots, const isci_davidson_opts *opts,
                            const double *guess, int nguess, int *slot)
{
    if (!e || !h || !slot) { set_error("NULL argument"); return ISCI_E_INVALID; }
    if (nroots < 1 || nroots > ISCI_MAX_ROOTS || nroots > h->dim) { set_error("bad nroots"); return ISCI_E_INVALID; }
    if (nguess < 0 || (nguess > 0 && !guess)) { set_error("bad guess"); return ISCI_E_INVALID; }
    Slot *sl = new (std::nothrow) Slot();
    if (!sl) { set_error("host allocation failed"); return ISCI_E_OOM; }
    sl->h = h;
    sl->k = nroots;
    sl->dim = h->dim;
    sl->o = normalized_opts(opts);
    isci_status st = slot_init(e, sl, guess, nguess);
    if (st != ISCI_OK) { (void)hipStreamSynchronize(e->s); slot_free(sl); return st; }
    int id = -1;
    for (size_t i = 0; i < e->slots.size(); ++i)
        if (!e->slots[i]) { id = (int)i; break; }
    if (id < 0) { id = (int)e->slots.size(); e->slots.push_back(nullptr); }
    e->slots[id] = sl;
    *slot = id;
    return ISCI_OK;
}

isci_status isci_engine_step(isci_engine e, int *nactive)
{
    if (!e) { set_error("NULL engine"); return ISCI_E_INVALID; }
    return engine_step(e, nactive);
}

isci_status isci_engine_result(isci_engine e, int slot, int *done, double *energies, double *vectors,
                               isci_davidson_info *info)
{
    if (!e || slot < 0 || slot >= (int)e->slots.size() || !e->slots[slot]) { set_error("bad slot"); return ISCI_E_INVALID; }
    Slot *sl = e->slots[slot];
    if (done) *done = sl->done ? 1 : 0;
    if (energies)
        for (int j = 0; j < sl->k; ++j) energies[j] = sl->theta[j];
    if (vectors && sl->done) {
        ISCI_HIP(hipMemcpyAsync(vectors, sl->X, sizeof(double) * (size_t)sl->k * sl->dim, hipMemcpyDeviceToDevice, e->s));
        ISCI_HIP(hipStreamSynchronize(e->s));
    }
    if (info) {
        info->iterations = sl->iter;
        info->converged = sl->conv ? 1 : 0;
        info->sigma_calls = sl->nsig;
        for (int j = 0; j < ISCI_MAX_ROOTS; ++j) info->residual[j] = j < sl->k ? sl->rn[j] : 0.0;
    }
    return sl->done ? sl->status : ISCI_OK;
}

isci_status isci_engine_release(isci_engine e, int slot)
{
    if (!e || slot < 0 || slot >= (int)e->slots.size() || !e->slots[slot]) { set_error("bad slot"); return ISCI_E_INVALID; }
    (void)hipStreamSynchronize(e->s);
    slot_free(e->slots[slot]);
    e->slots[slot] = nullptr;
    return ISCI_OK;
}

isci_status isci_engine_sigma(isci_engine e, int n, const isci_handle *hds, const int *nvec,
                              const double *const *c, const int64_t *ldc, double *const *sigma,
                              const int64_t *lds)
{
    if (!e || n < 0 || (n > 0 && (!hds || !nvec || !c || !ldc || !sigma || !lds))) {
        set_error("NULL argument");
        return ISCI_E_INVALID;
    }
    for (int i = 0; i < n; ++i)
        if (!hds[i] || nvec[i] < 1 || !c[i] || !sigma[i] || ldc[i] < hds[i]->dim || lds[i] < hds[i]->dim) {
            set_error("bad batch entry");
            return ISCI_E_INVALID;
        }
    return batch_sigma(e, n, hds, nvec, c, ldc, sigma, lds);
}

void isci_engine_destroy(isci_engine e)
{
    if (!e) return;
    (void)hipStreamSynchronize(e->s);
    delete e->pool;
    for (Slot *sl : e->slots) slot_free(sl);
    if (e->d_args) (void)hipFree(e->d_args);
    if (e->h_args) (void)hipHostFree(e->h_args);
    if (e->d_vecs) (void)hipFree(e->d_vecs);
    if (e->h_vecs) (void)hipHostFree(e->h_vecs);
    if (e->arena_d) (void)hipFree(e->arena_d);
    if (e->arena_ev) (void)hipEventDestroy(e->arena_ev);
    if (e->arena_h) (void)hipHostFree(e->arena_h);
    if (e->res_d) (void)hipFree(e->res_d);
    if (e->res_h) (void)hipHostFree(e->res_h);
    for (hipStream_t st : e->side) {
        (void)hipStreamSynchronize(st);
        (void)hipStreamDestroy(st);
    }
    for (hipEvent_t ev : e->side_ev) (void)hipEventDestroy(ev);
    delete e;
}

isci_status isci_davidson(isci_handle c, int nroots, const isci_davidson_opts *opts, const double *guess,
                          int nguess, double *energies, double *vectors, isci_davidson_info *info,
                          hipStream_t s)
{
    if (!c || !energies) { set_error("NULL argument"); return ISCI_E_INVALID; }
    isci_engine e = nullptr;
    isci_status st = isci_engine_create(&e, s);
    if (st != ISCI_OK) return st;
    int slot = -1;
    st = isci_engine_add(e, c, nroots, opts, guess, nguess, &slot);
    if (st != ISCI_OK) { isci_engine_destroy(e); return st; }
    int nact = 1;
    while (nact > 0) {
        st = isci_engine_step(e, &nact);
        if (st != ISCI_OK) { isci_engine_destroy(e); return st; }
        int done = 0;
        isci_engine_result(e, slot, &done, nullptr, nullptr, nullptr);
        if (done) break;
    }
    st = isci_engine_result(e, slot, nullptr, energies, vectors, info);
    isci_engine_destroy(e);
    return st;
}

}  // extern "C"
