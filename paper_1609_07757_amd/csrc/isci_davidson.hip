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

// After the enqueued appends of this round (count n, first at basis index
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

// ---- phase A: one fused sigma launch over the new basis vectors of every active slot
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
        hs.push_back(sl->h);
        nv.push_back(nnew);
        cv.push_back(sl->V + (size_t)sl->mdone * sl->dim);
        sv.push_back(sl->W + (size_t)sl->mdone * sl->dim);
        ld.push_back(sl->dim);
        sl->nsig += nnew;
    }
    return fused_sigma(e, (int)hs.size(), hs.data(), nv.data(), cv.data(), ld.data(), sv.data(), ld.data());
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
    // ---- phase B: new columns of G = V^T W_new
    for (Slot *sl : act) {
        const int nnew = sl->m - sl->mdone;
        st = dots(sl->V, sl->dim, sl->m, sl->W + (size_t)sl->mdone * sl->dim, sl->dim, nnew, sl->dim, sl->small,
                  sl->partial, sl->nblk, s);
        if (st != ISCI_OK) return st;
        ISCI_HIP(hipMemcpyAsync(sl->hsmall, sl->small, sizeof(double) * sl->m * nnew, hipMemcpyDeviceToHost, s));
    }
    ISCI_HIP(hipStreamSynchronize(s));
    // ---- phase C (host): projected eigenproblem; then Ritz vectors,
    // residuals and preconditioned corrections on the device
    for (Slot *sl : act) {
        const int m = sl->m, mdone = sl->mdone, nnew = m - mdone, mmax = sl->mmax;
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < nnew; ++j) {
                const double v = sl->hsmall[(size_t)i * nnew + j];
                sl->G[(size_t)i * mmax + mdone + j] = v;
                if (i < mdone) sl->G[(size_t)(mdone + j) * mmax + i] = v;
            }
        for (int i = mdone; i < m; ++i)
            for (int j = mdone; j < i; ++j) {
                const double a = 0.5 * (sl->G[(size_t)i * mmax + j] + sl->G[(size_t)j * mmax + i]);
                sl->G[(size_t)i * mmax + j] = a;
                sl->G[(size_t)j * mmax + i] = a;
            }
        sl->mdone = m;
        std::vector<double> Gm((size_t)m * m);
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < m; ++j) Gm[(size_t)i * m + j] = sl->G[(size_t)i * mmax + j];
        jacobi_eigh(m, Gm, sl->evals, sl->Z);
        const int kr = std::min(sl->kk, m);
        sl->kr = kr;
        double *hY = sl->hsmall;                       // [kr][m], then theta[kr]
        for (int j = 0; j < kr; ++j)
            for (int i = 0; i < m; ++i) hY[(size_t)j * m + i] = sl->Z[(size_t)i * m + j];
        for (int j = 0; j < kr; ++j) sl->theta[j] = hY[(size_t)kr * m + j] = sl->evals[j];
        double *dY = sl->small, *dth = sl->small + (size_t)kr * m, *dn = dth + kr;
        ISCI_HIP(hipMemcpyAsync(dY, hY, sizeof(double) * ((size_t)kr * m + kr), hipMemcpyHostToDevice, s));
        if ((st = lincomb(sl->V, sl->dim, m, dY, kr, sl->X, sl->dim, sl->dim, 0.0, s)) != ISCI_OK) return st;
        if ((st = lincomb(sl->W, sl->dim, m, dY, kr, sl->R, sl->dim, sl->dim, 0.0, s)) != ISCI_OK) return st;
        k_resid_precond<<<grid1(sl->dim), 256, 0, s>>>(sl->R, sl->X, sl->D, dth, kr, sl->dim, sl->dim, sl->T);
        ISCI_HIP(hipGetLastError());
        if ((st = dots(sl->R, sl->dim, kr, sl->R, sl->dim, kr, sl->dim, dn, sl->partial, sl->nblk, s)) != ISCI_OK)
            return st;
        ISCI_HIP(hipMemcpyAsync(sl->hsmall + (size_t)kr * m + kr, dn, sizeof(double) * kr * kr,
                                hipMemcpyDeviceToHost, s));
    }
    ISCI_HIP(hipStreamSynchronize(s));
    // ---- phase D (host): convergence, corrections, thick restart, CGS2
    for (Slot *sl : act) {
        const int m = sl->m, kr = sl->kr, k = sl->k;
        const double *rr = sl->hsmall + (size_t)kr * m + kr;
        sl->iter += 1;
        bool conv = kr >= k;
        for (int j = 0; j < kr; ++j) {
            sl->rn[j] = sqrt(std::max(0.0, rr[(size_t)j * kr + j]));
            if (j < k) conv = conv && sl->rn[j] <= sl->o.tol_residual && fabs(sl->theta[j] - sl->prev[j]) <= sl->o.tol_energy;
        }
        for (int j = 0; j < kr; ++j) sl->prev[j] = sl->theta[j];
        sl->conv = conv;
        if (conv || sl->iter >= sl->o.max_iter) {
            sl->done = true;
            sl->status = conv ? ISCI_OK : ISCI_E_NOT_CONVERGED;
            continue;
        }
        sl->pick.clear();
        for (int j = 0; j < kr && (int)sl->pick.size() < sl->block; ++j)
            if (sl->rn[j] > sl->o.tol_residual) sl->pick.push_back(j);
        if (sl->pick.empty())
            for (int j = 0; j < kr && (int)sl->pick.size() < sl->block; ++j) sl->pick.push_back(j);
        if (m + (int)sl->pick.size() > sl->mmax) {
            // thick restart: keep the lowest `keep` Ritz vectors
            const int keep = std::min(m, sl->keep_max);
            double *hYk = sl->hsmall;
            for (int j = 0; j < keep; ++j)
                for (int i = 0; i < m; ++i) hYk[(size_t)j * m + i] = sl->Z[(size_t)i * m + j];
            double *dYk = sl->small;
            ISCI_HIP(hipMemcpyAsync(dYk, hYk, sizeof(double) * (size_t)keep * m, hipMemcpyHostToDevice, s));
            if ((st = lincomb(sl->V, sl->dim, m, dYk, keep, sl->X, sl->dim, sl->dim, 0.0, s)) != ISCI_OK) return st;
            ISCI_HIP(hipMemcpyAsync(sl->V, sl->X, sizeof(double) * (size_t)keep * sl->dim, hipMemcpyDeviceToDevice, s));
            if ((st = lincomb(sl->W, sl->dim, m, dYk, keep, sl->X, sl->dim, sl->dim, 0.0, s)) != ISCI_OK) return st;
            ISCI_HIP(hipMemcpyAsync(sl->W, sl->X, sizeof(double) * (size_t)keep * sl->dim, hipMemcpyDeviceToDevice, s));
            ISCI_HIP(hipMemcpyAsync(sl->X, sl->V, sizeof(double) * (size_t)kr * sl->dim, hipMemcpyDeviceToDevice, s));
            // the host copy of hYk must stay valid until the copy above ran
            ISCI_HIP(hipStreamSynchronize(s));
            sl->m = keep;
            sl->mdone = keep;
            std::fill(sl->G.begin(), sl->G.end(), 0.0);
            for (int j = 0; j < keep; ++j) sl->G[(size_t)j * sl->mmax + j] = sl->evals[j];
        }
        const int m0 = sl->m;
        int n = 0;
        for (int j : sl->pick) {
            if (sl->m >= sl->mmax) break;
            if ((st = cgs2_enqueue(sl, sl->T + (size_t)j * sl->dim, n, s)) != ISCI_OK) return st;
            ++n;
        }
        sl->pick.assign(1, m0);          // remember where this round's appends start
        sl->pick.push_back(n);
        ISCI_HIP(hipMemcpyAsync(sl->hscal, sl->scal, sizeof(double) * 3 * std::max(n, 1), hipMemcpyDeviceToHost, s));
    }
    ISCI_HIP(hipStreamSynchronize(s));
    for (Slot *sl : act) {
        if (sl->done) continue;
        const int m0 = sl->pick[0], n = sl->pick[1];
        if ((st = cgs2_finish(sl, m0, n, s)) != ISCI_OK) return st;
        if (sl->m == m0) {   // stagnation: no new direction
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
    return fused_sigma(e, n, hds, nvec, c, ldc, sigma, lds);
}

void isci_engine_destroy(isci_engine e)
{
    if (!e) return;
    (void)hipStreamSynchronize(e->s);
    for (Slot *sl : e->slots) slot_free(sl);
    if (e->d_args) (void)hipFree(e->d_args);
    if (e->h_args) (void)hipHostFree(e->h_args);
    if (e->d_vecs) (void)hipFree(e->d_vecs);
    if (e->h_vecs) (void)hipHostFree(e->h_vecs);
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
