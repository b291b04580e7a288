// Internal definitions of libisci (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/isci.h"

#define ISCI_MAXN 4          // electrons per spin handled by the kernels
#define ISCI_MAXNORB 255     // orbitals fit in one byte
#define ISCI_MAXLEV 8        // level tables sized for 2 * ISCI_MAXN
#define ISCI_NKERNEL_IDS 8   // ISCI_KERNEL_* ids of the timing hook

namespace isci {

// Binomial table C(x, k) for x < 256, k <= ISCI_MAXN (+1 for counting).
constexpr int kBinomK = ISCI_MAXN + 1;

// Strings of one spin, sorted by (level, colex).  The level is the number
// of electrons in orbitals >= nocc (nocc = n: the excitation level; a GAS
// boundary b: the outer-space electrons).  Within level k the index is
// lev_off[k] + colexrank(outer orbitals - nocc) * C(nocc, n - k)
// + colexrank(inner orbitals), colexrank({e_1 < ... < e_m}) = sum C(e_i, i).
struct SpinTab {
    int n;                       // electrons of this spin
    int nocc;                    // level boundary: orbitals below it are inner (= n, or the GAS boundary)
    int nvirt;                   // norb - nocc
    int maxlev;                  // highest level present (<= L)
    int nstr;                    // number of strings with level <= maxlev
    int lev_off[ISCI_MAXLEV + 2];
    int occ_mult[ISCI_MAXN + 1]; // C(nocc, n - k)
    int le[ISCI_MAXLEV + 2];     // number of strings with level <= l (l = 0..L)
};

// alpha-beta product tiles: 64-column groups per tile (one per wave) and
// parts of the chunk list per tile (waves per tile = kAbCW * kAbSplit)
// (build-time tuning knobs ISCI_AB_CW / ISCI_AB_SPLIT; defaults measured best)
#ifndef ISCI_AB_CW
#define ISCI_AB_CW 2
#endif
#ifndef ISCI_AB_SPLIT
#define ISCI_AB_SPLIT 2
#endif
constexpr int kAbCW = ISCI_AB_CW;
constexpr int kAbSplit = ISCI_AB_SPLIT;
constexpr int kAbTile = 64 * kAbCW;   // columns per tile
// columns of T whose tiles run together on one XCD (a multiple of kAbTile;
// build-time knob ISCI_AB_SLAB_COLS)
#ifndef ISCI_AB_SLAB_COLS
#define ISCI_AB_SLAB_COLS 512
#endif
constexpr int kAbSlabCols = ISCI_AB_SLAB_COLS > kAbTile ? ISCI_AB_SLAB_COLS : kAbTile;
static_assert(kAbSlabCols % kAbTile == 0, "slab width must be a multiple of the tile width");

// One workgroup of the alpha-beta product: row block pair g (-1: idle
// workgroup), first column c0 of its kAbTile-column slab, its chunk list from
// eb, and the list ends end[l] that admit source classes <= l.
struct AbBlk {
    int g, c0, eb, pad;
    int end[3], pad2;
};

// Device tables owned by a handle.
struct DevTabs {
    uint32_t *astr = nullptr, *bstr = nullptr;  // packed strings (8 bits per orbital)
    int8_t *alev = nullptr, *blev = nullptr;
    int64_t *rowstart = nullptr;                // [nstr_a + 1]
    // one-body list, CSR over p: (q, h_pq)
    int *h_off = nullptr;
    uint8_t *h_q = nullptr;
    double *h_v = nullptr;
    // same-spin list, CSR over pair index P(p>r) = p(p-1)/2 + r: (q<<8 | s, value)
    int *ss_off = nullptr;
    uint16_t *ss_qs = nullptr;
    double *ss_v = nullptr;
    // alpha-beta list, CSR over (p, q, r): (s, (pq|rs))
    long long *ab_off = nullptr;
    uint8_t *ab_s = nullptr;
    double *ab_v = nullptr;
    // alpha (p -> active q) list: q with at least one kept (pq|rs)
    int *pq_off = nullptr;
    uint8_t *pq_q = nullptr;
    // diagonal units
    double *hd = nullptr;    // h_pp
    double *jj = nullptr;    // (pp|qq)
    double *ssd = nullptr;   // (pp|qq) - (pq|qp)
    unsigned long long *counters = nullptr;  // [2 * ISCI_NBUCKET] kept, terms
    int2 *plan = nullptr;                     // work items (alpha row, first beta target)
    // two-electron spins: index of string {a, b} (a != b) in layout order,
    // -1 when a == b or the string is above the level cut
    int *apidx = nullptr, *bpidx = nullptr;
    // alpha-beta MFMA tiles (two electrons per spin): orbitals grouped in
    // blocks of 4 (occupied block padded with -1); per ordered row-block pair
    // (A,B) a CSR list of column chunks (q, S-block) with their 16x4 values
    // (pq|rs), p in A, r in B, s in S, laid out in MFMA operand-A lane order
    int16_t *blk_orb = nullptr;     // [nblk][4] orbital of each block slot, -1: padding
    int *chunk_off = nullptr;       // [nblk*nblk + 1]
    int2 *chunk_desc = nullptr;     // (q, S)
    double *chunk_val = nullptr;    // [nchunk][64]
    uchar4 *quads = nullptr;        // target tiles (X, P, Y, R) with X<=P, Y<=R, level <= L
    double *hscreen = nullptr;      // [norb][norb] h with screened units set to 0 (one-body kernels)
    double *hpad = nullptr;         // [kObMaxNorb][kObMaxNorb] the same, zero padded (matrix-core one-body)
    double *hpadT = nullptr;        // above kObMaxNorb: [P][P], P = 16 ceil(norb / 16), the same, zero padded
    unsigned long long *hkmask = nullptr;   // [16] per 16-orbital tile of targets a: bit ks set when
                                            // some kept h_qa has q in [4 ks, 4 ks + 4) (norb <= 256)
    // alpha row of the ordered pair (x, q): start and length (-1 / 0 when
    // {x,q} is not a string of the space)
    long long *arow_base = nullptr;
    int *arow_len = nullptr;
    int *chunk_cls = nullptr;       // [nblk*nblk][3] chunks per source level class
    // alpha-beta class as unfold -> block-sparse product -> fold:
    // column offset of each spectator block pair ([nblk][nblk], -1 above
    // the level cut), packed (x, y, v) per column, T rows (q, S, T offset,
    // width) of every (q, S) that opens a chunk, per chunk (T offset, width),
    // row block pairs holding chunks, S offset per row block pair (-1: none),
    // and the per-call operands T and S
    int *abx_gofs = nullptr;
    int *abx_col = nullptr;
    int4 *abx_trow = nullptr;
    int2 *abx_tq = nullptr;         // [norb][nblk]: (T offset of row 0, width) of the rows of (q, S); width 0: none
    int2 *abx_chunk = nullptr;
    int *abx_ctof = nullptr;        // [nchunk + 8]: T offset of each chunk's row 0 (its width follows from its class)
    int *abx_rows = nullptr;
    long long *abx_soff = nullptr;
    AbBlk *abx_blk = nullptr;       // [8 * abx_xmax]: the product tile of each workgroup
    // packed chunks: per row block pair and class, the non-empty (q, s)
    // columns of its chunks four at a time (no all-zero column)
    int4 *abx_pchunk = nullptr;     // [npchunk]: T offsets of the four rows a packed chunk reads
    double *pchunk_val = nullptr;   // [npchunk][64]: values in MFMA operand-A lane order
    AbBlk *abx_pblk = nullptr;      // [8 * abx_pxmax]: product tiles over the packed chunk lists
    double *abx_T = nullptr;
    double *abx_S = nullptr;
    double *abx_S2 = nullptr;       // second S (one-body overlap: both passes' products before the folds)
    // narrow layouts of the packed product for passes of one and of two
    // vectors (one or two vector slots per spectator pair instead of four):
    // each has its own T (zero where no determinant writes) and tables; S
    // is shared with the four-slot layout
    struct AbxNarrow {
        int *gofs = nullptr;
        int2 *tq = nullptr;
        long long *soff = nullptr;
        int4 *pchunk = nullptr;
        AbBlk *pblk = nullptr;
        double *T = nullptr;
    } abxn[2];
    double *obT_c = nullptr;        // [obT_nv][dim] transposed CI block (beta one-body above kObMaxNorb,
                                    // full-CI alpha one-body)
    double *obT_s = nullptr;        // [obT_nv][dim] its one-body image
    // the beta columns of level <= L - 2 (every alpha pair present) as rows
    // [j][alpha string] for up to 8 vectors, their alpha-class image, and
    // the row starts j * nstr_a of that block
    double *obS_c = nullptr, *obS_s = nullptr;
    int64_t *obS_rs = nullptr;
    // density matrices: vectors in the spin-swapped layout (rows = beta
    // strings holding alpha prefixes), allocated by the first density call
    double *d1T = nullptr;          // [kD1Chunk][dim]
    double *d1part = nullptr;       // [kGramGroups][kD1Chunk][norb][norb] partial Gram sums
    // two-body density matrices (two electrons per spin), allocated by the
    // first isci_density2 call: a Gram matrix (max(nstr^2, norb^4)), the
    // pair tensor (norb^4), one vector in the spin-swapped layout, and the
    // row tables of the three Gram products
    double *d2G = nullptr, *d2M = nullptr, *d2cT = nullptr;
    int64_t *d2rs = nullptr;        // [nstr_a + nstr_b + norb^2] row starts: alpha rows, swapped rows, M rows
    int *d2rl = nullptr;            // the same rows' lengths
};

struct SigmaArgs {
    int norb, L;
    double tau;
    SpinTab sa, sb;
    const uint32_t *astr, *bstr;
    const int8_t *alev, *blev;
    const int64_t *rowstart;
    const int *h_off; const uint8_t *h_q; const double *h_v;
    const int *ss_off; const uint16_t *ss_qs; const double *ss_v;
    const long long *ab_off; const uint8_t *ab_s; const double *ab_v;
    const int *pq_off; const uint8_t *pq_q;
    const double *hd, *jj, *ssd;
    const int *apidx, *bpidx;
    int variant;             // 1: general strings, 2: two-electron pair tables, 3: pair + MFMA alpha-beta
    int classes;             // bit 0 one-body, bit 1 same-spin, bit 2 alpha-beta (pair kernel)
    int accumulate;          // pair kernel adds into sigma instead of overwriting
    int nblk;
    int ab_b, ab_nib;        // orbital blocks: inner orbitals 0..ab_b-1 in ab_nib blocks, outer ones after
    const int16_t *blk_orb;
    const int *chunk_off;
    const int2 *chunk_desc;
    const double *chunk_val;
    const uchar4 *quads;
    const long long *arow_base;
    const int *arow_len;
    const int *chunk_cls;
    const int *abx_gofs;
    const int *abx_col;
    const int4 *abx_trow;
    const int2 *abx_tq;
    const int2 *abx_chunk;
    const int *abx_rows;
    const long long *abx_soff;
    const AbBlk *abx_blk;
    const int *abx_ctof;
    const int4 *abx_pchunk;
    const double *pchunk_val;
    const AbBlk *abx_pblk;
    int nchunk;              // chunks of W; chunk_val holds one more, all zero
    double *abx_T, *abx_S;
    int abx_pcols[3];        // columns valid for sources / targets of class 0, 1, 2
    int abx_vs;              // vector slots per spectator pair in the product operands (4, 2 or 1)
};

// Orbital blocks of the matrix-core path: the inner orbitals 0..b-1 (the
// two occupied ones for the excitation hierarchy, the inner space of a GAS
// boundary) in blocks of four from 0, the last one short when b is not a
// multiple of four, then the outer orbitals in blocks of four from b; a
// block's level is 1 when it is outer.  Blocks follow orbital order.
__device__ __forceinline__ int ab_block(const SigmaArgs &A, int o)
{
    return o < A.ab_b ? (o >> 2) : A.ab_nib + ((o - A.ab_b) >> 2);
}
__device__ __forceinline__ int ab_slot(const SigmaArgs &A, int o) { return o < A.ab_b ? (o & 3) : ((o - A.ab_b) & 3); }
__device__ __forceinline__ int ab_width(const SigmaArgs &A, int B) { return B < A.ab_nib ? min(4, A.ab_b - 4 * B) : 4; }
__device__ __forceinline__ int ab_outer(const SigmaArgs &A, int B) { return B >= A.ab_nib ? 1 : 0; }
// orbital of slot i (0..3) of block B, -1 for padding
__device__ __forceinline__ int ab_orbital(const SigmaArgs &A, int B, int i)
{
    const int o = B < A.ab_nib ? 4 * B + i : A.ab_b + 4 * (B - A.ab_nib) + i;
    return (B < A.ab_nib ? o < A.ab_b : o < A.norb) ? o : -1;
}

// Workgroup b of a launch over the determinant rows that starts no empty
// workgroup: the alpha strings of level k (contiguous from sa.lev_off[k])
// hold sb.le[L - k] beta targets each, in ceil(len / 256) workgroups of
// 256.  Gives the row ia, its first target j0 and its length; the level
// walk is uniform and reads only kernel arguments.  The launch has one
// workgroup per 256 targets of each row (isci_ctx::nplan in all).
__device__ __forceinline__ void row_block(const SigmaArgs &A, int b, int &ia, int &j0, int &len)
{
    for (int k = 0;; ++k) {
        const int nr = A.sa.lev_off[k + 1] - A.sa.lev_off[k];
        const int l = A.sb.le[A.L - k];
        const int nbk = (l + 255) >> 8;
        if (b < nr * nbk || k >= A.sa.maxlev) {
            const int r = b / nbk;
            ia = A.sa.lev_off[k] + r;
            j0 = (b - r * nbk) << 8;
            len = l;
            return;
        }
        b -= nr * nbk;
    }
}

// One sigma job of a fused multi-instance launch: instance `inst`, nv (<= 8)
// vectors at c / s with leading dimensions ldc / lds; its work items are
// plan[0..nitems) of the instance (one alpha row, 256 beta targets each)
// and occupy the global item range [item0, item0 + nitems).
struct BatchVec {
    int inst, nv;
    const double *c;
    double *s;
    int64_t ldc, lds;
    const int2 *plan;
    int nitems, item0;
};

}  // namespace isci

struct isci_ctx {
    int norb = 0, na = 0, nb = 0, L = 0;
    double tau = 0.0;
    int device = 0;
    int64_t dim = 0;
    isci::SpinTab sa{}, sb{};
    isci::DevTabs d;
    isci_stats stats{};
    std::vector<void *> allocs;
    // caller's device memory provider (alloc == nullptr: hipMalloc / hipFree)
    isci_allocator allocator{};
    hipStream_t alloc_stream = nullptr;
    std::vector<int32_t> h_aorb, h_borb, h_alev, h_blev;  // host string tables
    std::vector<int64_t> h_rowstart;
    int max_rowlen = 0;
    int nplan = 0;           // work items of one sigma job (blocks of 256 beta targets)
    int sigma_variant = 0;   // ISCI_SIGMA_AUTO / _GENERAL / _PAIR / _MFMA
    int gas_bnd = 0;         // two-space GAS boundary orbital (0: the excitation hierarchy)
    int nblk = 0, nchunk = 0, nquad = 0;
    int ab_b = 2, ab_nib = 1;         // orbital blocks: inner orbitals 0..ab_b-1 in ab_nib blocks
    bool have_abx = false;   // alpha-beta product path built
    bool ab_gather = false;  // ISCI_OPT_AB_PATH = ISCI_AB_GATHER
    int abx_ntrow = 0, abx_nrows = 0, abx_pcols[3] = {0, 0, 0};
    int abx_xmax = 0;        // longest XCD tile run
    int abx_pxmax = 0;       // the same over the packed chunk lists (0: not built)
    int npchunk = 0;         // packed chunks
    // narrow layouts (index 0: one vector slot, 1: two), built with the product path
    bool have_abxn[2] = {false, false};
    int abxn_pcols[2][3] = {{0, 0, 0}, {0, 0, 0}}, abxn_pxmax[2] = {0, 0};
    int ab_kernel = ISCI_AB_PACKED;  // ISCI_OPT_AB_PRODUCT: packed wide-load k_ab_gemm (default), wide, plain, pipe
    int ob_kernel = ISCI_ONEBODY_TRANSPOSED;   // ISCI_OPT_ONEBODY_KERNEL
    int obT_nv = 4;                            // vectors of the transposed one-body scratch (4 or 8)
    bool ob_side = true;     // ISCI_OPT_ONEBODY_STREAM: one-body kernels on the side stream (else in line)
    int64_t nkept_h = 0, nkept_ab = 0;
    bool have_tiles = false;
    bool onebody_in_tiles = false;   // chunk values carry the one-body units (h/2 (x) identity)
    int ob_place = 0;                // ISCI_OB_* requested at create
    // optional per-kernel timing: HIP events recorded around each launch on
    // the launch stream, summed when read
    bool profile = false;
    std::vector<hipEvent_t> prof_ev[ISCI_NKERNEL_IDS];   // start/stop pairs
    // side stream of the matrix-core one-body classes, which run beside the
    // alpha-beta unfolds and products; fork / join events
    hipStream_t ob_stream = nullptr;
    hipEvent_t ob_fork = nullptr, ob_join = nullptr;
    size_t abx_sbytes = 0;
    // scratch for the eigensolver (grown on demand)
    std::vector<void *> work;
};

namespace isci {

// error plumbing
void set_error(const std::string &msg);
isci_status hip_fail(hipError_t e, const char *what);
#define ISCI_CHECK(call)                                            \
    do {                                                            \
        isci_status _st = (call);                                   \
        if (_st != ISCI_OK) return _st;                             \
    } while (0)
#define ISCI_HIP(call)                                              \
    do {                                                            \
        hipError_t _e = (call);                                     \
        if (_e != hipSuccess) return isci::hip_fail(_e, #call);     \
    } while (0)

void *dev_alloc(isci_ctx *c, size_t bytes);
SigmaArgs sigma_args(const isci_ctx *c);

// side = false runs the one-body kernels of the overlap path on `s` too,
// in the same order relative to the products and folds (same results, bit
// for bit): for callers that already overlap many handles on several streams
isci_status launch_sigma(const isci_ctx *c, int nvec, const double *cv, int64_t ldc,
                         double *sv, int64_t lds, hipStream_t s, bool side = true);
// records a start (begin=true) or stop event for kernel id `k` when profiling
isci_status prof_mark(const isci_ctx *c, int k, bool begin, hipStream_t s);
isci_status launch_diag(const isci_ctx *c, double *diag, hipStream_t s);
// alpha-beta class as unfold + block-sparse product + fold (writes sigma)
isci_status launch_ab_product(const isci_ctx *c, int nv, const double *cv, int64_t ldc, double *sv, int64_t lds,
                              hipStream_t s);
// its two halves: unfold + product into the S buffer Sbuf, and the fold
// from Sbuf (accumulate: add into sigma instead of writing it)
isci_status launch_ab_unfold_gemm(const isci_ctx *c, int nv, const double *cv, int64_t ldc, double *Sbuf,
                                  hipStream_t s);
isci_status launch_ab_fold(const isci_ctx *c, int nv, const double *Sbuf, double *sv, int64_t lds, bool accumulate,
                           hipStream_t s);
// one-body classes on matrix cores (two electrons per spin, norb <= kObMaxNorb)
constexpr int kObMaxNorb = 80;
// largest orbital count accepted with two electrons per spin (the
// spectator-form one-body kernels are compared with the oracle up to 199)
constexpr int kPairMaxNorb = 200;
bool onebody_mfma_ok(const isci_ctx *c);
// beta one-body class above kObMaxNorb on the rows themselves (excitation
// hierarchy, a full beta row fits LDS)
bool onebody_beta_rows_ok(const isci_ctx *c);
// first: the beta classes write sigma (they cover every element) instead
// of adding, and the alpha classes add
isci_status launch_onebody_mfma(const isci_ctx *c, int nv, const double *cv, int64_t ldc, double *sv, int64_t lds,
                                hipStream_t s, bool first = false);
// alpha one-body class on matrix cores above kObMaxNorb (spectator form, up
// to 256 orbitals; adds into sigma)
isci_status launch_onebody_alpha_large(const isci_ctx *c, int nv, const double *cv, int64_t ldc, double *sv,
                                       int64_t lds, hipStream_t s);
// beta one-body class above kObMaxNorb: the alpha class of the transposed
// block (nv <= 4; adds into sigma)
isci_status launch_onebody_beta_large(const isci_ctx *c, int nv, const double *cv, int64_t ldc, double *sv,
                                      int64_t lds, hipStream_t s);
isci_status launch_sigma_batched(const SigmaArgs *args_dev, const BatchVec *vecs_dev, int njobs, int nitems,
                                 int nvmax, int grid, hipStream_t s);

// device vector helpers used by the eigensolver
isci_status dots(const double *A, int64_t lda, int m, const double *B, int64_t ldb, int k,
                 int64_t n, double *out_dev, double *partial, int nblk, hipStream_t s);
int dots_blocks(int64_t n);
isci_status lincomb(const double *V, int64_t ldv, int m, const double *Y /*dev [k][m]*/, int k,
                    double *out, int64_t ldo, int64_t n, double beta, hipStream_t s);
// eigen-decomposition of a small symmetric matrix A (m x m, row major):
// eigenvalues w ascending, eigenvectors as columns of Z (Z[i * m + j])
void sym_eigh(int m, const std::vector<double> &A, std::vector<double> &w, std::vector<double> &Z);

}  // namespace isci
