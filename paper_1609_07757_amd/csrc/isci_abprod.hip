// Alpha-beta class (two electrons per spin) as unfold -> block-sparse
// product on FP64 matrix cores -> fold.
//
// With T[x][q][y][s] = sgn(q - x) sgn(s - y) c({x,q},{y,s}) (the CI vector
// as an antisymmetric pair tensor in each spin; zero where {x,q} or {y,s}
// is not a string or the determinant lies above the excitation cut), the
// alpha-beta class (Eq. sigma, the alpha-beta part, with the separable
// phase of its final equation) is
//   T'[x][p][y][r] = S[x][p][y][r] - S[p][x][y][r] - S[x][p][r][y] + S[p][x][r][y],
//   S[x][p][y][r]  = sum_{q,s} (pq|rs) T[x][q][y][s],
// S and T indexed [alpha spectator][alpha active][beta spectator][beta
// active].  For fixed spectators (x, y) this is a product with the
// screened matrix W[(p, r), (q, s)] = (pq|rs); over all spectators and the
// vectors of a pass it is a block-sparse GEMM whose columns are (x, y, v).
//
// Orbitals come in blocks of four, inner and outer apart (for the
// excitation hierarchy block 0 holds the two occupied orbitals; with a GAS
// boundary the inner space takes the first blocks); W is stored as 16 x 4
// chunks (rows (p, r) of a row block pair, columns (q, four s of an S
// block)), ordered inside a row block pair by the class [q outer] +
// [S outer].  Columns are grouped by spectator block pair (C, D), low level
// first (level = [C outer] + [D outer]), each level section padded with
// zero columns to a multiple of 64; a group has slots(C) * slots(D) * 4
// columns (fewer slots for a short inner block).  A
// source or target of class k only has the spectator groups of level
// <= L - k, which is a prefix of the columns: pcols[k].
//
//  * unfold: every (q, S) that opens a chunk gets 4 rows of T, pcols[class]
//    wide; each determinant scatters its values into T once per call;
//  * product: a workgroup takes one row block pair and kAbTile (128)
//    columns; each wave four 16-column tiles; K runs over the chunks whose class leaves
//    the columns valid (a prefix of the chunk list); S gets 16 rows x
//    pcols[class of the row block pair];
//  * fold: every determinant sums its four role readings of S and writes
//    sigma (the first class written; the others add).
#include <hip/hip_runtime.h>

#include "isci_device.h"
#include "isci_internal.h"

namespace isci {

typedef double v4d_ab __attribute__((ext_vector_type(4)));


// Unfold by scatter: one thread per determinant ({a0<a1}, {b0<b1}) of the
// space reads its VS vector values (coalesced; VS = 4 vector slots, or 1 or
// 2 in the narrow layouts) and writes them, with the role sign, to its four
// places in T, one per reading (alpha spectator x, active q) x (beta
// spectator y, active s):
//   T[(q, s)][(x, y, v)] = sgn(q - x) sgn(s - y) c_v({x,q},{y,s}).
// Every entry of T belongs to at most one determinant; entries that belong
// to none were zeroed when T was allocated.  Vectors v >= nv write zeros.
template <int VS>
__global__ __launch_bounds__(256) void k_ab_unfold(SigmaArgs A, int nv, const double *__restrict__ c, int64_t ldc)
{
    int ia, j0, len;
    row_block(A, blockIdx.x, ia, j0, len);
    const int jb = j0 + threadIdx.x;
    if (jb >= len) return;
    const int nb = A.nblk;
    const uint32_t as = A.astr[ia], bs = A.bstr[jb];
    const int a0 = as & 0xff, a1 = (as >> 8) & 0xff, b0 = bs & 0xff, b1 = (bs >> 8) & 0xff;
    const int64_t addr = A.rowstart[ia] + jb;
    double cv[VS];
#pragma unroll
    for (int v = 0; v < VS; ++v) cv[v] = v < nv ? c[(int64_t)v * ldc + addr] : 0.0;
#pragma unroll
    for (int ra = 0; ra < 2; ++ra) {
        const int x = ra ? a1 : a0, q = ra ? a0 : a1;   // alpha spectator, active
#pragma unroll
        for (int rb = 0; rb < 2; ++rb) {
            const int y = rb ? b1 : b0, s = rb ? b0 : b1;
            const int2 tq = A.abx_tq[q * nb + ab_block(A, s)];
            if (tq.y == 0) continue;   // no chunk reads this row
            const int D = ab_block(A, y);
            const int col = A.abx_gofs[ab_block(A, x) * nb + D] + (ab_slot(A, x) * ab_width(A, D) + ab_slot(A, y)) * VS;
            double *dst = A.abx_T + (size_t)tq.x + (size_t)ab_slot(A, s) * tq.y + col;
            const double f = (ra ^ rb) ? -1.0 : 1.0;   // sgn(q - x) sgn(s - y)
#pragma unroll
            for (int v = 0; v < VS; ++v) dst[v] = f * cv[v];
        }
    }
}

// S for one row block pair and 64 CW columns (one tile).  The tiles, ordered
// column slab by column slab, are split at setup into eight contiguous
// runs of about equal work; workgroups are dealt to the eight XCDs
// round-robin, so workgroup b takes tile b / 8 of run b % 8 (its whole
// description is one table entry, read with one scalar load): each XCD
// sweeps the row block pairs of a few slabs, and the slab of T they read
// stays in its own L2.  Within a tile, wave w takes the 64 columns
// (w % CW) and the (w / CW)-th of KS contiguous parts of the chunk list
// (more waves in flight per tile); the parts are summed through LDS in a
// fixed order.
// (at most 80 VGPRs: six waves per SIMD, six 4-wave workgroups per CU with
// the default 2 x 2 wave shape)
// WIDE: each lane fetches two adjacent columns with one 16-byte load (two
// loads per chunk instead of four), so the four 16-column N tiles of a
// wave are the even and odd columns of its two 32-column halves; S is
// stored two columns per lane in the same order.
// PACKED (with WIDE): the packed chunk lists, whose four K columns may come
// from different T rows (one offset per column, selected per lane group).
template <int CW, int KS, bool WIDE, bool PACKED>
__global__ __launch_bounds__(64 * CW * KS) __attribute__((amdgpu_waves_per_eu(6))) void k_ab_gemm(SigmaArgs A)
{
    static_assert(!PACKED || WIDE, "packed chunks use the 16-byte loads");
    __shared__ double red[KS > 1 ? KS - 1 : 1][CW][16][64];
    const int nb = A.nblk;
    const AbBlk tb = PACKED ? A.abx_pblk[blockIdx.x] : A.abx_blk[blockIdx.x];   // one scalar load: the tile
    if (tb.g < 0) return;
    const int g = tb.g;
    const int Ab = g / nb, Bb = g % nb;
    const int m = ab_outer(A, Ab) + ab_outer(A, Bb);
    // wave index made explicitly uniform: the chunk range and the chunk
    // table reads below then compile to scalar loads, which retire apart
    // from the vector loads of the operands
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int cw = wave % CW, part = wave / CW;
    const int c0 = tb.c0 + cw * 64;
    const int swidth = A.abx_pcols[m];
    const bool active = c0 < swidth;
    // chunks whose class keeps these columns valid: classes l with
    // c0 < pcols[max(l, m)], a prefix of the class-ordered list
    const int eb = tb.eb;
    int ee = eb;
    for (int l = 0; l < 3; ++l)
        if (c0 < A.abx_pcols[max(l, m)]) ee = tb.end[l];
    // parts cut at multiples of four chunks (the loop's step), so only the
    // last part runs zero-padded steps
    const int step = ((ee - eb + KS - 1) / KS + 3) & ~3;
    const int e0 = min(ee, eb + step * part);
    const int e1 = min(ee, eb + step * (part + 1));
    const int k = lane >> 4, n = lane & 15;
    v4d_ab acc[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) acc[u] = v4d_ab{0.0, 0.0, 0.0, 0.0};
    // two stages of two chunks, ping-ponged; loads are unconditional
    // (clamped chunk index, zero selected past the end) so waiting for one
    // stage never waits for the other
    double ax[2], bx[2][4], ay[2], by[2][4];
    auto load2 = [&](int e, double *a, double (*b)[4]) {
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int eu = min(e + u, e1 - 1);
            if (PACKED) {
                const int4 r4 = A.abx_pchunk[eu];   // T offsets of the chunk's four rows
                const int ro = k == 0 ? r4.x : (k == 1 ? r4.y : (k == 2 ? r4.z : r4.w));
                const double av = A.pchunk_val[(size_t)eu * 64 + lane];
                a[u] = e + u < e1 ? av : 0.0;
                const double2 *src = (const double2 *)(A.abx_T + (size_t)ro + c0 + 2 * n);
                const double2 lo = src[0], hi = src[16];
                b[u][0] = lo.x; b[u][1] = lo.y; b[u][2] = hi.x; b[u][3] = hi.y;
                continue;
            }
            const int2 tx = A.abx_chunk[eu];   // (T offset of the chunk's row 0, row width)
            const double av = A.chunk_val[(size_t)eu * 64 + lane];
            a[u] = e + u < e1 ? av : 0.0;
            if (WIDE) {
                // columns c0 + 32 h + 2 n + j -> N tile 2 h + j
                const double2 *src = (const double2 *)(A.abx_T + (size_t)tx.x + (size_t)k * tx.y + c0 + 2 * n);
                const double2 lo = src[0], hi = src[16];
                b[u][0] = lo.x; b[u][1] = lo.y; b[u][2] = hi.x; b[u][3] = hi.y;
            } else {
                const double *src = A.abx_T + (size_t)tx.x + (size_t)k * tx.y + c0 + n;
#pragma unroll
                for (int q = 0; q < 4; ++q) b[u][q] = src[16 * q];
            }
        }
    };
    auto mma2 = [&](const double *a, const double (*b)[4]) {
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u], b[u][q], acc[q], 0, 0, 0);
    };
    if (active && e0 < e1) {
        load2(e0, ax, bx);
        for (int e = e0; e < e1; e += 4) {
            load2(e + 2, ay, by);
            mma2(ax, bx);
            load2(e + 4, ax, bx);
            mma2(ay, by);
        }
    }
    if (KS > 1) {
        if (part > 0)
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int gg = 0; gg < 4; ++gg) red[part - 1][cw][4 * q + gg][lane] = acc[q][gg];
        __syncthreads();
        if (part > 0) return;
#pragma unroll
        for (int p2 = 0; p2 < KS - 1; ++p2)
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int gg = 0; gg < 4; ++gg) acc[q][gg] += red[p2][cw][4 * q + gg][lane];
    }
    if (!active) return;
    // element gg of lane l: row 4 gg + l / 16 (alpha active slot gg, beta active slot l / 16), column l % 16
    if (WIDE) {
        double2 *Sb = (double2 *)(A.abx_S + (size_t)A.abx_soff[g] + (size_t)k * swidth + c0 + 2 * n);
#pragma unroll
        for (int gg = 0; gg < 4; ++gg) {
            Sb[(size_t)gg * 2 * swidth] = double2{acc[0][gg], acc[1][gg]};
            Sb[(size_t)gg * 2 * swidth + 16] = double2{acc[2][gg], acc[3][gg]};
        }
    } else {
        double *Sb = A.abx_S + (size_t)A.abx_soff[g] + (size_t)k * swidth + c0 + n;
#pragma unroll
        for (int gg = 0; gg < 4; ++gg)
#pragma unroll
            for (int q = 0; q < 4; ++q) Sb[(size_t)gg * 4 * swidth + 16 * q] = acc[q][gg];
    }
}

// The product of k_ab_gemm with an explicit two-stage software pipeline:
// the chunks of a wave's list are taken U at a time; while the MFMAs of one
// stage run, the operand loads of the next stage are in flight and the
// chunk table of the stage after it is read (scalar loads one stage early,
// so no operand address waits on the scalar cache).  The table holds only
// each chunk's T offset; the row width follows from the chunk's class (the
// list is class ordered).  Loads past the end of the list read the all-zero
// chunk behind the last one (and a valid T row), so no value is selected
// after it is loaded.  Scheduling barriers keep every load of a stage ahead
// of the previous stage's MFMAs.  Tiles, waves and the K split as in
// k_ab_gemm; same sums in the same order per K part.
template <int CW, int KS, int U>
__global__ __launch_bounds__(64 * CW * KS) void k_ab_pipe(SigmaArgs A)
{
    __shared__ double red[KS > 1 ? KS - 1 : 1][CW][16][64];
    const int nb = A.nblk;
    const AbBlk tb = A.abx_blk[blockIdx.x];   // one scalar load: the tile of this workgroup
    if (tb.g < 0) return;
    const int g = tb.g;
    const int Ab = g / nb, Bb = g % nb;
    const int m = ab_outer(A, Ab) + ab_outer(A, Bb);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int cw = wave % CW, part = wave / CW;
    const int c0 = tb.c0 + cw * 64;
    const int swidth = A.abx_pcols[m];
    const bool active = c0 < swidth;
    const int eb = tb.eb;
    int ee = eb;
    for (int l = 0; l < 3; ++l)
        if (c0 < A.abx_pcols[max(l, m)]) ee = tb.end[l];
    // parts cut at multiples of 2 U chunks (one loop step)
    const int step = ((ee - eb + KS - 1) / KS + 2 * U - 1) / (2 * U) * (2 * U);
    const int e0 = min(ee, eb + step * part);
    const int e1 = min(ee, eb + step * (part + 1));
    const int k = lane >> 4, n = lane & 15;
    const int zc = A.nchunk;
    const int w0 = A.abx_pcols[0], w1 = A.abx_pcols[1], w2 = A.abx_pcols[2];
    const int end0 = tb.end[0], end1 = tb.end[1];
    const double *Tb = A.abx_T + c0 + n;
    const double *Va = A.chunk_val + lane;
    v4d_ab acc[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[q] = v4d_ab{0.0, 0.0, 0.0, 0.0};
    double ax[U], bx[U][4], ay[U], by[U][4];
    int tx[U], ty[U];
    auto fetch_tab = [&](int e, int *t) {
#pragma unroll
        for (int u = 0; u < U; ++u) t[u] = A.abx_ctof[min(e + u, e1 - 1)];
    };
    auto issue = [&](int e, const int *t, double *a, double (*b)[4]) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int eu = e + u, ec = min(eu, e1 - 1);
            const int wd = ec >= end1 ? w2 : (ec >= end0 ? w1 : w0);
            const double *src = Tb + (size_t)t[u] + (size_t)k * wd;
            a[u] = Va[(size_t)(eu < e1 ? eu : zc) * 64];
#pragma unroll
            for (int q = 0; q < 4; ++q) b[u][q] = src[16 * q];
        }
    };
    auto mma = [&](const double *a, const double (*b)[4]) {
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u], b[u][q], acc[q], 0, 0, 0);
    };
    if (active && e0 < e1) {
        fetch_tab(e0, tx);
        issue(e0, tx, ax, bx);
        fetch_tab(e0 + U, ty);
        for (int e = e0; e < e1; e += 2 * U) {
            issue(e + U, ty, ay, by);
            fetch_tab(e + 2 * U, tx);
            __builtin_amdgcn_sched_barrier(0);
            mma(ax, bx);
            __builtin_amdgcn_sched_barrier(0);
            issue(e + 2 * U, tx, ax, bx);
            fetch_tab(e + 3 * U, ty);
            __builtin_amdgcn_sched_barrier(0);
            mma(ay, by);
            __builtin_amdgcn_sched_barrier(0);
        }
    }
    if (KS > 1) {
        if (part > 0)
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int gg = 0; gg < 4; ++gg) red[part - 1][cw][4 * q + gg][lane] = acc[q][gg];
        __syncthreads();
        if (part > 0) return;
#pragma unroll
        for (int p2 = 0; p2 < KS - 1; ++p2)
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int gg = 0; gg < 4; ++gg) acc[q][gg] += red[p2][cw][4 * q + gg][lane];
    }
    if (!active) return;
    double *Sb = A.abx_S + (size_t)A.abx_soff[g] + (size_t)k * swidth + c0 + n;
#pragma unroll
    for (int gg = 0; gg < 4; ++gg)
#pragma unroll
        for (int q = 0; q < 4; ++q) Sb[(size_t)gg * 4 * swidth + 16 * q] = acc[q][gg];
}

// sigma({a0 < a1}, {b0 < b1}) = sum over the four readings (alpha
// spectator, alpha active) x (beta spectator, beta active) of S, sign - per
// spin whose spectator is the larger orbital
template <int VS>
__global__ __launch_bounds__(256) void k_ab_fold(SigmaArgs A, int nv, double *__restrict__ sg, int64_t lds,
                                                 int accumulate)
{
    int ia, j0, len;
    row_block(A, blockIdx.x, ia, j0, len);
    const int jb = j0 + threadIdx.x;
    if (jb >= len) return;
    const int nb = A.nblk;
    const uint32_t as = A.astr[ia], bs = A.bstr[jb];
    const int a0 = as & 0xff, a1 = (as >> 8) & 0xff, b0 = bs & 0xff, b1 = (bs >> 8) & 0xff;
    double acc[VS];
#pragma unroll
    for (int v = 0; v < VS; ++v) acc[v] = 0.0;
#pragma unroll
    for (int ra = 0; ra < 2; ++ra) {
        const int xs = ra ? a1 : a0, xa = ra ? a0 : a1;   // alpha spectator, active
#pragma unroll
        for (int rb = 0; rb < 2; ++rb) {
            const int ys = rb ? b1 : b0, ya = rb ? b0 : b1;
            const int g = ab_block(A, xa) * nb + ab_block(A, ya);
            const long long so = A.abx_soff[g];
            if (so < 0) continue;
            const int m = ab_outer(A, ab_block(A, xa)) + ab_outer(A, ab_block(A, ya));
            const int C = ab_block(A, xs), D = ab_block(A, ys);
            const int col = A.abx_gofs[C * nb + D] + (ab_slot(A, xs) * ab_width(A, D) + ab_slot(A, ys)) * VS;
            const int row = ab_slot(A, xa) * 4 + ab_slot(A, ya);
            const double *src = A.abx_S + (size_t)so + (size_t)row * A.abx_pcols[m] + col;
            const double f = (ra ^ rb) ? -1.0 : 1.0;
#pragma unroll
            for (int v = 0; v < VS; ++v) acc[v] += f * src[v];
        }
    }
    double *dst = sg + A.rowstart[ia] + jb;
    if (accumulate) {
        double old[VS];
#pragma unroll
        for (int v = 0; v < VS; ++v) old[v] = dst[(int64_t)min(v, nv - 1) * lds];
#pragma unroll
        for (int v = 0; v < VS; ++v)
            if (v < nv) dst[(int64_t)v * lds] = old[v] + acc[v];
    } else {
#pragma unroll
        for (int v = 0; v < VS; ++v)
            if (v < nv) dst[(int64_t)v * lds] = acc[v];
    }
}

// A pass of one or two vectors takes the narrow layout with that many
// vector slots per spectator pair (a quarter or half of the four-slot
// operands and product) when it is built and the packed product is
// selected; returns its index, or -1 for the four-slot layout
static int narrow_layout(const isci_ctx *cx, int nv)
{
    const int w = nv - 1;
    if (w < 0 || w > 1 || !cx->have_abxn[w] || cx->ab_kernel != ISCI_AB_PACKED || cx->abxn_pxmax[w] <= 0) return -1;
    return w;
}

// arguments of the product path for a pass of nv vectors
static SigmaArgs product_args(const isci_ctx *cx, int nv)
{
    SigmaArgs A = sigma_args(cx);
    const int w = narrow_layout(cx, nv);
    if (w >= 0) {
        const auto &x = cx->d.abxn[w];
        A.abx_vs = w + 1;
        A.abx_gofs = x.gofs;
        A.abx_tq = x.tq;
        A.abx_soff = x.soff;
        A.abx_pchunk = x.pchunk;
        A.abx_pblk = x.pblk;
        A.abx_T = x.T;
        for (int k = 0; k < 3; ++k) A.abx_pcols[k] = cx->abxn_pcols[w][k];
    }
    return A;
}

isci_status launch_ab_unfold_gemm(const isci_ctx *cx, int nv, const double *c, int64_t ldc, double *Sbuf,
                                  hipStream_t st)
{
    SigmaArgs A = product_args(cx, nv);
    A.abx_S = Sbuf;
    const int w = narrow_layout(cx, nv);
    if (cx->abx_ntrow > 0) {
        ISCI_CHECK(prof_mark(cx, ISCI_KERNEL_AB_UNFOLD, true, st));
        if (w == 0)
            k_ab_unfold<1><<<(unsigned)cx->nplan, 256, 0, st>>>(A, nv, c, ldc);
        else if (w == 1)
            k_ab_unfold<2><<<(unsigned)cx->nplan, 256, 0, st>>>(A, nv, c, ldc);
        else
            k_ab_unfold<4><<<(unsigned)cx->nplan, 256, 0, st>>>(A, nv, c, ldc);
        ISCI_CHECK(prof_mark(cx, ISCI_KERNEL_AB_UNFOLD, false, st));
    }
    if (cx->abx_nrows > 0) {
        ISCI_CHECK(prof_mark(cx, ISCI_KERNEL_AB_GEMM, true, st));
        const dim3 grid((unsigned)(8 * cx->abx_xmax)), block(64 * kAbCW * kAbSplit);
        if (w >= 0)
            k_ab_gemm<kAbCW, kAbSplit, true, true><<<dim3((unsigned)(8 * cx->abxn_pxmax[w])), block, 0, st>>>(A);
        else if (cx->ab_kernel == ISCI_AB_PACKED && cx->abx_pxmax > 0)
            k_ab_gemm<kAbCW, kAbSplit, true, true><<<dim3((unsigned)(8 * cx->abx_pxmax)), block, 0, st>>>(A);
        else if (cx->ab_kernel == ISCI_AB_PIPE)
            k_ab_pipe<kAbCW, kAbSplit, 2><<<grid, block, 0, st>>>(A);
        else if (cx->ab_kernel == ISCI_AB_WIDE || cx->ab_kernel == ISCI_AB_PACKED)
            k_ab_gemm<kAbCW, kAbSplit, true, false><<<grid, block, 0, st>>>(A);
        else
            k_ab_gemm<kAbCW, kAbSplit, false, false><<<grid, block, 0, st>>>(A);
        ISCI_CHECK(prof_mark(cx, ISCI_KERNEL_AB_GEMM, false, st));
    }
    ISCI_HIP(hipGetLastError());
    return ISCI_OK;
}

isci_status launch_ab_fold(const isci_ctx *cx, int nv, const double *Sbuf, double *s, int64_t lds, bool accumulate,
                           hipStream_t st)
{
    SigmaArgs A = product_args(cx, nv);
    A.abx_S = const_cast<double *>(Sbuf);
    ISCI_CHECK(prof_mark(cx, ISCI_KERNEL_AB_FOLD, true, st));
    if (A.abx_vs == 1)
        k_ab_fold<1><<<(unsigned)cx->nplan, 256, 0, st>>>(A, nv, s, lds, accumulate ? 1 : 0);
    else if (A.abx_vs == 2)
        k_ab_fold<2><<<(unsigned)cx->nplan, 256, 0, st>>>(A, nv, s, lds, accumulate ? 1 : 0);
    else
        k_ab_fold<4><<<(unsigned)cx->nplan, 256, 0, st>>>(A, nv, s, lds, accumulate ? 1 : 0);
    ISCI_CHECK(prof_mark(cx, ISCI_KERNEL_AB_FOLD, false, st));
    ISCI_HIP(hipGetLastError());
    return ISCI_OK;
}

isci_status launch_ab_product(const isci_ctx *cx, int nv, const double *c, int64_t ldc, double *s, int64_t lds,
                              hipStream_t st)
{
    ISCI_CHECK(launch_ab_unfold_gemm(cx, nv, c, ldc, cx->d.abx_S, st));
    return launch_ab_fold(cx, nv, cx->d.abx_S, s, lds, false, st);
}

}  // namespace isci
