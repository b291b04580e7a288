/*
 * isci.h -- C ABI of libisci, an FP64 implementation for AMD MI355X
 * (gfx950) of the sigma-vector step sigma = H c of the Integral Screened
 * Configuration Interaction method (Sorensen, Bauch & Madsen, "The
 * Integral Screened Configuration Interaction Method"), plus the
 * eigensolver around it.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Hamiltonian: Eq. ham / index_un of the paper, spin-restricted orbitals:
 *   H = sum_pq h_pq (E^a_pq + E^b_pq)
 *     + 1/2 sum_pqrs (pq|rs) sum_{s,s'} a+_{p s} a+_{r s'} a_{s s'} a_{q s},
 * with g_pqrs = (pq|rs) in chemists' order.  h is read from its lower
 * triangle (p >= q) and eri from its canonical element (p>=q, r>=s,
 * (p,q) >= (r,s) lexicographically); the other positions are never read,
 * so the caller may pass a tensor that is only filled there.
 *
 * Screening (section "The ISCI and Integral screening", Eqs. sigma_int
 * and sigma_split): every elementary integral unit with |unit| <= tau is
 * removed from H (ties at exactly tau are dropped).  The units are h_pq
 * (one-body), the antisymmetrised same-spin coefficient (pq|rs) - (ps|rq)
 * formed by one subtraction (Eq. index_re), and the raw (pq|rs) of the
 * alpha-beta class.  tau = 0 keeps every non-zero unit.
 *
 * CI space (Eqs. ci_ansatz, ci_hierarchy): the reference occupies
 * orbitals 0..n-1 of each spin; the level of a string is its number of
 * electrons in orbitals >= n; the space holds every (alpha, beta) string
 * pair with level_a + level_b <= max_excitation (2 CISD, 3 CISDT, 4
 * CISDTQ; a value >= na + nb gives full CI).
 *
 * Vector layout (all vectors, device memory, FP64): per spin the strings
 * (ascending orbital sets) are sorted by (level, colex order -- highest
 * orbital compared first).  Rows are alpha strings in that order; the row
 * of an alpha string of level k holds the beta strings of level
 * <= max_excitation - k, which is a prefix of the beta order.  The
 * determinant |Ia Ib> = (prod_{p in Ia, ascending} a+_{p alpha})
 * (prod_{q in Ib, ascending} a+_{q beta}) |vac> sits at
 * rowstart(Ia) + index(Ib).  isci_strings / isci_rowstart export the
 * tables so a caller can map by occupation.
 *
 * Streams and ownership: device pointers belong to the caller.  Every
 * entry point that takes a stream enqueues its work on that stream in
 * stream order and returns without synchronising, except isci_create
 * (one synchronisation to size the screened lists) and isci_davidson
 * (one small device-to-host copy per iteration, and a final
 * synchronisation).  A handle owns its device tables and frees them in
 * isci_destroy.  A handle is not thread safe; distinct handles may be
 * used concurrently on distinct streams.
 *
 * Errors: functions return an isci_status and never throw.  Argument
 * errors are detected before anything is enqueued.  isci_last_error()
 * returns a per-thread message for the last failure.
 *
 * Limits of this build: norb <= 255 (<= 200 with two electrons of each
 * spin), 0 <= na, nb <= 4, dim < 2^62, nvec >= 1 (vectors are processed
 * in chunks of 8).  isci_create refuses (ISCI_E_INVALID) integrals that
 * hold a NaN or an infinity in a position it reads.
 */
#ifndef ISCI_H
#define ISCI_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct isci_ctx *isci_handle;

typedef enum {
    ISCI_OK = 0,
    ISCI_E_INVALID = -1,        /* bad argument; nothing was enqueued */
    ISCI_E_OOM = -2,            /* device allocation failed */
    ISCI_E_HIP = -3,            /* a HIP runtime call failed */
    ISCI_E_NOT_CONVERGED = -4,  /* Davidson hit max_iter; best estimates returned */
    ISCI_E_UNSUPPORTED = -5     /* outside the limits of this build */
} isci_status;

#define ISCI_NBUCKET 42
#define ISCI_MAX_ROOTS 32

/* Screening statistics.  Buckets follow the paper's Hamiltonian classes
 * (Eqs. class_to_ex_dx .. the_end): 0..3 one-body alpha and 4..7 one-body
 * beta indexed 2 e_p + e_q; 8..16 same-spin alpha and 17..25 same-spin
 * beta indexed 3 (#virtual creators) + (#virtual annihilators); 26..41
 * alpha-beta indexed 8 e_p + 4 e_q + 2 e_r + e_s, where e_x = 1 if orbital
 * x is virtual for its spin (x >= n).  kept[b] counts kept integral units
 * (one-body (p,q) pairs, same-spin (p>r, q>s) pairs, alpha-beta (p,q,r,s)
 * quadruples); terms[b] counts the (unit, source determinant, target
 * determinant) products one sigma vector performs -- the paper's
 * operation-count unit. */
typedef struct {
    int64_t dim;
    int64_t nstr_alpha, nstr_beta;
    int64_t kept[ISCI_NBUCKET];
    int64_t terms[ISCI_NBUCKET];
    int64_t kept_total;
    int64_t terms_total;
    int64_t device_bytes;       /* bytes of device memory owned by the handle */
} isci_stats;

typedef struct {
    double tol_residual;        /* converged when every root has ||r||_2 <= this (default 1e-7) */
    double tol_energy;          /* ... and |dE| <= this between iterations (default 1e-11) */
    int max_iter;               /* default 200 */
    int max_subspace;           /* default max(32, 6 (nroots + 2)) */
    int block;                  /* correction vectors per iteration (default nroots + 2) */
} isci_davidson_opts;

typedef struct {
    int iterations;
    int converged;              /* 1 if every root met both tolerances */
    int sigma_calls;            /* sigma vectors computed */
    double residual[ISCI_MAX_ROOTS];
} isci_davidson_info;

/* Set defaults in *o. */
void isci_davidson_defaults(isci_davidson_opts *o);

/* Build a handle: validate, enumerate strings and the row layout, build
 * the screened integral lists on the device (one pass over h and eri),
 * count kept units and sigma terms per bucket, and tabulate the diagonal
 * units.  h: device [norb*norb]; eri: device [norb^4] ((pq|rs) at
 * ((p*norb+q)*norb+r)*norb+s).  Both are only read during this call (in
 * stream order; the call synchronises the stream before returning).
 * Errors: ISCI_E_INVALID for NULL pointers, norb < 1, electron counts
 * outside [0, norb], max_excitation < 0, tau negative, NaN or infinite,
 * and for a NaN or infinity in any element that is read (one device pass
 * over them before the lists are built: such a unit would fail
 * |unit| > tau and vanish silently); ISCI_E_UNSUPPORTED beyond the limits
 * above; ISCI_E_OOM / ISCI_E_HIP on device failures (the handle is not
 * created). */
isci_status isci_create(isci_handle *out, const double *h, const double *eri, int norb,
                        int nalpha, int nbeta, int max_excitation, double tau,
                        hipStream_t stream);

/* Where the matrix-core path (two electrons per spin) applies the kept
 * one-body units.  With two electrons of a spin, sum_r E_rr equals 2 on the
 * whole space, so h_pq E^alpha_pq = sum_r (h_pq / 2) E^alpha_pq E^beta_rr
 * (and likewise for beta): the units can ride in the alpha-beta tiles, at
 * the price of the tiles they open.  SEPARATE keeps them in their own
 * kernels; TILES puts them in the tiles; AUTO puts them in the tiles when
 * that adds at most one tile in eight or the space has at most 65536
 * determinants (there the extra launches cost more than the extra tiles).
 * Below three orbitals the tiles always carry them.  The sigma vector is
 * the same either way (up to rounding order). */
#define ISCI_OB_AUTO 0
#define ISCI_OB_SEPARATE 1
#define ISCI_OB_TILES 2

/* Device memory provider for a handle's resident tables (screened lists,
 * string and row tables, the product path's operand and result blocks):
 * for callers that keep device memory in their own pool (a framework's
 * caching allocator).  alloc returns `bytes` of device memory usable in
 * stream order on `stream`, or NULL (isci_create then fails with
 * ISCI_E_OOM and frees what it took); free releases one block.  Both are
 * called on the creating thread with the stream given to isci_create_ex,
 * alloc during isci_create_ex and free during isci_destroy (which first
 * waits for all work on the device, so no launch still reads a block).
 * Temporaries of isci_create itself use hipMallocAsync on that stream. */
typedef struct {
    void *(*alloc)(size_t bytes, hipStream_t stream, void *ctx);
    void (*free)(void *p, hipStream_t stream, void *ctx);
    void *ctx;
} isci_allocator;

/* Distance screening (the paper's proposal, in its discussion of the
 * screening results, of an additional integral screening by the distance
 * between orbitals, the route to linear scaling): with orb_dist (host,
 * [norb][norb] distances d(p, q) >= 0, read during creation only) and
 * max_dist > 0, every integral unit whose orbitals are not all within
 * max_dist of each other is removed from H as well: h_pq when d(p, q) >
 * max_dist, a two-electron unit over p, q, r, s when any of the six
 * pairwise distances exceeds it.  The handle then applies the Hamiltonian of
 * the integrals with those elements set to zero (screened by the usual rule
 * besides).  orb_dist NULL or max_dist == 0: off.  ISCI_E_INVALID when
 * orb_dist is given with a NaN or negative max_dist, or (screening on) holds
 * a NaN, infinite or negative distance.  A matrix that is not symmetric is
 * read as max(d(p, q), d(q, p)) for the pair p, q. */
typedef struct {
    int onebody;                      /* ISCI_OB_* (default ISCI_OB_AUTO) */
    const isci_allocator *allocator;  /* NULL: hipMalloc / hipFree; else
                                         both function pointers set; the
                                         struct is copied at creation */
    const double *orb_dist;           /* host [norb][norb] or NULL (no distance screening) */
    double max_dist;                  /* distance screening radius; 0: off */
    int gas_boundary;                 /* two-space GAS restriction (below); 0: off */
} isci_create_opts;

/* Two-space GAS restriction (section "Generalized Active Space"; the
 * restriction to at most one electron in the continuum in the appendix on
 * CAAB types): with gas_boundary = b, max(nalpha, nbeta) <= b <= norb, the
 * orbitals split into an inner space 0..b-1 and an outer space b..norb-1,
 * a string's level is its number of electrons in the outer space, and
 * max_excitation limits the outer electrons, alpha plus beta.  The space is
 * then every determinant of the inner orbitals (full CI there) with at most
 * max_excitation electrons in the outer ones; b = n_sigma for both spins is
 * the excitation hierarchy of Eq. ci_hierarchy (the default, 0).  The
 * layout is unchanged in form: strings sorted by (level, colex), the row of
 * a level-k alpha string holding the beta strings of level <= L - k.  With
 * two electrons per spin such a handle runs the matrix-core path with its
 * orbital blocks split at b (inner blocks first) and the one-body units
 * carried in the alpha-beta tiles (the separate one-body kernels take
 * orbitals 0 and 1 as the occupied ones; onebody = ISCI_OB_SEPARATE is
 * overridden); other electron counts run the general-string kernel.  The
 * densities apply as for any handle (isci_density1 and
 * isci_density1_noalloc for b <= 16, else ISCI_E_UNSUPPORTED).
 * ISCI_E_INVALID for b outside [max(nalpha, nbeta), norb]. */

/* isci_create with build options; opts may be NULL (defaults).  Returns
 * ISCI_E_INVALID for an unknown onebody value or an allocator with a NULL
 * function pointer. */
isci_status isci_create_ex(isci_handle *out, const double *h, const double *eri, int norb,
                           int nalpha, int nbeta, int max_excitation, double tau,
                           const isci_create_opts *opts, hipStream_t stream);

/* A handle built from factored two-electron integrals,
 *   (pq|rs) = sum_{K < naux} L^K_pq L^K_rs,
 * without forming the dense norb^4 tensor: the list builders form each
 * integral they need from the factors (at its canonical indices, K
 * ascending, every product and partial sum rounded once, no fused
 * multiply-add) when the screened lists are built, so each is computed
 * once and the sigma steps only fetch the kept units: the paper's minimum
 * integral calculation (section "First part" of the implementation: the
 * integrals of a Hamiltonian type computed once and fetched by every
 * block) applied to the screening of Eqs. sigma_int / sigma_split.  A
 * builder skips a unit without forming it when the Cauchy-Schwarz bound
 * |(pq|rs)| <= |L_pq| |L_rs| (with a margin for rounding) shows it would be
 * screened; the kept units and their values are exactly those of a dense
 * tensor assembled in the same order, so the handle behaves as one built
 * by isci_create_ex from that tensor.  Lfac: device [naux][norb][norb]
 * (L^K_pq at (K norb + p) norb + q), read during this call only; only the
 * elements p >= q are used (the lower triangle of each L^K).  The call
 * takes 8 (naux + 1) norb^2 bytes of temporaries instead of the 8 norb^4
 * bytes of a dense tensor.  Other arguments, the result and the errors as
 * isci_create_ex; ISCI_E_INVALID also for naux < 1, and for a non-finite
 * factor element that is used or a factor norm whose square overflows. */
isci_status isci_create_factored(isci_handle *out, const double *h, const double *Lfac, int naux, int norb,
                                 int nalpha, int nbeta, int max_excitation, double tau,
                                 const isci_create_opts *opts, hipStream_t stream);

/* Number of determinants of the truncated space: the terms of the CI
 * expansion (Eq. ci_ansatz) kept by the excitation hierarchy cut at
 * max_excitation (Eq. ci_hierarchy), counted per (alpha, beta) string
 * pair with level_a + level_b <= max_excitation.  *dim (host) receives the
 * length of every vector the handle reads or writes.  ISCI_E_INVALID if
 * hd or dim is NULL.  No device work. */
isci_status isci_dim(isci_handle hd, int64_t *dim);

/* sigma[v*lds + I] = sum_J (H_tau)_IJ c[v*ldc + J] for v < nvec, all I
 * (Eq. sigma).  c and sigma are device arrays of nvec vectors with leading
 * dimensions ldc, lds >= dim; sigma is overwritten and must not overlap c.
 * Asynchronous on `stream`.  The handle owns the call's scratch (unfolded
 * operand, products, transposed block) and a side stream that it forks
 * from and joins back to `stream` with events, so calls on one handle must
 * be ordered (one stream at a time, or synchronised); different handles
 * may run concurrently. */
isci_status isci_sigma(isci_handle hd, int nvec, const double *c, int64_t ldc,
                       double *sigma, int64_t lds, hipStream_t stream);

/* A sigma call recorded as a HIP graph, for callers that apply H_tau many
 * times to the same buffers (their own iterative solvers, serving loops
 * that reuse work vectors): one graph launch replaces the call's kernel
 * launches and its side-stream fork and join.
 *
 * isci_sigma_graph_create records isci_sigma(hd, nvec, c, ldc, sigma, lds)
 * (same arguments, same checks, same errors) by stream capture on a private
 * stream and instantiates it; nothing runs at creation.  Each
 * isci_graph_launch then computes sigma from the current contents of c,
 * exactly as the recorded call would (Eq. sigma), asynchronously on
 * `stream`.  The graph keeps the pointers c and sigma and uses the
 * handle's scratch: the caller keeps c, sigma and the handle alive until
 * isci_graph_destroy, and orders launches with the handle's other sigma
 * calls (one at a time).  The kernel path is the one the handle had at
 * creation; options set later do not change it.  Refused (ISCI_E_INVALID)
 * while kernel profiling is enabled on the handle.  *out is NULL on
 * failure. */
typedef struct isci_graph_s *isci_graph;
isci_status isci_sigma_graph_create(isci_handle hd, int nvec, const double *c, int64_t ldc,
                                    double *sigma, int64_t lds, isci_graph *out);
isci_status isci_graph_launch(isci_graph g, hipStream_t stream);
void isci_graph_destroy(isci_graph g);

/* diag[I] = (H_tau)_II, the Slater-Condon diagonal of determinant I of
 * the Hamiltonian of Eq. ham: the diagonal integrals of the classes present
 * in each diagonal block (section "The excitation class formalism", the
 * paper's list of classes of the reference block, of which only the
 * diagonal integrals are used), i.e. h_pp per occupied orbital,
 * (pp|qq) - (pq|qp) per same-spin pair and (pp|qq) per alpha-beta pair,
 * each unit kept by the same rule |unit| > tau as sigma.  diag: device
 * array of length dim, written (caller-owned).  Asynchronous on stream.
 * ISCI_E_INVALID for NULL arguments; ISCI_E_HIP if the launch fails. */
isci_status isci_diag(isci_handle hd, double *diag, hipStream_t stream);

/* One-body density matrix of each vector, by spin (the paper's density
 * matrices, Eq. d1, with the spin-orbital indices of one spin):
 *   d1[((v * 2 + s) * norb + p) * norb + q] = <c_v| a+_{p s} a_{q s} |c_v>,
 * s = 0 alpha, 1 beta, for v < nvec (1..65535).  c: device, nvec vectors
 * with leading dimension ldc >= dim, not normalised by the call (the trace
 * of the s block is n_s * |c_v|^2).  d1: device, nvec * 2 * norb^2 doubles,
 * overwritten, must not overlap c.  Every determinant pair connected by
 * a+_p a_q counts; the screening threshold plays no part.  Deterministic
 * (fixed summation order).  The beta block is computed from the vectors
 * transposed into the spin-swapped layout, eight at a time.  The handle
 * allocates on its first density call, and keeps until it is destroyed,
 * 64 * 8 * norb^2 doubles of partial sums and, with beta electrons, 8 * dim
 * doubles for the transposed vectors.  Calls on one handle share these
 * buffers and must be ordered.  Otherwise asynchronous on
 * `stream`.  Errors: ISCI_E_INVALID for NULL pointers, nvec or ldc out of
 * range, overlap; ISCI_E_OOM if the buffer cannot be allocated. */
isci_status isci_density1(isci_handle hd, int nvec, const double *c, int64_t ldc, double *d1,
                          hipStream_t stream);

/* Two-body density matrices of each vector by spin block (the paper's
 * density matrices, Eq. d2, with spin-orbital indices):
 *   d2[(((v * 3 + b) * norb + p) * norb + q) * norb^2 + r * norb + s]
 *     = <c_v| a+_{p S} a+_{r S'} a_{s S'} a_{q S} |c_v>,
 * b = 0: S = S' = alpha; b = 1: S = alpha, S' = beta; b = 2: S = S' = beta
 * (the block S = beta, S' = alpha is block 1 with (p, q) and (r, s)
 * exchanged), for v < nvec (1..65535).  The energy of a vector is
 * sum_pq h_pq D1_pq + 1/2 sum_pqrs (pq|rs) D2_pqrs summed over the spin
 * blocks.  Two electrons of each spin and at most 128 orbitals
 * (ISCI_E_UNSUPPORTED otherwise).  Each block is a Gram product on the
 * matrix cores: same-spin blocks from the rows of c (alpha) or of its
 * spin-swapped copy (beta), the alpha-beta block from the pair tensor
 * M[(p, r)][(x, y)] = sgn(p - x) sgn(r - y) c({x, p}, {y, r}).  c: device,
 * nvec vectors with leading dimension ldc >= dim, not normalised by the
 * call; d2: device, nvec * 3 * norb^4 doubles, overwritten, must not
 * overlap c.  The screening threshold plays no part.  Deterministic.  The
 * handle allocates on its first call, and keeps until it is destroyed,
 * about 16 norb^4 + 8 dim bytes of scratch.  Calls on one handle share it
 * and must be ordered; otherwise asynchronous on `stream`.  Errors:
 * ISCI_E_INVALID for NULL pointers, nvec or ldc out of range, overlap;
 * ISCI_E_OOM if the scratch cannot be allocated. */
isci_status isci_density2(isci_handle hd, int nvec, const double *c, int64_t ldc, double *d2,
                          hipStream_t stream);

/* isci_density1 without any device allocation, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc).  Same arguments, results and
 * errors as isci_density1 (bit for bit the same d1), but the partial sums
 * and the transposed vectors live in a static 64 MiB device array of the
 * library (one per GPU, held until the process ends) instead of buffers
 * owned by the handle; the vectors go through it in passes of up to eight,
 * as many as fit.  ISCI_E_UNSUPPORTED (with a message naming the bytes
 * needed) when one vector does not fit: 8 * (64 norb^2 + dim) bytes with
 * beta electrons, 8 * 64 norb^2 without; ISCI_E_INVALID when the current
 * device is not the handle's.  Calls on one GPU share the array, so calls
 * that overlap in time on one GPU (different streams, threads or handles)
 * race: order them.  The array needs no initial contents. */
isci_status isci_density1_noalloc(isci_handle hd, int nvec, const double *c, int64_t ldc, double *d1,
                                  hipStream_t stream);

/* Lowest nroots eigenpairs of H_tau, the eigenvalue problem of Eq. hcec
 * that the paper solves by repeated sigma steps (Eq. sigma) inside an
 * iterative optimiser (Davidson or Lanczos, in the text after Eq. sigma):
 * here block Davidson (FP64, device resident; the small projected
 * eigenproblem is solved on the host), with the diagonal of isci_diag as
 * preconditioner.  Errors: ISCI_E_INVALID for NULL hd or energies, nroots
 * outside [1, min(dim, ISCI_MAX_ROOTS)] or bad options; ISCI_E_OOM when the
 * subspace does not fit; ISCI_E_HIP on a runtime failure.  guess: device
 * [nguess][dim] or NULL (unit vectors on the lowest diagonal entries,
 * ties to the lowest address).  energies: host [nroots].  vectors: device
 * [nroots][dim] or NULL.  info may be NULL.  Returns ISCI_E_NOT_CONVERGED
 * with the best estimates when max_iter is reached. */
isci_status isci_davidson(isci_handle hd, int nroots, const isci_davidson_opts *opts,
                          const double *guess, int nguess, double *energies, double *vectors,
                          isci_davidson_info *info, hipStream_t stream);

/* Propagation of CI vectors under H_tau by the short-iterative
 * Arnoldi-Lanczos method: the optimiser the paper uses for the CI
 * coefficients (propagation in imaginary time, application section: thousands
 * of sigma steps), and real-time propagation for dynamics.  Each of nsteps
 * steps of length dt builds a Krylov basis of H_tau from the current vector
 * (each new direction orthogonalised against the two latest basis vectors
 * and then once against the whole basis), stops when
 * the residual estimate of the step falls below tol |u| or at `krylov`
 * vectors, and applies exp(-T dt) (imaginary) or exp(-i T dt) (real) of the
 * projected matrix.  Coefficient screening (the paper's proposal in its
 * section on the distribution of coefficients): after every step the
 * elements of modulus <= coef_tau are set to zero (0: off).
 *   imaginary = 1: c_re (device [dim]) <- exp(-H dt) c_re, normalised after
 *                  every step; c_im is not read (may be NULL);
 *   imaginary = 0: c_re + i c_im <- exp(-i H dt) (c_re + i c_im) (both device
 *                  [dim], distinct).
 * Vectors are updated in place.  The call allocates its Krylov basis
 * ((krylov + 1) dim doubles per real chain) for its own duration and
 * synchronises the stream once per Krylov vector (the stopping test runs
 * small host eigenproblems).  info (may be NULL): energy <c|H|c>/<c|c> of the result
 * (one more sigma), its norm, sigma vectors computed, Krylov size of the
 * last step and coefficients zeroed by the last screening.  Errors:
 * ISCI_E_INVALID for NULL handle or c_re, a missing or aliased c_im in real
 * time, dt negative or not finite, nsteps < 0, krylov outside 1..128,
 * negative tol or coef_tau; ISCI_E_OOM when the basis does not fit. */
typedef struct {
    int krylov;         /* largest Krylov basis per step (default 16) */
    int imaginary;      /* 1: imaginary time (default), 0: real time */
    double tol;         /* Krylov residual tolerance relative to |u| (default 1e-12) */
    double coef_tau;    /* coefficient screening threshold (default 0: off) */
} isci_propagate_opts;

typedef struct {
    double energy;
    double norm;
    int sigma_calls;
    int krylov_last;
    int64_t screened_last;
} isci_propagate_info;

void isci_propagate_defaults(isci_propagate_opts *o);
isci_status isci_propagate(isci_handle hd, double *c_re, double *c_im, double dt, int nsteps,
                           const isci_propagate_opts *opts, isci_propagate_info *info, hipStream_t stream);

/* Host copies of the string tables of one spin: the occupation strings
 * that build the determinants of Eq. ci_ansatz, with their excitation
 * level (electrons in virtual orbitals, the particle rank of the spin's
 * part of the excitation operator of Eq. ci_hierarchy).  orbitals
 * [nstr][n] (ascending) and level [nstr] in layout order, host arrays
 * owned by the caller; either pointer may be NULL; *nstr (host) receives
 * the count.  spin 0 is alpha, 1 beta.  ISCI_E_INVALID for a NULL handle,
 * a NULL nstr or spin outside {0, 1}.  No device work. */
isci_status isci_strings(isci_handle hd, int spin, int32_t *orbitals, int32_t *level,
                         int64_t *nstr);

/* Host copy of the row starts of the vector layout (the alpha-major
 * arrangement of the space of Eqs. ci_ansatz / ci_hierarchy described at
 * the top of this file): rowstart[nstr_alpha + 1], host array owned by
 * the caller; row Ia occupies [rowstart[Ia], rowstart[Ia + 1]).
 * ISCI_E_INVALID for NULL arguments.  No device work. */
isci_status isci_rowstart(isci_handle hd, int64_t *rowstart);

/* Screening statistics (host struct). */
isci_status isci_get_stats(isci_handle hd, isci_stats *s);

/* ---------------------------------------------------------------------
 * Multi-instance eigensolver engine (batched and served Davidson solves).
 *
 * An engine owns a stream and any number of Davidson solves ("slots"),
 * each on its own handle.  isci_engine_step advances every unfinished slot
 * by one Davidson iteration: one fused sigma launch covers the new basis
 * vectors of all slots (a persistent grid over a work list of (slot, alpha
 * row, beta block) items, heaviest first), followed by each slot's block
 * algebra; three host synchronisations per step serve all slots together.
 * Slots may be added and released between steps (continuous batching).
 * A slot's arithmetic does not depend on which other slots share the
 * engine, so a solve gives the same energies alone or in a mix.
 * isci_davidson is an engine with a single slot.
 * ------------------------------------------------------------------- */
typedef struct isci_engine_s *isci_engine;

isci_status isci_engine_create(isci_engine *out, hipStream_t stream);

/* Launch shape of the fused sigma: grid = persistent workgroups (0: one per
 * work item); heaviest_first orders work items by estimated cost. */
isci_status isci_engine_config(isci_engine e, int grid, int heaviest_first);

/* Admit a Davidson solve (allocates its subspace on the device, builds the
 * initial basis; synchronises the engine stream).  guess as in
 * isci_davidson.  *slot receives the slot id. */
isci_status isci_engine_add(isci_engine e, isci_handle hd, int nroots, const isci_davidson_opts *opts,
                            const double *guess, int nguess, int *slot);

/* One Davidson iteration for every unfinished slot; *nactive (may be
 * NULL) receives the number of slots that were advanced. */
isci_status isci_engine_step(isci_engine e, int *nactive);

/* State of a slot: *done = 1 when converged or stopped.  energies (host
 * [nroots]) hold the current Ritz values; vectors (device [nroots][dim])
 * are written only when done.  Returns the slot's final status once done
 * (ISCI_OK or ISCI_E_NOT_CONVERGED), ISCI_OK before. */
isci_status isci_engine_result(isci_engine e, int slot, int *done, double *energies, double *vectors,
                               isci_davidson_info *info);

/* Free a slot's device memory (its id may be reused). */
isci_status isci_engine_release(isci_engine e, int slot);

/* Fused sigma over n handles in one launch on the engine stream:
 * sigma_i = H_i c_i for nvec[i] vectors with leading dimensions ldc[i],
 * lds[i] (host arrays of device pointers).  Asynchronous. */
isci_status isci_engine_sigma(isci_engine e, int n, const isci_handle *hds, const int *nvec,
                              const double *const *c, const int64_t *ldc, double *const *sigma,
                              const int64_t *lds);

void isci_engine_destroy(isci_engine e);

/* Device bytes a Davidson solve of nroots roots on this handle allocates
 * (the admission footprint; the handle's own tables are in
 * isci_stats.device_bytes).  -1 on bad arguments. */
int64_t isci_davidson_footprint(isci_handle hd, int nroots, const isci_davidson_opts *opts);

/* Per-handle options.
 *   ISCI_OPT_SIGMA_KERNEL: ISCI_SIGMA_AUTO (default: two electrons per spin
 *   use the matrix-core path; other electron counts the general kernel),
 *   ISCI_SIGMA_GENERAL
 *   (string algebra for any electron count), ISCI_SIGMA_PAIR (two-electron
 *   pair tables; ISCI_E_UNSUPPORTED otherwise), ISCI_SIGMA_MFMA (pair
 *   tables, alpha-beta class on FP64 matrix cores; two electrons per spin).
 *   All give the same sigma up to rounding. */
#define ISCI_OPT_SIGMA_KERNEL 1
#define ISCI_SIGMA_AUTO 0
#define ISCI_SIGMA_GENERAL 1
#define ISCI_SIGMA_PAIR 2
#define ISCI_SIGMA_MFMA 3   /* FP64 matrix cores for the alpha-beta and one-body classes, pair kernel for same-spin */
/*   ISCI_OPT_AB_PATH (matrix-core path only): ISCI_AB_AUTO (default: the
 *   unfold / block-sparse product / fold path whenever its operands were
 *   built, i.e. fit in 2 GiB), ISCI_AB_GATHER (the gathered tile kernel).
 *   Both give the same sigma up to rounding. */
#define ISCI_OPT_AB_PATH 2
#define ISCI_AB_AUTO 0
#define ISCI_AB_GATHER 1
/*   ISCI_OPT_AB_PRODUCT (unfold / product / fold path only, for tuning):
 *   the kernel of the block-sparse product (the alpha-beta classes, Eqs.
 *   h200ca..h200ab among them, as one screened matrix of (pq|rs) applied
 *   to the unfolded vectors), one row block pair per workgroup tile:
 *   ISCI_AB_PACKED (default) as WIDE over packed chunks (per row block
 *   pair and source class, the (q, s) columns that hold a kept value, four
 *   per chunk: no all-zero K column); ISCI_AB_WIDE with a two-chunk
 *   ping-pong and 16-byte operand loads and stores (two adjacent columns
 *   per lane) over the (q, four-orbital block of s) chunks; ISCI_AB_PLAIN
 *   the same with 8-byte ones; ISCI_AB_PIPE with an explicit two-stage
 *   software pipeline (chunk table read one stage early).  Same sigma up to
 *   rounding order (WIDE and PLAIN: the same sums in the same order, bit
 *   for bit). */
#define ISCI_OPT_AB_PRODUCT 3
#define ISCI_AB_PLAIN 0
#define ISCI_AB_PIPE 1
#define ISCI_AB_WIDE 2
#define ISCI_AB_PACKED 3
/*   ISCI_OPT_ONEBODY_KERNEL (matrix-core one-body classes up to 80
 *   orbitals, for tuning): ISCI_ONEBODY_TRANSPOSED (default) runs the alpha
 *   class on the beta columns that hold every alpha pair (all columns in
 *   full CI, those of level <= L - 2 otherwise) as the beta class of that
 *   block transposed (contiguous rows); ISCI_ONEBODY_SINGLE takes two
 *   columns per workgroup there;
 *   ISCI_ONEBODY_SPECTATOR runs the whole alpha class in the spectator form
 *   used above 80 orbitals (U[a][x][j] = sum_q h_aq T_j[q][x], the rows
 *   {q, x} read directly, no transposes).  Above 80 orbitals the option
 *   picks the beta class: ISCI_ONEBODY_ROWS (default there for the
 *   excitation hierarchy where a row holding every beta pair fits a
 *   workgroup's LDS, up to 202 orbitals; ISCI_E_UNSUPPORTED elsewhere) runs
 *   it on the rows themselves, any other value as the alpha class of the
 *   transposed block.  Same sigma up to rounding order. */
#define ISCI_OPT_ONEBODY_KERNEL 5
#define ISCI_ONEBODY_SINGLE 1
#define ISCI_ONEBODY_TRANSPOSED 2
#define ISCI_ONEBODY_SPECTATOR 3
#define ISCI_ONEBODY_ROWS 4
/*   ISCI_OPT_ONEBODY_STREAM (matrix-core path with separate one-body
 *   kernels, for tuning): ISCI_ONEBODY_SIDE (default) runs the one-body
 *   classes on the handle's side stream beside the alpha-beta unfolds and
 *   products; ISCI_ONEBODY_INLINE runs them before those on the caller's
 *   stream.  The same kernels in the same order per element: identical
 *   sigma. */
#define ISCI_OPT_ONEBODY_STREAM 6
#define ISCI_ONEBODY_SIDE 0
#define ISCI_ONEBODY_INLINE 1
isci_status isci_set_option(isci_handle hd, int option, int value);

/* Kernel timing hook (for measurement).  When enabled, HIP events are
 * recorded on the launch stream around every sigma kernel launch of the
 * handle; isci_profile_read synchronises those events and returns the
 * summed milliseconds and launch count of one kernel since the last read,
 * then clears them.  Kernel ids: */
#define ISCI_KERNEL_GENERAL 0   /* k_sigma_generic: all classes, any electron count */
#define ISCI_KERNEL_PAIR 1      /* k_sigma_n2: all classes, two electrons per spin */
#define ISCI_KERNEL_AB_MFMA 2   /* k_sigma_ab_mfma: alpha-beta class on matrix cores, gathered operands
                                   (when the product path's operands would exceed 2 GiB) */
#define ISCI_KERNEL_PAIR_REST 3 /* k_sigma_n2 restricted to the classes the MFMA path leaves */
#define ISCI_KERNEL_ONEBODY 4   /* one-body classes, two electrons per spin (matrix-core products, or
                                   k_ob_alpha_spec, also on the transposed block for beta, above 80 orbitals) */
#define ISCI_KERNEL_AB_UNFOLD 5 /* k_ab_unfold: alpha-beta class, CI block unfolded into the product operand */
#define ISCI_KERNEL_AB_GEMM 6   /* k_ab_gemm: alpha-beta class, block-sparse product on matrix cores */
#define ISCI_KERNEL_AB_FOLD 7   /* k_ab_fold: alpha-beta class, role readings summed into sigma */
isci_status isci_profile(isci_handle hd, int enable);
isci_status isci_profile_read(isci_handle hd, int kernel, double *total_ms, int64_t *launches);

/* Measurement aid (not part of the method), for benchmarks that re-measure
 * the chip's FP64 peaks: enqueues `blocks` workgroups of 256 threads that
 * each run `iters` steps of independent FP64 chains on register operands,
 * kind 0 on the matrix cores (16x16x4 MFMA, eight chains per wave), kind 1
 * as vector FMAs (sixteen chains per lane), and write one value per thread
 * to out (device, blocks * 256 doubles).  *flops receives the floating-point
 * operations enqueued; time the call with events on `stream`. */
isci_status isci_probe_fp64(int kind, int64_t iters, int blocks, double *out, double *flops,
                            hipStream_t stream);

void isci_destroy(isci_handle hd);
const char *isci_status_string(isci_status s);
const char *isci_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* ISCI_H */
