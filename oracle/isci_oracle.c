/*
 * TEST INFRASTRUCTURE ONLY.  Plain, slow CPU oracle for the sigma step of
 * the Integral Screened Configuration Interaction (ISCI) method (Sorensen,
 * Bauch & Madsen, "The Integral Screened Configuration Interaction
 * Method").  Only tests/, the smoke check and the benchmark's CPU-baseline
 * leg may load this library.  It shares no code with the HIP library.
 *
 * What is computed -- the plain definition, not the paper's algorithm:
 *
 *   sigma_I = sum_J (H_tau)_IJ c_J
 *
 * where H_tau is the CI Hamiltonian (Eq. ham / index_un, spin-restricted,
 * g_pqrs = (pq|rs) in chemists' order) in the truncated CI space
 * (Eq. ci_ansatz / ci_hierarchy: all determinants whose alpha plus beta
 * excitation level is at most L), with every elementary integral unit of
 * magnitude <= tau removed (Eq. sigma_int / sigma_split).  Matrix elements
 * are Slater-Condon sums of such units; each unit is kept iff |unit| > tau:
 *
 *   diagonal:      [h_pp] per occupied p (both spins)
 *                  [(pp|qq) - (pq|qp)] per same-spin occupied pair p<q
 *                  [(pp|qq)] per alpha p, beta q
 *   single q->p:   sign * ( [h_pq] + sum_{k same spin, common} [(pq|kk) - (pk|kq)]
 *                                  + sum_{k opposite spin}      [(pq|kk)] )
 *   double same:   sign * [(pq|rs) - (ps|rq)]      ({q,s} -> {p,r})
 *   double ab:     sign * [(pq|rs)]                (alpha q->p, beta s->r)
 *
 * The same-spin unit is the antisymmetrised coefficient of Eq. index_re
 * (formed by one subtraction), the alpha-beta unit the raw (pq|rs).
 * Signs come from applying the operator word to the ordered creator list
 * of J and counting transpositions, the symbolic manipulation described
 * with Eqs. contract and add: an annihilator is moved to its partner
 * (sign (-1)^position), a creator is prepended and then sorted into place
 * (sign (-1)^inversions).  A determinant is the product of alpha creators
 * (ascending orbital) followed by beta creators (ascending), alpha before
 * beta as in Eq. index_re.
 *
 * Integrals are read through their canonical representative
 * (p>=q, r>=s, (p,q)>=(r,s); h with p>=q), so every unit is formed from
 * the same doubles whatever the labelling.
 *
 * Blocks guarded by ORC_PLANT_* macros are deliberate mistakes used only
 * by the mutation test (tests/test_oracle_mutants.py), which checks that
 * the pins catch them; the normal build defines none of them.
 *
 * Layout of the CI vector: per spin the strings (ascending orbital sets of
 * n electrons) are sorted by excitation level (number of electrons in
 * orbitals >= n, the reference occupying 0..n-1) and then in colex order
 * (highest orbital compared first).  Row Ia (alpha string) holds the beta
 * strings of level <= L - level(Ia), which is a prefix of the beta order;
 * addr = rowstart(Ia) + index(Ib).
 *
 * Two-space GAS restriction (section "Generalized Active Space"): with a
 * boundary orbital b (n <= b <= norb for both spins) the level of a string
 * is instead its number of electrons in orbitals >= b, so the space holds
 * every determinant of the orbitals 0..b-1 (full CI there) with at most L
 * electrons, alpha plus beta, in the outer space b..norb-1.  b = n per spin
 * is the CI hierarchy above.  The one-body/same-spin/alpha-beta bucket of a
 * unit classifies its orbitals as inner (< boundary) or outer.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OMAXN 16           /* electrons per spin */
#define OSPIN 1024         /* key offset of beta spin orbitals */
#define NBUCKET 42

typedef struct {
    int norb, n, maxlev, bnd;  /* bnd: level = # electrons in orbitals >= bnd */
    int64_t nstr;
    int32_t *orbs;         /* [nstr][n], ascending */
    int32_t *lev;          /* [nstr] */
} ostr_t;

typedef struct {
    int norb, na, nb, L;
    ostr_t a, b;
    int64_t *rowstart;     /* [a.nstr + 1] */
    int64_t *bprefix;      /* [L + 2]: # beta strings with level <= l */
    int64_t dim;
} ospace_t;

/* ------------------------------------------------------------------ */
/* strings                                                            */

static int g_cmp_n;        /* comparator context (setup is single threaded) */

static int cmp_level_colex(const int32_t *x, int lx, const int32_t *y, int ly, int n)
{
    if (lx != ly) return lx < ly ? -1 : 1;
    for (int i = n - 1; i >= 0; --i)
        if (x[i] != y[i]) return x[i] < y[i] ? -1 : 1;
    return 0;
}

typedef struct { int32_t lev; int32_t o[OMAXN]; } str_rec;

static int qsort_cmp(const void *pa, const void *pb)
{
    const str_rec *x = (const str_rec *)pa, *y = (const str_rec *)pb;
    return cmp_level_colex(x->o, x->lev, y->o, y->lev, g_cmp_n);
}

static int build_strings(ostr_t *S, int norb, int n, int maxlev, int bnd)
{
    S->norb = norb; S->n = n; S->maxlev = maxlev; S->bnd = bnd;
    /* count all n-subsets with level <= maxlev by enumeration */
    int64_t cap = 1024, cnt = 0;
    str_rec *buf = (str_rec *)malloc(sizeof(str_rec) * cap);
    if (!buf) return -1;
    int idx[OMAXN];
    for (int i = 0; i < n; ++i) idx[i] = i;
    for (;;) {
        int lev = 0;
#if defined(ORC_PLANT_GAS_LEVEL)
        for (int i = 0; i < n; ++i) lev += (idx[i] >= n);
#else
        for (int i = 0; i < n; ++i) lev += (idx[i] >= bnd);
#endif
        if (lev <= maxlev) {
            if (cnt == cap) {
                cap *= 2;
                str_rec *nb = (str_rec *)realloc(buf, sizeof(str_rec) * cap);
                if (!nb) { free(buf); return -1; }
                buf = nb;
            }
            memset(&buf[cnt], 0, sizeof(str_rec));
            buf[cnt].lev = lev;
            for (int i = 0; i < n; ++i) buf[cnt].o[i] = idx[i];
            cnt++;
        }
        /* next n-subset in lexicographic order */
        int i = n - 1;
        while (i >= 0 && idx[i] == norb - n + i) --i;
        if (i < 0) break;
        idx[i]++;
        for (int j = i + 1; j < n; ++j) idx[j] = idx[j - 1] + 1;
    }
    g_cmp_n = n;
    qsort(buf, (size_t)cnt, sizeof(str_rec), qsort_cmp);
    S->nstr = cnt;
    S->orbs = (int32_t *)malloc(sizeof(int32_t) * (size_t)(cnt * (n > 0 ? n : 1)));
    S->lev = (int32_t *)malloc(sizeof(int32_t) * (size_t)cnt);
    for (int64_t k = 0; k < cnt; ++k) {
        S->lev[k] = buf[k].lev;
        for (int i = 0; i < n; ++i) S->orbs[k * n + i] = buf[k].o[i];
    }
    free(buf);
    return 0;
}

/* index of a string (ascending orbitals o[], level lev) or -1 */
static int64_t find_string(const ostr_t *S, const int32_t *o, int lev)
{
    int64_t lo = 0, hi = S->nstr - 1;
    while (lo <= hi) {
        int64_t mid = (lo + hi) / 2;
        int c = cmp_level_colex(S->orbs + mid * S->n, S->lev[mid], o, lev, S->n);
        if (c == 0) return mid;
        if (c < 0) lo = mid + 1; else hi = mid - 1;
    }
    return -1;
}

static int level_of(const int32_t *o, int n, int bnd)
{
    int l = 0;
#if defined(ORC_PLANT_GAS_LEVEL)
    (void)bnd;
    for (int i = 0; i < n; ++i) l += (o[i] >= n);
#else
    for (int i = 0; i < n; ++i) l += (o[i] >= bnd);
#endif
    return l;
}

/* ------------------------------------------------------------------ */
/* operator words acting on ordered creator lists                     */

/* Apply word ops[0..nops-1] (leftmost first; the rightmost acts first) to
 * the product of creators keys[0..nk-1] acting on the vacuum.  type +1 is
 * a creator, -1 an annihilator.  Returns the number of creators left (in
 * product order) in out[], the sign in *sign, or -1 if the result is 0. */
static int apply_word(int nops, const int *type, const int *op, int nk, const int *keys,
                      int *out, int *sign)
{
    int list[2 * OMAXN + 8];
    int len = nk, s = 1;
    for (int i = 0; i < nk; ++i) list[i] = keys[i];
    for (int w = nops - 1; w >= 0; --w) {
        int k = op[w];
        int pos = -1;
        for (int i = 0; i < len; ++i) if (list[i] == k) { pos = i; break; }
        if (type[w] > 0) {
            if (pos >= 0) return -1;              /* a+_k a+_k = 0 */
            for (int i = len; i > 0; --i) list[i] = list[i - 1];
            list[0] = k;
            len++;
        } else {
            if (pos < 0) return -1;               /* a_k on a state without k */
            if (pos & 1) s = -s;                  /* move a_k past pos creators */
            for (int i = pos; i < len - 1; ++i) list[i] = list[i + 1];
            len--;
        }
    }
    for (int i = 0; i < len; ++i) out[i] = list[i];
    *sign = s;
    return len;
}

/* Sort a creator product into ascending (order=+1) or descending (order=-1)
 * order, multiplying *sign by (-1)^(number of transpositions). */
static void sort_creators(int len, int *list, int order, int *sign)
{
    for (int i = 1; i < len; ++i)                 /* insertion sort, adjacent swaps */
        for (int j = i; j > 0; --j) {
            int bad = order > 0 ? (list[j - 1] > list[j]) : (list[j - 1] < list[j]);
            if (!bad) break;
            int t = list[j]; list[j] = list[j - 1]; list[j - 1] = t;
            *sign = -*sign;
        }
}

/* <I| word |J> for determinants given as ascending key lists; returns 0 if
 * the word does not map J onto I. */
static int word_sign(int nops, const int *type, const int *op, int nj, const int *jkeys,
                     int ni, const int *ikeys)
{
    int out[2 * OMAXN + 8], s;
    int len = apply_word(nops, type, op, nj, jkeys, out, &s);
    if (len != ni) return 0;
    sort_creators(len, out, +1, &s);
    for (int i = 0; i < len; ++i) if (out[i] != ikeys[i]) return 0;
    return s;
}

/* ------------------------------------------------------------------ */
/* integrals through the canonical representative                     */

static inline double geri(const double *eri, int n, int p, int q, int r, int s)
{
    int t;
    if (p < q) { t = p; p = q; q = t; }
    if (r < s) { t = r; r = s; s = t; }
    if (p < r || (p == r && q < s)) { t = p; p = r; r = t; t = q; q = s; s = t; }
    return eri[(((int64_t)p * n + q) * n + r) * n + s];
}

static inline double gh(const double *h, int n, int p, int q)
{
    if (p < q) { int t = p; p = q; q = t; }
    return h[(int64_t)p * n + q];
}

/* ------------------------------------------------------------------ */
/* space                                                              */

/* bnd = 0: the CI hierarchy (boundary n per spin); else the two-space
 * restriction with boundary orbital bnd, max(na, nb) <= bnd <= norb */
static int space_init(ospace_t *S, int norb, int na, int nb, int L, int bnd)
{
    memset(S, 0, sizeof(*S));
    if (norb < 1 || na < 0 || nb < 0 || na > norb || nb > norb || L < 0) return -1;
    if (na > OMAXN || nb > OMAXN || norb >= OSPIN) return -1;
    if (bnd != 0 && (bnd < na || bnd < nb || bnd > norb)) return -1;
    S->norb = norb; S->na = na; S->nb = nb; S->L = L;
    if (build_strings(&S->a, norb, na, L, bnd ? bnd : na) || build_strings(&S->b, norb, nb, L, bnd ? bnd : nb))
        return -1;
    S->bprefix = (int64_t *)calloc((size_t)L + 2, sizeof(int64_t));
    for (int64_t k = 0; k < S->b.nstr; ++k)
        for (int l = S->b.lev[k]; l <= L; ++l) S->bprefix[l]++;
    S->rowstart = (int64_t *)malloc(sizeof(int64_t) * (size_t)(S->a.nstr + 1));
    int64_t acc = 0;
    for (int64_t k = 0; k < S->a.nstr; ++k) {
        S->rowstart[k] = acc;
        acc += S->bprefix[L - S->a.lev[k]];
    }
    S->rowstart[S->a.nstr] = acc;
    S->dim = acc;
    return 0;
}

static void space_free(ospace_t *S)
{
    free(S->a.orbs); free(S->a.lev); free(S->b.orbs); free(S->b.lev);
    free(S->rowstart); free(S->bprefix);
}

static int64_t row_of(const ospace_t *S, int64_t t)
{
    int64_t lo = 0, hi = S->a.nstr - 1;
    while (lo < hi) {                     /* last row with rowstart <= t */
        int64_t mid = (lo + hi + 1) / 2;
        if (S->rowstart[mid] <= t) lo = mid; else hi = mid - 1;
    }
    return lo;
}

/* address of (alpha orbitals, beta orbitals) or -1 if outside the space */
static int64_t address(const ospace_t *S, const int32_t *ao, const int32_t *bo)
{
    int la = level_of(ao, S->na, S->a.bnd), lb = level_of(bo, S->nb, S->b.bnd);
    if (la + lb > S->L) return -1;
    int64_t ia = find_string(&S->a, ao, la), ib = find_string(&S->b, bo, lb);
    if (ia < 0 || ib < 0) return -1;
    return S->rowstart[ia] + ib;
}

/* ------------------------------------------------------------------ */
/* visiting the units of one row of H                                  */

typedef struct {
    const double *h, *eri;
    double tau;
    int norb, na, nb;
} oints_t;

/* callback: J address, signed unit value (sign * unit), bucket, kept flag */
typedef void (*unit_fn)(void *ctx, int64_t j, double signed_unit, int bucket, int kept);

static inline int ev(int p, int nocc) { return p >= nocc; }

/* bucket numbering: 0..3 one-body alpha (e_p*2+e_q), 4..7 one-body beta,
 * 8..16 same-spin alpha (3*#virt creators + #virt annihilators), 17..25
 * same-spin beta, 26..41 alpha-beta (8 e_p + 4 e_q + 2 e_r + e_s). */
static inline int b_one(int spin, int p, int q, int nocc)
{ return 4 * spin + 2 * ev(p, nocc) + ev(q, nocc); }
static inline int b_ss(int spin, int p, int r, int q, int s, int nocc)
{ return 8 + 9 * spin + 3 * (ev(p, nocc) + ev(r, nocc)) + ev(q, nocc) + ev(s, nocc); }
static inline int b_ab(int p, int q, int r, int s, int na, int nb)
{ return 26 + 8 * ev(p, na) + 4 * ev(q, na) + 2 * ev(r, nb) + ev(s, nb); }

static inline void emit(unit_fn fn, void *ctx, const oints_t *I, int64_t j, int sign,
                        double unit, int bucket)
{
#if defined(ORC_PLANT_KEEP_GE)
    int kept = fabs(unit) >= I->tau;
#else
    int kept = fabs(unit) > I->tau;
#endif
    fn(ctx, j, sign * unit, bucket, kept);
}

static inline int contains(const int32_t *o, int n, int p)
{
    for (int i = 0; i < n; ++i) if (o[i] == p) return 1;
    return 0;
}

/* replace orbital `from` by `to` in the ascending list o (length n) -> out (ascending) */
static void replace_sorted(const int32_t *o, int n, int from, int to, int32_t *out)
{
    int k = 0;
    for (int i = 0; i < n; ++i) if (o[i] != from) out[k++] = o[i];
    out[k++] = to;
    for (int i = k - 1; i > 0 && out[i - 1] > out[i]; --i) { int32_t t = out[i]; out[i] = out[i - 1]; out[i - 1] = t; }
}

static void keys_of(const int32_t *ao, int na, const int32_t *bo, int nb, int *keys)
{
    for (int i = 0; i < na; ++i) keys[i] = ao[i];
    for (int i = 0; i < nb; ++i) keys[na + i] = OSPIN + bo[i];
}

static void visit_row(const ospace_t *S, const oints_t *I, int64_t t, unit_fn fn, void *ctx)
{
    const int n = S->norb, na = S->na, nb = S->nb;
    const int ba = S->a.bnd, bb = S->b.bnd;   /* bucket classification: inner / outer */
    int64_t ia = row_of(S, t), ib = t - S->rowstart[ia];
    const int32_t *A = S->a.orbs + ia * na, *B = S->b.orbs + ib * nb;
    int ikeys[2 * OMAXN], jkeys[2 * OMAXN];
    keys_of(A, na, B, nb, ikeys);
    const double *h = I->h, *eri = I->eri;

    /* ---- diagonal ---- */
    for (int i = 0; i < na; ++i) emit(fn, ctx, I, t, 1, gh(h, n, A[i], A[i]), b_one(0, A[i], A[i], ba));
    for (int i = 0; i < nb; ++i) emit(fn, ctx, I, t, 1, gh(h, n, B[i], B[i]), b_one(1, B[i], B[i], bb));
    for (int i = 0; i < na; ++i)
        for (int j = i + 1; j < na; ++j) {
            int p = A[i], q = A[j];
            emit(fn, ctx, I, t, 1, geri(eri, n, p, p, q, q) - geri(eri, n, p, q, q, p),
                 b_ss(0, p, q, p, q, ba));
        }
    for (int i = 0; i < nb; ++i)
        for (int j = i + 1; j < nb; ++j) {
            int p = B[i], q = B[j];
            emit(fn, ctx, I, t, 1, geri(eri, n, p, p, q, q) - geri(eri, n, p, q, q, p),
                 b_ss(1, p, q, p, q, bb));
        }
#if !defined(ORC_PLANT_DROP_AB_DIAG)
    for (int i = 0; i < na; ++i)
        for (int j = 0; j < nb; ++j)
            emit(fn, ctx, I, t, 1, geri(eri, n, A[i], A[i], B[j], B[j]),
                 b_ab(A[i], A[i], B[j], B[j], ba, bb));
#endif

    int32_t J[OMAXN];
    /* ---- single excitations J -> I, same spin q -> p ---- */
    for (int spin = 0; spin < 2; ++spin) {
        const int32_t *X = spin ? B : A;          /* string that changes */
        const int32_t *Y = spin ? A : B;          /* other spin, spectator */
        int nx = spin ? nb : na, ny = spin ? na : nb;
        int bx = spin ? bb : ba;
        for (int i = 0; i < nx; ++i) {
            int p = X[i];
            for (int q = 0; q < n; ++q) {
                if (contains(X, nx, q)) continue;
                replace_sorted(X, nx, p, q, J);
                int64_t jaddr = spin ? address(S, A, J) : address(S, J, B);
                if (jaddr < 0) continue;
                if (spin) keys_of(A, na, J, nb, jkeys); else keys_of(J, na, B, nb, jkeys);
                int off = spin ? OSPIN : 0;
                int ty[2] = {+1, -1}, op[2] = {off + p, off + q};
                int sg = word_sign(2, ty, op, na + nb, jkeys, na + nb, ikeys);
                if (!sg) continue;
#if defined(ORC_PLANT_SINGLE_NOSIGN)
                sg = 1;
#endif
                emit(fn, ctx, I, jaddr, sg, gh(h, n, p, q), b_one(spin, p, q, bx));
                for (int k = 0; k < nx; ++k) {
                    int kk = X[k];
                    if (kk == p) continue;        /* common occupied, same spin */
#if defined(ORC_PLANT_DROP_SS_SINGLE)
                    continue;
#endif
                    emit(fn, ctx, I, jaddr, sg,
                         geri(eri, n, p, q, kk, kk) - geri(eri, n, p, kk, kk, q),
                         b_ss(spin, p, kk, q, kk, bx));
                }
                for (int k = 0; k < ny; ++k) {
                    int kk = Y[k];
                    emit(fn, ctx, I, jaddr, sg, geri(eri, n, p, q, kk, kk),
                         spin ? b_ab(kk, kk, p, q, ba, bb) : b_ab(p, q, kk, kk, ba, bb));
                }
            }
        }
    }

    /* ---- same-spin doubles {q,s} -> {p,r} ---- */
    int32_t T[OMAXN];
    for (int spin = 0; spin < 2; ++spin) {
        const int32_t *X = spin ? B : A;
        int nx = spin ? nb : na;
        int bx = spin ? bb : ba;
        int off = spin ? OSPIN : 0;
        for (int i = 0; i < nx; ++i)
            for (int j = i + 1; j < nx; ++j) {
                int p = X[i], r = X[j];
                for (int q = 0; q < n; ++q) {
                    if (contains(X, nx, q)) continue;
                    for (int s = q + 1; s < n; ++s) {
                        if (contains(X, nx, s)) continue;
                        replace_sorted(X, nx, p, q, T);
                        replace_sorted(T, nx, r, s, J);
                        int64_t jaddr = spin ? address(S, A, J) : address(S, J, B);
                        if (jaddr < 0) continue;
                        if (spin) keys_of(A, na, J, nb, jkeys); else keys_of(J, na, B, nb, jkeys);
                        int ty[4] = {+1, +1, -1, -1};
                        int op[4] = {off + p, off + r, off + s, off + q};
                        int sg = word_sign(4, ty, op, na + nb, jkeys, na + nb, ikeys);
                        if (!sg) continue;
#if defined(ORC_PLANT_SS_EXCHANGE)
                        emit(fn, ctx, I, jaddr, sg,
                             geri(eri, n, p, q, r, s) + geri(eri, n, p, s, r, q),
                             b_ss(spin, p, r, q, s, bx));
#else
                        emit(fn, ctx, I, jaddr, sg,
                             geri(eri, n, p, q, r, s) - geri(eri, n, p, s, r, q),
                             b_ss(spin, p, r, q, s, bx));
#endif
                    }
                }
            }
    }

    /* ---- alpha-beta doubles: alpha q -> p, beta s -> r ---- */
    int32_t JA[OMAXN], JB[OMAXN];
    for (int i = 0; i < na; ++i) {
        int p = A[i];
        for (int q = 0; q < n; ++q) {
            if (contains(A, na, q)) continue;
            replace_sorted(A, na, p, q, JA);
            for (int k = 0; k < nb; ++k) {
                int r = B[k];
                for (int s = 0; s < n; ++s) {
                    if (contains(B, nb, s)) continue;
                    replace_sorted(B, nb, r, s, JB);
                    int64_t jaddr = address(S, JA, JB);
                    if (jaddr < 0) continue;
                    keys_of(JA, na, JB, nb, jkeys);
                    int ty[4] = {+1, +1, -1, -1};
                    int op[4] = {p, OSPIN + r, OSPIN + s, q};
                    int sg = word_sign(4, ty, op, na + nb, jkeys, na + nb, ikeys);
                    if (!sg) continue;
#if defined(ORC_PLANT_AB_SIGN)
                    sg = -sg;
#endif
#if defined(ORC_PLANT_AB_INDEX)
                    emit(fn, ctx, I, jaddr, sg, geri(eri, n, p, r, q, s), b_ab(p, q, r, s, ba, bb));
#else
                    emit(fn, ctx, I, jaddr, sg, geri(eri, n, p, q, r, s), b_ab(p, q, r, s, ba, bb));
#endif
                }
            }
        }
    }
}

/* ------------------------------------------------------------------ */
/* exported API (ctypes)                                               */

void *orc_space_create_gas(int norb, int na, int nb, int L, int bnd)
{
    ospace_t *S = (ospace_t *)calloc(1, sizeof(ospace_t));
    if (!S) return NULL;
    if (space_init(S, norb, na, nb, L, bnd)) { space_free(S); free(S); return NULL; }
    return S;
}

void *orc_space_create(int norb, int na, int nb, int L) { return orc_space_create_gas(norb, na, nb, L, 0); }

void orc_space_destroy(void *h) { if (h) { space_free((ospace_t *)h); free(h); } }
int64_t orc_space_dim(void *h) { return ((ospace_t *)h)->dim; }
int64_t orc_space_nstr(void *h, int spin) { ospace_t *S = (ospace_t *)h; return spin ? S->b.nstr : S->a.nstr; }

int orc_space_strings(void *h, int spin, int32_t *orbs, int32_t *lev)
{
    ospace_t *S = (ospace_t *)h;
    ostr_t *T = spin ? &S->b : &S->a;
    if (orbs && T->n) memcpy(orbs, T->orbs, sizeof(int32_t) * (size_t)(T->nstr * T->n));
    if (lev) memcpy(lev, T->lev, sizeof(int32_t) * (size_t)T->nstr);
    return 0;
}

int orc_space_rowstart(void *h, int64_t *rowstart)
{
    ospace_t *S = (ospace_t *)h;
    memcpy(rowstart, S->rowstart, sizeof(int64_t) * (size_t)(S->a.nstr + 1));
    return 0;
}

int64_t orc_space_address(void *h, const int32_t *ao, const int32_t *bo)
{
    return address((ospace_t *)h, ao, bo);
}

/* sigma */
typedef struct { int nvec; const double *c; int64_t ldc; long double acc[64]; } sig_ctx;

static void sig_cb(void *vctx, int64_t j, double su, int bucket, int kept)
{
    (void)bucket;
    if (!kept) return;
    sig_ctx *x = (sig_ctx *)vctx;
    for (int v = 0; v < x->nvec; ++v) x->acc[v] += (long double)su * (long double)x->c[v * x->ldc + j];
}

/* out[v * ntarget + i] = sigma_v(targets[i]); targets == NULL means all
 * addresses 0..dim-1 (then ntarget must equal dim). nvec <= 64. */
int orc_sigma(void *hs, const double *h, const double *eri, double tau, int nvec,
              const double *c, int64_t ldc, int64_t ntarget, const int64_t *targets, double *out)
{
    ospace_t *S = (ospace_t *)hs;
    if (nvec < 1 || nvec > 64) return -1;
    oints_t I = {h, eri, tau, S->norb, S->na, S->nb};
    int64_t nt = targets ? ntarget : S->dim;
    #pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < nt; ++i) {
        int64_t t = targets ? targets[i] : i;
        sig_ctx x;
        x.nvec = nvec; x.c = c; x.ldc = ldc;
        for (int v = 0; v < nvec; ++v) x.acc[v] = 0.0L;
        visit_row(S, &I, t, sig_cb, &x);
        for (int v = 0; v < nvec; ++v) out[(int64_t)v * nt + i] = (double)x.acc[v];
    }
    return 0;
}

/* diagonal H_II (kept units only) */
typedef struct { int64_t self; long double acc; } diag_ctx;
static void diag_cb(void *vctx, int64_t j, double su, int bucket, int kept)
{
    (void)bucket;
    diag_ctx *x = (diag_ctx *)vctx;
#if defined(ORC_PLANT_DIAG_ROWSUM)
    (void)j;
    if (kept) x->acc += su;
#elif defined(ORC_PLANT_DIAG_UNSCREENED)
    (void)kept;
    if (j == x->self) x->acc += su;
#else
    if (kept && j == x->self) x->acc += su;
#endif
}

int orc_diag(void *hs, const double *h, const double *eri, double tau,
             int64_t ntarget, const int64_t *targets, double *out)
{
    ospace_t *S = (ospace_t *)hs;
    oints_t I = {h, eri, tau, S->norb, S->na, S->nb};
    int64_t nt = targets ? ntarget : S->dim;
    #pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < nt; ++i) {
        int64_t t = targets ? targets[i] : i;
        diag_ctx x = {t, 0.0L};
        visit_row(S, &I, t, diag_cb, &x);
        out[i] = (double)x.acc;
    }
    return 0;
}

/* per-bucket counts of kept (and all) units over the whole space */
typedef struct { int64_t kept[NBUCKET], all[NBUCKET]; } cnt_ctx;
static void cnt_cb(void *vctx, int64_t j, double su, int bucket, int kept)
{
    (void)j; (void)su;
    cnt_ctx *x = (cnt_ctx *)vctx;
    x->all[bucket]++;
    if (kept) x->kept[bucket]++;
}

int orc_terms(void *hs, const double *h, const double *eri, double tau,
              int64_t *kept, int64_t *all)
{
    ospace_t *S = (ospace_t *)hs;
    oints_t I = {h, eri, tau, S->norb, S->na, S->nb};
    for (int b = 0; b < NBUCKET; ++b) { kept[b] = 0; all[b] = 0; }
    #pragma omp parallel
    {
        cnt_ctx x;
        memset(&x, 0, sizeof(x));
        #pragma omp for schedule(dynamic, 16)
        for (int64_t t = 0; t < S->dim; ++t) visit_row(S, &I, t, cnt_cb, &x);
        #pragma omp critical
        for (int b = 0; b < NBUCKET; ++b) { kept[b] += x.kept[b]; all[b] += x.all[b]; }
    }
    return 0;
}

/* dense H_tau (row-major dim x dim) for tiny spaces */
typedef struct { double *row; } dense_ctx;
static void dense_cb(void *vctx, int64_t j, double su, int bucket, int kept)
{
    (void)bucket;
    if (kept) ((dense_ctx *)vctx)->row[j] += su;
}

int orc_dense_h(void *hs, const double *h, const double *eri, double tau, double *H)
{
    ospace_t *S = (ospace_t *)hs;
    oints_t I = {h, eri, tau, S->norb, S->na, S->nb};
    memset(H, 0, sizeof(double) * (size_t)(S->dim * S->dim));
    #pragma omp parallel for schedule(dynamic, 4)
    for (int64_t t = 0; t < S->dim; ++t) {
        dense_ctx x = {H + t * S->dim};
        visit_row(S, &I, t, dense_cb, &x);
    }
    return 0;
}

/* B(tau) = max_I sum_J |sum of dropped units in H_IJ|, an upper bound on
 * ||H_0 - H_tau||_2 (the matrix is symmetric, so the infinity norm bounds
 * the spectral norm). */
typedef struct { int64_t *js; double *vs; int64_t n, cap; } drop_ctx;
static void drop_cb(void *vctx, int64_t j, double su, int bucket, int kept)
{
    (void)bucket;
    if (kept) return;
    drop_ctx *x = (drop_ctx *)vctx;
    for (int64_t i = 0; i < x->n; ++i) if (x->js[i] == j) { x->vs[i] += su; return; }
    if (x->n == x->cap) {
        x->cap = x->cap ? 2 * x->cap : 256;
        x->js = (int64_t *)realloc(x->js, sizeof(int64_t) * (size_t)x->cap);
        x->vs = (double *)realloc(x->vs, sizeof(double) * (size_t)x->cap);
    }
    x->js[x->n] = j; x->vs[x->n] = su; x->n++;
}

int orc_dropped_bound(void *hs, const double *h, const double *eri, double tau, double *bound)
{
    ospace_t *S = (ospace_t *)hs;
    oints_t I = {h, eri, tau, S->norb, S->na, S->nb};
    double best = 0.0;
    #pragma omp parallel
    {
        drop_ctx x = {NULL, NULL, 0, 0};
        double mine = 0.0;
        #pragma omp for schedule(dynamic, 16)
        for (int64_t t = 0; t < S->dim; ++t) {
            x.n = 0;
            visit_row(S, &I, t, drop_cb, &x);
            double r = 0.0;
            for (int64_t i = 0; i < x.n; ++i) r += fabs(x.vs[i]);
            if (r > mine) mine = r;
        }
        #pragma omp critical
        if (mine > best) best = mine;
        free(x.js); free(x.vs);
    }
    *bound = best;
    return 0;
}

/* Symbolic manipulation of an operator word on the vacuum (Eqs. contract
 * and add): ops given left to right; returns the number of creators left
 * (written to out[] in product order, then sorted if order != 0), the sign
 * in *sign, or -1 when the word annihilates the vacuum. */
int orc_apply_word(int nops, const int *type, const int *op, int order, int *out, int *sign)
{
    if (nops > 2 * OMAXN) return -2;
    int len = apply_word(nops, type, op, 0, NULL, out, sign);
    if (len < 0) return -1;
    if (order) sort_creators(len, out, order, sign);
    return len;
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
