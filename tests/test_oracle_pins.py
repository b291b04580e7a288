"""Pins of the CPU oracle against facts the paper and the mathematics fix.

None of these tests compares the oracle with itself: each check is an
independent construction (closed forms, textbook linear algebra, the
paper's printed numbers and worked examples, an integral-driven count).
"""
import os
from itertools import combinations
from math import comb

import numpy as np
import pytest

import oracle as O
from isci_inputs import recipe_a, recipe_b, recipe_random, random_vectors

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- P1
def _table_norb():
    rows = []
    for line in open(os.path.join(GOLDEN, "table_norb.txt")):
        line = line.split("#")[0].strip()
        if not line:
            continue
        f = line.split()
        rows.append((int(f[0]), int(f[1]), [None if x == "-" else int(x) for x in f[2:5]]))
    return rows


def test_table_norb_closed_form():
    """Closed-form dimension reproduces every entry of the paper's table."""
    rows = _table_norb()
    assert len(rows) == 15
    n = 0
    for _R, norb, counts in rows:
        for L, want in zip((2, 3, 4), counts):
            if want is None:
                continue
            assert O.dim_closed_form(norb, 2, 2, L) == want
            n += 1
    assert n == 15 + 7 + 5


@pytest.mark.parametrize("norb,L", [(106, 2), (142, 2), (106, 3), (250, 2)])
def test_table_norb_enumeration(norb, L):
    """The oracle's explicit string enumeration and row layout give the
    paper's printed counts."""
    want = {r[1]: r[2] for r in _table_norb()}[norb][L - 2]
    S = O.Space(norb, 2, 2, L)
    assert S.dim == want


def _brute_dets(norb, na, nb, L):
    out = []
    for a in combinations(range(norb), na):
        la = sum(x >= na for x in a)
        for b in combinations(range(norb), nb):
            lb = sum(x >= nb for x in b)
            if la + lb <= L:
                out.append((a, b))
    return out


@pytest.mark.parametrize("norb,na,nb,L", [(7, 2, 2, 2), (8, 2, 2, 3), (6, 3, 2, 2),
                                          (6, 2, 2, 4), (5, 1, 2, 1), (6, 0, 2, 2),
                                          (7, 3, 3, 6)])
def test_layout_brute_force(norb, na, nb, L):
    """Every determinant appears exactly once; rows are alpha strings in
    (level, colex) order; each row holds a prefix of the beta order."""
    S = O.Space(norb, na, nb, L)
    dets = S.determinants()
    brute = _brute_dets(norb, na, nb, L)
    assert S.dim == len(brute) == len(set(dets))
    assert set(dets) == set(brute)

    def key(s, n):
        return (sum(x >= n for x in s), tuple(sorted(s, reverse=True)))

    ao, _ = S.strings(0)
    bo, _ = S.strings(1)
    ka = [key(tuple(r), na) for r in ao]
    kb = [key(tuple(r), nb) for r in bo]
    assert ka == sorted(ka) and kb == sorted(kb)
    for i, (a, b) in enumerate(dets):
        assert S.address(a, b) == i


# ---------------------------------------------------------------- P2
def _sign_examples():
    m = {"a": 1, "b": 2, "c": 3, "d": 4}
    for line in open(os.path.join(GOLDEN, "sign_examples.txt")):
        line = line.split("#")[0].strip()
        if not line:
            continue
        name, word, order, sign, res = [x.strip() for x in line.split("|")]
        ops = [(tok[0], m[tok[1]]) for tok in word.split()]
        yield name, ops, {"none": 0, "desc": -1, "asc": 1}[order], int(sign), [m[x] for x in res.split()]


@pytest.mark.parametrize("ex", list(_sign_examples()), ids=lambda e: e[0])
def test_paper_sign_examples(ex):
    _name, ops, order, sign, res = ex
    s, out = O.apply_word(ops, order)
    assert (s, out) == (sign, res)


def test_word_vanishing_cases():
    # a contraction that does not match returns no string
    assert O.apply_word([("-", 2), ("-", 1), ("+", 4), ("+", 3), ("+", 1)]) == (0, None)
    assert O.apply_word([("+", 1), ("+", 1)]) == (0, None)


# ---------------------------------------------------------------- P4
@pytest.mark.parametrize("recipe", ["A", "B", "R"])
@pytest.mark.parametrize("na,nb", [(2, 2), (3, 1), (1, 0)])
def test_reference_energy_closed_form(recipe, na, nb):
    norb = 7
    h, eri = _ints(recipe, norb, 3)
    S = O.Space(norb, na, nb, 2)
    e0 = np.zeros((1, S.dim))
    e0[0, 0] = 1.0
    sig = O.sigma(S, h, eri, 0.0, e0, targets=[0])[0, 0]
    assert abs(sig - O.e_ref_closed_form(h, eri, na, nb)) <= 1e-12 * max(1.0, abs(sig))


def _ints(recipe, norb, seed):
    if recipe == "A":
        return recipe_a(norb, seed=seed)
    if recipe == "B":
        return recipe_b(norb, seed=seed)
    return recipe_random(norb, seed=seed)


# ---------------------------------------------------------------- P5
@pytest.mark.parametrize("recipe", ["A", "B", "R"])
@pytest.mark.parametrize("norb,na,nb,L,tau", [(7, 2, 2, 2, 0.0), (7, 2, 2, 3, 1e-6),
                                              (6, 3, 2, 3, 0.0), (8, 2, 2, 4, 1e-3)])
def test_hermiticity(recipe, norb, na, nb, L, tau):
    h, eri = _ints(recipe, norb, 5)
    S = O.Space(norb, na, nb, L)
    H = O.dense_h(S, h, eri, tau)
    assert np.abs(H - H.T).max() <= 1e-13 * np.abs(H).max()
    u, v = random_vectors(S.dim, 2, 9)
    su, sv = O.sigma(S, h, eri, tau, np.stack([u, v]))
    assert abs(u @ sv - v @ su) <= 1e-12 * np.linalg.norm(u) * np.linalg.norm(v) * np.abs(H).max()


# ---------------------------------------------------------------- diagonal
def _slater_condon_diag(h, eri, A, B, tau):
    """Textbook Slater-Condon diagonal of the determinant with alpha
    orbitals A and beta orbitals B, as a sum of units (h_pp; per same-spin
    pair (pp|qq) - (pq|qp) formed by one subtraction; per alpha-beta pair
    (pp|qq)), each kept iff |unit| > tau."""
    units = [h[p, p] for p in A] + [h[p, p] for p in B]
    for S in (A, B):
        units += [eri[p, p, q, q] - eri[p, q, q, p] for i, p in enumerate(S) for q in S[i + 1:]]
    units += [eri[p, p, q, q] for p in A for q in B]
    return sum(u for u in units if abs(u) > tau)


@pytest.mark.parametrize("recipe", ["A", "B", "R"])
@pytest.mark.parametrize("norb,na,nb,L,tau", [(7, 2, 2, 2, 0.0), (7, 2, 2, 3, 1e-6), (6, 3, 2, 3, 0.0),
                                              (8, 2, 2, 4, 1e-3), (7, 3, 2, 3, 0.2), (6, 1, 1, 2, 0.05)])
def test_diag_slater_condon_and_dense_diagonal(recipe, norb, na, nb, L, tau):
    """The oracle diagonal (section on diagonal classes; Eq. ham) equals the
    Slater-Condon diagonal of every determinant, unit by unit under the
    strict keep rule, and the diagonal of the dense H_tau."""
    h, eri = _ints(recipe, norb, 5)
    h = 0.5 * (h + h.T)
    S = O.Space(norb, na, nb, L)
    d = O.diag(S, h, eri, tau)
    H = O.dense_h(S, h, eri, tau)
    scale = max(1.0, np.abs(d).max())
    assert np.abs(d - np.diag(H)).max() <= 1e-14 * scale
    ao, _ = S.strings(0)
    bo, _ = S.strings(1)
    rs = S.rowstart()
    ref = np.empty(S.dim)
    for ia in range(len(rs) - 1):
        for j in range(rs[ia + 1] - rs[ia]):
            ref[rs[ia] + j] = _slater_condon_diag(h, eri, list(ao[ia]), list(bo[j]), tau)
    assert np.abs(d - ref).max() <= 1e-13 * scale


def test_diag_closed_shell_relabelled_reference():
    """A closed-shell determinant (same orbitals in both spins) is the
    reference of the Hamiltonian with its orbitals relabelled to 0..n-1, so
    its diagonal element is that Hamiltonian's closed-form E_ref."""
    norb, n, L = 7, 2, 4
    h, eri = _ints("R", norb, 8)
    S = O.Space(norb, n, n, L)
    d = O.diag(S, h, eri, 0.0)
    ao, _ = S.strings(0)
    rs = S.rowstart()
    bo, _ = S.strings(1)
    checked = 0
    for ia in range(len(rs) - 1):
        for j in range(rs[ia + 1] - rs[ia]):
            if list(ao[ia]) != list(bo[j]):
                continue
            occ = list(ao[ia])
            perm = occ + [p for p in range(norb) if p not in occ]
            hp = h[np.ix_(perm, perm)]
            ep = eri[np.ix_(perm, perm, perm, perm)]
            e = O.e_ref_closed_form(hp, ep, n, n)
            assert abs(d[rs[ia] + j] - e) <= 1e-13 * max(1.0, abs(e))
            checked += 1
    assert checked == comb(norb, n)


# ---------------------------------------------------------------- P7
def test_noninteracting_limit():
    """eri = 0: FCI ground energy is the sum of the lowest na + nb orbital
    energies, and the alpha one-body action on the antisymmetric pair
    tensor is T' = h T + T h^T."""
    norb = 7
    h, _ = recipe_random(norb, seed=2)
    eri = np.zeros((norb,) * 4)
    S = O.Space(norb, 2, 2, 4)
    w = np.linalg.eigvalsh(O.dense_h(S, h, eri, 0.0))
    eps = np.linalg.eigvalsh(h)
    assert abs(w[0] - (2 * eps[:2].sum())) <= 1e-11

    # pair-tensor check on one vector
    dets = S.determinants()
    c = random_vectors(S.dim, 1, 4)[0]
    T = np.zeros((norb, norb, norb, norb))
    for val, ((a1, a2), (b1, b2)) in zip(c, dets):
        for (x, y, sa) in ((a1, a2, 1), (a2, a1, -1)):
            for (u, v, sb) in ((b1, b2, 1), (b2, b1, -1)):
                T[x, y, u, v] = sa * sb * val
    Tp = (np.einsum("pq,qbcd->pbcd", h, T) + np.einsum("pq,aqcd->apcd", h, T)
          + np.einsum("pq,abqd->abpd", h, T) + np.einsum("pq,abcq->abcp", h, T))
    sig = O.sigma(S, h, eri, 0.0, c[None])[0]
    want = np.array([Tp[a1, a2, b1, b2] for ((a1, a2), (b1, b2)) in dets])
    assert np.abs(sig - want).max() <= 1e-12 * np.abs(want).max()


# ---------------------------------------------------------------- P8
@pytest.mark.parametrize("seed", [0, 1])
def test_one_electron_per_spin_kronecker(seed):
    """na = nb = 1 FCI: H = h (x) 1 + 1 (x) h + G, G[(p,r),(q,s)] = (pq|rs).
    With an unstructured eri this fixes the integral index order."""
    norb = 6
    h, eri = recipe_random(norb, seed=seed)
    S = O.Space(norb, 1, 1, 2)
    H = O.dense_h(S, h, eri, 0.0)
    dets = S.determinants()
    idx = [a[0] * norb + b[0] for a, b in dets]
    I = np.eye(norb)
    K = np.kron(h, I) + np.kron(I, h) + eri.transpose(0, 2, 1, 3).reshape(norb * norb, norb * norb)
    K = K[np.ix_(idx, idx)]
    assert np.abs(H - K).max() <= 1e-13


# ---------------------------------------------------------------- P9
def test_fci_orbital_rotation_invariance():
    norb = 6
    h, eri = recipe_random(norb, seed=7)
    rng = np.random.default_rng(3)
    U, _ = np.linalg.qr(rng.normal(size=(norb, norb)))
    h2 = U.T @ h @ U
    eri2 = np.einsum("pqrs,pi,qj,rk,sl->ijkl", eri, U, U, U, U, optimize=True)
    S = O.Space(norb, 2, 2, 4)
    w1 = np.linalg.eigvalsh(O.dense_h(S, h, eri, 0.0))
    w2 = np.linalg.eigvalsh(O.dense_h(S, h2, eri2, 0.0))
    assert np.abs(w1 - w2).max() <= 1e-10


def test_fci_orbital_rotation_invariance_unequal_spins():
    norb = 6
    h, eri = recipe_random(norb, seed=8)
    rng = np.random.default_rng(4)
    U, _ = np.linalg.qr(rng.normal(size=(norb, norb)))
    h2 = U.T @ h @ U
    eri2 = np.einsum("pqrs,pi,qj,rk,sl->ijkl", eri, U, U, U, U, optimize=True)
    S = O.Space(norb, 3, 1, 4)
    w1 = np.linalg.eigvalsh(O.dense_h(S, h, eri, 0.0))
    w2 = np.linalg.eigvalsh(O.dense_h(S, h2, eri2, 0.0))
    assert np.abs(w1 - w2).max() <= 1e-10


# ---------------------------------------------------------------- P10
@pytest.mark.parametrize("L", [2, 3, 4])
def test_alpha_beta_swap_covariance(L):
    norb = 7
    h, eri = recipe_random(norb, seed=11)
    S = O.Space(norb, 2, 2, L)
    dets = S.determinants()
    pos = {d: i for i, d in enumerate(dets)}
    perm = np.array([pos[(b, a)] for a, b in dets])
    c = random_vectors(S.dim, 1, 2)[0]
    s1 = O.sigma(S, h, eri, 1e-3, c[perm][None])[0]
    s2 = O.sigma(S, h, eri, 1e-3, c[None])[0][perm]
    assert np.abs(s1 - s2).max() <= 1e-12 * np.abs(s2).max()


# ---------------------------------------------------------------- P6
@pytest.mark.parametrize("recipe,norb,L", [("A", 10, 4), ("B", 12, 2), ("A", 14, 2), ("B", 9, 3)])
def test_davidson_matches_dense(recipe, norb, L):
    h, eri = _ints(recipe, norb, 1)
    S = O.Space(norb, 2, 2, L)
    w = np.linalg.eigvalsh(O.dense_h(S, h, eri, 0.0))
    e, X, rn = O.davidson(S, h, eri, 0.0, nroots=2, tol=1e-9)
    assert np.all(rn <= 1e-9)
    assert np.abs(e - w[:2]).max() <= 1e-12 * max(1.0, abs(w[0])) + 1e-13


# ---------------------------------------------------------------- P11
@pytest.mark.parametrize("tau", [1e-6, 1e-4, 1e-2])
def test_screening_bound(tau):
    """Weyl: |lambda_k(H_0) - lambda_k(H_tau)| <= ||H_0 - H_tau||_2 <= B(tau)."""
    h, eri = recipe_a(10, seed=2)
    S = O.Space(10, 2, 2, 3)
    w0 = np.linalg.eigvalsh(O.dense_h(S, h, eri, 0.0))
    wt = np.linalg.eigvalsh(O.dense_h(S, h, eri, tau))
    B = O.dropped_bound(S, h, eri, tau)
    D = O.dense_h(S, h, eri, 0.0) - O.dense_h(S, h, eri, tau)
    # D carries the rounding of two dense sums; allow for it
    assert B >= np.abs(D).sum(axis=1).max() - 1e-13
    assert np.abs(w0 - wt).max() <= B + 1e-13
    if tau >= 1e-4:
        assert B > 0.0


def test_screening_tau_zero_is_exact():
    """tau = 0 drops only exact zeros, which contribute nothing."""
    h, eri = recipe_a(9, seed=3)
    eri = eri.copy()
    eri[np.abs(eri) < 1e-9] = 0.0
    S = O.Space(9, 2, 2, 3)
    assert O.dropped_bound(S, h, eri, 0.0) == 0.0


def test_strict_threshold():
    """A unit exactly equal to tau is dropped (keep rule |I| > tau)."""
    norb = 5
    h, eri = recipe_random(norb, seed=5)
    tau = abs(h[3, 1])
    S = O.Space(norb, 1, 0, 1)
    H = O.dense_h(S, h, eri, tau)
    # one alpha electron, no beta: H is h restricted to the (level<=1) space
    ao, _ = S.strings(0)
    idx = [int(r[0]) for r in ao]
    want = h[np.ix_(idx, idx)].copy()
    want[np.abs(want) <= tau] = 0.0
    assert np.array_equal(H, want)


# ---------------------------------------------------------------- P12
def _integral_driven_counts(h, eri, norb, L, tau, boundary=None):
    """Independent count for na = nb = 2, written in the paper's loop
    order: integral indices outside, spectator strings inside.  A string's
    level counts its electrons in orbitals >= boundary (default n)."""
    n = 2
    b = n if boundary is None else boundary
    e = (np.arange(norb) >= b).astype(int)
    # number of beta strings with level <= l
    nb_le = [sum(comb(b, n - k) * comb(norb - b, k) for k in range(0, min(l, 2) + 1)) if l >= 0 else 0
             for l in range(0, 5)]

    def nble(l):
        return nb_le[l] if l >= 0 else 0

    one = 0
    for p in range(norb):
        for q in range(norb):
            if abs(h[max(p, q), min(p, q)]) <= tau:
                continue
            for x in range(norb):
                if x in (p, q):
                    continue
                la = max(e[x] + e[p], e[x] + e[q])
                one += nble(L - la)
    one *= 2  # alpha and beta
    ss = 0
    for p in range(norb):
        for r in range(p):
            for q in range(norb):
                for s in range(q):
                    val = eri[p, q, r, s] - eri[p, s, r, q]
                    if abs(val) <= tau:
                        continue
                    la = max(e[p] + e[r], e[q] + e[s])
                    ss += nble(L - la)
    ss *= 2
    ab = 0
    ex = e
    for p in range(norb):
        for q in range(norb):
            for r in range(norb):
                for s in range(norb):
                    if abs(eri[p, q, r, s]) <= tau:
                        continue
                    for x in range(norb):
                        if x in (p, q):
                            continue
                        for y in range(norb):
                            if y in (r, s):
                                continue
                            src = ex[x] + ex[q] + ex[y] + ex[s]
                            dst = ex[x] + ex[p] + ex[y] + ex[r]
                            if src <= L and dst <= L:
                                ab += 1
    return one, ss, ab


@pytest.mark.parametrize("recipe,norb,L,tau", [("R", 6, 2, 0.0), ("B", 7, 3, 1e-3), ("A", 8, 2, 1e-6)])
def test_term_counts_integral_driven(recipe, norb, L, tau):
    h, eri = _ints(recipe, norb, 3)
    S = O.Space(norb, 2, 2, L)
    kept, allc = O.terms(S, h, eri, tau)
    one, ss, ab = _integral_driven_counts(h, eri, norb, L, tau)
    assert kept[0:8].sum() == one
    assert kept[8:26].sum() == ss
    assert kept[26:42].sum() == ab
    if tau == 0.0:
        assert np.array_equal(kept, allc)
    assert len(O.bucket_names()) == 42


def test_term_count_alpha_beta_swap_symmetry():
    h, eri = recipe_b(8, seed=4)
    S = O.Space(8, 2, 2, 3)
    kept, _ = O.terms(S, h, eri, 1e-8)
    assert np.array_equal(kept[0:4], kept[4:8])
    assert np.array_equal(kept[8:17], kept[17:26])
    ab = kept[26:42].reshape(2, 2, 2, 2)
    assert np.array_equal(ab, ab.transpose(2, 3, 0, 1))


# ---------------------------------------------------------------- D1
# One-body density matrices (the paper's density-matrix subsection, Eq. d1).
_D1_SPACES = [(6, 2, 2, 2), (7, 3, 1, 3), (6, 2, 2, 4), (5, 1, 0, 1), (6, 3, 3, 6), (7, 2, 1, 2)]


@pytest.mark.parametrize("norb,na,nb,L", _D1_SPACES)
def test_density1_single_determinant_occupations(norb, na, nb, L):
    """A single determinant has the occupation numbers of its strings on
    the diagonal of each spin block and nothing off it."""
    S = O.Space(norb, na, nb, L)
    dets = S.determinants()
    for k in sorted({0, S.dim // 3, S.dim - 1}):
        e = np.zeros((1, S.dim))
        e[0, k] = -1.5
        d = O.density1(S, e)[0]
        want = np.zeros((2, norb, norb))
        for s, orbs in enumerate(dets[k]):
            for o in orbs:
                want[s, o, o] = 2.25
        np.testing.assert_array_equal(d, want)


@pytest.mark.parametrize("norb,na,nb,L", _D1_SPACES)
def test_density1_trace_and_symmetry(norb, na, nb, L):
    S = O.Space(norb, na, nb, L)
    c = random_vectors(S.dim, 3, seed=norb + L)
    d = O.density1(S, c)
    nn = (c * c).sum(1)
    for s, n in enumerate((na, nb)):
        np.testing.assert_allclose(np.trace(d[:, s], axis1=1, axis2=2), n * nn, rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(d, d.transpose(0, 1, 3, 2), rtol=0, atol=1e-13 * np.abs(d).max())


@pytest.mark.parametrize("norb,na,nb,L", _D1_SPACES)
def test_density1_one_body_energy_against_dense_h(norb, na, nb, L):
    """<c|H1|c> with H1 the oracle's dense Hamiltonian for zero two-electron
    integrals equals sum_pq h_pq (D1a + D1b)_pq, for several random
    symmetric h (each draw weighs every element differently)."""
    S = O.Space(norb, na, nb, L)
    c = random_vectors(S.dim, 2, seed=7 * norb + L)
    d = O.density1(S, c)
    eri = np.zeros((norb,) * 4)
    rng = np.random.default_rng(norb * 31 + L)
    for _ in range(3):
        h = rng.standard_normal((norb, norb))
        h = h + h.T
        H = O.dense_h(S, h, eri, 0.0)
        for v in range(2):
            e = c[v] @ H @ c[v]
            assert abs(e - (h * (d[v, 0] + d[v, 1])).sum()) <= 1e-12 * max(1.0, abs(e))


def test_density1_alpha_beta_swap():
    """With as many alpha as beta electrons the space is closed under the
    spin swap (Ia, Ib) -> (Ib, Ia); the swapped vector's alpha block is the
    original beta block and vice versa."""
    norb, n, L = 7, 2, 3
    S = O.Space(norb, n, n, L)
    c = random_vectors(S.dim, 2, seed=3)
    dets = S.determinants()
    perm = np.array([S.address(b, a) for a, b in dets])
    assert (perm >= 0).all() and len(set(perm.tolist())) == S.dim
    cs = np.zeros_like(c)
    cs[:, perm] = c
    d, ds = O.density1(S, c), O.density1(S, cs)
    np.testing.assert_allclose(ds[:, 0], d[:, 1], rtol=0, atol=1e-13)
    np.testing.assert_allclose(ds[:, 1], d[:, 0], rtol=0, atol=1e-13)


@pytest.mark.parametrize("norb,na,nb,L", [(5, 2, 2, 2), (5, 3, 1, 2), (4, 2, 2, 4)])
def test_density1_brute_force_words(norb, na, nb, L):
    """Every element by brute force: for each determinant and each (p, q),
    the word a+_p a_q applied to the spin's creator string through
    apply_word (pinned by the paper's worked sign examples), the target's
    address in the space, and the coefficient product."""
    S = O.Space(norb, na, nb, L)
    c = random_vectors(S.dim, 1, seed=11)[0]
    want = np.zeros((2, norb, norb))
    for k, (a, b) in enumerate(S.determinants()):
        for s, orbs in enumerate((a, b)):
            for p in range(norb):
                for q in range(norb):
                    sg, out = O.apply_word([("+", p), ("-", q)] + [("+", o) for o in orbs], 1)
                    if not sg:
                        continue
                    j = S.address(out, b) if s == 0 else S.address(a, out)
                    if j < 0:
                        continue
                    want[s, p, q] += sg * c[j] * c[k]
    np.testing.assert_allclose(O.density1(S, c[None])[0], want, rtol=0, atol=1e-13)


# ---------------------------------------------------------------- factored integrals
@pytest.mark.parametrize("norb,naux,seed", [(6, 4, 0), (9, 18, 1), (12, 5, 2)])
def test_assemble_factored_gram_structure(norb, naux, seed):
    """(pq|rs) = sum_K L^K_pq L^K_rs is a Gram matrix over the pair index:
    positive semidefinite, rank <= naux, symmetric under (pq) <-> (rs), with
    |(pq|rs)|^2 <= (pq|pq)(rs|rs); with symmetric factors it has the 8-fold
    symmetry exactly (each term is formed from the same two doubles)."""
    from isci_inputs.recipes import factors_a
    rng = np.random.default_rng(seed)
    Lr = rng.standard_normal((naux, norb, norb))
    E = O.assemble_factored(Lr)
    M = E.reshape(norb * norb, norb * norb)
    assert np.array_equal(M, M.T)
    w = np.linalg.eigvalsh(M)
    assert w.min() >= -1e-12 * w.max()
    assert np.sum(w > 1e-10 * w.max()) <= naux
    d = np.diag(M)
    assert np.all(M ** 2 <= np.outer(d, d) * (1 + 1e-12) + 1e-300)
    _h, Ls = factors_a(norb, float(norb), naux, seed)
    Ls = 0.5 * (Ls + Ls.transpose(0, 2, 1))
    Es = O.assemble_factored(Ls)
    for perm in [(1, 0, 2, 3), (0, 1, 3, 2), (2, 3, 0, 1), (3, 2, 1, 0)]:
        assert np.array_equal(Es, Es.transpose(perm))


def test_assemble_factored_matches_matrix_product_assembly():
    """The same recipe-A factors assembled by the inputs module (one matrix
    product) agree within rounding."""
    from isci_inputs.recipes import assemble_eri, factors_a
    _h, L = factors_a(14, 14.0, 28, 3)
    a = O.assemble_factored(L)
    b = assemble_eri(L)
    assert np.abs(a - b).max() <= 1e-14 * np.abs(b).max()


# ---------------------------------------------------------------- two-body density matrices
_D2_SPACES = [(6, 2, 2, 2), (5, 3, 1, 3), (5, 2, 1, 2), (5, 1, 1, 2), (5, 0, 2, 2), (6, 2, 2, 4)]


def _d2_total(d2):
    """sum over the spin blocks of <a+_p a+_r a_s a_q>: aa + ab + ba + bb,
    ba[p,q,r,s] = ab[r,s,p,q]."""
    return d2[:, 0] + d2[:, 1] + d2[:, 1].transpose(0, 3, 4, 1, 2) + d2[:, 2]


@pytest.mark.parametrize("norb,na,nb,L", _D2_SPACES)
def test_density2_energy_identity(norb, na, nb, L):
    """<c|H|c> from the oracle sigma equals sum h D1 + 1/2 sum (pq|rs) D2 for
    integrals with no symmetry beyond the 8-fold one."""
    h, eri = _ints("R", norb, 11)
    S = O.Space(norb, na, nb, L)
    c = random_vectors(S.dim, 2, seed=5)
    e = np.einsum("vi,vi->v", c, O.sigma(S, h, eri, 0.0, c))
    d1 = O.density1(S, c)
    d2 = O.density2(S, c)
    e1 = np.einsum("pq,vpq->v", h, d1[:, 0] + d1[:, 1])
    e2 = 0.5 * np.einsum("pqrs,vpqrs->v", eri, _d2_total(d2))
    assert np.abs(e1 + e2 - e).max() <= 1e-12 * np.abs(e).max()


@pytest.mark.parametrize("norb,na,nb,L", _D2_SPACES)
def test_density2_traces_and_reduction(norb, na, nb, L):
    S = O.Space(norb, na, nb, L)
    c = random_vectors(S.dim, 2, seed=6)
    nn = (c * c).sum(1)
    d1 = O.density1(S, c)
    d2 = O.density2(S, c)
    tr = np.einsum("vbpprr->vb", d2)
    assert np.allclose(tr[:, 0], na * (na - 1) * nn, rtol=1e-12, atol=1e-12)
    assert np.allclose(tr[:, 1], na * nb * nn, rtol=1e-12, atol=1e-12)
    assert np.allclose(tr[:, 2], nb * (nb - 1) * nn, rtol=1e-12, atol=1e-12)
    # the other spin's number operator, or the same spin's minus one
    assert np.allclose(np.einsum("vpqrr->vpq", d2[:, 1]), nb * d1[:, 0], atol=1e-12)
    assert np.allclose(np.einsum("vpprs->vrs", d2[:, 1]), na * d1[:, 1], atol=1e-12)
    assert np.allclose(np.einsum("vpqrr->vpq", d2[:, 0]), (na - 1) * d1[:, 0], atol=1e-12)
    assert np.allclose(np.einsum("vpqrr->vpq", d2[:, 2]), (nb - 1) * d1[:, 1], atol=1e-12)


@pytest.mark.parametrize("norb,na,nb,L", _D2_SPACES[:3])
def test_density2_symmetries(norb, na, nb, L):
    S = O.Space(norb, na, nb, L)
    c = random_vectors(S.dim, 1, seed=2)
    d2 = O.density2(S, c)
    for b in (0, 2):
        assert np.allclose(d2[:, b], -d2[:, b].transpose(0, 3, 2, 1, 4), atol=1e-13)
        assert np.allclose(d2[:, b], -d2[:, b].transpose(0, 1, 4, 3, 2), atol=1e-13)
    for b in range(3):   # real vectors: <a+p a+r a_s a_q> = <a+q a+s a_r a_p>
        assert np.allclose(d2[:, b], d2[:, b].transpose(0, 2, 1, 4, 3), atol=1e-13)


def test_density2_single_determinant():
    norb, na, nb, L = 6, 2, 2, 2
    S = O.Space(norb, na, nb, L)
    ao, _ = S.strings(0)
    bo, _ = S.strings(1)
    rs = S.rowstart()
    i = 3
    k = 2
    c = np.zeros((1, S.dim))
    c[0, rs[i] + k] = 1.0
    d2 = O.density2(S, c)
    A, B = [int(x) for x in ao[i]], [int(x) for x in bo[k]]
    want = np.zeros((3, norb, norb, norb, norb))
    for p in A:
        for r in B:
            want[1, p, p, r, r] = 1.0
    for blk, occ in ((0, A), (2, B)):
        for p in occ:
            for r in occ:
                if p != r:
                    want[blk, p, p, r, r] = 1.0
                    want[blk, p, r, r, p] = -1.0
    assert np.array_equal(d2[0], want)


# ---------------------------------------------------------------- propagation
def test_propagate_exact_properties():
    norb, L, tau = 7, 2, 0.0
    h, eri = _ints("R", norb, 4)
    S = O.Space(norb, 2, 2, L)
    re, im = random_vectors(S.dim, 2, seed=3)
    c = re + 1j * im
    H = O.dense_h(S, h, eri, tau)
    c1 = O.propagate_exact(S, h, eri, tau, re, im, 0.7, imaginary=False)
    assert abs(np.linalg.norm(c1) - np.linalg.norm(c)) <= 1e-12 * np.linalg.norm(c)
    e0 = np.real(np.vdot(c, H @ c))
    assert abs(np.real(np.vdot(c1, H @ c1)) - e0) <= 1e-11 * abs(e0)
    c2 = O.propagate_exact(S, h, eri, tau, np.real(c1), np.imag(c1), 0.5, imaginary=False)
    c12 = O.propagate_exact(S, h, eri, tau, re, im, 1.2, imaginary=False)
    assert np.abs(c2 - c12).max() <= 1e-12 * np.abs(c12).max()
    # short-time difference quotient against the oracle sigma
    d = 1e-6
    cd = O.propagate_exact(S, h, eri, tau, re, im, d, imaginary=False)
    hc = O.sigma(S, h, eri, tau, np.stack([re, im]))
    want = -1j * (hc[0] + 1j * hc[1])
    assert np.abs((cd - c) / d - want).max() <= 1e-4 * np.abs(want).max()
    # imaginary time: difference quotient of the normalised flow and the
    # long-time limit (lowest eigenvector, up to sign)
    u = re / np.linalg.norm(re)
    ud = O.propagate_exact(S, h, eri, tau, u, None, d)
    hu = O.sigma(S, h, eri, tau, u[None])[0]
    want = -(hu - (u @ hu) * u)
    assert np.abs((ud - u) / d - want).max() <= 1e-4 * np.abs(want).max()
    uinf = O.propagate_exact(S, h, eri, tau, u, None, 400.0)
    w = np.linalg.eigvalsh(H)
    assert abs(uinf @ (H @ uinf) - w[0]) <= 1e-10


def test_propagate_exact_coefficient_screening():
    """Screened stepping: a threshold below every coefficient changes
    nothing (the steps compose to the unscreened flow); one screened step
    is the unscreened step with its small entries zeroed, checked element by
    element; the screened imaginary-time vector stays above the lowest
    eigenvalue (variational) and approaches it as the threshold falls."""
    norb, L, tau = 8, 2, 0.0
    h, eri = _ints("R", norb, 6)
    S = O.Space(norb, 2, 2, L)
    re, im = random_vectors(S.dim, 2, seed=5)
    a = O.propagate_exact(S, h, eri, tau, re, im, 1.0, imaginary=False, nsteps=5, coef_tau=1e-300)
    b = O.propagate_exact(S, h, eri, tau, re, im, 1.0, imaginary=False)
    assert np.abs(a - b).max() <= 1e-12 * np.abs(b).max()
    u = np.zeros(S.dim)
    u[0] = 1.0
    one = O.propagate_exact(S, h, eri, tau, u, None, 0.4)
    t1 = float(np.median(np.abs(one)))
    scr = O.propagate_exact(S, h, eri, tau, u, None, 0.4, nsteps=1, coef_tau=t1)
    for i in range(S.dim):
        assert scr[i] == (0.0 if abs(one[i]) <= t1 else one[i])
    assert 0 < int(np.sum(scr == 0.0)) < S.dim
    H = O.dense_h(S, h, eri, tau)
    w, V = np.linalg.eigh(H)
    w0, a0 = w[0], np.sort(np.abs(V[:, 0]))
    gaps = []
    # thresholds that cut about 40 %, 20 % and 5 % of the ground state
    for thr in (a0[int(0.4 * S.dim)], a0[int(0.2 * S.dim)], a0[int(0.05 * S.dim)]):
        c = O.propagate_exact(S, h, eri, tau, u, None, 200.0, nsteps=100, coef_tau=thr)
        e = (c @ (H @ c)) / (c @ c)
        assert e >= w0 - 1e-12
        gaps.append(e - w0)
    assert gaps[0] > gaps[1] > gaps[2]


# ---------------------------------------------------------------- distance screening
def test_mask_by_distance_brute_force_and_limits():
    norb = 5
    h, eri = _ints("R", norb, 2)
    x = np.array([0.0, 1.0, 2.5, 4.0, 7.0])
    dist = np.abs(x[:, None] - x[None, :])
    hm, em = O.mask_by_distance(h, eri, dist, 3.0)
    for p in range(norb):
        for q in range(norb):
            assert hm[p, q] == (h[p, q] if dist[p, q] <= 3.0 else 0.0)
            for r in range(norb):
                for s in range(norb):
                    orbs = (p, q, r, s)
                    ok = all(dist[a, b] <= 3.0 for a in orbs for b in orbs)
                    assert em[p, q, r, s] == (eri[p, q, r, s] if ok else 0.0)
    h2, e2 = O.mask_by_distance(h, eri, dist, 100.0)
    assert np.array_equal(h2, h) and np.array_equal(e2, eri)
    h3, e3 = O.mask_by_distance(h, eri, dist, 0.5)
    assert np.array_equal(h3, np.diag(np.diag(h)))
    keep = np.zeros_like(eri)
    for p in range(norb):
        keep[p, p, p, p] = eri[p, p, p, p]
    assert np.array_equal(e3, keep)
    # a non-symmetric matrix reads as the pair maximum
    rng = np.random.default_rng(1)
    da = dist * rng.uniform(0.5, 1.5, dist.shape)
    ha, ea = O.mask_by_distance(h, eri, da, 3.0)
    hb, eb = O.mask_by_distance(h, eri, np.maximum(da, da.T), 3.0)
    assert np.array_equal(ha, hb) and np.array_equal(ea, eb)
    assert np.array_equal(ea, ea.transpose(1, 0, 2, 3)) and np.array_equal(ea, ea.transpose(2, 3, 0, 1))


# ---------------------------------------------------------------- GAS (two spaces)
# Section "Generalized Active Space": the orbitals split at a boundary b
# into an inner space 0..b-1 (full CI there) and an outer space b..norb-1
# holding at most L electrons, alpha plus beta.  b = n is the CI hierarchy.
_GAS_SPACES = [(8, 2, 2, 1, 4), (8, 2, 2, 2, 3), (8, 2, 2, 0, 5), (9, 3, 2, 1, 4),
               (7, 2, 2, 3, 4), (7, 2, 1, 2, 5), (7, 2, 2, 1, 7), (6, 0, 2, 1, 3)]


def _brute_gas(norb, na, nb, L, b):
    out = []
    for a in combinations(range(norb), na):
        for bb in combinations(range(norb), nb):
            if sum(x >= b for x in a) + sum(x >= b for x in bb) <= L:
                out.append((a, bb))
    return out


@pytest.mark.parametrize("norb,na,nb,L,b", _GAS_SPACES)
def test_gas_layout_brute_force(norb, na, nb, L, b):
    """The space is exactly the determinants with at most L electrons in
    the outer orbitals, each once; strings in (outer count, colex) order;
    rows hold prefixes of the beta order; the closed form counts it."""
    S = O.Space(norb, na, nb, L, boundary=b)
    dets = S.determinants()
    brute = _brute_gas(norb, na, nb, L, b)
    assert S.dim == len(brute) == len(set(dets)) == O.dim_closed_form(norb, na, nb, L, boundary=b)
    assert set(dets) == set(brute)
    ao, _ = S.strings(0)
    bo, _ = S.strings(1)
    key = lambda r: (sum(int(x) >= b for x in r), tuple(sorted((int(x) for x in r), reverse=True)))
    assert [key(r) for r in ao] == sorted(key(r) for r in ao)
    assert [key(r) for r in bo] == sorted(key(r) for r in bo)
    for i, (a, bb) in enumerate(dets):
        assert S.address(a, bb) == i


def test_gas_boundary_at_n_is_the_hierarchy_and_at_norb_is_fci():
    for norb, na, nb, L in [(8, 2, 2, 2), (7, 3, 2, 3)]:
        S, G = O.Space(norb, na, nb, L), O.Space(norb, na, nb, L, boundary=max(na, nb))
        if na == nb:
            assert S.determinants() == G.determinants()
    F = O.Space(7, 2, 2, 4)
    for L in (0, 1, 3):
        assert O.Space(7, 2, 2, L, boundary=7).dim == F.dim
    with pytest.raises(ValueError):
        O.Space(7, 3, 2, 1, boundary=2)        # boundary below an electron count
    with pytest.raises(ValueError):
        O.Space(7, 2, 2, 1, boundary=8)


@pytest.mark.parametrize("recipe", ["B", "R"])
@pytest.mark.parametrize("norb,na,nb,L,b", [(8, 2, 2, 1, 4), (7, 2, 2, 2, 3), (7, 3, 2, 1, 4)])
@pytest.mark.parametrize("tau", [0.0, 1e-3])
def test_gas_h_is_the_fci_submatrix(recipe, norb, na, nb, L, b, tau):
    """A matrix element depends only on its two determinants: the GAS
    Hamiltonian (dense, sigma and diagonal) is the full-CI one restricted
    to the GAS determinants (the full-CI H is pinned by the closed forms,
    the noninteracting and one-electron limits and rotation invariance)."""
    h, eri = _ints(recipe, norb, 11)
    G = O.Space(norb, na, nb, L, boundary=b)
    F = O.Space(norb, na, nb, na + nb)
    idx = np.array([F.address(a, bb) for a, bb in G.determinants()])
    HF = O.dense_h(F, h, eri, tau)
    HG = O.dense_h(G, h, eri, tau)
    assert np.array_equal(HG, HF[np.ix_(idx, idx)])
    c = random_vectors(G.dim, 2, 4)
    assert np.allclose(O.sigma(G, h, eri, tau, c), c @ HF[np.ix_(idx, idx)].T, rtol=0, atol=1e-12)
    # the diagonal is summed in long double, the dense matrix in double
    assert np.allclose(O.diag(G, h, eri, tau), np.diag(HF)[idx], rtol=0, atol=1e-13 * np.abs(HF).max())


def test_gas_no_outer_electrons_is_inner_fci():
    """L = 0 keeps every electron in the inner orbitals: the spectrum is the
    full CI of the integrals cut to those orbitals (a smaller problem built
    independently)."""
    h, eri = recipe_b(9, seed=2)
    b = 5
    G = O.Space(9, 2, 2, 0, boundary=b)
    F = O.Space(b, 2, 2, 4)
    eg = np.linalg.eigvalsh(O.dense_h(G, h, eri, 0.0))
    ef = np.linalg.eigvalsh(O.dense_h(F, h[:b, :b].copy(), eri[:b, :b, :b, :b].copy(), 0.0))
    assert G.dim == F.dim
    assert np.allclose(eg, ef, rtol=0, atol=1e-12)


def test_gas_variational_nesting():
    """Spaces nested by L give non-increasing lowest energies (Cauchy
    interlacing), equal to full CI once L reaches every electron."""
    h, eri = recipe_a(8, seed=1)
    b = 4
    e = [np.linalg.eigvalsh(O.dense_h(O.Space(8, 2, 2, L, boundary=b), h, eri, 0.0))[0] for L in range(5)]
    ef = np.linalg.eigvalsh(O.dense_h(O.Space(8, 2, 2, 4), h, eri, 0.0))[0]
    assert all(e[i + 1] <= e[i] + 1e-12 for i in range(4))
    assert e[0] > e[-1] + 1e-6
    assert abs(e[-1] - ef) <= 1e-12


@pytest.mark.parametrize("recipe,norb,L,b,tau", [("R", 7, 1, 4, 0.0), ("B", 8, 2, 3, 1e-3), ("A", 8, 1, 5, 1e-6)])
def test_gas_term_counts_integral_driven(recipe, norb, L, b, tau):
    h, eri = _ints(recipe, norb, 3)
    S = O.Space(norb, 2, 2, L, boundary=b)
    kept, _ = O.terms(S, h, eri, tau)
    one, ss, ab = _integral_driven_counts(h, eri, norb, L, tau, boundary=b)
    assert kept[0:8].sum() == one
    assert kept[8:26].sum() == ss
    assert kept[26:42].sum() == ab
