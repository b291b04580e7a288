"""ctypes binding of the C oracle plus numpy reference pieces.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Parity status:

* ``Space`` (strings, levels, row starts, addresses): pinned by the
  closed-form space dimension, which reproduces the paper's table of
  determinant counts (application section, table of orbitals and
  coefficients), and by brute-force enumeration in the tests.  With a
  two-space boundary (section "Generalized Active Space"): by brute-force
  filtering of every determinant by its outer-space electron count and the
  matching closed form; the boundary-level count is checked by a planted
  mistake (level counted from n) that these pins reject.
* ``sigma`` / ``dense_h`` / ``diag`` on two-space spaces: pinned as the
  restriction of the pinned full-CI matrix to the space's determinants, by
  the full CI of the cut integrals when no outer electron is allowed, and
  by variational nesting in the outer-electron limit.
* ``sigma`` / ``dense_h``: pinned by the closed-form reference energy,
  Hermiticity, the non-interacting limit, the one-electron-per-spin
  Kronecker construction, orbital-rotation invariance of FCI, alpha/beta
  swap covariance and exact diagonalisation (tests/test_oracle_*.py).
* ``diag``: pinned by the textbook Slater-Condon diagonal of every
  determinant (unit by unit under the keep rule), by the diagonal of the
  pinned ``dense_h``, and by the closed-form reference energy of the
  relabelled Hamiltonian for closed-shell determinants; two planted
  mistakes (whole row summed, screened units counted) are rejected.
* ``apply_word``: pinned by the paper's two worked sign examples
  (Eqs. contract and add).
* ``terms``: pinned by an independent closed-form count in the tests.
* ``dropped_bound``: pinned by the Weyl inequality against exact spectra.
* ``davidson``: pinned by dense diagonalisation on small spaces.
* ``assemble_factored``: pinned by the Gram structure of the definition
  (the (pq),(rs) matrix is positive semidefinite of rank <= naux, symmetric,
  and obeys the Cauchy-Schwarz bound) and by agreement within rounding with
  the inputs module's matrix-product assembly of the same factors.
* ``density2``: pinned by the energy identity <c|H|c> = sum h D1 + 1/2 sum
  (pq|rs) D2 against the oracle sigma for generic integrals, traces and
  partial traces (electron-pair counts, reduction to ``density1``),
  same-spin antisymmetry, Hermiticity and single determinants; planted
  mistakes are rejected.
* ``propagate_exact``: pinned by the properties that fix the exponential:
  real time keeps the norm and the energy, steps compose (t1 then t2 is
  t1 + t2), the short-time difference quotient is -i H c (resp. -(H - E) c)
  with H c from the oracle sigma, and imaginary time tends to the lowest
  eigenvector; its coefficient screening by a threshold below every
  coefficient (no change), one step checked element by element, and the
  variational bound of the screened vector.
* ``mask_by_distance``: pinned by brute-force enumeration of every element
  on tiny inputs, and by its limits (a radius above every distance changes
  nothing; below every non-zero distance only the one-orbital units p = q = r
  = s and h_pp survive).
* ``density1``: pinned by single determinants (occupation numbers), the
  trace (electron count), the one-body energy against ``dense_h`` with the
  two-electron integrals set to zero, the alpha/beta swap, and brute force
  through ``apply_word`` on tiny spaces.
"""
from __future__ import annotations

import ctypes
import os
from math import comb

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.environ.get("ISCI_ORACLE_LIB") or os.path.join(HERE, "liboracle.so")

NBUCKET = 42
_i64 = ctypes.c_int64
_dp = ctypes.POINTER(ctypes.c_double)
_i64p = ctypes.POINTER(ctypes.c_int64)
_i32p = ctypes.POINTER(ctypes.c_int32)
_ip = ctypes.POINTER(ctypes.c_int)

_LIB = None

# Mutation switches for the pin tests (a planted mistake; never set in use).
_PLANT = set(os.environ.get("ISCI_ORACLE_PLANT", "").split(","))


def lib():
    """Load liboracle.so, building it first if it is absent."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIBPATH):
            from .build import build
            build()
        L = ctypes.CDLL(LIBPATH)
        L.orc_space_create.restype = ctypes.c_void_p
        L.orc_space_create.argtypes = [ctypes.c_int] * 4
        L.orc_space_create_gas.restype = ctypes.c_void_p
        L.orc_space_create_gas.argtypes = [ctypes.c_int] * 5
        L.orc_space_destroy.argtypes = [ctypes.c_void_p]
        L.orc_space_dim.restype = _i64
        L.orc_space_dim.argtypes = [ctypes.c_void_p]
        L.orc_space_nstr.restype = _i64
        L.orc_space_nstr.argtypes = [ctypes.c_void_p, ctypes.c_int]
        L.orc_space_strings.argtypes = [ctypes.c_void_p, ctypes.c_int, _i32p, _i32p]
        L.orc_space_rowstart.argtypes = [ctypes.c_void_p, _i64p]
        L.orc_space_address.restype = _i64
        L.orc_space_address.argtypes = [ctypes.c_void_p, _i32p, _i32p]
        L.orc_sigma.argtypes = [ctypes.c_void_p, _dp, _dp, ctypes.c_double, ctypes.c_int,
                                _dp, _i64, _i64, _i64p, _dp]
        L.orc_diag.argtypes = [ctypes.c_void_p, _dp, _dp, ctypes.c_double, _i64, _i64p, _dp]
        L.orc_terms.argtypes = [ctypes.c_void_p, _dp, _dp, ctypes.c_double, _i64p, _i64p]
        L.orc_dense_h.argtypes = [ctypes.c_void_p, _dp, _dp, ctypes.c_double, _dp]
        L.orc_dropped_bound.argtypes = [ctypes.c_void_p, _dp, _dp, ctypes.c_double, _dp]
        L.orc_apply_word.argtypes = [ctypes.c_int, _ip, _ip, ctypes.c_int, _ip, _ip]
        L.orc_num_threads.restype = ctypes.c_int
        _LIB = L
    return _LIB


def _p(a, t=_dp):
    return a.ctypes.data_as(t)


def _ints(h, eri):
    h = np.ascontiguousarray(h, dtype=np.float64)
    eri = np.ascontiguousarray(eri, dtype=np.float64)
    n = h.shape[0]
    if h.shape != (n, n) or eri.shape != (n, n, n, n):
        raise ValueError("h must be [norb,norb] and eri [norb]^4")
    return h, eri


def num_threads() -> int:
    return int(lib().orc_num_threads())


class Space:
    """Truncated CI space of the oracle (strings and determinant addresses).

    Strings per spin: ascending orbital sets sorted by (excitation level,
    colex); row Ia holds the beta strings of level <= L - level(Ia).

    ``boundary`` (section "Generalized Active Space", two spaces): if given,
    a string's level is its number of electrons in orbitals >= boundary
    instead of >= n, so the space is the full CI of the orbitals below the
    boundary with at most ``level`` electrons (alpha plus beta) above it.
    """

    def __init__(self, norb: int, nalpha: int, nbeta: int, level: int, boundary: int | None = None):
        self.norb, self.nalpha, self.nbeta, self.level = norb, nalpha, nbeta, level
        self.boundary = boundary
        self._h = lib().orc_space_create_gas(norb, nalpha, nbeta, level, int(boundary or 0))
        if not self._h:
            raise ValueError("invalid space")
        self.dim = int(lib().orc_space_dim(self._h))

    def close(self):
        if self._h:
            lib().orc_space_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def nstr(self, spin: int) -> int:
        return int(lib().orc_space_nstr(self._h, spin))

    def strings(self, spin: int):
        n = self.nbeta if spin else self.nalpha
        ns = self.nstr(spin)
        orbs = np.zeros((ns, max(n, 1)), dtype=np.int32)
        lev = np.zeros(ns, dtype=np.int32)
        lib().orc_space_strings(self._h, spin, _p(orbs, _i32p), _p(lev, _i32p))
        return orbs[:, :n].copy(), lev

    def rowstart(self):
        rs = np.zeros(self.nstr(0) + 1, dtype=np.int64)
        lib().orc_space_rowstart(self._h, _p(rs, _i64p))
        return rs

    def address(self, alpha, beta) -> int:
        a = np.ascontiguousarray(sorted(alpha), dtype=np.int32)
        b = np.ascontiguousarray(sorted(beta), dtype=np.int32)
        if a.size == 0:
            a = np.zeros(1, dtype=np.int32)
        if b.size == 0:
            b = np.zeros(1, dtype=np.int32)
        return int(lib().orc_space_address(self._h, _p(a, _i32p), _p(b, _i32p)))

    def determinants(self):
        """List of (alpha tuple, beta tuple) in address order."""
        ao, _ = self.strings(0)
        bo, _ = self.strings(1)
        rs = self.rowstart()
        out = []
        for ia in range(len(ao)):
            for ib in range(int(rs[ia + 1] - rs[ia])):
                out.append((tuple(int(x) for x in ao[ia]), tuple(int(x) for x in bo[ib])))
        return out


def sigma(space: Space, h, eri, tau: float, c, targets=None) -> np.ndarray:
    """sigma_v(I) = sum_J (H_tau)_IJ c_v(J) for I in targets (default all).

    c is [nvec][dim]; returns [nvec][len(targets)]."""
    h, eri = _ints(h, eri)
    c = np.ascontiguousarray(np.atleast_2d(c), dtype=np.float64)
    nvec = c.shape[0]
    if c.shape[1] != space.dim:
        raise ValueError("c has wrong length")
    if targets is None:
        nt = space.dim
        tp = None
    else:
        tg = np.ascontiguousarray(targets, dtype=np.int64)
        nt = tg.size
        tp = _p(tg, _i64p)
    out = np.zeros((nvec, nt))
    for v0 in range(0, nvec, 64):
        v1 = min(nvec, v0 + 64)
        cc = np.ascontiguousarray(c[v0:v1])
        oo = np.zeros((v1 - v0, nt))
        rc = lib().orc_sigma(space._h, _p(h), _p(eri), float(tau), v1 - v0, _p(cc),
                             space.dim, nt, tp, _p(oo))
        if rc:
            raise RuntimeError("orc_sigma failed")
        out[v0:v1] = oo
    return out


def diag(space: Space, h, eri, tau: float, targets=None) -> np.ndarray:
    h, eri = _ints(h, eri)
    if targets is None:
        nt, tp = space.dim, None
    else:
        tg = np.ascontiguousarray(targets, dtype=np.int64)
        nt, tp = tg.size, _p(tg, _i64p)
    out = np.zeros(nt)
    lib().orc_diag(space._h, _p(h), _p(eri), float(tau), nt, tp, _p(out))
    return out


def terms(space: Space, h, eri, tau: float):
    """(kept, all) unit counts per bucket (42 buckets, see bucket_names())."""
    h, eri = _ints(h, eri)
    kept = np.zeros(NBUCKET, dtype=np.int64)
    allc = np.zeros(NBUCKET, dtype=np.int64)
    lib().orc_terms(space._h, _p(h), _p(eri), float(tau), _p(kept, _i64p), _p(allc, _i64p))
    return kept, allc


def dense_h(space: Space, h, eri, tau: float) -> np.ndarray:
    if space.dim > 20000:
        raise ValueError("dense H only for tiny spaces")
    h, eri = _ints(h, eri)
    H = np.zeros((space.dim, space.dim))
    lib().orc_dense_h(space._h, _p(h), _p(eri), float(tau), _p(H))
    return H


def dropped_bound(space: Space, h, eri, tau: float) -> float:
    h, eri = _ints(h, eri)
    b = np.zeros(1)
    lib().orc_dropped_bound(space._h, _p(h), _p(eri), float(tau), _p(b))
    return float(b[0])


def apply_word(word, order: int = 0):
    """word: list of ('+', k) creators / ('-', k) annihilators, left to right,
    acting on the vacuum.  Returns (sign, creators) or (0, None)."""
    n = len(word)
    ty = np.array([1 if t == "+" else -1 for t, _ in word], dtype=np.intc)
    op = np.array([k for _, k in word], dtype=np.intc)
    out = np.zeros(max(n, 1), dtype=np.intc)
    sg = np.zeros(1, dtype=np.intc)
    ln = lib().orc_apply_word(n, _p(ty, _ip), _p(op, _ip), int(order), _p(out, _ip), _p(sg, _ip))
    if ln < 0:
        return 0, None
    return int(sg[0]), [int(x) for x in out[:ln]]


def bucket_names():
    names = []
    ov = "ov"
    for spin in "ab":
        for ep in range(2):
            for eq in range(2):
                names.append(f"1b_{spin}_{ov[ep]}{ov[eq]}")
    for spin in ("aa", "bb"):
        for nc in range(3):
            for na in range(3):
                names.append(f"ss_{spin}_c{nc}a{na}")
    for ep in range(2):
        for eq in range(2):
            for er in range(2):
                for es in range(2):
                    names.append(f"ab_{ov[ep]}{ov[eq]}|{ov[er]}{ov[es]}")
    return names


def dim_closed_form(norb: int, nalpha: int, nbeta: int, level: int, boundary: int | None = None) -> int:
    """sum over ka + kb <= level of C(ba,na-ka) C(norb-ba,ka) C(bb,nb-kb) C(norb-bb,kb),
    with the boundary b_sigma = n_sigma (the CI hierarchy) unless given."""
    ba = nalpha if boundary is None else boundary
    bb = nbeta if boundary is None else boundary
    tot = 0
    for ka in range(0, nalpha + 1):
        for kb in range(0, nbeta + 1):
            if ka + kb <= level:
                tot += (comb(ba, nalpha - ka) * comb(norb - ba, ka)
                        * comb(bb, nbeta - kb) * comb(norb - bb, kb))
    return tot


def e_ref_closed_form(h, eri, nalpha: int, nbeta: int) -> float:
    """E_ref = sum_i h_ii + 1/2 sum_ij [(ii|jj) - delta_{spin} (ij|ji)] over
    the occupied spin orbitals of the reference (orbitals 0..n-1 per spin)."""
    occ = [(i, 0) for i in range(nalpha)] + [(i, 1) for i in range(nbeta)]
    e = sum(h[i, i] for i, _ in occ)
    for i, si in occ:
        for j, sj in occ:
            e += 0.5 * eri[i, i, j, j]
            if si == sj:
                e -= 0.5 * eri[i, j, j, i]
    return float(e)


def assemble_factored(L) -> np.ndarray:
    """Dense (pq|rs) = sum_K L^K_pq L^K_rs from factors L [naux][norb][norb],
    summed K by K in ascending order with each product and each partial sum
    rounded once (numpy elementwise operations, no fused multiply-add): the
    definition of factored integrals written out in the order the library's
    factored handles use, so both sides screen the same doubles."""
    L = np.ascontiguousarray(L, dtype=np.float64)
    naux, n, n2 = L.shape
    if n != n2:
        raise ValueError("L must be [naux][norb][norb]")
    out = np.zeros((n, n, n, n))
    for K in range(naux):
        out = out + np.multiply.outer(L[K], L[K])
    return out


def dense_eigh(space: Space, h, eri, tau: float):
    H = dense_h(space, h, eri, tau)
    return np.linalg.eigh(H)


def davidson(space: Space, h, eri, tau: float, nroots: int = 1, tol: float = 1e-8,
             maxiter: int = 200, max_subspace: int | None = None, diagonal=None):
    """Textbook Davidson (Davidson 1975) on the oracle sigma.

    Returns (energies, vectors [nroots][dim], residual norms)."""
    dim = space.dim
    D = diag(space, h, eri, tau) if diagonal is None else diagonal
    k = min(nroots, dim)
    mmax = max_subspace or max(24, 8 * k)
    mmax = min(mmax, dim)
    order = np.argsort(D, kind="stable")
    V = np.zeros((dim, min(dim, max(k, 2 * k))))
    for i in range(V.shape[1]):
        V[order[i], i] = 1.0
    W = sigma(space, h, eri, tau, V.T).T
    theta = None
    rn = None
    for _ in range(maxiter):
        G = V.T @ W
        G = 0.5 * (G + G.T)
        th, y = np.linalg.eigh(G)
        th, y = th[:k], y[:, :k]
        X = V @ y
        R = W @ y - X * th
        rn = np.linalg.norm(R, axis=0)
        theta = th
        if np.all(rn <= tol):
            return th, X.T, rn
        new = []
        for i in range(k):
            if rn[i] <= tol:
                continue
            den = th[i] - D
            den = np.where(np.abs(den) < 1e-8, np.copysign(1e-8, den), den)
            new.append(R[:, i] / den)
        if V.shape[1] + len(new) > mmax:
            V = X.copy()
            W = W @ y
            Q, _ = np.linalg.qr(V)
            # re-express W in the orthonormalised basis
            W = sigma(space, h, eri, tau, Q.T).T
            V = Q
        add = []
        for t in new:
            for _rep in range(2):
                t = t - V @ (V.T @ t)
                for a in add:
                    t = t - a * (a @ t)
            nrm = np.linalg.norm(t)
            if nrm > 1e-10:
                add.append(t / nrm)
        if not add:
            break
        A = np.stack(add, axis=1)
        WA = sigma(space, h, eri, tau, A.T).T
        V = np.hstack([V, A])
        W = np.hstack([W, WA])
    return theta, (V @ np.linalg.eigh(0.5 * (V.T @ W + W.T @ V))[1][:, :k]).T, rn


def _excite(orbs, p, q):
    """a+_p a_q on the ascending creator string `orbs`: (sign, new string) or
    None.  a_q moves past the creators left of q; a+_p is then moved from the
    front to its ascending place past the creators below p."""
    if q not in orbs:
        return None
    k = orbs.index(q)
    rest = orbs[:k] + orbs[k + 1:]
    if p in rest:
        return None
    below = sum(1 for x in rest if x < p)
    if "D1_HALF_SIGN" in _PLANT:
        below = 0
    sign = -1 if (k + below) % 2 else 1
    return sign, tuple(sorted(rest + (p,)))


def density1(space: Space, c) -> np.ndarray:
    """One-body density matrix of each vector, by spin: the paper's D1 (its
    density-matrix subsection, Eq. d1) with spin-orbital indices
    restricted to one spin, d[v, s, p, q] = <c_v| a+_{p s} a_{q s} |c_v>,
    s = 0 alpha, 1 beta.

    Every (source determinant, replacement q -> p) pair that lands in the
    space contributes sign * c(target) * c(source).  An alpha replacement
    keeps the beta string, so the pair's contributions along a row are one
    dot product over the beta strings both rows hold (rows are prefixes of
    the beta list); a beta replacement stays inside its alpha row.  The
    alpha creators stand left of the beta ones, and a+ a moved past them is
    even, so beta replacements carry only their own sign."""
    c = np.atleast_2d(np.asarray(c, dtype=np.float64))
    nv = c.shape[0]
    norb = space.norb
    ao, _ = space.strings(0)
    bo, _ = space.strings(1)
    rs = space.rowstart()
    ln = np.diff(rs)
    amap = {tuple(int(x) for x in o): i for i, o in enumerate(ao)}
    bmap = {tuple(int(x) for x in o): i for i, o in enumerate(bo)}
    d = np.zeros((nv, 2, norb, norb))
    for i, o in enumerate(ao):
        src = tuple(int(x) for x in o)
        for q in src:
            for p in range(norb):
                r = _excite(src, p, q)
                if r is None or r[1] not in amap:
                    continue
                j = amap[r[1]]
                m = int(max(ln[i], ln[j]) if "D1_LONG_ROW" in _PLANT else min(ln[i], ln[j]))
                d[:, 0, p, q] += r[0] * np.einsum("vk,vk->v", c[:, rs[j]:rs[j] + m], c[:, rs[i]:rs[i] + m])
    K, J, P, Q, S = [], [], [], [], []
    for k, o in enumerate(bo):
        src = tuple(int(x) for x in o)
        for q in src:
            for p in range(norb):
                r = _excite(src, p, q)
                if r is None or r[1] not in bmap:
                    continue
                K.append(k); J.append(bmap[r[1]]); P.append(p); Q.append(q); S.append(r[0])
    K, J, P, Q, S = (np.array(x, dtype=np.int64) for x in (K, J, P, Q, S))
    for i in range(len(ao)):
        sel = (K < ln[i]) & (J < ln[i])
        if not sel.any():
            continue
        vals = S[sel] * c[:, rs[i] + J[sel]] * c[:, rs[i] + K[sel]]
        if "D1_BETA_PAST_ALPHA" in _PLANT and space.nalpha % 2:
            vals = -vals
        for v in range(nv):
            np.add.at(d[v, 1], (P[sel], Q[sel]), vals[v])
    return d


def _word(orbs, ops):
    """Apply an operator word to the ascending creator string `orbs`: ops
    are (kind, orbital) pairs in the order they act (rightmost operator of
    the word first), kind '-' annihilates (sign (-1)^position), '+' creates
    at the front and sorts into place (sign (-1)^(#creators below)).
    Returns (sign, new string) or None when the word gives zero."""
    cur = list(orbs)
    sign = 1
    for kind, x in ops:
        if kind == "-":
            if x not in cur:
                return None
            k = cur.index(x)
            sign = -sign if k % 2 else sign
            del cur[k]
        else:
            if x in cur:
                return None
            below = sum(1 for y in cur if y < x)
            sign = -sign if below % 2 else sign
            cur.append(x)
            cur.sort()
    return sign, tuple(cur)


def density2(space: Space, c) -> np.ndarray:
    """Two-body density matrices of each vector by spin block: the paper's
    D2 (its density-matrix subsection, Eq. d2) with spin-orbital indices,
    d[v, b, p, q, r, s] = <c_v| a+_{p S} a+_{r S'} a_{s S'} a_{q S} |c_v>,
    b = 0: S = S' = alpha, 1: S = alpha, S' = beta, 2: S = S' = beta.  The
    block S = beta, S' = alpha is d[v, 1] with (p, q) and (r, s) exchanged.

    Every (source determinant, word) pair that lands in the space adds
    sign * c(target) * c(source), the sign from applying the word to the
    ordered creators.  Same-spin words act on one spin's string (the other
    string is unchanged: alpha words pair rows over the beta strings both
    hold; beta words stay in a row, and passing the alpha creators with an
    even number of operators costs no sign).  The alpha-beta word equals
    (a+_{p a} a_{q a})(a+_{r b} a_{s b}) (a_{q a} moved past two beta
    operators), so its sign is the product of the two replacements'."""
    c = np.atleast_2d(np.asarray(c, dtype=np.float64))
    nv = c.shape[0]
    n = space.norb
    ao, _ = space.strings(0)
    bo, _ = space.strings(1)
    rs = space.rowstart()
    ln = np.diff(rs)
    amap = {tuple(int(x) for x in o): i for i, o in enumerate(ao)}
    bmap = {tuple(int(x) for x in o): i for i, o in enumerate(bo)}
    d = np.zeros((nv, 3, n, n, n, n))
    # alpha-alpha: pair rows over the beta strings both hold
    for i, o in enumerate(ao):
        src = tuple(int(x) for x in o)
        for q in src:
            for s_ in src:
                for p in range(n):
                    for r in range(n):
                        w = _word(src, [("-", q), ("-", s_), ("+", r), ("+", p)])
                        if w is None or w[1] not in amap:
                            continue
                        j = amap[w[1]]
                        m = int(min(ln[i], ln[j]))
                        d[:, 0, p, q, r, s_] += w[0] * np.einsum("vk,vk->v", c[:, rs[j]:rs[j] + m],
                                                                 c[:, rs[i]:rs[i] + m])
    # beta words of one row, tabulated once: source k, target j, sign
    def beta_words(two):
        tab = []
        for k, o in enumerate(bo):
            src = tuple(int(x) for x in o)
            for q in src:
                for s_ in (src if two else [None]):
                    for p in range(n):
                        for r in (range(n) if two else [None]):
                            ops = [("-", q), ("-", s_), ("+", r), ("+", p)] if two else [("-", q), ("+", p)]
                            w = _word(src, ops)
                            if w is None or w[1] not in bmap:
                                continue
                            tab.append((k, bmap[w[1]], p, q, r, s_, w[0]))
        return tab
    bb = beta_words(True)
    for i in range(len(ao)):
        for k, j, p, q, r, s_, sg in bb:
            if k < ln[i] and j < ln[i]:
                d[:, 2, p, q, r, s_] += sg * c[:, rs[i] + j] * c[:, rs[i] + k]
    # alpha-beta: an alpha replacement q -> p times a beta replacement s -> r
    b1 = beta_words(False)
    for i, o in enumerate(ao):
        src = tuple(int(x) for x in o)
        for q in src:
            for p in range(n):
                w = _word(src, [("-", q), ("+", p)])
                if w is None or w[1] not in amap:
                    continue
                j = amap[w[1]]
                for k, jb, r, s_, _u1, _u2, sb in b1:
                    if k < ln[i] and jb < ln[j]:
                        sgn = w[0] * (1 if "D2_AB_NO_BETA_SIGN" in _PLANT else sb)
                        d[:, 1, p, q, r, s_] += sgn * c[:, rs[j] + jb] * c[:, rs[i] + k]
    if "D2_AA_SWAP_QS" in _PLANT:
        d[:, 0] = d[:, 0].transpose(0, 1, 4, 3, 2).copy()
    return d


def propagate_exact(space: Space, h, eri, tau: float, c_re, c_im=None, t: float = 0.0, imaginary: bool = True,
                    nsteps: int = 1, coef_tau: float = 0.0):
    """exp(-H_tau t) c normalised (imaginary time) or exp(-i H_tau t) (c_re +
    i c_im) (real time) for tiny spaces, by the spectral decomposition of
    the dense H_tau: the propagation the library's short-iterative
    Arnoldi-Lanczos steps approximate.  With coef_tau > 0 the time t is
    taken in nsteps equal steps and, after each (and after the
    normalisation in imaginary time), every coefficient of modulus <=
    coef_tau is set to zero: the screening of small CI coefficients the
    paper proposes.  Returns a real vector (imaginary) or a complex one
    (real time)."""
    H = dense_h(space, h, eri, tau)
    w, V = np.linalg.eigh(0.5 * (H + H.T))
    c = np.asarray(c_re, dtype=np.float64) + (0.0 if c_im is None else 1j * np.asarray(c_im, dtype=np.float64))
    steps = nsteps if coef_tau > 0.0 else 1
    dt = t / steps
    for _ in range(steps):
        y = V.T @ c
        if imaginary:
            c = np.real(V @ (np.exp(-(w - w[0]) * dt) * y))
            c = c / np.linalg.norm(c)
        else:
            c = V @ (np.exp(-1j * w * dt) * y)
        if coef_tau > 0.0:
            c = np.where(np.abs(c) <= coef_tau, 0.0, c)
    return c


def mask_by_distance(h, eri, dist, dmax: float):
    """Distance screening of the integrals: h_pq set to zero when d(p, q) >
    dmax, (pq|rs) when any of the six distances among p, q, r, s exceeds
    dmax (the additional distance-dependent screening the paper proposes).
    Returns masked copies."""
    h = np.array(h, dtype=np.float64)
    eri = np.array(eri, dtype=np.float64)
    d = np.asarray(dist, dtype=np.float64)
    far = (d > dmax) | (d.T > dmax)     # a pair is as far as its larger entry
    h[far] = 0.0
    n = h.shape[0]
    I = np.arange(n)
    p, q, r, s = np.meshgrid(I, I, I, I, indexing="ij")
    span_far = far[p, q] | far[p, r] | far[p, s] | far[q, r] | far[q, s] | far[r, s]
    eri[span_far] = 0.0
    return h, eri
