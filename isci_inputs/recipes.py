"""Seeded integral recipes (one-electron h and two-electron (pq|rs)).

Recipe A is the synthetic stand-in for the paper's beryllium FE-DVR
integrals (application section, basis and set-up): local orbitals on a
1D box of length ``box`` with one orbital per unit length, so that
integrals between distant orbitals decay below the screening threshold.

    x_p   = p * box / norb + U(-0.05, 0.05)          (draw 1: jitter)
    eps_p = sort(U(-2, 1))                           (draw 2)
    X_K   ~ U(0, box),  K = 1..naux                  (draw 3)
    h_pq  = eps_p delta_pq - 0.5 exp(-|x_p - x_q|)
    L^K_pq = 0.7 g_p(X_K) g_q(X_K),  g_p(x) = exp(-(x - x_p)^2 / 2)
    (pq|rs) = sum_K L^K_pq L^K_rs

Recipe A makes (pq|rs) symmetric in all four indices, so every same-spin
antisymmetrised coefficient (ps|rq) - (pq|rs) is rounding noise.  Recipe B
multiplies L^K_pq by (1 + 0.3 cos(x_p - x_q)), which keeps the 8-fold
permutational symmetry and positive semidefiniteness but breaks the
total symmetry, so the same-spin class carries real weight.  The random
recipe draws an unstructured 8-fold symmetric tensor for tests that must
see every index permutation.

Nothing here implements the CI method: these functions only produce the
arrays that both the oracle and the library take as input.
"""
from __future__ import annotations

import numpy as np


def _grid(norb: int, box: float, naux: int, seed: int):
    rng = np.random.default_rng(seed)
    x = np.arange(norb, dtype=np.float64) * (box / norb) + rng.uniform(-0.05, 0.05, norb)
    eps = np.sort(rng.uniform(-2.0, 1.0, norb))
    X = rng.uniform(0.0, box, naux)
    return x, eps, X


def orbital_centres(norb: int, box: float, naux: int, seed: int) -> np.ndarray:
    """Centres x_p of the recipe's local orbitals (the same draw as the
    integrals of that seed), for distance matrices |x_p - x_q|."""
    return _grid(norb, box, naux, seed)[0]


def _h_of(x, eps):
    h = -0.5 * np.exp(-np.abs(x[:, None] - x[None, :]))
    h[np.diag_indices_from(h)] += eps
    return symmetrize_h(h)


def factors_a(norb: int, box: float, naux: int, seed: int, recipe: str = "A"):
    """Return (h, Lfac) with Lfac[K, p, q] = L^K_pq for recipe A or B."""
    x, eps, X = _grid(norb, box, naux, seed)
    g = np.exp(-0.5 * (X[:, None] - x[None, :]) ** 2)          # [K, p]
    L = 0.7 * g[:, :, None] * g[:, None, :]                     # [K, p, q]
    if recipe == "B":
        L = L * (1.0 + 0.3 * np.cos(x[:, None] - x[None, :]))[None]
    elif recipe != "A":
        raise ValueError(recipe)
    return _h_of(x, eps), L


def assemble_eri(L: np.ndarray) -> np.ndarray:
    """(pq|rs) = sum_K L[K,p,q] L[K,r,s] as one dense norb^4 array."""
    K, n, _ = L.shape
    M = L.reshape(K, n * n)
    return (M.T @ M).reshape(n, n, n, n)


def recipe_a(norb: int, box: float | None = None, naux: int | None = None,
             seed: int = 0, canonical: bool = True):
    """Recipe A.  Defaults follow the workloads: box = norb, naux = 2 box."""
    box = float(norb) if box is None else float(box)
    naux = int(round(2 * box)) if naux is None else int(naux)
    h, L = factors_a(norb, box, naux, seed, "A")
    eri = assemble_eri(L)
    return h, (canonicalize_eri(eri) if canonical else eri)


def recipe_b(norb: int, box: float | None = None, naux: int | None = None,
             seed: int = 0, canonical: bool = True):
    box = float(norb) if box is None else float(box)
    naux = int(round(2 * box)) if naux is None else int(naux)
    h, L = factors_a(norb, box, naux, seed, "B")
    eri = assemble_eri(L)
    return h, (canonicalize_eri(eri) if canonical else eri)


def recipe_random(norb: int, seed: int = 0, hscale: float = 1.0,
                  gscale: float = 0.3, canonical: bool = True):
    """Unstructured h (symmetric) and 8-fold symmetric (pq|rs)."""
    rng = np.random.default_rng(seed)
    h = rng.normal(scale=hscale, size=(norb, norb))
    h = symmetrize_h(h)
    eri = rng.normal(scale=gscale, size=(norb, norb, norb, norb))
    return h, (canonicalize_eri(eri) if canonical else eri)


def symmetrize_h(h: np.ndarray) -> np.ndarray:
    """Copy the lower triangle (p >= q) onto the upper one."""
    h = np.array(h, dtype=np.float64, copy=True)
    iu = np.triu_indices(h.shape[0], 1)
    h[iu] = h.T[iu]
    return h


def canonicalize_eri(eri: np.ndarray) -> np.ndarray:
    """Copy each canonical element (p>=q, r>=s, (p,q)>=(r,s)) to its 8 images.

    The result is exactly (bit-for-bit) invariant under p<->q, r<->s and
    (pq)<->(rs).
    """
    E = np.asarray(eri, dtype=np.float64)
    n = E.shape[0]
    i = np.arange(n)
    ge = (i[:, None] >= i[None, :])                       # [p, q]: p >= q
    E = np.where(ge[:, :, None, None], E, E.transpose(1, 0, 2, 3))
    E = np.where(ge[None, None, :, :], E, E.transpose(0, 1, 3, 2))
    hi = np.maximum(i[:, None], i[None, :])
    lo = np.minimum(i[:, None], i[None, :])
    key = hi * n + lo                                     # pair order on (max, min)
    keep = key[:, :, None, None] >= key[None, None, :, :]
    E = np.where(keep, E, E.transpose(2, 3, 0, 1))
    return np.ascontiguousarray(E)


def random_vectors(dim: int, nvec: int, seed: int) -> np.ndarray:
    """[nvec][dim] standard normal vectors."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((nvec, dim))
