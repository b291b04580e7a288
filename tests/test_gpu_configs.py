"""GPU parity at the benchmark configurations' full sizes and at the
largest orbital counts the served workload reaches: sampled targets (row
ends included) against the CPU oracle, the tolerance scaled by the oracle's
values on those targets; Davidson energies of the 30-orbital CISDT
workload against the oracle's own Davidson (stored by
tests/golden/make_davidson_cisdt_n30.py).

Bar: sigma |delta| <= 1e-12 * ||sigma||_inf (Eq. sigma; screened units
removed as in Eqs. sigma_int / sigma_split), energies within 1e-10 Eh."""
import os

import numpy as np
import pytest

import oracle as O
from isci_inputs import random_vectors, recipe_a, workload

from gpu_common import create, gpu_sigma, sample_targets, sampled_ok, torch_dev

pytestmark = pytest.mark.gpu
TOL = 1e-12
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _sampled(hd, S, h, eri, tau, nvec, nsamp, seed):
    c = random_vectors(S.dim, nvec, seed=seed)
    got = gpu_sigma(hd, c)
    tg = sample_targets(S.rowstart(), S.dim, nsamp, seed=seed + 1)
    ref = O.sigma(S, h, eri, tau, c, targets=tg)
    ok, err = sampled_ok(got, tg, ref, TOL)
    assert ok, err


@pytest.mark.parametrize("tau", [0.0, 1e-10])
def test_cisdt_n60_tau_sweep(tau):
    """CISDT, 60 orbitals: tau = 0 keeps every non-zero unit (about 48 times
    the tau = 1e-14 list), tau = 1e-10 drops more."""
    W = workload("cisdt_n60")
    h, eri = W.integrals()
    print(f"cisdt_n60 tau={tau:g}", flush=True)
    hd = create(h, eri, W.norb, 2, 2, W.level, tau)
    S = O.Space(W.norb, 2, 2, W.level)
    _sampled(hd, S, h, eri, tau, 2, 300, seed=40)


def test_cisdt_n120():
    """The largest box of the box-length scan: CISDT, 120 orbitals."""
    W = workload("cisdt_n120")
    h, eri = W.integrals()
    print("cisdt_n120", flush=True)
    hd = create(h, eri, W.norb, 2, 2, W.level, W.tau)
    S = O.Space(W.norb, 2, 2, W.level)
    _sampled(hd, S, h, eri, W.tau, 2, 300, seed=41)


def test_cisdt_n160_workload():
    """The served-size CISDT workload (160 orbitals, tau 1e-12, 4 vectors),
    a larger sample."""
    W = workload("cisdt_n160")
    h, eri = W.integrals()
    print("cisdt_n160", flush=True)
    hd = create(h, eri, W.norb, 2, 2, W.level, W.tau)
    S = O.Space(W.norb, 2, 2, W.level)
    _sampled(hd, S, h, eri, W.tau, W.nvec, 1500, seed=42)


@pytest.mark.parametrize("norb", [176, 199])
def test_cisdt_largest_orbital_counts(norb):
    """CISDT above 160 orbitals: the spectator-form one-body kernel with 11
    and 13 orbital tiles (199 orbitals needs the fourth 64-row mask).  Both
    sides read only the canonical element of (pq|rs), so the tensor is
    passed as assembled."""
    tau = 1e-12
    h, eri = recipe_a(norb, seed=4, canonical=False)
    print(f"cisdt norb={norb}", flush=True)
    hd = create(h, eri, norb, 2, 2, 3, tau)
    S = O.Space(norb, 2, 2, 3)
    _sampled(hd, S, h, eri, tau, 2, 300, seed=43)


def _golden_energies():
    vals = []
    for line in open(os.path.join(GOLDEN, "davidson_cisdt_n30.txt")):
        line = line.strip()
        if line and not line.startswith("#"):
            vals.append(float(line))
    return np.array(vals)


def test_davidson_cisdt_n30_against_oracle():
    """CISDT, 30 orbitals (the smallest box of the scan): the library's
    Davidson energies against the oracle's Davidson, 1e-10 Eh."""
    import paper_1609_07757_amd as isci
    torch_dev()
    ref = _golden_energies()
    W = workload("cisdt_n30")
    h, eri = W.integrals()
    hd = create(h, eri, W.norb, 2, 2, W.level, W.tau)
    e, _, info = isci.isci_davidson(hd, nroots=len(ref), tol_residual=1e-8, max_iter=600)
    assert info["converged"]
    assert np.abs(e - ref).max() <= 1e-10, (e, ref)


@pytest.mark.parametrize("where", ["eri", "h", "eri_inf"])
def test_nonfinite_integrals_rejected(where):
    """A NaN or infinity among the integrals read (the canonical elements of
    eri, the lower triangle of h) is refused with ISCI_E_INVALID before any
    list is built; one in a position that is never read is ignored."""
    import paper_1609_07757_amd as isci
    torch_dev()
    norb = 8
    h, eri = recipe_a(norb, seed=2)
    h = h.copy()
    eri = eri.copy()
    if where == "eri":
        eri[5, 2, 3, 1] = np.nan           # canonical: 5 >= 2, 3 >= 1, (5,2) >= (3,1)
    elif where == "h":
        h[6, 1] = np.nan                   # lower triangle
    else:
        eri[4, 4, 0, 0] = np.inf
    with pytest.raises(isci.IsciError) as ex:
        create(h, eri, norb, 2, 2, 2, 1e-12)
    assert ex.value.status == -1
    h2, eri2 = recipe_a(norb, seed=2)
    eri2 = eri2.copy()
    h2 = h2.copy()
    eri2[2, 5, 1, 3] = np.nan              # not canonical (2 < 5): never read
    h2[1, 6] = np.nan                      # upper triangle: never read
    hd = create(h2, eri2, norb, 2, 2, 2, 1e-12)
    c = random_vectors(hd.dim, 1, seed=1)
    assert np.all(np.isfinite(gpu_sigma(hd, c)))
