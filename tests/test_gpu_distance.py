"""GPU: distance screening (isci_create_opts.orb_dist / max_dist, the
additional distance-dependent screening of Sec. 2).  A handle built with a
radius must equal, bit for bit, a handle built from integrals the oracle
masked by the same radius (oracle.mask_by_distance): same kept units, same
sigma; and the sigma must match the oracle's on the masked integrals.
Dense and factored integrals are both covered.

Bar: sigma |delta| <= 1e-12 * ||sigma||_inf; tables and counts exact."""
import numpy as np
import pytest

import oracle as O
from isci_inputs import random_vectors
from isci_inputs.recipes import factors_a

from gpu_common import gpu_sigma, rel_err, torch_dev

pytestmark = pytest.mark.gpu
TOL = 1e-12


def _chain(norb, seed, spacing=1.0):
    rng = np.random.default_rng(seed)
    x = spacing * np.arange(norb) + 0.2 * rng.uniform(-1, 1, norb)
    return np.abs(x[:, None] - x[None, :])


@pytest.mark.parametrize("norb,na,nb,lev,tau,dmax,nvec", [
    (10, 2, 2, 3, 1e-12, 3.5, 2), (12, 2, 2, 2, 0.0, 5.0, 1), (8, 3, 2, 4, 1e-8, 2.5, 3),
    (9, 1, 1, 2, 0.0, 1.5, 1), (14, 2, 2, 4, 1e-10, 6.0, 2)])
def test_distance_screened_handle(norb, na, nb, lev, tau, dmax, nvec):
    import paper_1609_07757_amd as isci
    torch, dev = torch_dev()
    h, L = factors_a(norb, float(norb), 2 * norb, 3)
    eri = O.assemble_factored(L)
    dist = _chain(norb, 11)
    hm, em = O.mask_by_distance(h, eri, dist, dmax)
    ht = torch.from_numpy(np.ascontiguousarray(h)).to(dev)
    hd = isci.isci_create(ht, torch.from_numpy(eri).to(dev), norb, na, nb, lev, tau,
                          orb_dist=dist, max_dist=dmax)
    hf = isci.isci_create_factored(ht, torch.from_numpy(np.ascontiguousarray(L)).to(dev), norb, na, nb, lev,
                                   tau, orb_dist=dist, max_dist=dmax)
    hr = isci.isci_create(torch.from_numpy(hm).to(dev), torch.from_numpy(em).to(dev), norb, na, nb, lev, tau)
    hu = isci.isci_create(ht, torch.from_numpy(eri).to(dev), norb, na, nb, lev, tau)
    torch.cuda.synchronize()
    S = O.Space(norb, na, nb, lev)
    c = random_vectors(S.dim, nvec, seed=5)
    g = gpu_sigma(hd, c)
    assert rel_err(g, O.sigma(S, hm, em, tau, c)) <= TOL
    sd, sf, sr, su = (isci.isci_get_stats(x) for x in (hd, hf, hr, hu))
    for s in (sf, sr):
        assert np.array_equal(s["kept"], sd["kept"]) and np.array_equal(s["terms"], sd["terms"])
    assert np.array_equal(g, gpu_sigma(hf, c))
    assert np.array_equal(g, gpu_sigma(hr, c))
    assert np.array_equal(isci.isci_diag(hd).cpu().numpy(), isci.isci_diag(hr).cpu().numpy())
    assert int(np.sum(sd["kept"])) < int(np.sum(su["kept"]))


def test_distance_asymmetric_matrix_reads_pair_maximum():
    """A non-symmetric distance matrix acts as its elementwise maximum with
    its transpose, whichever order a unit's orbitals are named in."""
    import paper_1609_07757_amd as isci
    torch, dev = torch_dev()
    norb = 9
    h, L = factors_a(norb, 9.0, 18, 6)
    eri = O.assemble_factored(L)
    rng = np.random.default_rng(3)
    d = _chain(norb, 4) * rng.uniform(0.6, 1.4, (norb, norb))
    np.fill_diagonal(d, 0.0)
    ht, et = torch.from_numpy(h).to(dev), torch.from_numpy(eri).to(dev)
    a = isci.isci_create(ht, et, norb, 2, 2, 3, 0.0, orb_dist=d, max_dist=3.0)
    b = isci.isci_create(ht, et, norb, 2, 2, 3, 0.0, orb_dist=np.maximum(d, d.T), max_dist=3.0)
    S = O.Space(norb, 2, 2, 3)
    c = random_vectors(S.dim, 2, seed=2)
    g = gpu_sigma(a, c)
    assert np.array_equal(g, gpu_sigma(b, c))
    hm, em = O.mask_by_distance(h, eri, d, 3.0)
    assert rel_err(g, O.sigma(S, hm, em, 0.0, c)) <= TOL


def test_distance_radius_above_all_changes_nothing():
    import paper_1609_07757_amd as isci
    torch, dev = torch_dev()
    norb = 10
    h, L = factors_a(norb, float(norb), 20, 4)
    eri = O.assemble_factored(L)
    dist = _chain(norb, 2)
    ht, et = torch.from_numpy(h).to(dev), torch.from_numpy(eri).to(dev)
    a = isci.isci_create(ht, et, norb, 2, 2, 4, 1e-12, orb_dist=dist, max_dist=1e3)
    b = isci.isci_create(ht, et, norb, 2, 2, 4, 1e-12)
    c = random_vectors(O.Space(norb, 2, 2, 4).dim, 2, seed=1)
    assert np.array_equal(gpu_sigma(a, c), gpu_sigma(b, c))
    assert np.array_equal(isci.isci_get_stats(a)["kept"], isci.isci_get_stats(b)["kept"])


def test_distance_argument_errors():
    import paper_1609_07757_amd as isci
    torch, dev = torch_dev()
    norb = 6
    h, L = factors_a(norb, 6.0, 12, 1)
    eri = O.assemble_factored(L)
    ht, et = torch.from_numpy(h).to(dev), torch.from_numpy(eri).to(dev)
    with pytest.raises(ValueError):
        isci.isci_create(ht, et, norb, 2, 2, 2, 0.0, orb_dist=np.zeros((norb, norb + 1)), max_dist=1.0)
    bad = _chain(norb, 1)
    bad[1, 2] = np.nan
    with pytest.raises(RuntimeError):
        isci.isci_create(ht, et, norb, 2, 2, 2, 0.0, orb_dist=bad, max_dist=1.0)
