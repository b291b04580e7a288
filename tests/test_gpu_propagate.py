"""GPU: short-iterative Arnoldi-Lanczos propagation (isci_propagate) in
real and imaginary time against the oracle's exact propagation (spectral
decomposition of the dense H_tau) on small spaces; imaginary-time
convergence to the Davidson ground state; real-time conservation of norm
and energy at a larger size; coefficient screening."""
import numpy as np
import pytest

import oracle as O
from isci_inputs import random_vectors, recipe_a, recipe_b, workload

from gpu_common import create, torch_dev

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("recipe,norb,L,tau", [("B", 8, 2, 0.0), ("A", 10, 3, 1e-12), ("B", 7, 4, 1e-10)])
def test_real_time_against_exact(recipe, norb, L, tau):
    import paper_1609_07757_amd as isci
    torch, dev = torch_dev()
    h, eri = (recipe_a if recipe == "A" else recipe_b)(norb, seed=2)
    S = O.Space(norb, 2, 2, L)
    hd = create(h, eri, norb, 2, 2, L, tau)
    re, im = random_vectors(S.dim, 2, seed=4)
    cr, ci = torch.from_numpy(re.copy()).to(dev), torch.from_numpy(im.copy()).to(dev)
    dt, n = 0.3, 4
    info = isci.isci_propagate(hd, cr, dt, n, c_im=ci, imaginary=False, krylov=24, tol=1e-14)
    got = cr.cpu().numpy() + 1j * ci.cpu().numpy()
    want = O.propagate_exact(S, h, eri, tau, re, im, dt * n, imaginary=False)
    assert np.abs(got - want).max() <= 1e-10 * np.abs(want).max()
    assert abs(info["norm"] - np.linalg.norm(re + 1j * im)) <= 1e-10 * info["norm"]


@pytest.mark.parametrize("recipe,norb,L,tau", [("B", 8, 2, 0.0), ("A", 9, 4, 1e-12)])
def test_imaginary_time_against_exact(recipe, norb, L, tau):
    import paper_1609_07757_amd as isci
    torch, dev = torch_dev()
    h, eri = (recipe_a if recipe == "A" else recipe_b)(norb, seed=5)
    S = O.Space(norb, 2, 2, L)
    hd = create(h, eri, norb, 2, 2, L, tau)
    u = random_vectors(S.dim, 1, seed=6)[0]
    u /= np.linalg.norm(u)
    cu = torch.from_numpy(u.copy()).to(dev)
    isci.isci_propagate(hd, cu, 0.2, 5, krylov=24, tol=1e-14)
    want = O.propagate_exact(S, h, eri, tau, u, None, 1.0)
    assert np.abs(cu.cpu().numpy() - want).max() <= 1e-10


def test_imaginary_time_reaches_ground_state():
    """The paper's optimiser: imaginary-time propagation of the CISD/20
    workload converges to the Davidson ground-state energy."""
    import paper_1609_07757_amd as isci
    torch, dev = torch_dev()
    W = workload("cisd_n20")
    h, eri = W.integrals()
    hd = create(h, eri, W.norb, 2, 2, W.level, W.tau)
    e_dav, _, _ = isci.isci_davidson(hd, nroots=1, tol_residual=1e-9)
    c = torch.zeros(hd.dim, dtype=torch.float64, device=dev)
    c[0] = 1.0
    info = isci.isci_propagate(hd, c, 5.0, 60, krylov=16)
    assert abs(info["energy"] - e_dav[0]) <= 1e-9, (info, e_dav)
    assert abs(info["norm"] - 1.0) <= 1e-12


def test_real_time_conserves_norm_and_energy_cisdt_n30():
    import paper_1609_07757_amd as isci
    torch, dev = torch_dev()
    W = workload("cisdt_n30")
    h, eri = W.integrals()
    hd = create(h, eri, W.norb, 2, 2, W.level, W.tau)
    re, im = random_vectors(hd.dim, 2, seed=8)
    cr, ci = torch.from_numpy(re.copy()).to(dev), torch.from_numpy(im.copy()).to(dev)
    i0 = isci.isci_propagate(hd, cr.clone(), 0.0, 0, c_im=ci.clone(), imaginary=False)
    i1 = isci.isci_propagate(hd, cr, 0.2, 5, c_im=ci, imaginary=False, krylov=24, tol=1e-13)
    assert abs(i1["norm"] - i0["norm"]) <= 1e-10 * i0["norm"]
    assert abs(i1["energy"] - i0["energy"]) <= 1e-9 * abs(i0["energy"])


def _screen_margin(S, h, eri, tau, re, im, dt, nsteps, thr, imaginary):
    """Smallest distance between a coefficient modulus and the threshold over
    the oracle's screened steps (the comparison below needs it well above
    the propagators' rounding)."""
    c_re, c_im = re, im
    margin = np.inf
    for _ in range(nsteps):
        c = O.propagate_exact(S, h, eri, tau, c_re, c_im, dt, imaginary=imaginary)
        margin = min(margin, float(np.abs(np.abs(c) - thr).min()))
        c = O.propagate_exact(S, h, eri, tau, c_re, c_im, dt, imaginary=imaginary, nsteps=1, coef_tau=thr)
        c_re, c_im = np.real(c), (np.imag(c) if not imaginary else None)
    return margin


@pytest.mark.parametrize("recipe,norb,L,imaginary,thr", [("B", 8, 2, True, 1e-4), ("A", 10, 3, True, 1e-5),
                                                          ("B", 8, 3, False, 1e-3), ("A", 9, 2, False, 1e-4)])
def test_coefficient_screening_against_oracle(recipe, norb, L, imaginary, thr):
    """Each step is followed by the screening of coefficients of modulus <=
    thr (after the normalisation in imaginary time), as in the oracle."""
    import paper_1609_07757_amd as isci
    torch, dev = torch_dev()
    h, eri = (recipe_a if recipe == "A" else recipe_b)(norb, seed=5)
    S = O.Space(norb, 2, 2, L)
    hd = create(h, eri, norb, 2, 2, L, 0.0)
    re = np.zeros(S.dim)
    re[0] = 1.0
    im = None if imaginary else np.zeros(S.dim)
    dt, n = 0.25, 6
    assert _screen_margin(S, h, eri, 0.0, re, im, dt, n, thr, imaginary) > 1e-8
    want = O.propagate_exact(S, h, eri, 0.0, re, im, dt * n, imaginary=imaginary, nsteps=n, coef_tau=thr)
    cr = torch.from_numpy(re.copy()).to(dev)
    ci = None if imaginary else torch.from_numpy(im.copy()).to(dev)
    info = isci.isci_propagate(hd, cr, dt, n, c_im=ci, imaginary=imaginary, krylov=32, tol=1e-14, coef_tau=thr)
    got = cr.cpu().numpy() + (0.0 if imaginary else 1j * ci.cpu().numpy())
    assert np.array_equal(got == 0, want == 0)
    assert np.abs(got - want).max() <= 1e-10
    assert info["screened_last"] > 0


def test_coefficient_screening_cisd_n20():
    """The CISD/20 workload: screened imaginary-time energies stay above the
    unscreened ground state (variational) and approach it as the threshold
    falls."""
    import paper_1609_07757_amd as isci
    torch, dev = torch_dev()
    W = workload("cisd_n20")
    h, eri = W.integrals()
    hd = create(h, eri, W.norb, 2, 2, W.level, W.tau)
    c0 = torch.zeros(hd.dim, dtype=torch.float64, device=dev)
    c0[0] = 1.0
    e = {}
    for thr in (0.0, 1e-8, 1e-6, 1e-4):
        v = c0.clone()
        info = isci.isci_propagate(hd, v, 5.0, 60, krylov=16, coef_tau=thr)
        e[thr] = info["energy"]
        if thr >= 1e-6:
            assert info["screened_last"] > 0
            assert int((v == 0).sum()) >= info["screened_last"]
    assert e[1e-8] >= e[0.0] - 1e-10 and e[1e-6] >= e[0.0] - 1e-10 and e[1e-4] >= e[0.0] - 1e-10
    assert e[1e-4] - e[0.0] > e[1e-6] - e[0.0] > e[1e-8] - e[0.0] - 1e-10
