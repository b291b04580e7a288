"""One-body density matrices on the GPU (isci_density1) against the oracle.

Every element against oracle.density1 (tolerance 1e-12 of the largest
element, the sigma bar), on small spaces and on the 60-orbital CISDT space
of the sigma benchmark (400,491 determinants, 8 vectors).  There also the
properties that hold at any size: the trace of each spin block (electron
count times |c|^2), symmetry, and the one-body energy sum_pq h_pq (D1a +
D1b)_pq against c . sigma of a handle built with the same h, zero
two-electron integrals and no screening."""
import ctypes

import numpy as np
import pytest

import oracle as O
from isci_inputs import random_vectors, recipe_a, recipe_b, recipe_random, workload

from gpu_common import create, torch_dev

pytestmark = pytest.mark.gpu

TOL = 1e-12


def _ints(recipe, norb, seed):
    return {"A": recipe_a, "B": recipe_b}.get(recipe, recipe_random)(norb, seed=seed)


def _gpu_d1(hd, c, ld=None):
    import paper_1609_07757_amd as isci
    torch, dev = torch_dev()
    nvec, dim = c.shape
    ld = ld or dim
    cbuf = torch.full((nvec, ld), float("nan"), dtype=torch.float64, device=dev)
    cbuf[:, :dim] = torch.from_numpy(c).to(dev)
    out = torch.full((nvec, 2, hd.norb, hd.norb), float("nan"), dtype=torch.float64, device=dev)
    if ld == dim:
        isci.isci_density1(hd, cbuf, out)
    else:
        from paper_1609_07757_amd import _lib
        st = _lib.load().isci_density1(hd.ptr, nvec, ctypes.c_void_p(cbuf.data_ptr()), ld,
                                       ctypes.c_void_p(out.data_ptr()),
                                       ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
        _lib.check(st)
    torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize("recipe,norb,na,nb,L", [
    ("A", 6, 2, 2, 2), ("B", 7, 3, 1, 3), ("R", 8, 4, 4, 3), ("A", 9, 2, 2, 3), ("R", 5, 1, 0, 1),
    ("B", 6, 3, 3, 6), ("A", 12, 2, 2, 4), ("A", 20, 2, 2, 2), ("B", 10, 3, 2, 3), ("A", 30, 2, 2, 3),
    ("R", 7, 2, 1, 2), ("R", 6, 1, 1, 2),
    # above 64 orbitals the output has several 64 x 64 tiles
    ("A", 100, 2, 2, 1), ("B", 70, 2, 2, 2), ("R", 66, 3, 2, 1), ("A", 130, 1, 1, 2), ("R", 90, 2, 1, 2)])
def test_density1_parity(recipe, norb, na, nb, L):
    h, eri = _ints(recipe, norb, 3)
    print(f"density1 parity {recipe} norb={norb} na={na} nb={nb} L={L}", flush=True)
    hd = create(h, eri, norb, na, nb, L, 1e-12)
    S = O.Space(norb, na, nb, L)
    c = random_vectors(S.dim, 3, seed=norb * 7 + L)
    c /= np.linalg.norm(c, axis=1, keepdims=True)
    got = _gpu_d1(hd, c)
    want = O.density1(S, c)
    assert np.abs(got - want).max() <= TOL * np.abs(want).max()


def test_density1_padded_leading_dimension_and_repeat():
    norb, na, nb, L = 9, 2, 2, 3
    h, eri = recipe_b(norb, seed=2)
    hd = create(h, eri, norb, na, nb, L, 1e-10)
    S = O.Space(norb, na, nb, L)
    c = random_vectors(S.dim, 2, seed=1)
    a = _gpu_d1(hd, c, ld=S.dim + 37)
    b = _gpu_d1(hd, c, ld=S.dim + 37)
    assert np.array_equal(a, b), "density1 is not reproducible"
    want = O.density1(S, c)
    assert np.abs(a - want).max() <= TOL * np.abs(want).max()


def test_density1_cisdt_n60():
    """Bench-size space (CISDT, 60 orbitals, 8 vectors): every element
    against the oracle, traces, symmetry and the one-body energy identity
    against the library's own sigma."""
    import paper_1609_07757_amd as isci
    torch, dev = torch_dev()
    W = workload("cisdt_n60")
    h, _eri = W.integrals()
    print("density1 cisdt_n60 properties", flush=True)
    hd = create(h, np.zeros((W.norb,) * 4), W.norb, W.nalpha, W.nbeta, W.level, 0.0)
    c = torch.from_numpy(random_vectors(hd.dim, 8, seed=21)).to(dev)
    d = isci.isci_density1(hd, c)
    sg = isci.isci_sigma(hd, c)
    torch.cuda.synchronize()
    d = d.cpu().numpy()
    cn = c.cpu().numpy()
    want = O.density1(O.Space(W.norb, W.nalpha, W.nbeta, W.level), cn)
    assert np.abs(d - want).max() <= TOL * np.abs(want).max()
    e = (cn * sg.cpu().numpy()).sum(1)
    nn = (cn * cn).sum(1)
    scale = np.abs(d).max()
    for v in range(8):
        for s, n in enumerate((W.nalpha, W.nbeta)):
            assert abs(np.trace(d[v, s]) - n * nn[v]) <= 1e-12 * n * nn[v]
            assert np.abs(d[v, s] - d[v, s].T).max() <= TOL * scale
        e1 = (h * (d[v, 0] + d[v, 1])).sum()
        assert abs(e1 - e[v]) <= 1e-11 * np.abs(h).sum() * scale


def test_density1_cisdt_n160_properties():
    """Served-size space (CISDT, 160 orbitals, 7,963,991 determinants, 4
    vectors, nine output tiles): traces, symmetry and the one-body energy
    identity against the library's sigma for zero two-electron integrals."""
    import paper_1609_07757_amd as isci
    torch, dev = torch_dev()
    W = workload("cisdt_n160")
    h, _eri = W.integrals()
    del _eri
    print("density1 cisdt_n160 properties", flush=True)
    hd = create(h, np.zeros((W.norb,) * 4), W.norb, W.nalpha, W.nbeta, W.level, 0.0)
    c = torch.from_numpy(random_vectors(hd.dim, 4, seed=23)).to(dev)
    d = isci.isci_density1(hd, c)
    sg = isci.isci_sigma(hd, c)
    torch.cuda.synchronize()
    d = d.cpu().numpy()
    cn = c.cpu().numpy()
    e = (cn * sg.cpu().numpy()).sum(1)
    nn = (cn * cn).sum(1)
    scale = np.abs(d).max()
    for v in range(4):
        for s_, n in enumerate((W.nalpha, W.nbeta)):
            assert abs(np.trace(d[v, s_]) - n * nn[v]) <= 1e-12 * n * nn[v]
            # (symmetric by construction off the diagonal tiles: the
            # reduction mirrors the upper tiles, so no symmetry check here)
        e1 = (h * (d[v, 0] + d[v, 1])).sum()
        assert abs(e1 - e[v]) <= 1e-11 * np.abs(h).sum() * scale


def test_density1_cisd_n130_two_electrons_per_spin():
    """Two electrons per spin above 128 orbitals (three 64 x 64 output
    tiles per spin block, 82,305 determinants): every element against the
    oracle."""
    norb = 130
    h, eri = recipe_a(norb, seed=5, canonical=False)
    print("density1 cisd norb=130 2a2b", flush=True)
    hd = create(h, eri, norb, 2, 2, 2, 1e-12)
    del eri
    S = O.Space(norb, 2, 2, 2)
    c = random_vectors(S.dim, 2, seed=31)
    c /= np.linalg.norm(c, axis=1, keepdims=True)
    got = _gpu_d1(hd, c)
    want = O.density1(S, c)
    assert np.abs(got - want).max() <= TOL * np.abs(want).max()


@pytest.mark.parametrize("nvec", [9, 10])
def test_density1_more_than_eight_vectors(nvec):
    """Vectors beyond the first eight go through a second pass (offsets into
    c, the output and the transposed copy)."""
    norb, L = 14, 3
    h, eri = recipe_b(norb, seed=6)
    hd = create(h, eri, norb, 2, 2, L, 1e-12)
    S = O.Space(norb, 2, 2, L)
    c = random_vectors(S.dim, nvec, seed=nvec)
    got = _gpu_d1(hd, c)
    want = O.density1(S, c)
    assert np.abs(got - want).max() <= TOL * np.abs(want).max()
