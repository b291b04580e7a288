"""GPU: the two-space GAS restriction (isci_create_opts.gas_boundary, the
section "Generalized Active Space" and the single-continuum-electron
restriction of the appendix on CAAB types): full CI in the orbitals below
the boundary, at most max_excitation electrons above it.  Compared with
the oracle built on the same space (oracle.Space(..., boundary=b)).

Bar: sigma |delta| <= 1e-12 * ||sigma||_inf (the oracle's); strings, row
starts and term counts exact; Davidson energies within 1e-10 Eh of the
oracle's dense spectrum."""
import functools

import numpy as np
import pytest

import oracle as O
from isci_inputs import random_vectors, recipe_a, recipe_b

from gpu_common import gpu_sigma, rel_err, sample_targets, sampled_ok, torch_dev

pytestmark = pytest.mark.gpu
TOL = 1e-12


def _gas(h, eri, norb, na, nb, L, tau, b, kernel=0):
    import paper_1609_07757_amd as isci
    torch, dev = torch_dev()
    ht = torch.from_numpy(np.ascontiguousarray(h)).to(dev)
    et = torch.from_numpy(np.ascontiguousarray(eri)).to(dev)
    hd = isci.isci_create(ht, et, norb, na, nb, L, tau, gas_boundary=b)
    torch.cuda.synchronize()
    if kernel:
        isci.isci_set_option(hd, isci.OPT_SIGMA_KERNEL, kernel)
    return hd


@pytest.mark.parametrize("recipe,norb,na,nb,L,b,tau,nvec", [
    ("A", 12, 2, 2, 1, 5, 0.0, 2), ("B", 12, 2, 2, 2, 4, 1e-8, 3), ("A", 14, 2, 2, 1, 3, 1e-12, 1),
    ("B", 10, 3, 2, 2, 4, 0.0, 2), ("A", 9, 2, 1, 1, 4, 1e-10, 2), ("B", 10, 1, 1, 1, 3, 0.0, 1),
    ("A", 11, 2, 2, 0, 6, 1e-12, 2), ("B", 9, 3, 3, 2, 5, 1e-9, 1)])
def test_gas_sigma_matches_oracle(recipe, norb, na, nb, L, b, tau, nvec):
    """Every element of sigma: for two electrons per spin on the
    matrix-core path (blocks split at the boundary, one-body units in the
    tiles; the unfold / product / fold route and the gathered tile kernel),
    the pair-table kernel and the general-string kernel; for other electron
    counts on the general-string kernel."""
    import paper_1609_07757_amd as isci
    h, eri = (recipe_a if recipe == "A" else recipe_b)(norb, seed=3)
    S = O.Space(norb, na, nb, L, boundary=b)
    hd = _gas(h, eri, norb, na, nb, L, tau, b)
    assert isci.isci_dim(hd) == S.dim
    c = random_vectors(S.dim, nvec, seed=7)
    ref = O.sigma(S, h, eri, tau, c)
    got = gpu_sigma(hd, c)
    assert rel_err(got, ref) <= TOL
    if na == 2 and nb == 2:
        for kern in (isci.SIGMA_GENERAL, isci.SIGMA_PAIR):
            hk = _gas(h, eri, norb, na, nb, L, tau, b, kernel=kern)
            assert rel_err(gpu_sigma(hk, c), ref) <= TOL
        hm = _gas(h, eri, norb, na, nb, L, tau, b, kernel=isci.SIGMA_MFMA)
        isci.isci_set_option(hm, isci.OPT_AB_PATH, isci.AB_GATHER)
        assert rel_err(gpu_sigma(hm, c), ref) <= TOL


@pytest.mark.parametrize("norb,na,nb,L,b", [(12, 2, 2, 1, 5), (10, 3, 2, 2, 4), (9, 2, 1, 2, 9)])
def test_gas_strings_rows_and_term_counts_exact(norb, na, nb, L, b):
    import paper_1609_07757_amd as isci
    h, eri = recipe_b(norb, seed=5)
    tau = 1e-9
    S = O.Space(norb, na, nb, L, boundary=b)
    hd = _gas(h, eri, norb, na, nb, L, tau, b)
    for spin in (0, 1):
        go, gl = isci.isci_strings(hd, spin)
        oo, ol = S.strings(spin)
        assert np.array_equal(go, oo) and np.array_equal(gl, ol)
    assert np.array_equal(isci.isci_rowstart(hd), S.rowstart())
    kept, _ = O.terms(S, h, eri, tau)
    st = isci.isci_get_stats(hd)
    assert np.array_equal(np.asarray(st["terms"], dtype=np.int64), kept)
    d = isci.isci_diag(hd).cpu().numpy()
    assert rel_err(d[None], O.diag(S, h, eri, tau)[None]) <= TOL


def test_gas_boundary_at_norb_is_fci():
    """b = norb leaves no outer orbital: the handle is full CI whatever the
    limit.  Every string then has level 0, so the strings are in plain
    colex order: the determinants are the full-CI ones in another order,
    and sigma is the full-CI sigma (hierarchy layout) permuted."""
    norb = 8
    h, eri = recipe_a(norb, seed=2)
    F = O.Space(norb, 2, 2, 4)
    G = O.Space(norb, 2, 2, 1, boundary=norb)
    perm = np.array([F.address(a, b) for a, b in G.determinants()])
    assert np.array_equal(np.sort(perm), np.arange(F.dim))
    hd = _gas(h, eri, norb, 2, 2, 1, 1e-12, norb)
    c = random_vectors(F.dim, 2, seed=4)
    assert rel_err(gpu_sigma(hd, c[:, perm]), O.sigma(F, h, eri, 1e-12, c)[:, perm]) <= TOL


def test_gas_davidson_energies():
    """Davidson on the GAS handle against the dense spectrum of the
    oracle's matrix on the same space, and the nesting of the ground
    energy in the outer-electron limit."""
    import paper_1609_07757_amd as isci
    norb, b = 12, 5
    h, eri = recipe_a(norb, seed=1)
    e0 = []
    for L in (0, 1, 2):
        S = O.Space(norb, 2, 2, L, boundary=b)
        ref = np.linalg.eigvalsh(O.dense_h(S, h, eri, 0.0))[:3]
        hd = _gas(h, eri, norb, 2, 2, L, 0.0, b)
        e, _v, info = isci.isci_davidson(hd, nroots=3, tol_residual=1e-8)
        assert info["converged"]
        assert np.abs(np.asarray(e) - ref).max() <= 1e-10
        e0.append(e[0])
    assert e0[0] > e0[1] > e0[2]


@functools.lru_cache(maxsize=1)
def _ints200():
    return recipe_a(200, seed=1)


@pytest.mark.parametrize("L,nvec", [(1, 8), (2, 2)])
def test_gas_outer_electrons_sampled(L, nvec):
    """200 orbitals, 16 inner: at most one electron outside them (the
    benchmark's shape, 720,960 determinants, eight vectors) and at most two
    (13.4 million determinants): sampled targets, row ends included."""
    norb, b, tau = 200, 16, 1e-12
    h, eri = _ints200()
    S = O.Space(norb, 2, 2, L, boundary=b)
    hd = _gas(h, eri, norb, 2, 2, L, tau, b)
    c = random_vectors(S.dim, nvec, seed=21)
    got = gpu_sigma(hd, c)
    tg = sample_targets(S.rowstart(), S.dim, 300, seed=5)
    ok, err = sampled_ok(got, tg, O.sigma(S, h, eri, tau, c, targets=tg), TOL)
    assert ok, err


def test_gas_gathered_tiles_above_128_orbitals():
    """The gathered tile kernel without its LDS lookup tables (above 128
    orbitals) on a GAS handle: sampled targets against the oracle."""
    import paper_1609_07757_amd as isci
    norb, b, L, tau = 140, 12, 1, 1e-12
    h, eri = recipe_a(norb, seed=2)
    S = O.Space(norb, 2, 2, L, boundary=b)
    hd = _gas(h, eri, norb, 2, 2, L, tau, b, kernel=isci.SIGMA_MFMA)
    isci.isci_set_option(hd, isci.OPT_AB_PATH, isci.AB_GATHER)
    c = random_vectors(S.dim, 2, seed=4)
    got = gpu_sigma(hd, c)
    tg = sample_targets(S.rowstart(), S.dim, 300, seed=6)
    ok, err = sampled_ok(got, tg, O.sigma(S, h, eri, tau, c, targets=tg), TOL)
    assert ok, err


@pytest.mark.parametrize("norb,na,nb,L,b,nvec", [(12, 2, 2, 1, 5, 2), (40, 2, 2, 1, 16, 3), (10, 3, 2, 2, 4, 1),
                                                  (18, 2, 2, 2, 16, 2), (9, 2, 1, 1, 9, 1)])
def test_gas_density1_matches_oracle(norb, na, nb, L, b, nvec):
    """One-body densities of a GAS handle (the Gram form's second phase over
    the pairs of up to 16 inner rows), and the allocation-free entry point
    bit for bit against it."""
    import paper_1609_07757_amd as isci
    torch, dev = torch_dev()
    h, eri = recipe_b(norb, seed=8)
    S = O.Space(norb, na, nb, L, boundary=b)
    hd = _gas(h, eri, norb, na, nb, L, 1e-12, b)
    c = random_vectors(S.dim, nvec, seed=3)
    ct = torch.from_numpy(c).to(dev)
    got = isci.isci_density1(hd, ct).cpu().numpy()
    want = O.density1(S, c)
    assert np.abs(got - want).max() <= TOL * np.abs(want).max()
    d1 = torch.empty((nvec, 2, norb, norb), dtype=torch.float64, device=dev)
    isci.isci_density1_noalloc(hd, ct, d1)
    torch.cuda.synchronize()
    assert np.array_equal(d1.cpu().numpy(), got)


@pytest.mark.parametrize("norb,L,b", [(12, 1, 5), (10, 2, 4), (14, 1, 8)])
def test_gas_density2_matches_oracle(norb, L, b):
    import paper_1609_07757_amd as isci
    torch, dev = torch_dev()
    h, eri = recipe_a(norb, seed=6)
    S = O.Space(norb, 2, 2, L, boundary=b)
    hd = _gas(h, eri, norb, 2, 2, L, 0.0, b)
    c = random_vectors(S.dim, 2, seed=12)
    got = isci.isci_density2(hd, torch.from_numpy(c).to(dev)).cpu().numpy()
    want = O.density2(S, c)
    assert np.abs(got - want).max() <= TOL * np.abs(want).max()


def test_gas_errors():
    import paper_1609_07757_amd as isci
    from paper_1609_07757_amd import _lib
    torch, dev = torch_dev()
    norb = 8
    h, eri = recipe_a(norb, seed=0)
    ht = torch.from_numpy(h).to(dev)
    et = torch.from_numpy(eri).to(dev)
    for b in (1, norb + 1):
        with pytest.raises(isci.IsciError) as ei:
            isci.isci_create(ht, et, norb, 2, 2, 1, 0.0, gas_boundary=b)
        assert ei.value.status == _lib.ISCI_E_INVALID
    with pytest.raises(isci.IsciError):
        isci.isci_create(ht, et, norb, 3, 2, 1, 0.0, gas_boundary=2)
    # one-body densities: at most 16 inner orbitals
    norb = 20
    h, eri = recipe_a(norb, seed=0)
    hd = isci.isci_create(torch.from_numpy(h).to(dev), torch.from_numpy(eri).to(dev), norb, 2, 2, 1, 0.0,
                          gas_boundary=17)
    c = torch.zeros((1, isci.isci_dim(hd)), dtype=torch.float64, device=dev)
    with pytest.raises(isci.IsciError) as ei:
        isci.isci_density1(hd, c)
    assert ei.value.status == _lib.ISCI_E_UNSUPPORTED
    d1 = torch.zeros((1, 2, norb, norb), dtype=torch.float64, device=dev)
    with pytest.raises(isci.IsciError) as ei:
        isci.isci_density1_noalloc(hd, c, d1)
    assert ei.value.status == _lib.ISCI_E_UNSUPPORTED


def test_gas_factored_and_distance_screened():
    """A GAS handle built from factors equals the one built from the dense
    tensor of the same factors bit for bit; with distance screening it
    matches the oracle on the masked integrals."""
    import paper_1609_07757_amd as isci
    from isci_inputs.recipes import factors_a, orbital_centres
    torch, dev = torch_dev()
    norb, L, b, tau = 14, 1, 6, 1e-12
    h, Lf = factors_a(norb, float(norb), 2 * norb, 4)
    eri = O.assemble_factored(Lf)
    S = O.Space(norb, 2, 2, L, boundary=b)
    c = random_vectors(S.dim, 2, seed=9)
    ht = torch.from_numpy(np.ascontiguousarray(h)).to(dev)
    hd = isci.isci_create(ht, torch.from_numpy(eri).to(dev), norb, 2, 2, L, tau, gas_boundary=b)
    hf = isci.isci_create_factored(ht, torch.from_numpy(np.ascontiguousarray(Lf)).to(dev), norb, 2, 2, L, tau,
                                   gas_boundary=b)
    torch.cuda.synchronize()
    g = gpu_sigma(hd, c)
    assert np.array_equal(g, gpu_sigma(hf, c))
    assert rel_err(g, O.sigma(S, h, eri, tau, c)) <= TOL
    x = orbital_centres(norb, float(norb), 2 * norb, 4)
    dist = np.abs(x[:, None] - x[None, :])
    hm, em = O.mask_by_distance(h, eri, dist, 4.0)
    hs = isci.isci_create(ht, torch.from_numpy(eri).to(dev), norb, 2, 2, L, tau, gas_boundary=b,
                          orb_dist=dist, max_dist=4.0)
    torch.cuda.synchronize()
    assert rel_err(gpu_sigma(hs, c), O.sigma(S, hm, em, tau, c)) <= TOL


def test_gas_engine_and_propagation():
    """GAS handles in the multi-solve engine beside a hierarchy handle give
    the energies of their own Davidson solves and of the oracle's dense
    spectrum; imaginary-time propagation on a GAS handle falls to the
    lowest of them."""
    import paper_1609_07757_amd as isci
    torch, dev = torch_dev()
    cases = [(12, 1, 5, 2), (10, 2, 4, 1)]
    handles, refs = [], []
    for norb, L, b, nroots in cases:
        h, eri = recipe_a(norb, seed=norb)
        S = O.Space(norb, 2, 2, L, boundary=b)
        refs.append(np.linalg.eigvalsh(O.dense_h(S, h, eri, 0.0))[:nroots])
        handles.append((_gas(h, eri, norb, 2, 2, L, 0.0, b), nroots))
    h, eri = recipe_a(10, seed=3)
    hh = isci.isci_create(torch.from_numpy(h).to(dev), torch.from_numpy(eri).to(dev), 10, 2, 2, 2, 0.0)
    refs.append(np.linalg.eigvalsh(O.dense_h(O.Space(10, 2, 2, 2), h, eri, 0.0))[:1])
    handles.append((hh, 1))
    eng = isci.isci_engine_create()
    slots = [isci.isci_engine_add(eng, hd, nroots=k, tol_residual=1e-8) for hd, k in handles]
    for _ in range(400):
        if isci.isci_engine_step(eng) == 0:
            break
    for s, (hd, k), ref in zip(slots, handles, refs):
        done, e, _v, info = isci.isci_engine_result(eng, s)
        assert done and info["converged"]
        assert np.abs(e - ref).max() <= 1e-10
        e1, _, _ = isci.isci_davidson(hd, nroots=k, tol_residual=1e-8)
        assert np.abs(e1 - ref).max() <= 1e-10
    eng.destroy()
    hd, _ = handles[0]
    c0 = torch.from_numpy(random_vectors(hd.dim, 1, seed=2)[0]).to(dev)
    info = isci.isci_propagate(hd, c0, 0.5, 120)   # t = 60: 3.6e-12 above the ground energy (gap 0.21)
    assert abs(info["energy"] - refs[0][0]) <= 1e-8


@pytest.mark.parametrize("norb,na,nb,L,b", [(3, 2, 2, 1, 2), (4, 2, 2, 1, 3), (5, 2, 2, 0, 5), (6, 2, 2, 2, 2),
                                           (9, 2, 2, 3, 6), (23, 2, 2, 2, 7), (21, 2, 2, 1, 13)])
def test_gas_edges(norb, na, nb, L, b):
    """Tiny spaces (fewer than three orbitals outside or inside), the
    boundary at n (the hierarchy, with the one-body units in the tiles),
    limits above what the outer space can hold, and boundaries that cut an
    orbital block (7, 13) with several outer blocks."""
    import paper_1609_07757_amd as isci
    h, eri = recipe_b(norb, seed=norb + b)
    tau = 1e-12
    S = O.Space(norb, na, nb, L, boundary=b)
    hd = _gas(h, eri, norb, na, nb, L, tau, b)
    assert isci.isci_dim(hd) == S.dim
    c = random_vectors(S.dim, 3, seed=b)
    got = gpu_sigma(hd, c)
    assert rel_err(got, O.sigma(S, h, eri, tau, c)) <= TOL
    if b == na:
        from gpu_common import create
        assert rel_err(gpu_sigma(create(h, eri, norb, na, nb, L, tau), c), got) <= TOL
