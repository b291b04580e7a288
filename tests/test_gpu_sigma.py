"""GPU parity: the HIP sigma path (through the C ABI) against the CPU
oracle on the same seeded inputs.

Bar: integer string / address tables and term counts bit-exact; sigma
elementwise |delta| <= 1e-12 * ||sigma||_inf (FP64).
"""
import numpy as np
import pytest

import oracle as O
from isci_inputs import canonicalize_eri, random_vectors, recipe_a, recipe_b, recipe_random

from gpu_common import create, gpu_sigma, rel_err, sample_targets, sampled_ok, torch_dev

pytestmark = pytest.mark.gpu
TOL = 1e-12


def _ints(recipe, norb, seed):
    if recipe == "A":
        return recipe_a(norb, seed=seed)
    if recipe == "B":
        return recipe_b(norb, seed=seed)
    return recipe_random(norb, seed=seed)


CASES = [
    # recipe, norb, na, nb, L, tau, nvec
    ("B", 8, 2, 2, 2, 0.0, 1),
    ("B", 10, 2, 2, 3, 1e-10, 3),
    ("R", 7, 2, 2, 4, 0.0, 2),
    ("A", 12, 2, 2, 2, 1e-14, 8),
    ("B", 9, 3, 2, 3, 1e-8, 9),
    ("R", 6, 3, 3, 6, 1e-3, 1),
    ("R", 8, 4, 3, 3, 1e-6, 2),
    ("R", 6, 1, 1, 2, 0.0, 4),
    ("B", 7, 1, 0, 1, 0.0, 1),
    ("R", 6, 0, 2, 2, 0.0, 1),
    ("B", 11, 2, 1, 2, 1e-9, 5),
    ("R", 5, 2, 2, 0, 0.0, 1),     # reference only
    ("R", 6, 2, 2, 1, 1e-4, 2),    # singles only
    ("R", 4, 4, 4, 8, 0.0, 1),     # no virtual orbitals
    ("B", 20, 2, 2, 2, 1e-14, 1),  # CISD 20 orbitals, recipe B
    ("B", 16, 2, 2, 3, 1e-12, 17),
    ("B", 26, 2, 2, 3, 1e-12, 2),  # 26 orbitals: two 16-orbital tiles, ragged
    ("A", 72, 2, 2, 2, 1e-12, 3),  # 72 orbitals: five 16-orbital tiles
    ("A", 90, 2, 2, 2, 1e-12, 2),  # above the one-body matrix-core limit (80 orbitals)
    ("A", 84, 2, 2, 1, 1e-12, 3),  # CIS above 80 orbitals: reference-row and virtual tails only
    ("R", 2, 2, 2, 2, 0.0, 1),     # two orbitals, one determinant (one-body units in the tiles)
    ("R", 3, 2, 2, 2, 0.0, 2),     # one virtual orbital
]


@pytest.mark.parametrize("variant", [1, 2, 3, 4, 5])
@pytest.mark.parametrize("case", CASES, ids=lambda c: "-".join(map(str, c)))
def test_sigma_parity(case, variant):
    """variant 1: general string kernel; 2: pair tables; 3: matrix-core
    path (alpha-beta unfold / product / fold; these small spaces take the
    one-body units into the tiles); 4: matrix-core path with the gathered
    alpha-beta tile kernel; 5: matrix-core path with the one-body kernels
    (2-5 need two electrons per spin)."""
    recipe, norb, na, nb, L, tau, nvec = case
    if variant > 1 and not (na == 2 and nb == 2):
        pytest.skip("pair kernels need two electrons per spin")
    h, eri = _ints(recipe, norb, 3)
    hd = create(h, eri, norb, na, nb, L, tau, variant)
    S = O.Space(norb, na, nb, L)
    assert hd.dim == S.dim
    c = random_vectors(S.dim, nvec, seed=11)
    got = gpu_sigma(hd, c)
    ref = O.sigma(S, h, eri, tau, c)
    assert rel_err(got, ref) <= TOL


@pytest.mark.parametrize("case", [("B", 10, 2, 2, 3), ("R", 8, 3, 1, 4), ("R", 7, 0, 3, 2),
                                  ("A", 30, 2, 2, 3), ("R", 9, 4, 4, 2)])
def test_strings_and_rowstart_bitexact(case):
    import paper_1609_07757_amd as isci
    recipe, norb, na, nb, L = case
    h, eri = _ints(recipe, norb, 1)
    hd = create(h, eri, norb, na, nb, L, 0.0)
    S = O.Space(norb, na, nb, L)
    for spin in (0, 1):
        go, gl = isci.isci_strings(hd, spin)
        oo, ol = S.strings(spin)
        assert np.array_equal(go, oo) and np.array_equal(gl, ol)
    assert np.array_equal(isci.isci_rowstart(hd), S.rowstart())


@pytest.mark.parametrize("case", [("B", 8, 2, 2, 3, 1e-9), ("R", 7, 2, 2, 2, 0.0), ("A", 10, 2, 2, 4, 1e-14),
                                  ("R", 7, 3, 2, 3, 0.2), ("B", 9, 2, 1, 2, 1e-6), ("R", 6, 1, 1, 2, 0.0)])
def test_term_counts_bitexact(case):
    import paper_1609_07757_amd as isci
    recipe, norb, na, nb, L, tau = case
    h, eri = _ints(recipe, norb, 2)
    hd = create(h, eri, norb, na, nb, L, tau)
    S = O.Space(norb, na, nb, L)
    kept, _ = O.terms(S, h, eri, tau)
    st = isci.isci_get_stats(hd)
    assert np.array_equal(st["terms"], kept)
    assert st["terms_total"] == int(kept.sum())


@pytest.mark.parametrize("case", [("B", 10, 2, 2, 3, 1e-10), ("R", 7, 3, 2, 4, 1e-3), ("A", 20, 2, 2, 2, 1e-14)])
def test_diag_parity(case):
    import paper_1609_07757_amd as isci
    torch, dev = torch_dev()
    recipe, norb, na, nb, L, tau = case
    h, eri = _ints(recipe, norb, 4)
    hd = create(h, eri, norb, na, nb, L, tau)
    d = isci.isci_diag(hd).cpu().numpy()
    S = O.Space(norb, na, nb, L)
    ref = O.diag(S, h, eri, tau)
    assert rel_err(d, ref) <= TOL


def test_noncanonical_positions_are_ignored():
    """Only canonical elements of eri (and the lower triangle of h) are read."""
    norb, L, tau = 8, 3, 1e-9
    h, eri = recipe_b(norb, seed=6)
    rng = np.random.default_rng(0)
    noisy = eri + rng.normal(scale=1e-3, size=eri.shape)
    noisy = noisy.copy()
    canon = canonicalize_eri(noisy)
    hn = h + np.triu(rng.normal(scale=1e-3, size=h.shape), 1)
    S = O.Space(norb, 2, 2, L)
    c = random_vectors(S.dim, 2, seed=3)
    g1 = gpu_sigma(create(hn, noisy, norb, 2, 2, L, tau), c)
    g2 = gpu_sigma(create(np.tril(hn) + np.tril(hn, -1).T, canon, norb, 2, 2, L, tau), c)
    assert np.array_equal(g1, g2)
    ref = O.sigma(S, hn, noisy, tau, c)
    assert rel_err(g1, ref) <= TOL


def test_everything_screened():
    norb = 8
    h, eri = recipe_b(norb, seed=1)
    tau = 1e6
    hd = create(h, eri, norb, 2, 2, 3, tau)
    c = random_vectors(hd.dim, 1, seed=1)
    assert np.all(gpu_sigma(hd, c) == 0.0)


def test_leading_dimension_and_no_overrun():
    norb = 9
    h, eri = recipe_b(norb, seed=2)
    S = O.Space(norb, 2, 2, 3)
    hd = create(h, eri, norb, 2, 2, 3, 1e-10)
    c = random_vectors(S.dim, 3, seed=2)
    got = gpu_sigma(hd, c, ld=S.dim + 37)
    assert rel_err(got, O.sigma(S, h, eri, 1e-10, c)) <= TOL


def test_hermiticity_large():
    """u . H v == v . H u at a size beyond the dense oracle."""
    norb, L = 40, 3
    h, eri = recipe_b(norb, seed=9)
    hd = create(h, eri, norb, 2, 2, L, 1e-12)
    u, v = random_vectors(hd.dim, 2, seed=4)
    s = gpu_sigma(hd, np.stack([u, v]))
    a, b = u @ s[1], v @ s[0]
    assert abs(a - b) <= 1e-12 * np.linalg.norm(u) * np.linalg.norm(v) * max(1.0, np.abs(s).max())


@pytest.mark.parametrize("variant", [3, 4, 2, 1, 6])
@pytest.mark.parametrize("wl,nsamp,nvec", [("cisd_n20", None, 1), ("cisdt_n30", 600, 2),
                                           ("cisdt_n60", 300, 8), ("fci_n48", 200, 8)])
def test_sigma_workloads(wl, nsamp, nvec, variant):
    """Named workloads (recipe A): full comparison for the small one, sampled
    targets (row ends included) at full size for the others; every path."""
    from isci_inputs import workload
    W = workload(wl)
    h, eri = W.integrals()
    hd = create(h, eri, W.norb, W.nalpha, W.nbeta, W.level, W.tau, variant)
    S = O.Space(W.norb, W.nalpha, W.nbeta, W.level)
    assert hd.dim == S.dim
    c = random_vectors(S.dim, nvec, seed=21)
    got = gpu_sigma(hd, c)
    if nsamp is None:
        ref = O.sigma(S, h, eri, W.tau, c)
        assert rel_err(got, ref) <= TOL
    else:
        tg = sample_targets(S.rowstart(), S.dim, nsamp, seed=5)
        ref = O.sigma(S, h, eri, W.tau, c, targets=tg)
        ok, err = sampled_ok(got, tg, ref, TOL)
        assert ok, err


@pytest.mark.parametrize("variant", [5, 3])
@pytest.mark.parametrize("norb,L", [(130, 2), (84, 3), (150, 3)])
def test_sigma_large_orbitals_sampled(variant, norb, L):
    """Above the LDS pair-block limit of the one-body kernels the alpha class
    runs in spectator form (up to four 64-row masks).  CISD 130 orbitals:
    virtual spectators through the narrow kernel and the reference-row
    tail; CISDT 84 and 150 orbitals: virtual spectators through the
    matrix-core spectator kernel (165 and 297 columns).  Sampled targets
    (row ends included) against the oracle."""
    tau = 1e-12
    h, eri = recipe_a(norb, seed=4)
    hd = create(h, eri, norb, 2, 2, L, tau, variant)
    S = O.Space(norb, 2, 2, L)
    c = random_vectors(S.dim, 2, seed=17)
    got = gpu_sigma(hd, c)
    tg = sample_targets(S.rowstart(), S.dim, 400, seed=9)
    ref = O.sigma(S, h, eri, tau, c, targets=tg)
    ok, err = sampled_ok(got, tg, ref, TOL)
    assert ok, err


@pytest.mark.parametrize("norb,L,nvec", [(97, 2, 2), (199, 3, 1)])
def test_spectator_kernel_edges(norb, L, nvec):
    """Spectator-form one-body classes at 7 and 13 target tiles (CISD 97
    and CISDT 199 orbitals, several vectors at 97): the oracle on sampled
    targets, row ends included."""
    tau = 1e-12
    h, eri = recipe_a(norb, seed=6)
    hd = create(h, eri, norb, 2, 2, L, tau, 5)
    S = O.Space(norb, 2, 2, L)
    c = random_vectors(S.dim, nvec, seed=19)
    got = gpu_sigma(hd, c)
    tg = sample_targets(S.rowstart(), S.dim, 300, seed=13)
    ref = O.sigma(S, h, eri, tau, c, targets=tg)
    ok, err = sampled_ok(got, tg, ref, TOL)
    assert ok, err


@pytest.mark.parametrize("norb,L,nvec", [(81, 1, 1), (97, 2, 4), (84, 3, 3), (90, 4, 2)])
def test_beta_rows_match_transposed(norb, L, nvec):
    """Above 80 orbitals the beta one-body class runs on the rows themselves
    (rows holding every beta pair staged whole, rows capped at level 1 or 0
    eight to a workgroup): CIS 81 orbitals (capped rows only), CISD 97,
    CISDT 84 (both kinds), full CI 90 (whole rows only), orbital counts off
    the 16-orbital tiles.  Every element against the transposed-block route
    (same terms, other summation order) and sampled targets, row ends
    included, against the oracle; the row route is refused at 80 orbitals,
    and the transposed route's scratch is allocated only when that route is
    selected.  These sizes run the row kernel with its pair-code table; 176
    and 199 orbitals (test_gpu_configs) run its rank-formula form."""
    import paper_1609_07757_amd as isci
    tau = 1e-12
    h, eri = recipe_a(norb, seed=8)
    hd = create(h, eri, norb, 2, 2, L, tau, 5)
    S = O.Space(norb, 2, 2, L)
    c = random_vectors(S.dim, nvec, seed=31)
    print(f"beta rows norb={norb} L={L} nvec={nvec}", flush=True)
    rows = gpu_sigma(hd, c)   # the default above 80 orbitals
    held = isci.isci_get_stats(hd)["device_bytes"]
    isci.isci_set_option(hd, isci.OPT_ONEBODY_KERNEL, isci.ONEBODY_TRANSPOSED)
    # the transposed route's scratch (a 4-vector block and its image) is
    # allocated only when that route is selected
    assert isci.isci_get_stats(hd)["device_bytes"] - held == 2 * 4 * 8 * S.dim
    tr = gpu_sigma(hd, c)
    isci.isci_set_option(hd, isci.OPT_ONEBODY_KERNEL, isci.ONEBODY_ROWS)
    assert np.array_equal(gpu_sigma(hd, c), rows)   # deterministic
    assert rel_err(rows, tr) <= 1e-13
    tg = sample_targets(S.rowstart(), S.dim, 300, seed=12)
    ok, err = sampled_ok(rows, tg, O.sigma(S, h, eri, tau, c, targets=tg), TOL)
    assert ok, err
    h80, eri80 = recipe_b(12, seed=2)
    hs = create(h80, eri80, 12, 2, 2, 2, 0.0, 5)
    with pytest.raises(isci.IsciError):
        isci.isci_set_option(hs, isci.OPT_ONEBODY_KERNEL, isci.ONEBODY_ROWS)


@pytest.mark.parametrize("k,tau", [(0, 0.0), (1, 1e-14), (2, 1e-10)])
def test_sigma_tau_sweep_cisdt_n30(k, tau):
    from isci_inputs import workload
    W = workload("cisdt_n30")
    h, eri = W.integrals()
    hd = create(h, eri, W.norb, 2, 2, 3, tau)
    S = O.Space(W.norb, 2, 2, 3)
    c = random_vectors(S.dim, 1, seed=8)
    got = gpu_sigma(hd, c)
    tg = sample_targets(S.rowstart(), S.dim, 400, seed=100 + k)
    ref = O.sigma(S, h, eri, tau, c, targets=tg)
    ok, err = sampled_ok(got, tg, ref, TOL)
    assert ok, err


def test_pair_kernel_rejected_for_other_electron_counts():
    import paper_1609_07757_amd as isci
    h, eri = recipe_b(7, seed=1)
    hd = create(h, eri, 7, 3, 2, 2, 0.0)
    with pytest.raises(isci.IsciError):
        isci.isci_set_option(hd, isci.OPT_SIGMA_KERNEL, isci.SIGMA_PAIR)


def test_ab_path_option():
    import paper_1609_07757_amd as isci
    h, eri = recipe_b(9, seed=1)
    hd = create(h, eri, 9, 2, 2, 2, 0.0, 3)
    with pytest.raises(isci.IsciError):
        isci.isci_set_option(hd, isci.OPT_AB_PATH, 7)
    c = random_vectors(hd.dim, 3, seed=2)
    a = gpu_sigma(hd, c)
    isci.isci_set_option(hd, isci.OPT_AB_PATH, isci.AB_GATHER)
    b = gpu_sigma(hd, c)
    isci.isci_set_option(hd, isci.OPT_AB_PATH, isci.AB_AUTO)
    assert rel_err(b, a) <= TOL
    assert np.array_equal(gpu_sigma(hd, c), a)   # same path again: bit-identical


@pytest.mark.parametrize("wl,nsamp,nvec", [("cisd_n20", None, 3), ("cisdt_n30", 400, 8), ("fci_n48", 200, 8),
                                            ("cisdt_n60", 200, 5)])
def test_ab_product_kernels(wl, nsamp, nvec):
    """The kernels of the block-sparse alpha-beta product against the oracle:
    8-byte, pipelined and 16-byte loads bit for bit with each other (same K
    parts, same order within each), the packed chunks to rounding."""
    import paper_1609_07757_amd as isci
    from isci_inputs import workload
    W = workload(wl)
    h, eri = W.integrals()
    hd = create(h, eri, W.norb, 2, 2, W.level, W.tau, 5)
    S = O.Space(W.norb, 2, 2, W.level)
    c = random_vectors(S.dim, nvec, seed=22)
    tg = None if nsamp is None else sample_targets(S.rowstart(), S.dim, nsamp, seed=6)
    ref = O.sigma(S, h, eri, W.tau, c, targets=tg)
    outs = []
    for val in (isci.AB_PLAIN, isci.AB_PIPE, isci.AB_WIDE, isci.AB_PACKED):
        isci.isci_set_option(hd, isci.OPT_AB_PRODUCT, val)
        got = gpu_sigma(hd, c)
        outs.append(got)
        if tg is None:
            assert rel_err(got, ref) <= TOL, val
        else:
            ok, err = sampled_ok(got, tg, ref, TOL)
            assert ok, (val, err)
    # the same chunks in the same order: bit for bit; the packed chunks
    # group the same products differently: rounding only
    assert np.array_equal(outs[0], outs[1]) and np.array_equal(outs[0], outs[2])
    assert rel_err(outs[3], outs[0]) <= 1e-13


@pytest.mark.parametrize("recipe,norb,L,tau,nvec,nsamp", [("B", 12, 2, 1e-12, 3, None), ("B", 16, 4, 0.0, 5, None),
                                                          ("A", 30, 3, 1e-14, 8, 400), ("A", 48, 4, 1e-14, 8, 300),
                                                          ("A", 60, 3, 1e-14, 4, 300), ("B", 77, 2, 1e-12, 2, 300)])
def test_onebody_kernels(recipe, norb, L, tau, nvec, nsamp):
    """The one-body classes in their own kernels (one-body units kept out of
    the alpha-beta tiles), 12 to 77 orbitals (one to five 16-orbital
    tiles): two-column alpha kernel, and the alpha class through the
    transposed block where every column holds every pair (full CI, 16 and 48
    orbitals), on the side stream and in line, and the spectator form at
    every size; each against the oracle."""
    import paper_1609_07757_amd as isci
    h, eri = _ints(recipe, norb, 7)
    hd = create(h, eri, norb, 2, 2, L, tau, 5)
    S = O.Space(norb, 2, 2, L)
    c = random_vectors(S.dim, nvec, seed=23)
    tg = None if nsamp is None else sample_targets(S.rowstart(), S.dim, nsamp, seed=7)
    ref = O.sigma(S, h, eri, tau, c, targets=tg)
    for kern, stream in ((isci.ONEBODY_SINGLE, isci.ONEBODY_SIDE), (isci.ONEBODY_TRANSPOSED, isci.ONEBODY_SIDE),
                         (isci.ONEBODY_TRANSPOSED, isci.ONEBODY_INLINE), (isci.ONEBODY_SPECTATOR, isci.ONEBODY_SIDE)):
        isci.isci_set_option(hd, isci.OPT_ONEBODY_KERNEL, kern)
        isci.isci_set_option(hd, isci.OPT_ONEBODY_STREAM, stream)
        got = gpu_sigma(hd, c)
        if tg is None:
            assert rel_err(got, ref) <= TOL, kern
        else:
            ok, err = sampled_ok(got, tg, ref, TOL)
            assert ok, (kern, err)


@pytest.mark.parametrize("norb,L,b,ob", [(12, 4, 0, "auto"), (20, 3, 0, "auto"), (24, 2, 0, "separate"),
                                        (16, 1, 6, "auto"), (48, 4, 0, "auto")])
def test_narrow_layouts_match_four_slot_passes(norb, L, b, ob):
    """Passes of one and of two vectors run the product on the narrow
    operand layouts (one or two vector slots per spectator pair); every
    vector's sigma equals, bit for bit, the same vector computed inside a
    four-vector call, and five- and six-vector calls (a four-slot pass and a
    one- or two-slot pass) match both."""
    import paper_1609_07757_amd as isci
    torch, dev = torch_dev()
    h, eri = recipe_a(norb, seed=9)
    ht, et = torch.from_numpy(h).to(dev), torch.from_numpy(eri).to(dev)
    place = {"auto": isci.OB_AUTO, "separate": isci.OB_SEPARATE}[ob]
    hd = isci.isci_create(ht, et, norb, 2, 2, L, 1e-12, onebody=place, gas_boundary=b)
    torch.cuda.synchronize()
    c = random_vectors(hd.dim, 6, seed=4)
    s4 = np.concatenate([gpu_sigma(hd, c[:4]), gpu_sigma(hd, c[2:6])[2:]])
    s5 = gpu_sigma(hd, c[:5])
    s6 = gpu_sigma(hd, c)
    assert np.array_equal(s6, s4)
    assert np.array_equal(s5, s4[:5])
    for v in range(6):
        assert np.array_equal(gpu_sigma(hd, c[v:v + 1])[0], s4[v])
    for v in range(0, 6, 2):
        assert np.array_equal(gpu_sigma(hd, c[v:v + 2]), s4[v:v + 2])
    assert np.array_equal(gpu_sigma(hd, c[1:4]), s4[1:4])
    if norb <= 24:
        S = O.Space(norb, 2, 2, L, boundary=b or None)
        assert rel_err(s6, O.sigma(S, h, eri, 1e-12, c)) <= TOL
