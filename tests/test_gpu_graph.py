"""GPU: a sigma call recorded as a HIP graph (isci_sigma_graph_create) and
replayed through the C ABI.

Bar: every replay equals the eager isci_sigma on the same inputs bit for
bit (the graph holds the same kernels in the same order), and the oracle
within the sigma bar |delta| <= 1e-12 * ||sigma||_inf.  Replays are
interleaved with eager work on the same handle and stream, and the input
buffer is rewritten between replays (the graph reads it at launch)."""
import numpy as np
import pytest

import oracle as O
from isci_inputs import random_vectors, recipe_b

from gpu_common import create, torch_dev

pytestmark = pytest.mark.gpu
TOL = 1e-12


def _check(hd, S, h, eri, tau, nvec, nsamp=None, seed=3):
    import paper_1609_07757_amd as isci
    from gpu_common import sample_targets, sampled_ok
    torch, dev = torch_dev()
    c1 = torch.from_numpy(random_vectors(S.dim, nvec, seed=seed)).to(dev)
    c2 = torch.from_numpy(random_vectors(S.dim, nvec, seed=seed + 1)).to(dev)
    e1 = isci.isci_sigma(hd, c1)
    e2 = isci.isci_sigma(hd, c2)
    cbuf = c1.clone()
    sbuf = torch.full_like(c1, float("nan"))
    g = isci.isci_sigma_graph_create(hd, cbuf, sbuf)
    torch.cuda.synchronize()
    assert torch.isnan(sbuf).all(), "graph creation must not run the call"
    other = torch.empty_like(c1)
    for rep in range(3):
        sbuf.fill_(float("nan"))
        g.launch()
        isci.isci_sigma(hd, c2, other)          # eager work between replays
        torch.cuda.synchronize()
        assert torch.equal(sbuf, e1), f"replay {rep}"
        assert torch.equal(other, e2)
    cbuf.copy_(c2)
    g.launch()
    torch.cuda.synchronize()
    assert torch.equal(sbuf, e2), "replay after the input changed"
    g.destroy()
    got = e1.cpu().numpy()
    cn = c1.cpu().numpy()
    if nsamp is None:
        ref = O.sigma(S, h, eri, tau, cn)
        assert np.abs(got - ref).max() <= TOL * max(np.abs(ref).max(), 1.0)
    else:
        tg = sample_targets(S.rowstart(), S.dim, nsamp, seed=11)
        ref = O.sigma(S, h, eri, tau, cn, targets=tg)
        ok, err = sampled_ok(got, tg, ref, TOL)
        assert ok, err


@pytest.mark.parametrize("variant,nvec", [(0, 1), (1, 3), (2, 9), (3, 5), (6, 2)])
def test_graph_replay_small(variant, nvec):
    """Recipe B (same-spin units present), 10 orbitals, CISDT: every kernel
    family, nvec across the 8-vector chunk boundary."""
    h, eri = recipe_b(10, seed=2)
    tau = 1e-12
    hd = create(h, eri, 10, 2, 2, 3, tau, variant)
    _check(hd, O.Space(10, 2, 2, 3), h, eri, tau, nvec)


@pytest.mark.parametrize("wl,variant,nvec,nsamp", [("cisd_n20", 0, 1, None), ("cisdt_n30", 5, 8, 500),
                                                   ("cisdt_n60", 0, 8, 300)])
def test_graph_replay_workloads(wl, variant, nvec, nsamp):
    """Named workloads; variant 5 / the default at 60 orbitals run the
    one-body classes on the handle's side stream, so the fork and join are
    part of the graph."""
    from isci_inputs import workload
    W = workload(wl)
    h, eri = W.integrals()
    hd = create(h, eri, W.norb, W.nalpha, W.nbeta, W.level, W.tau, variant)
    _check(hd, O.Space(W.norb, W.nalpha, W.nbeta, W.level), h, eri, W.tau, nvec, nsamp)


def test_graph_refusals():
    import paper_1609_07757_amd as isci
    torch, dev = torch_dev()
    h, eri = recipe_b(8, seed=1)
    hd = create(h, eri, 8, 2, 2, 2, 0.0)
    c = torch.zeros((2, hd.dim), dtype=torch.float64, device=dev)
    with pytest.raises(isci.IsciError):
        isci.isci_sigma_graph_create(hd, c, c)            # sigma overlaps c
    isci.isci_profile(hd, True)
    with pytest.raises(isci.IsciError):
        isci.isci_sigma_graph_create(hd, c)               # profiling enabled
    isci.isci_profile(hd, False)
    g = isci.isci_sigma_graph_create(hd, c)
    g.launch()
    torch.cuda.synchronize()
    g.destroy()
    with pytest.raises(ValueError):
        g.launch()
