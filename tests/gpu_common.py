"""Helpers for the GPU tests: upload seeded inputs, call the C ABI, pick
sampled targets.  Imported only by tests marked gpu."""
from __future__ import annotations

import numpy as np


def torch_dev():
    import torch
    if not torch.cuda.is_available():
        import pytest
        pytest.skip("no GPU")
    return torch, torch.device("cuda:0")


def create(h, eri, norb, na, nb, L, tau, variant=0):
    """variant 0: automatic; 1-3: isci.SIGMA_* kernel; 4: matrix-core path
    with the gathered alpha-beta tile kernel; 5 / 6: matrix-core path with
    the one-body units in their own kernels / in the alpha-beta tiles."""
    import paper_1609_07757_amd as isci
    torch, dev = torch_dev()
    ht = torch.from_numpy(np.ascontiguousarray(h)).to(dev)
    et = torch.from_numpy(np.ascontiguousarray(eri)).to(dev)
    ob = {5: isci.OB_SEPARATE, 6: isci.OB_TILES}.get(variant, isci.OB_AUTO)
    hd = isci.isci_create(ht, et, norb, na, nb, L, tau, onebody=ob)
    torch.cuda.synchronize()
    del ht, et
    if variant == 4:
        # matrix-core path with the gathered alpha-beta tile kernel
        isci.isci_set_option(hd, isci.OPT_SIGMA_KERNEL, isci.SIGMA_MFMA)
        isci.isci_set_option(hd, isci.OPT_AB_PATH, isci.AB_GATHER)
    elif variant in (5, 6):
        isci.isci_set_option(hd, isci.OPT_SIGMA_KERNEL, isci.SIGMA_MFMA)
    elif variant:
        isci.isci_set_option(hd, isci.OPT_SIGMA_KERNEL, variant)
    return hd


def gpu_sigma(hd, c, ld=None):
    """c: numpy [nvec][dim] -> numpy sigma [nvec][dim] (optionally padded ld)."""
    import paper_1609_07757_amd as isci
    torch, dev = torch_dev()
    nvec, dim = c.shape
    ld = ld or dim
    cbuf = torch.zeros((nvec, ld), dtype=torch.float64, device=dev)
    cbuf[:, :dim] = torch.from_numpy(c).to(dev)
    sbuf = torch.full((nvec, ld), float("nan"), dtype=torch.float64, device=dev)
    if ld == dim:
        isci.isci_sigma(hd, cbuf, sbuf)
    else:
        from paper_1609_07757_amd import _lib
        import ctypes
        st = _lib.load().isci_sigma(hd.ptr, nvec, ctypes.c_void_p(cbuf.data_ptr()), ld,
                                    ctypes.c_void_p(sbuf.data_ptr()), ld,
                                    ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
        _lib.check(st)
    torch.cuda.synchronize()
    out = sbuf.cpu().numpy()
    if ld != dim:
        assert np.all(np.isnan(out[:, dim:])), "sigma wrote past dim"
    return out[:, :dim]


def sample_targets(rowstart, dim, n, seed):
    """Random addresses plus the first and last element of the first, last
    and a few middle rows (row ends are the ragged tails)."""
    rng = np.random.default_rng(seed)
    t = set(rng.integers(0, dim, size=min(n, dim)).tolist())
    nrow = len(rowstart) - 1
    for r in {0, 1, nrow // 2, nrow - 2, nrow - 1}:
        if 0 <= r < nrow and rowstart[r + 1] > rowstart[r]:
            t.add(int(rowstart[r]))
            t.add(int(rowstart[r + 1] - 1))
    return np.array(sorted(t), dtype=np.int64)


def rel_err(a, b):
    scale = np.abs(b).max()
    return float(np.abs(a - b).max() / (scale if scale > 0 else 1.0))


def sampled_ok(got, tg, ref, tol):
    """Sampled parity: |got[:, tg] - ref| <= tol * ||ref||_inf, the scale
    taken from the oracle's values on the sampled targets (never from the
    GPU's output)."""
    scale = np.abs(ref).max()
    err = np.abs(got[:, tg] - ref).max()
    return err <= tol * (scale if scale > 0 else 1.0), err / (scale if scale > 0 else 1.0)
