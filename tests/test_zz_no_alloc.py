"""GPU: isci_density1_noalloc (the allocation-free variant of
isci_density1, working in the library's static device scratch) through the
C ABI, against isci_density1 on two calls in a row, the second on a smaller
space, and against the oracle; a space whose single vector does not fit the
scratch is refused."""
import ctypes

import numpy as np
import pytest

import oracle as O
from isci_inputs import random_vectors, recipe_b, workload

from gpu_common import create, torch_dev

pytestmark = pytest.mark.gpu
TOL = 1e-12


def _both(hd, c_np):
    import paper_1609_07757_amd as isci
    torch, dev = torch_dev()
    c = torch.from_numpy(c_np).to(dev)
    nv, n = c.shape[0], hd.norb
    ref = isci.isci_density1(hd, c)
    out = torch.full((nv, 2, n, n), float("nan"), dtype=torch.float64, device=dev)
    isci.isci_density1_noalloc(hd, c, out)
    torch.cuda.synchronize()
    return out.cpu().numpy(), ref.cpu().numpy()


def test_noalloc_two_calls_second_smaller():
    # first call: full CI, 48 orbitals, 8 vectors (the scratch takes five
    # vectors per pass: two passes)
    W = workload("fci_n48")
    h, eri = W.integrals()
    print("noalloc call 1: fci_n48, 8 vectors", flush=True)
    hd = create(h, eri, W.norb, 2, 2, W.level, W.tau)
    got, ref = _both(hd, random_vectors(hd.dim, 8, seed=3))
    assert np.abs(got - ref).max() <= TOL * np.abs(ref).max()
    assert np.array_equal(got, ref)
    hd.destroy()
    # second call, smaller space: the scratch keeps the first call's contents
    print("noalloc call 2: recipe B, 11 orbitals CISDT, 2 vectors", flush=True)
    norb = 11
    h, eri = recipe_b(norb, seed=4)
    hd = create(h, eri, norb, 2, 2, 3, 1e-12)
    c = random_vectors(hd.dim, 2, seed=5)
    got, ref = _both(hd, c)
    assert np.abs(got - ref).max() <= TOL * np.abs(ref).max()
    want = O.density1(O.Space(norb, 2, 2, 3), c)
    assert np.abs(got - want).max() <= TOL * np.abs(want).max()


def test_noalloc_refuses_a_vector_larger_than_the_scratch():
    import paper_1609_07757_amd as isci
    from paper_1609_07757_amd import _lib
    torch, dev = torch_dev()
    norb, na, nb, L = 40, 4, 4, 4          # 23,805,835 determinants: 190 MB per vector
    h, eri = recipe_b(norb, seed=1)
    hd = create(h, eri, norb, na, nb, L, 1e-12)
    c = torch.zeros((1, hd.dim), dtype=torch.float64, device=dev)
    out = torch.zeros((1, 2, norb, norb), dtype=torch.float64, device=dev)
    st = _lib.load().isci_density1_noalloc(hd.ptr, 1, ctypes.c_void_p(c.data_ptr()), hd.dim,
                                           ctypes.c_void_p(out.data_ptr()),
                                           ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == isci.E_UNSUPPORTED
    assert b"static scratch" in _lib.load().isci_last_error()
