"""GPU: a handle whose resident tables come from the caller's allocator
(isci_create_opts.allocator), here torch's caching allocator.

Checks: the handle's device bytes show up in torch's allocated total
after creation and leave it after isci_destroy; sigma and the diagonal
equal those of a handle built with hipMalloc bit for bit (same tables,
same kernels)."""
import numpy as np
import pytest

from isci_inputs import random_vectors

from gpu_common import torch_dev

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("wl,onebody", [("cisd_n20", 0), ("cisdt_n30", 1)])
def test_torch_allocator_handle(wl, onebody):
    import paper_1609_07757_amd as isci
    from isci_inputs import workload
    torch, dev = torch_dev()
    W = workload(wl)
    h, eri = W.integrals()
    ht = torch.from_numpy(np.ascontiguousarray(h)).to(dev)
    et = torch.from_numpy(np.ascontiguousarray(eri)).to(dev)
    ref = isci.isci_create(ht, et, W.norb, 2, 2, W.level, W.tau, onebody=onebody)
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    hd = isci.isci_create(ht, et, W.norb, 2, 2, W.level, W.tau, onebody=onebody, allocator="torch")
    torch.cuda.synchronize()
    held = torch.cuda.memory_allocated() - before
    nbytes = isci.isci_get_stats(hd)["device_bytes"]
    assert nbytes > 0 and held >= nbytes
    c = torch.from_numpy(random_vectors(hd.dim, 5, seed=4)).to(dev)
    assert torch.equal(isci.isci_sigma(hd, c), isci.isci_sigma(ref, c))
    assert torch.equal(isci.isci_diag(hd), isci.isci_diag(ref))
    e1 = isci.isci_davidson(hd, nroots=1)[0]
    e2 = isci.isci_davidson(ref, nroots=1)[0]
    assert np.array_equal(np.asarray(e1), np.asarray(e2))
    del c
    hd.destroy()
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() - before == 0
