"""Device-side assembly of recipe-A/B integrals (input preparation).

The random draws come from the same numpy generator as isci_inputs.recipes
(so a workload has one definition); only the dense (pq|rs) = sum_K L^K_pq
L^K_rs product runs on the GPU through torch, which keeps large inputs
(norb up to 200: 12.8 GB) off the host.  Values can differ from the host
assembly in the last bit (different summation order); every consumer gets
the arrays it is handed, so this does not affect parity checks, which use
one assembly for both sides.
"""
from __future__ import annotations

import numpy as np

from .recipes import factors_a


def integrals_on_device(norb: int, box: float, naux: int, seed: int, recipe: str = "A", device="cuda"):
    import torch
    h, L = factors_a(norb, box, naux, seed, recipe)
    Lt = torch.from_numpy(np.ascontiguousarray(L.reshape(L.shape[0], norb * norb))).to(device)
    eri = (Lt.t() @ Lt).reshape(norb, norb, norb, norb)
    del Lt
    return torch.from_numpy(h).to(device), eri


def factors_on_device(norb: int, box: float, naux: int, seed: int, recipe: str = "A", device="cuda"):
    """(h, L) on the device, L[K, p, q] = L^K_pq as drawn by the recipe: the
    input of a factored handle, 8 (naux + 1) norb^2 bytes instead of the
    8 norb^4 of the dense tensor."""
    import torch
    h, L = factors_a(norb, box, naux, seed, recipe)
    return torch.from_numpy(h).to(device), torch.from_numpy(np.ascontiguousarray(L)).to(device)
