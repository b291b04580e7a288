"""MI355X (gfx950) FP64 library for the sigma step of Integral Screened
Configuration Interaction (Sorensen, Bauch & Madsen).

The compute lives in ``libisci.so`` (HIP kernels behind the C ABI of
``include/isci.h``).  This module is a thin binding with the same entry
point names; PyTorch only supplies device memory (tensors) and streams.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _lib
from ._lib import IsciDavidsonInfo, IsciDavidsonOpts, IsciError, IsciStats, check

__all__ = ["Handle", "isci_create", "isci_dim", "isci_sigma", "isci_diag", "isci_davidson",
           "isci_strings", "isci_rowstart", "isci_get_stats", "isci_destroy", "IsciError",
           "lib_path", "BUCKET_NAMES", "Engine", "isci_engine_create", "isci_engine_config",
           "isci_engine_add", "isci_engine_step", "isci_engine_result", "isci_engine_release",
           "isci_engine_sigma", "isci_engine_destroy", "isci_davidson_footprint", "isci_set_option",
           "SIGMA_AUTO", "SIGMA_GENERAL", "SIGMA_PAIR", "SIGMA_MFMA", "OPT_AB_PATH", "AB_AUTO",
           "AB_GATHER", "SigmaGraph", "isci_sigma_graph_create", "torch_allocator", "isci_density1",
           "isci_density1_noalloc", "isci_create_factored", "isci_density2", "isci_propagate"]

OPT_SIGMA_KERNEL = 1
SIGMA_AUTO, SIGMA_GENERAL, SIGMA_PAIR, SIGMA_MFMA = 0, 1, 2, 3
OPT_AB_PATH = 2
AB_AUTO, AB_GATHER = 0, 1
# kernel of the block-sparse alpha-beta product (tuning; same sigma up to rounding order)
OPT_AB_PRODUCT = 3
AB_PLAIN, AB_PIPE, AB_WIDE, AB_PACKED = 0, 1, 2, 3
# one-body kernel where every column holds every pair (tuning)
OPT_ONEBODY_KERNEL = 5
ONEBODY_SINGLE, ONEBODY_TRANSPOSED, ONEBODY_SPECTATOR, ONEBODY_ROWS = 1, 2, 3, 4
# one-body kernels beside the alpha-beta products on a side stream, or in line (tuning)
OPT_ONEBODY_STREAM = 6
ONEBODY_SIDE, ONEBODY_INLINE = 0, 1
# isci_create_opts.onebody: where the matrix-core path applies the one-body units
OB_AUTO, OB_SEPARATE, OB_TILES = 0, 1, 2
# isci_status codes
OK, E_INVALID, E_OOM, E_HIP, E_NOT_CONVERGED, E_UNSUPPORTED = 0, -1, -2, -3, -4, -5


def isci_set_option(hd, option: int, value: int):
    check(_lib.load().isci_set_option(hd.ptr, int(option), int(value)), "isci_set_option")


def lib_path() -> str:
    return _lib.LIBPATH


def _torch():
    import torch
    return torch


def _stream_ptr(stream):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


def _dev_f64(t, name):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda" or t.dtype != torch.float64:
        raise TypeError(f"{name} must be a CUDA float64 tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


class Handle:
    """Owns an isci_handle; destroyed with the object or by isci_destroy."""

    def __init__(self, ptr, norb, nalpha, nbeta, level, tau, keep=None):
        self._ptr = ptr
        self._keep = keep   # the allocator callbacks, alive until isci_destroy
        self.norb, self.nalpha, self.nbeta, self.level, self.tau = norb, nalpha, nbeta, level, tau
        self.dim = isci_dim(self)

    @property
    def ptr(self):
        if self._ptr is None:
            raise ValueError("handle destroyed")
        return self._ptr

    def destroy(self):
        if self._ptr is not None:
            _lib.load().isci_destroy(self._ptr)
            self._ptr = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def torch_allocator():
    """An isci_allocator that takes the handle's device memory from torch's
    caching allocator (torch.cuda.caching_allocator_alloc / _delete)."""
    torch = _torch()

    def _alloc(nbytes, stream, ctx):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), stream=int(stream or 0))
        except Exception:
            return None

    def _free(p, stream, ctx):
        try:
            torch.cuda.caching_allocator_delete(int(p))
        except Exception:
            pass

    return _lib.IsciAllocator(_lib.ALLOC_FN(_alloc), _lib.FREE_FN(_free), None)


def _create_opts(onebody, allocator, orb_dist, max_dist, norb, gas_boundary=0):
    if isinstance(allocator, str):
        if allocator != "torch":
            raise ValueError("allocator must be None, 'torch' or an IsciAllocator")
        allocator = torch_allocator()
    dist = None
    if orb_dist is not None:
        dist = np.ascontiguousarray(orb_dist, dtype=np.float64)
        if dist.shape != (norb, norb):
            raise ValueError("orb_dist must be [norb, norb]")
    opts = _lib.IsciCreateOpts(int(onebody), ctypes.pointer(allocator) if allocator is not None else None,
                               dist.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if dist is not None else None,
                               float(max_dist), int(gas_boundary or 0))
    return opts, allocator, dist


def isci_create(h, eri, norb: int, nalpha: int, nbeta: int, max_excitation: int, tau: float,
                stream=None, onebody: int = OB_AUTO, allocator=None, orb_dist=None, max_dist: float = 0.0,
                gas_boundary: int = 0) -> Handle:
    """Build a handle (isci_create_ex; onebody is one of OB_*).  allocator:
    None (hipMalloc), "torch" (torch's caching allocator) or an
    _lib.IsciAllocator.  orb_dist (host [norb, norb]) with max_dist > 0:
    distance screening (units whose orbitals are not all within max_dist
    are removed).  gas_boundary b > 0: the two-space GAS restriction (full
    CI of orbitals 0..b-1, at most max_excitation electrons in b..norb-1)."""
    L = _lib.load()
    hp = _dev_f64(h, "h")
    ep = _dev_f64(eri, "eri")
    if h.numel() != norb * norb or eri.numel() != norb ** 4:
        raise ValueError("h must hold norb^2 and eri norb^4 elements")
    out = ctypes.c_void_p()
    opts, allocator, _dist = _create_opts(onebody, allocator, orb_dist, max_dist, norb, gas_boundary)
    st = L.isci_create_ex(ctypes.byref(out), hp, ep, int(norb), int(nalpha), int(nbeta),
                          int(max_excitation), float(tau), ctypes.byref(opts), _stream_ptr(stream))
    check(st, "isci_create")
    return Handle(out, norb, nalpha, nbeta, max_excitation, tau, keep=allocator)


def isci_create_factored(h, Lfac, norb: int, nalpha: int, nbeta: int, max_excitation: int, tau: float,
                         stream=None, onebody: int = OB_AUTO, allocator=None, orb_dist=None,
                         max_dist: float = 0.0, gas_boundary: int = 0) -> Handle:
    """Build a handle from factored integrals (pq|rs) = sum_K L^K_pq L^K_rs,
    Lfac of shape [naux, norb, norb] on the device, with no dense norb^4
    tensor (isci_create_factored)."""
    L = _lib.load()
    hp = _dev_f64(h, "h")
    lp = _dev_f64(Lfac, "Lfac")
    if h.numel() != norb * norb or Lfac.dim() != 3 or tuple(Lfac.shape[1:]) != (norb, norb):
        raise ValueError("h must hold norb^2 elements and Lfac be [naux, norb, norb]")
    out = ctypes.c_void_p()
    opts, allocator, _dist = _create_opts(onebody, allocator, orb_dist, max_dist, norb, gas_boundary)
    st = L.isci_create_factored(ctypes.byref(out), hp, lp, int(Lfac.shape[0]), int(norb), int(nalpha), int(nbeta),
                                int(max_excitation), float(tau), ctypes.byref(opts), _stream_ptr(stream))
    check(st, "isci_create_factored")
    return Handle(out, norb, nalpha, nbeta, max_excitation, tau, keep=allocator)


def isci_dim(hd: Handle) -> int:
    d = ctypes.c_int64()
    check(_lib.load().isci_dim(hd.ptr, ctypes.byref(d)), "isci_dim")
    return int(d.value)


def isci_sigma(hd: Handle, c, sigma=None, stream=None):
    """sigma = H_tau c for c of shape [nvec, dim] (or [dim]); returns sigma."""
    torch = _torch()
    squeeze = c.dim() == 1
    c2 = c.unsqueeze(0) if squeeze else c
    if c2.shape[-1] != hd.dim:
        raise ValueError("c has wrong length")
    if sigma is None:
        sigma = torch.empty_like(c2)
    s2 = sigma.unsqueeze(0) if sigma.dim() == 1 else sigma
    st = _lib.load().isci_sigma(hd.ptr, int(c2.shape[0]), _dev_f64(c2, "c"), int(c2.stride(0)),
                                _dev_f64(s2, "sigma"), int(s2.stride(0)), _stream_ptr(stream))
    check(st, "isci_sigma")
    return sigma.squeeze(0) if (squeeze and sigma.dim() == 2) else sigma


class SigmaGraph:
    """One sigma call recorded as a HIP graph (isci_sigma_graph_create).
    Holds the handle and both tensors so they outlive the graph."""

    def __init__(self, ptr, hd: Handle, c, sigma, squeeze: bool):
        self._ptr, self.handle, self.c, self.sigma, self._squeeze = ptr, hd, c, sigma, squeeze

    def launch(self, stream=None):
        """sigma = H_tau c from the current contents of c; returns sigma."""
        if self._ptr is None:
            raise ValueError("graph destroyed")
        check(_lib.load().isci_graph_launch(self._ptr, _stream_ptr(stream)), "isci_graph_launch")
        return self.sigma.squeeze(0) if self._squeeze else self.sigma

    def destroy(self):
        if self._ptr is not None:
            _lib.load().isci_graph_destroy(self._ptr)
            self._ptr = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def isci_sigma_graph_create(hd: Handle, c, sigma=None) -> SigmaGraph:
    """Record isci_sigma(hd, c, sigma) as a graph; launch() replays it."""
    torch = _torch()
    squeeze = c.dim() == 1
    c2 = c.unsqueeze(0) if squeeze else c
    if c2.shape[-1] != hd.dim:
        raise ValueError("c has wrong length")
    if sigma is None:
        sigma = torch.empty_like(c2)
    s2 = sigma.unsqueeze(0) if sigma.dim() == 1 else sigma
    out = ctypes.c_void_p()
    st = _lib.load().isci_sigma_graph_create(hd.ptr, int(c2.shape[0]), _dev_f64(c2, "c"), int(c2.stride(0)),
                                             _dev_f64(s2, "sigma"), int(s2.stride(0)), ctypes.byref(out))
    check(st, "isci_sigma_graph_create")
    return SigmaGraph(out, hd, c2, s2, squeeze)


def isci_probe_fp64(kind: int, iters: int, blocks: int, out, stream=None) -> float:
    """Enqueue the FP64 issue-rate probe (kind 0 matrix cores, 1 vector FMA);
    returns the flops enqueued (a measurement aid, not part of the method)."""
    fl = ctypes.c_double()
    check(_lib.load().isci_probe_fp64(int(kind), int(iters), int(blocks), _dev_f64(out, "out"),
                                      ctypes.byref(fl), _stream_ptr(stream)), "isci_probe_fp64")
    return float(fl.value)


def isci_diag(hd: Handle, out=None, stream=None):
    torch = _torch()
    if out is None:
        out = torch.empty(hd.dim, dtype=torch.float64, device="cuda")
    check(_lib.load().isci_diag(hd.ptr, _dev_f64(out, "diag"), _stream_ptr(stream)), "isci_diag")
    return out


def isci_density1(hd: Handle, c, out=None, stream=None):
    """One-body density matrices by spin: out[v, s, p, q] = <c_v| a+_{p s}
    a_{q s} |c_v> (s = 0 alpha, 1 beta) for c of shape [nvec, dim] or [dim]."""
    torch = _torch()
    squeeze = c.dim() == 1
    c2 = c.unsqueeze(0) if squeeze else c
    if c2.shape[-1] != hd.dim:
        raise ValueError("c has wrong length")
    nv, n = int(c2.shape[0]), hd.norb
    if out is None:
        out = torch.empty((nv, 2, n, n), dtype=torch.float64, device=c2.device)
    if tuple(out.shape) != (nv, 2, n, n) or not out.is_contiguous():
        raise ValueError("out must be a contiguous [nvec, 2, norb, norb] tensor")
    check(_lib.load().isci_density1(hd.ptr, nv, _dev_f64(c2, "c"), int(c2.stride(0)), _dev_f64(out, "d1"),
                                    _stream_ptr(stream)), "isci_density1")
    return out[0] if squeeze else out


def isci_density2(hd: Handle, c, out=None, stream=None):
    """Two-body density matrices by spin block: out[v, b, p, q, r, s] =
    <c_v| a+_{p S} a+_{r S'} a_{s S'} a_{q S} |c_v> with (S, S') = (a, a),
    (a, b), (b, b) for b = 0, 1, 2; c of shape [nvec, dim] or [dim]."""
    torch = _torch()
    squeeze = c.dim() == 1
    c2 = c.unsqueeze(0) if squeeze else c
    if c2.shape[-1] != hd.dim:
        raise ValueError("c has wrong length")
    nv, n = int(c2.shape[0]), hd.norb
    shape = (nv, 3, n, n, n, n)
    if out is None:
        out = torch.empty(shape, dtype=torch.float64, device=c2.device)
    if tuple(out.shape) != shape or not out.is_contiguous():
        raise ValueError("out must be a contiguous [nvec, 3, norb, norb, norb, norb] tensor")
    check(_lib.load().isci_density2(hd.ptr, nv, _dev_f64(c2, "c"), int(c2.stride(0)), _dev_f64(out, "d2"),
                                    _stream_ptr(stream)), "isci_density2")
    return out[0] if squeeze else out


def isci_propagate(hd: Handle, c_re, dt: float, nsteps: int, c_im=None, imaginary: bool = True, krylov: int = 16,
                   tol: float = 1e-12, coef_tau: float = 0.0, stream=None) -> dict:
    """Short-iterative Arnoldi-Lanczos propagation in place: imaginary time
    c_re <- exp(-H dt) c_re (normalised) or real time (c_re + i c_im) <-
    exp(-i H dt) (c_re + i c_im), nsteps times; coef_tau > 0 zeroes small
    coefficients after every step.  Returns the info record as a dict."""
    L = _lib.load()
    o = _lib.IsciPropagateOpts()
    L.isci_propagate_defaults(ctypes.byref(o))
    o.krylov, o.imaginary, o.tol, o.coef_tau = int(krylov), 1 if imaginary else 0, float(tol), float(coef_tau)
    info = _lib.IsciPropagateInfo()
    if c_re.dim() != 1 or c_re.shape[0] != hd.dim or (c_im is not None and tuple(c_im.shape) != tuple(c_re.shape)):
        raise ValueError("c_re (and c_im) must be [dim] vectors")
    im = _dev_f64(c_im, "c_im") if c_im is not None else None
    check(L.isci_propagate(hd.ptr, _dev_f64(c_re, "c_re"), im, float(dt), int(nsteps), ctypes.byref(o),
                           ctypes.byref(info), _stream_ptr(stream)), "isci_propagate")
    return {"energy": info.energy, "norm": info.norm, "sigma_calls": info.sigma_calls,
            "krylov_last": info.krylov_last, "screened_last": info.screened_last}


def isci_density1_noalloc(hd: Handle, c, out, stream=None):
    """isci_density1 for callers that cannot allocate device memory: the
    caller passes the output, and the library works in its static scratch
    (no allocation by the library or this binding)."""
    if c.dim() != 2 or c.shape[-1] != hd.dim:
        raise ValueError("c must be [nvec, dim]")
    nv, n = int(c.shape[0]), hd.norb
    if tuple(out.shape) != (nv, 2, n, n) or not out.is_contiguous():
        raise ValueError("out must be a contiguous [nvec, 2, norb, norb] tensor")
    check(_lib.load().isci_density1_noalloc(hd.ptr, nv, _dev_f64(c, "c"), int(c.stride(0)), _dev_f64(out, "d1"),
                                            _stream_ptr(stream)), "isci_density1_noalloc")
    return out


def _opts(tol_residual=1e-7, tol_energy=1e-11, max_iter=200, max_subspace=0, block=0):
    o = IsciDavidsonOpts()
    _lib.load().isci_davidson_defaults(ctypes.byref(o))
    o.tol_residual, o.tol_energy, o.max_iter = tol_residual, tol_energy, max_iter
    o.max_subspace, o.block = max_subspace, block
    return o


def isci_davidson(hd: Handle, nroots: int = 1, tol_residual: float = 1e-7, tol_energy: float = 1e-11,
                  max_iter: int = 200, max_subspace: int = 0, block: int = 0, guess=None,
                  want_vectors: bool = False, stream=None, raise_on_nonconv: bool = True):
    """Lowest nroots eigenpairs.  Returns (energies ndarray, vectors or None, info dict)."""
    torch = _torch()
    L = _lib.load()
    o = IsciDavidsonOpts()
    L.isci_davidson_defaults(ctypes.byref(o))
    o.tol_residual, o.tol_energy, o.max_iter = tol_residual, tol_energy, max_iter
    o.max_subspace, o.block = max_subspace, block
    en = (ctypes.c_double * nroots)()
    info = IsciDavidsonInfo()
    vec = torch.empty((nroots, hd.dim), dtype=torch.float64, device="cuda") if want_vectors else None
    gp, ng = ctypes.c_void_p(0), 0
    if guess is not None:
        gp, ng = _dev_f64(guess, "guess"), int(guess.shape[0])
    st = L.isci_davidson(hd.ptr, int(nroots), ctypes.byref(o), gp, ng, en,
                         _dev_f64(vec, "vectors") if vec is not None else ctypes.c_void_p(0),
                         ctypes.byref(info), _stream_ptr(stream))
    inf = {"iterations": info.iterations, "converged": bool(info.converged),
           "sigma_calls": info.sigma_calls, "residual": list(info.residual)[:nroots], "status": st}
    if st != _lib.ISCI_OK and not (st == _lib.ISCI_E_NOT_CONVERGED and not raise_on_nonconv):
        check(st, "isci_davidson")
    return np.array(list(en)), vec, inf


def isci_strings(hd: Handle, spin: int):
    """(orbitals [nstr][n] int32, level [nstr] int32) in layout order."""
    L = _lib.load()
    ns = ctypes.c_int64()
    check(L.isci_strings(hd.ptr, int(spin), None, None, ctypes.byref(ns)), "isci_strings")
    n = hd.nbeta if spin else hd.nalpha
    orb = np.zeros((ns.value, max(n, 1)), dtype=np.int32)
    lev = np.zeros(ns.value, dtype=np.int32)
    check(L.isci_strings(hd.ptr, int(spin), orb.ctypes.data_as(ctypes.c_void_p),
                         lev.ctypes.data_as(ctypes.c_void_p), ctypes.byref(ns)), "isci_strings")
    return orb[:, :n].copy(), lev


def isci_rowstart(hd: Handle):
    na = isci_get_stats(hd)["nstr_alpha"]
    rs = np.zeros(na + 1, dtype=np.int64)
    check(_lib.load().isci_rowstart(hd.ptr, rs.ctypes.data_as(ctypes.c_void_p)), "isci_rowstart")
    return rs


def isci_get_stats(hd: Handle) -> dict:
    s = IsciStats()
    check(_lib.load().isci_get_stats(hd.ptr, ctypes.byref(s)), "isci_get_stats")
    return {"dim": s.dim, "nstr_alpha": s.nstr_alpha, "nstr_beta": s.nstr_beta,
            "kept": np.array(list(s.kept), dtype=np.int64), "terms": np.array(list(s.terms), dtype=np.int64),
            "kept_total": s.kept_total, "terms_total": s.terms_total, "device_bytes": s.device_bytes}


def isci_destroy(hd: Handle):
    hd.destroy()


def _bucket_names():
    names = []
    ov = "ov"
    for spin in "ab":
        for ep in range(2):
            for eq in range(2):
                names.append(f"1b_{spin}_{ov[ep]}{ov[eq]}")
    for spin in ("aa", "bb"):
        for nc in range(3):
            for na in range(3):
                names.append(f"ss_{spin}_c{nc}a{na}")
    for ep in range(2):
        for eq in range(2):
            for er in range(2):
                for es in range(2):
                    names.append(f"ab_{ov[ep]}{ov[eq]}|{ov[er]}{ov[es]}")
    return names


BUCKET_NAMES = _bucket_names()


# ---------------------------------------------------------------- engine

class Engine:
    """Owns an isci_engine (multi-instance Davidson + fused sigma)."""

    def __init__(self, ptr, stream):
        self._ptr = ptr
        self.stream = stream
        self.handles = {}

    @property
    def ptr(self):
        if self._ptr is None:
            raise ValueError("engine destroyed")
        return self._ptr

    def destroy(self):
        if self._ptr is not None:
            _lib.load().isci_engine_destroy(self._ptr)
            self._ptr = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def isci_engine_create(stream=None) -> Engine:
    out = ctypes.c_void_p()
    sp = _stream_ptr(stream)
    check(_lib.load().isci_engine_create(ctypes.byref(out), sp), "isci_engine_create")
    return Engine(out, sp)


def isci_engine_config(e: Engine, grid: int = 0, heaviest_first: bool = True):
    check(_lib.load().isci_engine_config(e.ptr, int(grid), 1 if heaviest_first else 0), "isci_engine_config")


def isci_engine_add(e: Engine, hd: Handle, nroots: int = 1, guess=None, **opts) -> int:
    slot = ctypes.c_int()
    o = _opts(**opts)
    gp, ng = ctypes.c_void_p(0), 0
    if guess is not None:
        gp, ng = _dev_f64(guess, "guess"), int(guess.shape[0])
    check(_lib.load().isci_engine_add(e.ptr, hd.ptr, int(nroots), ctypes.byref(o), gp, ng, ctypes.byref(slot)),
          "isci_engine_add")
    e.handles[slot.value] = (hd, nroots)
    return slot.value


def isci_engine_step(e: Engine) -> int:
    n = ctypes.c_int()
    check(_lib.load().isci_engine_step(e.ptr, ctypes.byref(n)), "isci_engine_step")
    return n.value


def isci_engine_result(e: Engine, slot: int, want_vectors: bool = False):
    """(done, energies, vectors or None, info)."""
    torch = _torch()
    hd, nroots = e.handles[slot]
    done = ctypes.c_int()
    en = (ctypes.c_double * nroots)()
    info = IsciDavidsonInfo()
    vec = None
    st = _lib.load().isci_engine_result(e.ptr, slot, ctypes.byref(done), en, None, ctypes.byref(info))
    if st not in (_lib.ISCI_OK, _lib.ISCI_E_NOT_CONVERGED):
        check(st, "isci_engine_result")
    if done.value and want_vectors:
        vec = torch.empty((nroots, hd.dim), dtype=torch.float64, device="cuda")
        _lib.load().isci_engine_result(e.ptr, slot, None, None, _dev_f64(vec, "vectors"), None)
    inf = {"iterations": info.iterations, "converged": bool(info.converged),
           "sigma_calls": info.sigma_calls, "residual": list(info.residual)[:nroots], "status": st}
    return bool(done.value), np.array(list(en)), vec, inf


def isci_engine_release(e: Engine, slot: int):
    check(_lib.load().isci_engine_release(e.ptr, int(slot)), "isci_engine_release")
    e.handles.pop(slot, None)


def isci_engine_sigma(e: Engine, handles, cs, sigmas):
    """Fused sigma: sigmas[i] = H_i cs[i] for every handle, one launch."""
    n = len(handles)
    H = (ctypes.c_void_p * n)(*[h.ptr for h in handles])
    NV = (ctypes.c_int * n)(*[int(c.shape[0]) if c.dim() == 2 else 1 for c in cs])
    C = (ctypes.c_void_p * n)(*[_dev_f64(c, "c").value for c in cs])
    S = (ctypes.c_void_p * n)(*[_dev_f64(s, "sigma").value for s in sigmas])
    LC = (ctypes.c_int64 * n)(*[int(c.stride(0)) if c.dim() == 2 else h.dim for c, h in zip(cs, handles)])
    LS = (ctypes.c_int64 * n)(*[int(s.stride(0)) if s.dim() == 2 else h.dim for s, h in zip(sigmas, handles)])
    check(_lib.load().isci_engine_sigma(e.ptr, n, H, NV, C, LC, S, LS), "isci_engine_sigma")


def isci_engine_destroy(e: Engine):
    e.destroy()


def isci_davidson_footprint(hd: Handle, nroots: int = 1, **opts) -> int:
    o = _opts(**opts)
    return int(_lib.load().isci_davidson_footprint(hd.ptr, int(nroots), ctypes.byref(o)))


KERNEL_NAMES = {0: "k_sigma_generic", 1: "k_sigma_n2", 2: "k_sigma_ab_mfma", 3: "k_sigma_n2(same-spin)",
                4: "onebody", 5: "k_ab_unfold", 6: "k_ab_gemm", 7: "k_ab_fold"}


def isci_profile(hd: Handle, enable: bool = True):
    check(_lib.load().isci_profile(hd.ptr, 1 if enable else 0), "isci_profile")


def isci_profile_read(hd: Handle) -> dict:
    """{kernel name: (total ms, launches)} of the launches recorded since the last read."""
    out = {}
    L = _lib.load()
    for k, name in KERNEL_NAMES.items():
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        check(L.isci_profile_read(hd.ptr, k, ctypes.byref(ms), ctypes.byref(n)), "isci_profile_read")
        if n.value:
            out[name] = (ms.value, n.value)
    return out
