"""Autotuner for the sigma kernels and the engine's fused launch.

Candidates are timed on the actual inputs with HIP events (through the C
ABI) and the fastest is applied; results are cached per shape in a JSON
file (``$ISCI_TUNE_CACHE``, default ``~/.cache/isci/tune.json``) so a
later process with the same shape skips the search.

Tunables
--------
* per handle: sigma kernel family (general string algebra, pair tables,
  pair tables + FP64 MFMA alpha-beta tiles) and, on the matrix-core path,
  the alpha-beta product kernel, the one-body kernel and whether the
  one-body classes run on the handle's side stream or in line
  (``tune_handle``);
* per engine: persistent grid size of the fused sigma launch and the
  order of its jobs (heaviest first or natural).
"""
from __future__ import annotations

import json
import math
import os

import paper_1609_07757_amd as isci

CACHE = os.environ.get("ISCI_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "isci", "tune.json"))


def _load():
    try:
        with open(CACHE) as f:
            return json.load(f)
    except Exception:
        return {}


def _save(d):
    try:
        os.makedirs(os.path.dirname(CACHE), exist_ok=True)
        with open(CACHE + ".tmp", "w") as f:
            json.dump(d, f, indent=1, sort_keys=True)
        os.replace(CACHE + ".tmp", CACHE)
    except OSError:
        pass


def _time(fn, reps, torch):
    s = torch.cuda.current_stream()
    fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        fn()
    e1.record(s)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def sigma_key(hd, nvec):
    tdec = "0" if hd.tau <= 0 else str(int(round(math.log10(hd.tau))))
    return f"sigma:{hd.norb}:{hd.nalpha}:{hd.nbeta}:{hd.level}:{tdec}:{nvec}"


def tune_sigma(hd, nvec: int = 1, reps: int = 3, use_cache: bool = True):
    """Pick the fastest sigma kernel for this handle and block size.
    Returns (variant, {variant: ms})."""
    import torch
    key = sigma_key(hd, nvec)
    cache = _load() if use_cache else {}
    if key in cache:
        v = int(cache[key]["variant"])
        isci.isci_set_option(hd, isci.OPT_SIGMA_KERNEL, v)
        return v, cache[key]["ms"]
    cands = [isci.SIGMA_GENERAL]
    if hd.nalpha == 2 and hd.nbeta == 2:
        cands = [isci.SIGMA_PAIR, isci.SIGMA_MFMA]
    c = torch.randn(nvec, hd.dim, dtype=torch.float64, device="cuda")
    sg = torch.empty_like(c)
    ms = {}
    for v in cands:
        isci.isci_set_option(hd, isci.OPT_SIGMA_KERNEL, v)
        ms[v] = _time(lambda: isci.isci_sigma(hd, c, sg), reps, torch)
    best = min(ms, key=ms.get)
    isci.isci_set_option(hd, isci.OPT_SIGMA_KERNEL, best)
    cache = _load()
    cache[key] = {"variant": best, "ms": {str(k): v for k, v in ms.items()}}
    _save(cache)
    return best, ms


def handle_key(hd, nvec):
    return sigma_key(hd, nvec).replace("sigma:", "handle:", 1)


def _apply(hd, cfg):
    """Set a handle configuration; False when the handle refuses it."""
    try:
        for opt, val in cfg:
            isci.isci_set_option(hd, opt, val)
        return True
    except isci.IsciError:
        return False


def handle_candidates(hd):
    """Option sets worth timing for this handle: the scalar pair kernel, and
    for two electrons per spin every combination of product kernel,
    one-body kernel (the alpha route up to 80 orbitals, the beta route above) and
    one-body stream on the matrix-core path."""
    if not (hd.nalpha == 2 and hd.nbeta == 2):
        return [((isci.OPT_SIGMA_KERNEL, isci.SIGMA_GENERAL),)]
    cands = [((isci.OPT_SIGMA_KERNEL, isci.SIGMA_PAIR),)]
    obk = [isci.ONEBODY_TRANSPOSED, isci.ONEBODY_SINGLE, isci.ONEBODY_SPECTATOR] if hd.norb <= 80 else \
        [isci.ONEBODY_ROWS, isci.ONEBODY_TRANSPOSED]
    for ab in (isci.AB_PACKED, isci.AB_WIDE, isci.AB_PLAIN, isci.AB_PIPE):
        for ob in obk:
            for st in (isci.ONEBODY_SIDE, isci.ONEBODY_INLINE):
                cands.append(((isci.OPT_SIGMA_KERNEL, isci.SIGMA_MFMA), (isci.OPT_AB_PRODUCT, ab),
                              (isci.OPT_ONEBODY_KERNEL, ob), (isci.OPT_ONEBODY_STREAM, st)))
    return cands


def tune_handle(hd, nvec: int = 1, reps: int = 3, use_cache: bool = True):
    """Pick the fastest option set of `handle_candidates` for this handle and
    block size, timed on the handle itself with HIP events; the winner is
    applied and cached per shape.  Returns (config, {index: ms})."""
    import torch
    key = handle_key(hd, nvec)
    cache = _load() if use_cache else {}
    if key in cache:
        cfg = tuple(tuple(x) for x in cache[key]["config"])
        if _apply(hd, cfg):
            return cfg, cache[key]["ms"]
    c = torch.randn(nvec, hd.dim, dtype=torch.float64, device="cuda")
    sg = torch.empty_like(c)
    ms = {}
    cands = handle_candidates(hd)
    for i, cfg in enumerate(cands):
        if not _apply(hd, cfg):
            continue
        ms[i] = _time(lambda: isci.isci_sigma(hd, c, sg), reps, torch)
    best = min(ms, key=ms.get)
    _apply(hd, cands[best])
    cache = _load()
    cache[key] = {"config": [list(x) for x in cands[best]], "ms": {str(k): v for k, v in ms.items()}}
    _save(cache)
    return cands[best], ms


def tune_engine(eng, handles, nvecs, reps: int = 3):
    """Pick grid size and job order of the engine's fused sigma launch for
    this set of handles.  Returns ((grid, heaviest_first), {cand: ms})."""
    import torch
    cs = [torch.randn(n, h.dim, dtype=torch.float64, device="cuda") for h, n in zip(handles, nvecs)]
    ss = [torch.empty_like(c) for c in cs]
    ms = {}
    for grid in (0, 1024, 2048, 4096, 8192):
        for order in (True, False):
            isci.isci_engine_config(eng, grid, order)
            ms[(grid, order)] = _time(lambda: isci.isci_engine_sigma(eng, handles, cs, ss), reps, torch)
    best = min(ms, key=ms.get)
    isci.isci_engine_config(eng, *best)
    return best, ms
