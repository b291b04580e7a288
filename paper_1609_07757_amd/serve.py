"""Serving loop for Davidson solves with continuous batching.

Requests arrive over time (each carries its integrals, norb, electron
counts, excitation level, tau and number of roots).  The loop admits
requests in arrival order while their device footprint fits the HBM
budget and a slot is free, adds them to a running multi-instance engine
(``isci_engine``) at the next iteration boundary, advances every admitted
solve by one Davidson iteration per step (one fused sigma launch for all
of them), and retires finished solves, freeing their memory for the
queue.  Latency is measured from arrival to energies.

The scheduler is written against a small executor interface so that its
admission and batching logic can be exercised on the CPU with a mock
executor; ``GpuExecutor`` drives the HIP library through the C ABI.
"""
from __future__ import annotations

import time
from collections import deque
from dataclasses import dataclass, field
from math import comb

import numpy as np


@dataclass
class Request:
    rid: int
    arrival: float              # seconds on the server clock
    norb: int
    nalpha: int
    nbeta: int
    level: int
    tau: float
    nroots: int
    payload: object = None      # executor-specific (integrals or a generator)
    naux: int = 0               # > 0: the payload gives factors L [naux][norb][norb] instead of a dense eri
    # filled by the server
    admitted: float | None = None
    finished: float | None = None
    energies: np.ndarray | None = None
    info: dict = field(default_factory=dict)
    status: str = "queued"      # queued | running | done | rejected | cancelled

    @property
    def latency(self):
        return None if self.finished is None else self.finished - self.arrival


def ci_dim(norb, na, nb, level):
    tot = 0
    for ka in range(na + 1):
        for kb in range(nb + 1):
            if ka + kb <= level:
                tot += comb(na, ka) * comb(norb - na, ka) * comb(nb, kb) * comb(norb - nb, kb)
    return tot


def davidson_bytes(dim: int, nroots: int) -> int:
    """Device bytes of one Davidson solve with default options (the same
    sizing rule as the library: nroots + 2 followed roots, subspace
    max(32, 6 (nroots + 2)), thick restart keeping <= 2 kk + 4 vectors)."""
    kk = min(dim, nroots + 2)
    mmax = min(max(32, 6 * kk, 2 * kk), dim)
    keep = max(kk, min(2 * kk + 4, mmax // 2))
    nscr = max(kk, keep)
    nblk = 1 if dim <= 2048 else min(256, max(1, (dim + 511) // 512))
    return 8 * dim * (2 * mmax + nscr + 2 * kk + 1) + 8 * (mmax * mmax + 8 * mmax + 64 + nblk * mmax * mmax + 3 * (mmax + 8))


def handle_bytes_estimate(norb: int, dim: int, naux: int = 0) -> int:
    """Admission estimate of what building a handle needs at its peak: the
    transient dense eri (8 norb^4), list offsets and tables sized for one
    kept alpha-beta unit in eight, the product operands (about 16 B per
    determinant and vector of a 4-vector pass, two result buffers, and the
    one- and two-vector layouts' own operands, three quarters of a pass's), and
    above 202 orbitals (where a row of every beta pair no longer fits LDS and
    the beta one-body class takes the transposed-block route) that route's
    blocks (64 B per determinant).  It is an estimate, not a bound: at tau = 0 the lists
    alone can exceed it.  The server therefore re-charges a running
    request by what its handle really holds (isci_stats.device_bytes, read
    after the build) and puts a request whose build ran out of memory back
    at the head of the queue.  With factored integrals (naux > 0) the
    transient is the factors and their transposed copy, 8 (2 naux + 1)
    norb^2 bytes, instead of the dense tensor."""
    n3 = norb ** 3
    lists = 8 * (n3 + 1) + 9 * norb ** 4 // 8 + 4 * norb * norb * 16
    strings = 8 * (norb * norb) * 4
    operands = 3 * 16 * 4 * dim + 48 * dim
    onebody = 64 * dim if norb > 202 else 0
    transient = 8 * (2 * naux + 1) * norb * norb if naux > 0 else 8 * norb ** 4
    return transient + lists + strings + 8 * dim + operands + onebody


# kept for callers of the earlier name
handle_bytes_bound = handle_bytes_estimate


class Server:
    """Continuous-batching scheduler.

    executor: object with
        footprint(req) -> int          device bytes needed while the request runs
        start(req) -> token            build the handle and admit the solve
        step() -> int                  one iteration for all running solves
        poll(token) -> (done, energies, info)
        finish(token)                  free the solve and its handle
    hbm_budget: bytes available for running requests.
    max_slots: concurrently running solves.
    clock: callable returning seconds (default time.perf_counter relative to run()).
    """

    def __init__(self, executor, hbm_budget: int, max_slots: int = 64, clock=None):
        self.ex = executor
        self.budget = int(hbm_budget)
        self.max_slots = int(max_slots)
        self.clock = clock
        self.used = 0
        self.queue: deque[Request] = deque()
        self.running: dict = {}          # token -> (req, bytes)
        self.done: list[Request] = []
        self.steps = 0
        self.peak_used = 0
        self.peak_running = 0
        self.oom_requeued = 0

    def _now(self):
        return self.clock() - self._t0

    def cancel(self, rid: int) -> bool:
        for r in list(self.queue):
            if r.rid == rid:
                self.queue.remove(r)
                r.status = "cancelled"
                self.done.append(r)
                return True
        for tok, (r, b) in list(self.running.items()):
            if r.rid == rid:
                self.ex.finish(tok)
                del self.running[tok]
                self.used -= b
                r.status = "cancelled"
                self.done.append(r)
                return True
        return False

    def _admit(self):
        """Admit queued requests in arrival order while they fit; a request
        larger than the whole budget is rejected; one that does not fit now
        waits (head of line) until memory frees up."""
        while self.queue and len(self.running) < self.max_slots:
            r = self.queue[0]
            need = int(self.ex.footprint(r))
            if need > self.budget:
                self.queue.popleft()
                r.status = "rejected"
                r.finished = self._now()
                self.done.append(r)
                continue
            if self.used + need > self.budget:
                break
            self.queue.popleft()
            try:
                tok = self.ex.start(r)
            except MemoryError:
                # the build ran out of device memory (the estimate was low):
                # back to the head of the queue until a running solve frees
                # memory; with nothing running there is nothing to wait for
                if not self.running:
                    r.status = "rejected"
                    r.finished = self._now()
                    self.done.append(r)
                    continue
                self.queue.appendleft(r)
                self.oom_requeued += 1
                break
            # charge what the request really holds from now on
            charge = getattr(self.ex, "charge", None)
            held = int(charge(tok)) if charge is not None else need
            r.admitted = self._now()
            r.status = "running"
            self.running[tok] = (r, held)
            self.used += held
            self.peak_used = max(self.peak_used, self.used)
        self.peak_running = max(self.peak_running, len(self.running))

    def _retire(self):
        for tok, (r, b) in list(self.running.items()):
            done, en, info = self.ex.poll(tok)
            if done:
                r.finished = self._now()
                r.energies = en
                r.info = info
                r.status = "done"
                self.ex.finish(tok)
                del self.running[tok]
                self.used -= b
                self.done.append(r)

    def run(self, requests, max_wall: float | None = None, progress=None, progress_every: float = 10.0):
        """Serve `requests` (sorted by arrival).  Returns the finished list.
        `progress(report)` is called about every `progress_every` seconds."""
        if self.clock is None:
            self.clock = time.perf_counter
        self._t0 = self.clock()
        pending = deque(sorted(requests, key=lambda r: r.arrival))
        next_report = progress_every
        while pending or self.queue or self.running:
            now = self._now()
            if progress is not None and now >= next_report:
                progress(dict(self.report(), t=now, queued=len(self.queue), running=len(self.running)))
                next_report = now + progress_every
            if max_wall is not None and now > max_wall:
                break
            while pending and pending[0].arrival <= now:
                self.queue.append(pending.popleft())
            self._admit()
            if self.running:
                self.ex.step()
                self.steps += 1
                self._retire()
            elif pending:
                wait = pending[0].arrival - self._now()
                if wait > 0:
                    self._sleep(wait)
        return self.done

    def _sleep(self, dt):
        if self.clock is time.perf_counter:
            time.sleep(min(dt, 0.05))
        elif hasattr(self.clock, "advance"):
            self.clock.advance(dt)

    def report(self):
        lat = np.array([r.latency for r in self.done if r.status == "done"])
        out = {"served": int(len(lat)), "rejected": sum(r.status == "rejected" for r in self.done),
               "steps": self.steps, "peak_running": self.peak_running, "peak_bytes": self.peak_used,
               "oom_requeued": self.oom_requeued}
        if len(lat):
            out.update({"p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
                        "mean_s": float(lat.mean())})
        return out


def pick_class(active, tclass, share: float) -> int:
    """Class to step next: with solves in both classes, the fast class (0)
    while its accumulated step time is at most `share` of the total, else
    the slow class (1); with one class busy, that class."""
    if active[0] and active[1]:
        return 0 if tclass[0] <= share * (tclass[0] + tclass[1]) else 1
    return 0 if active[0] else 1


class GpuExecutor:
    """Runs requests on the HIP library: integrals are produced on the
    device by `payload` (a callable returning (h, eri) CUDA tensors, or
    (h, L) factors when the request has naux > 0, built with
    isci_create_factored), the handle is built, the integrals are dropped,
    and the solve joins an engine.  Footprint = transient integrals +
    handle tables (estimate, then what the handle holds) + subspace.

    Two size classes, each in its own engine: solves of at most `fast_dim`
    determinants and the rest.  An engine step advances every solve of one
    class by one iteration, and the classes share the GPU by time: the fast
    class is stepped while its accumulated step time is below `fast_share`
    of the total, so small solves are not held to the pace of the largest
    ones (a size-based scheduling policy; each solve's arithmetic is the
    same in either class).  fast_dim = 0 puts every solve in one engine."""

    def __init__(self, davidson_opts=None, stream=None, fast_dim: int = 1_000_000, fast_share: float = 0.75,
                 tune: bool = False):
        import paper_1609_07757_amd as isci
        self.isci = isci
        self.tune = bool(tune)   # pick each handle's kernel options with tune.tune_handle (cached per shape)
        self.engs = [isci.isci_engine_create(stream), isci.isci_engine_create(stream)]
        self.opts = davidson_opts or {}
        self.fast_dim = int(fast_dim)
        self.fast_share = float(fast_share)
        self.sigma_vectors = 0
        self.handles = {}
        self._roots = {}
        self.active = [0, 0]
        self.tclass = [0.0, 0.0]

    def footprint(self, r: Request) -> int:
        dim = ci_dim(r.norb, r.nalpha, r.nbeta, r.level)
        return handle_bytes_estimate(r.norb, dim, r.naux) + davidson_bytes(dim, r.nroots)

    def start(self, r: Request):
        """Build the handle and admit the solve.  Raises MemoryError (after
        freeing what it took) when the device runs out of memory."""
        import torch
        hd = None
        try:
            h, ints = r.payload()
            if r.naux > 0:
                hd = self.isci.isci_create_factored(h, ints, r.norb, r.nalpha, r.nbeta, r.level, r.tau)
            else:
                hd = self.isci.isci_create(h, ints, r.norb, r.nalpha, r.nbeta, r.level, r.tau)
            del h, ints
            if self.tune:
                from paper_1609_07757_amd import tune
                tune.tune_handle(hd, nvec=min(r.nroots + 2, 8))
            cls = 0 if hd.dim <= self.fast_dim else 1
            slot = self.isci.isci_engine_add(self.engs[cls], hd, nroots=r.nroots, **self.opts)
        except torch.cuda.OutOfMemoryError as e:
            if hd is not None:
                hd.destroy()
            raise MemoryError(str(e)) from e
        except self.isci.IsciError as e:
            if hd is not None:
                hd.destroy()
            if e.status == self.isci.E_OOM:
                raise MemoryError(str(e)) from e
            raise
        tok = (cls, slot)
        self.handles[tok] = hd
        self._roots[tok] = r.nroots
        self.active[cls] += 1
        return tok

    def charge(self, tok) -> int:
        """Device bytes a running request holds: its handle's tables and its
        Davidson subspace (the dense eri is gone once the handle is built)."""
        hd = self.handles[tok]
        st = self.isci.isci_get_stats(hd)
        return int(st["device_bytes"]) + int(self.isci.isci_davidson_footprint(hd, self._roots[tok]))

    def step(self) -> int:
        """One engine step of the class that is behind its time share (the
        other class when one is empty); returns the number of solves it
        advanced."""
        cls = pick_class(self.active, self.tclass, self.fast_share)
        t0 = time.perf_counter()
        n = self.isci.isci_engine_step(self.engs[cls])
        self.tclass[cls] += time.perf_counter() - t0
        return n

    def poll(self, tok):
        cls, slot = tok
        done, en, _, info = self.isci.isci_engine_result(self.engs[cls], slot)
        if done:
            self.sigma_vectors += info["sigma_calls"]
        return done, en, info

    def finish(self, tok):
        cls, slot = tok
        self.isci.isci_engine_release(self.engs[cls], slot)
        hd = self.handles.pop(tok)
        self._roots.pop(tok, None)
        hd.destroy()
        self.active[cls] -= 1
        if not self.active[cls]:
            self.tclass = [0.0, 0.0]   # a new mix starts its share afresh

    def close(self):
        for e in self.engs:
            e.destroy()
