#!/usr/bin/env python3
"""Benchmark of the ISCI sigma step on one MI355X.

A step is one sigma product sigma = H_tau c over a block of nvec vectors
of the named workload (default: CISDTQ = full CI for 4 electrons, 48
orbitals in a 48 bohr box, 96 auxiliary points, tau = 1e-14, nvec = 8, the
largest plain single-GPU configuration), with inputs resident in HBM.  Prints one JSON line with sigma-vectors/s, screened
terms/s, the roofline position of the dominant kernel (timed with HIP
events on the launch stream), a CPU-oracle baseline timed on a bounded
sample of target determinants, and p50/p99 of Davidson solve latency on
the small CISD workload.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_PEAK_TFLOPS = 78.6      # 256 CU x 4 SIMD x 16 lanes x 2 flop (FMA) x 2.4 GHz
# revision of each kernel's code: stored HBM traffic (profiles/sigma_traffic.json)
# is used only when it was counted for the same revision
KERNEL_REV = {"k_ab_gemm": "slab-major tiles, scalar chunk table, step-aligned parts, 80 VGPRs, 16-byte operand loads, 128-column tiles in 512-column slabs, packed chunks, block levels from the level boundary"}
HBM_PEAK_GBS = 8000.0
METRIC = "σ-vectors/s + screened terms/s (% roofline); p50/p99 Davidson solve latency"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="fci_n48")
    ap.add_argument("--rows-factored", default="cisdt_n60", help="rows mode: workload of the factored and distance rows")
    ap.add_argument("--nvec", type=int, default=None)
    ap.add_argument("--tau", type=float, default=None)
    ap.add_argument("--kernel", choices=["auto", "general", "pair", "mfma"], default="auto")
    ap.add_argument("--ab", choices=["plain", "pipe", "wide", "packed"], default="packed",
                    help="kernel of the alpha-beta block-sparse product")
    ap.add_argument("--onebody", choices=["auto", "transposed", "single", "spectator", "rows"], default="auto",
                    help="one-body kernel on the rows / columns that hold every pair")
    ap.add_argument("--ob-place", choices=["auto", "separate", "tiles"], default="auto",
                    help="one-body units in their own kernels or inside the alpha-beta tiles (default: by chunk growth)")
    ap.add_argument("--onebody-stream", choices=["side", "inline"], default="side",
                    help="one-body kernels on the side stream beside the alpha-beta products, or in line")
    ap.add_argument("--skip-cpu", action="store_true", help="omit the CPU oracle baseline")
    ap.add_argument("--skip-davidson", action="store_true")
    ap.add_argument("--tune", action="store_true", help="batched mode: choose each handle's kernel options with tune.py")
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="target CPU oracle sample time")
    ap.add_argument("--skip-density", action="store_true", help="do not time the density matrices")
    ap.add_argument("--mode", choices=["sigma", "batched", "served", "copycal", "peaks", "sweep", "rows"], default="sigma",
                    help="sigma: headline line; batched: 64 uneven Davidson solves, engine vs plain loop; "
                         "served: Poisson request stream with continuous batching; copycal: plain device "
                         "copies of known size (calibrates the HBM byte counters); sweep: the CISDT "
                         "tau sweep at 60 orbitals and the box-length scan at 30 / 60 / 120 orbitals")
    ap.add_argument("--instances", type=int, default=64)
    ap.add_argument("--requests", type=int, default=120, help="served mode: requests (of the 2000-request stream)")
    ap.add_argument("--max-wall", type=float, default=240.0, help="served mode: wall-clock cap (s)")
    ap.add_argument("--hbm-budget-gb", type=float, default=200.0)
    ap.add_argument("--dense-eri", action="store_true",
                    help="served mode: requests carry dense eri tensors instead of factors")
    ap.add_argument("--fast-dim", type=int, default=1_000_000,
                    help="served mode: solves of at most this many determinants form the fast class (0: one class)")
    ap.add_argument("--fast-share", type=float, default=0.75, help="served mode: GPU time share of the fast class")
    ap.add_argument("--traffic-json", default=os.path.join(ROOT, "profiles", "sigma_traffic.json"),
                    help="HBM bytes per launch from rocprofv3 counters (optional)")
    return ap.parse_args()


def main():
    a = parse()
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: this build runs the sigma step on a single MI355X "
              "(no multi-GPU path); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    if a.mode == "batched":
        return bench_batched(a)
    if a.mode == "served":
        return bench_served(a)
    if a.mode == "copycal":
        return bench_copycal(a)
    if a.mode == "peaks":
        return bench_peaks(a)
    if a.mode == "rows":
        return bench_rows(a)
    if a.mode == "sweep":
        return bench_sweep(a)
    import numpy as np
    import torch

    import paper_1609_07757_amd as isci
    from isci_inputs import random_vectors, workload

    W = workload(a.workload)
    nvec = a.nvec or W.nvec
    tau = W.tau if a.tau is None else a.tau
    dev = torch.device("cuda:0")
    h, eri = W.integrals()
    hd = isci.isci_create(torch.from_numpy(h).to(dev), torch.from_numpy(eri).to(dev), W.norb,
                          W.nalpha, W.nbeta, W.level, tau,
                          onebody={"auto": isci.OB_AUTO, "separate": isci.OB_SEPARATE, "tiles": isci.OB_TILES}[a.ob_place],
                          gas_boundary=W.gas_boundary)
    variant = {"auto": isci.SIGMA_AUTO, "general": isci.SIGMA_GENERAL, "pair": isci.SIGMA_PAIR,
               "mfma": isci.SIGMA_MFMA}[a.kernel]
    isci.isci_set_option(hd, isci.OPT_SIGMA_KERNEL, variant)
    set_ab_product(isci, hd, a.ab)
    if a.onebody != "auto":   # auto: the handle's own choice
        isci.isci_set_option(hd, isci.OPT_ONEBODY_KERNEL,
                             {"single": isci.ONEBODY_SINGLE, "transposed": isci.ONEBODY_TRANSPOSED,
                              "spectator": isci.ONEBODY_SPECTATOR, "rows": isci.ONEBODY_ROWS}[a.onebody])
    isci.isci_set_option(hd, isci.OPT_ONEBODY_STREAM,
                         isci.ONEBODY_SIDE if a.onebody_stream == "side" else isci.ONEBODY_INLINE)
    st = isci.isci_get_stats(hd)
    dim = hd.dim
    c = torch.from_numpy(random_vectors(dim, nvec, seed=21)).to(dev)
    sg = torch.empty_like(c)
    stream = torch.cuda.current_stream()
    for _ in range(a.warmup):
        isci.isci_sigma(hd, c, sg, stream=stream)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(a.steps):
        isci.isci_sigma(hd, c, sg, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev_ms = e0.elapsed_time(e1)
    ms_per_step = ev_ms / a.steps
    # distribution of single steps (an event pair around each, outside the
    # timed region above)
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(a.steps)]
    for ea, eb in evs:
        ea.record(stream)
        isci.isci_sigma(hd, c, sg, stream=stream)
        eb.record(stream)
    torch.cuda.synchronize()
    step_ms = np.array([ea.elapsed_time(eb) for ea, eb in evs])
    # the same step recorded once as a HIP graph and replayed (one graph
    # launch per step instead of the call's kernel launches)
    sg_g = torch.empty_like(c)
    g = isci.isci_sigma_graph_create(hd, c, sg_g)
    for _ in range(a.warmup):
        g.launch(stream)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(a.steps):
        g.launch(stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_graph = e0.elapsed_time(e1) / a.steps
    graph_equal = bool(torch.equal(sg_g, sg))
    g.destroy()
    terms = int(st["terms_total"])
    tb = st["terms"]
    terms_ab = int(tb[26:42].sum())
    terms_rest = terms - terms_ab
    flops_step = 2.0 * terms * nvec
    sig_per_s = nvec * a.steps / (ev_ms * 1e-3)
    terms_per_s = terms * nvec * a.steps / (ev_ms * 1e-3)
    # per-kernel durations: HIP events recorded by the library around each
    # launch on this stream, over a second timed pass of the same steps
    isci.isci_profile(hd, True)
    for _ in range(a.steps):
        isci.isci_sigma(hd, c, sg, stream=stream)
    torch.cuda.synchronize()
    prof = isci.isci_profile_read(hd)
    isci.isci_profile(hd, False)
    # algorithmic flops each kernel performs per step (2 per sigma term per
    # vector); when no one-body launch shows up on the matrix-core path, its
    # terms ride in the alpha-beta tiles (dense integrals)
    terms_1b = int(tb[0:8].sum())
    ob_in_ab = "onebody" not in prof
    t_ab = terms_ab + (terms_1b if ob_in_ab else 0)
    kflops = {"k_sigma_generic": 2.0 * terms * nvec, "k_sigma_n2": 2.0 * terms * nvec,
              "k_sigma_ab_mfma": 2.0 * t_ab * nvec,
              "k_sigma_n2(same-spin)": 2.0 * (terms_rest - terms_1b) * nvec,
              "onebody": 2.0 * terms_1b * nvec,
              "k_ab_gemm": 2.0 * t_ab * nvec,
              # data movement only (no sigma terms): unfold and fold
              "k_ab_unfold": 0.0, "k_ab_fold": 0.0}
    kernels = {}
    for name, (tot_ms, nl) in prof.items():
        per_launch_ms = tot_ms / nl
        launches_per_step = nl / a.steps
        fl = kflops[name] / launches_per_step
        kernels[name] = {"avg_launch_ms": per_launch_ms, "launches_per_step": launches_per_step,
                         "share_of_step": tot_ms / a.steps / ms_per_step,
                         "algorithmic_flops_per_launch": fl,
                         "tflops": fl / (per_launch_ms * 1e-3) / 1e12}
    # dominant kernel: the largest time per step among those that do the
    # sigma arithmetic.  The one-body entry is a group of launches (its
    # timing marks bracket all of them); it competes when the recorded
    # times add up within the step, i.e. nothing ran beside it, so its time
    # is its own; beside the products on the side stream its duration
    # includes time shared with them, and the single kernels decide
    summed = sum(v["avg_launch_ms"] * v["launches_per_step"] for v in kernels.values())
    overlapped = summed > 1.02 * ms_per_step
    arith = [k for k in kernels if kflops.get(k, 0.0) > 0.0 and (k != "onebody" or not overlapped)] or list(kernels)
    dom = max(arith, key=lambda k: kernels[k]["avg_launch_ms"] * kernels[k]["launches_per_step"])
    kname = dom
    achieved = kernels[dom]["tflops"]
    nlaunch = kernels[dom]["launches_per_step"]
    traffic = None
    if os.path.exists(a.traffic_json):
        try:
            tj = json.load(open(a.traffic_json))
            key = f"{a.workload}:nvec{nvec}:tau{tau:g}"
            if key in tj and tj[key].get("kernel_version") == f"{kname}:{KERNEL_REV.get(kname, '')}":
                traffic = tj[key]["bytes_per_launch"]
        except Exception:
            traffic = None
    out = {
        "metric": METRIC,
        "value": sig_per_s,
        "unit": "σ-vectors/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (recipe A 1D local-orbital integrals, seeded)",
        "config": {"workload": a.workload, "norb": W.norb, "nalpha": W.nalpha, "nbeta": W.nbeta,
                   "max_excitation": W.level, "tau": tau, "nvec": nvec, "dim": dim,
                   "box": W.box_len, "naux": W.n_aux, "seed": W.seed, "ab_product": a.ab,
                   "onebody_kernel": a.onebody, "onebody_stream": a.onebody_stream,
                   **({"gas_boundary": W.gas_boundary} if W.gas_boundary else {})},
        "screened_terms_per_s": terms_per_s,
        "terms_per_vector": terms,
        "kept_integral_units": int(st["kept_total"]),
        "wall_s_timed": wall,
        "step_ms_p50": float(np.percentile(step_ms, 50)), "step_ms_p99": float(np.percentile(step_ms, 99)),
        "roofline": {"bound": "alu" if kname in ("k_sigma_generic", "k_sigma_n2", "k_sigma_n2(same-spin)") else "mfma",
                     "kernel": kname if kname != "onebody" else "onebody (group: the one-body class launches of a step)",
                     "kernels_overlapped": overlapped,
                     "achieved": achieved, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP64_PEAK_TFLOPS, "traffic": traffic,
                     "launches_per_step": nlaunch,
                     "avg_launch_ms": kernels[kname]["avg_launch_ms"],
                     "algorithmic_flops_per_launch": kernels[kname]["algorithmic_flops_per_launch"]},
        "step_tflops": flops_step / (ms_per_step * 1e-3) / 1e12,
        "step_frac_fp64": flops_step / (ms_per_step * 1e-3) / 1e12 / FP64_PEAK_TFLOPS,
        "kernels": kernels,
        "graph": {"ms_per_step": ms_graph, "sigma_vectors_per_s": nvec / (ms_graph * 1e-3),
                  "speedup_vs_calls": ms_per_step / ms_graph, "bitwise_equal_to_calls": graph_equal},
    }
    if not a.skip_density:
        out["density1"] = density1_timing(isci, torch, hd, c, stream, a.steps)
    if not a.skip_davidson:
        out["davidson"] = davidson_latency(isci, torch, dev)
    if not a.skip_cpu:
        out["cpu_baseline"] = cpu_baseline(W, h, eri, tau, nvec, dim, a.cpu_seconds)
    print(json.dumps(out), flush=True)


def set_ab_product(isci, hd, name):
    """Kernel of the alpha-beta product: plain ping-pong or software pipeline."""
    isci.isci_set_option(hd, isci.OPT_AB_PRODUCT, {"plain": isci.AB_PLAIN, "pipe": isci.AB_PIPE,
                                                   "wide": isci.AB_WIDE, "packed": isci.AB_PACKED}[name])


def density1_timing(isci, torch, hd, c, stream, steps):
    """One-body density matrices of the bench vectors (not part of the sigma
    step or its value), timed with HIP events on the launch stream.  Bytes a
    pass must move at least: the alpha pass reads c (8 B per determinant
    and vector), the beta pass transposes c (16 B) and reads the
    transposed copy (8 B): 32 B per determinant and vector."""
    d1 = isci.isci_density1(hd, c, stream=stream)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        isci.isci_density1(hd, c, d1, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    nv = int(c.shape[0])
    nb = 32.0 * hd.dim * nv
    tr = [float(torch.trace(d1[v, s]) / (c[v] @ c[v])) for v in range(nv) for s in range(2)]
    return {"ms_per_call": ms, "vectors": nv, "electrons_from_traces": [min(tr), max(tr)],
            "roofline": {"bound": "hbm", "achieved": nb / (ms * 1e-3) / 1e9, "peak": 8000.0, "unit": "GB/s",
                         "frac": nb / (ms * 1e-3) / 1e9 / 8000.0, "algorithmic_bytes": nb}}


def davidson_latency(isci, torch, dev, reps=9):
    """p50 / p99 latency of a full Davidson solve (create excluded) on the
    plain CISD workload (20 orbitals, lowest root)."""
    import numpy as np
    from isci_inputs import workload
    W = workload("cisd_n20")
    h, eri = W.integrals()
    hd = isci.isci_create(torch.from_numpy(h).to(dev), torch.from_numpy(eri).to(dev), W.norb, 2, 2,
                          W.level, W.tau)
    lat, en, iters = [], None, 0
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e, _, info = isci.isci_davidson(hd, nroots=1)
        lat.append(time.perf_counter() - t0)
        en, iters = float(e[0]), info["iterations"]
    lat = np.array(lat) * 1e3
    return {"workload": "cisd_n20", "p50_ms": float(np.percentile(lat, 50)),
            "p99_ms": float(np.percentile(lat, 99)), "energy": en, "iterations": iters, "solves": reps}


def cpu_baseline(W, h, eri, tau, nvec, dim, seconds):
    """The CPU oracle (plain Slater-Condon, OpenMP over targets) timed on a
    bounded sample of target determinants of the same workload, scaled to
    sigma-vectors/s."""
    import numpy as np
    import oracle as O
    from isci_inputs import random_vectors
    S = O.Space(W.norb, W.nalpha, W.nbeta, W.level, boundary=W.gas_boundary or None)
    c = random_vectors(dim, nvec, seed=21)
    rng = np.random.default_rng(0)
    n = 64
    t = 0.0
    while True:
        tg = np.sort(rng.choice(dim, size=min(n, dim), replace=False))
        t0 = time.perf_counter()
        O.sigma(S, h, eri, tau, c, targets=tg)
        t = time.perf_counter() - t0
        if t >= seconds or n >= dim:
            break
        n = int(min(dim, max(2 * n, n * seconds / max(t, 1e-3) * 1.05)))
    frac = len(tg) / dim
    value = nvec * frac / t
    out = {"value": value, "unit": "σ-vectors/s", "cores": O.num_threads(), "kind": "oracle",
           "sample": f"{len(tg)} of {dim} target determinants (random, seed 0), nvec={nvec}, "
                     f"{t:.1f} s; scaled by dim/sample"}
    out["single_core"] = cpu_baseline_one_core(W, tau, nvec, dim, max(2, len(tg) // max(1, O.num_threads())),
                                               seconds)
    return out


def cpu_baseline_one_core(W, tau, nvec, dim, ntarget, seconds):
    """The same oracle on one host core (a child process with
    OMP_NUM_THREADS=1), on a sample sized to take about `seconds`."""
    import subprocess
    code = ("import sys, time, json, numpy as np; sys.path.insert(0, %r); import oracle as O; "
            "from isci_inputs import random_vectors, workload; W = workload(%r); h, eri = W.integrals(); "
            "S = O.Space(W.norb, W.nalpha, W.nbeta, W.level, boundary=W.gas_boundary or None); "
            "c = random_vectors(%d, %d, seed=21); "
            "rng = np.random.default_rng(1); n = %d\n"
            "while True:\n"
            "    tg = np.sort(rng.choice(%d, size=min(n, %d), replace=False)); t0 = time.perf_counter(); "
            "O.sigma(S, h, eri, %r, c, targets=tg); t = time.perf_counter() - t0\n"
            "    if t >= %r * 0.6 or n >= %d: break\n"
            "    n = int(min(%d, max(2 * n, n * %r / max(t, 1e-3))))\n"
            "print(json.dumps({'n': int(len(tg)), 't': t, 'threads': O.num_threads()}))"
            % (ROOT, W.name, dim, nvec, max(2, ntarget // 8), dim, dim, tau, seconds, dim, dim, seconds))
    env = dict(os.environ, OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=600)
    if r.returncode != 0:
        return {"error": r.stderr[-400:]}
    d = json.loads(r.stdout.strip().splitlines()[-1])
    return {"value": nvec * d["n"] / dim / d["t"], "unit": "σ-vectors/s", "cores": d["threads"], "kind": "oracle",
            "sample": f"{d['n']} of {dim} target determinants (random, seed 1), nvec={nvec}, {d['t']:.1f} s; "
                      f"scaled by dim/sample"}


def _kernel_variant(isci, name):
    return {"auto": isci.SIGMA_AUTO, "general": isci.SIGMA_GENERAL, "pair": isci.SIGMA_PAIR,
            "mfma": isci.SIGMA_MFMA}[name]


def bench_batched(a):
    """64 uneven CI instances (norb 20-80, CISD/CISDT, 1-4 roots, tau 1e-12):
    every solve run one at a time (one instance per launch) vs all solves in
    one engine (one fused sigma launch per Davidson iteration).  Reports
    sigma-vectors/s of both, their ratio and the largest energy difference."""
    import numpy as np
    import torch
    import paper_1609_07757_amd as isci
    from isci_inputs.device import integrals_on_device
    from isci_inputs.workloads import batched_instances
    insts = batched_instances(a.instances)
    handles = []
    t0 = time.perf_counter()
    for W in insts:
        h, eri = integrals_on_device(W.norb, W.box_len, W.n_aux, W.seed)
        hd = isci.isci_create(h, eri, W.norb, 2, 2, W.level, W.tau)
        del h, eri
        isci.isci_set_option(hd, isci.OPT_SIGMA_KERNEL, _kernel_variant(isci, a.kernel))
        handles.append(hd)
    torch.cuda.synchronize()
    t_create = time.perf_counter() - t0
    t_tune, tuned = 0.0, {}
    if a.tune:
        # kernel options per handle from the tuner (timed on each handle,
        # cached per shape); outside the timed regions
        from paper_1609_07757_amd import tune
        t0 = time.perf_counter()
        for W, hd in zip(insts, handles):
            cfg, _ = tune.tune_handle(hd, nvec=min(W.nroots + 2, 8))
            tuned[str(cfg)] = tuned.get(str(cfg), 0) + 1
        torch.cuda.synchronize()
        t_tune = time.perf_counter() - t0
    # plain: one solve after the other
    t0 = time.perf_counter()
    plain_e, plain_sig = [], 0
    for W, hd in zip(insts, handles):
        e, _, info = isci.isci_davidson(hd, nroots=W.nroots)
        plain_e.append(e)
        plain_sig += info["sigma_calls"]
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    # batched: one engine, all slots
    eng = isci.isci_engine_create()
    t0 = time.perf_counter()
    slots = [isci.isci_engine_add(eng, hd, nroots=W.nroots) for W, hd in zip(insts, handles)]
    steps = 0
    while isci.isci_engine_step(eng) > 0:
        steps += 1
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    batch_e, batch_sig, iters = [], 0, []
    for sl in slots:
        done, e, _, info = isci.isci_engine_result(eng, sl)
        batch_e.append(e)
        batch_sig += info["sigma_calls"]
        iters.append(info["iterations"])
    dE = max(float(np.abs(x - y).max()) for x, y in zip(plain_e, batch_e))
    out = {"metric": "batched σ-vectors/s (64 uneven Davidson solves, one engine) vs plain loop",
           "value": batch_sig / t_batch, "unit": "σ-vectors/s", "n_gpus": 1,
           "higher_is_better": True, "dtype": "f64", "data": "synthetic (recipe A, per-instance seeds)",
           "config": {"workload": "batched64", "instances": len(insts), "tau": 1e-12,
                      "norb_range": [min(w.norb for w in insts), max(w.norb for w in insts)],
                      "kernel": a.kernel},
           "plain_sigma_vectors_per_s": plain_sig / t_plain, "speedup_vs_plain": (batch_sig / t_batch) / (plain_sig / t_plain),
           "plain_s": t_plain, "batched_s": t_batch, "engine_steps": steps, "create_s": t_create,
           "max_abs_energy_diff": dE, "sigma_vectors_plain": plain_sig, "sigma_vectors_batched": batch_sig,
           "max_iterations": max(iters), "tuned": bool(a.tune), "tune_s": t_tune, "tuned_configs": tuned}
    print(json.dumps(out), flush=True)


def bench_served(a):
    """Poisson stream (50 req/s) of Davidson solves, norb log-uniform in
    [40, 200], CISD/CISDT (CISDTQ when its dimension is below 5M), 1-3
    roots, tau 1e-12; admission by HBM footprint into a continuously
    batched engine.  Runs the first `requests` of the 2000-request stream
    (or until max_wall) and reports p50/p99 arrival-to-energy latency."""
    import numpy as np
    import torch
    from paper_1609_07757_amd.serve import GpuExecutor, Request, Server
    from isci_inputs.device import factors_on_device, integrals_on_device
    from isci_inputs.workloads import served_requests
    stream = served_requests(2000)[: a.requests]
    reqs = []
    for i, (t, W) in enumerate(stream):
        if a.dense_eri:
            def payload(W=W):
                return integrals_on_device(W.norb, W.box_len, W.n_aux, W.seed)
        else:
            def payload(W=W):
                return factors_on_device(W.norb, W.box_len, W.n_aux, W.seed)
        reqs.append(Request(i, t, W.norb, 2, 2, W.level, W.tau, W.nroots, payload=payload,
                            naux=0 if a.dense_eri else W.n_aux))
    ex = GpuExecutor(fast_dim=a.fast_dim, fast_share=a.fast_share)
    srv = Server(ex, hbm_budget=int(a.hbm_budget_gb * 2**30), max_slots=64)
    samples = []

    def progress(r):
        samples.append({k: r[k] for k in ("t", "queued", "running", "served") if k in r})
        print("served progress", json.dumps(r), file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    srv.run(reqs, max_wall=a.max_wall, progress=progress)
    wall = time.perf_counter() - t0
    rep = srv.report()
    done = [r for r in srv.done if r.status == "done"]
    last_arrival = max(r.arrival for r in reqs) if reqs else 0.0
    out = {"metric": "served Davidson solves: p50/p99 latency and σ throughput",
           "value": rep.get("p50_s"), "unit": "s (p50 latency)", "n_gpus": 1, "higher_is_better": False,
           "dtype": "f64", "data": "synthetic (recipe A, per-request seeds, Poisson arrivals)",
           "config": {"workload": "served_poisson50", "requests_offered": len(reqs), "rate_per_s": 50,
                      "tau": 1e-12, "hbm_budget_gb": a.hbm_budget_gb,
                      "fast_class_dim": a.fast_dim, "fast_class_share": a.fast_share,
                      "integrals": "dense eri" if a.dense_eri else "factors (isci_create_factored)"},
           "p50_s": rep.get("p50_s"), "p99_s": rep.get("p99_s"), "served": rep["served"],
           "rejected": rep["rejected"], "wall_s": wall, "sigma_vectors_per_s": ex.sigma_vectors / wall,
           "peak_concurrent": rep["peak_running"], "peak_bytes": rep["peak_bytes"],
           "norb_served": sorted(r.norb for r in done)[-3:],
           "offered_rate_per_s": len(reqs) / last_arrival if last_arrival > 0 else None,
           "sustained_rate_per_s": rep["served"] / wall if wall > 0 else None,
           "unfinished": len(reqs) - rep["served"] - rep["rejected"],
           "oom_requeued": rep.get("oom_requeued", 0), "queue_over_time": samples}
    ex.close()
    print(json.dumps(out), flush=True)


def _sigma_point(isci, torch, W, tau, nvec, steps, warmup):
    """sigma-vectors/s and terms of one workload at one tau (HIP-event timed
    calls on the current stream, inputs resident)."""
    from isci_inputs import random_vectors
    from isci_inputs.device import integrals_on_device
    h, eri = integrals_on_device(W.norb, W.box_len, W.n_aux, W.seed)
    hd = isci.isci_create(h, eri, W.norb, W.nalpha, W.nbeta, W.level, tau)
    del h, eri
    st = isci.isci_get_stats(hd)
    c = torch.from_numpy(random_vectors(hd.dim, nvec, seed=21)).to("cuda:0")
    sg = torch.empty_like(c)
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        isci.isci_sigma(hd, c, sg, stream=stream)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(steps):
        isci.isci_sigma(hd, c, sg, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    terms = int(st["terms_total"])
    out = {"workload": W.name, "norb": W.norb, "tau": tau, "nvec": nvec, "dim": hd.dim,
           "kept_units": int(st["kept_total"]), "terms_per_vector": terms, "ms_per_step": ms,
           "sigma_vectors_per_s": nvec / (ms * 1e-3), "screened_terms_per_s": terms * nvec / (ms * 1e-3),
           "tflops": 2.0 * terms * nvec / (ms * 1e-3) / 1e12}
    hd.destroy()
    del c, sg
    torch.cuda.empty_cache()
    return out


def bench_sweep(a):
    """The CISDT measurements beside the headline: the screening sweep at 60
    orbitals (tau = 0 / 1e-14 / 1e-10) and the box-length scan at fixed
    orbital density (30 / 60 / 120 orbitals, tau = 1e-14), with the fitted
    exponents of screened terms, determinants and sigma time against the box
    length (the paper's own exponents, measured on beryllium with another
    basis, are context only)."""
    import numpy as np
    import torch
    import paper_1609_07757_amd as isci
    from isci_inputs import workload
    nvec = a.nvec or 8
    tau_sweep = []
    for tau in (0.0, 1e-14, 1e-10):
        tau_sweep.append(_sigma_point(isci, torch, workload("cisdt_n60"), tau, nvec, a.steps, a.warmup))
        print("sweep", json.dumps(tau_sweep[-1]), file=sys.stderr, flush=True)
    scan = []
    for name in ("cisdt_n30", "cisdt_n60", "cisdt_n120"):
        W = workload(name)
        scan.append(_sigma_point(isci, torch, W, W.tau, nvec, a.steps, a.warmup))
        print("scan", json.dumps(scan[-1]), file=sys.stderr, flush=True)
    box = np.log([p["norb"] for p in scan])

    def fit(key):
        return float(np.polyfit(box, np.log([p[key] for p in scan]), 1)[0])
    out = {"metric": "σ-vectors/s and screened terms/s: CISDT tau sweep and box-length scan",
           "unit": "σ-vectors/s", "n_gpus": 1, "dtype": "f64",
           "data": "synthetic (recipe A 1D local-orbital integrals, seeded)",
           "config": {"workload": "cisdt_sweep", "nvec": nvec},
           "tau_sweep_cisdt_n60": tau_sweep, "box_scan": scan,
           "fitted_exponents_vs_box": {"terms": fit("terms_per_vector"), "dim": fit("dim"),
                                       "ms_per_step": fit("ms_per_step")},
           "paper_context": {"cisd": 1.24, "cisdt": 1.48, "cisdtq": 1.98,
                             "note": "the paper's flop-count exponents for beryllium in a finite-element basis; "
                                     "context only, not a target"}}
    print(json.dumps(out), flush=True)


def _events_ms(torch, stream, fn, reps):
    fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def bench_rows(a):
    """The rows that extend the sigma path, each timed on the device and set
    against its bound:
      * two-body densities (isci_density2) on the workload's vectors: HBM,
        the three spin blocks written once and c read once, 8 (3 norb^4 +
        dim) B per vector;
      * imaginary-time SIAL propagation (isci_propagate): time per step and
        the share its sigma calls take at the one-vector sigma rate;
      * handles from factors against dense handles: creation time, the
        bytes handed over, and the sigma of both (bit for bit);
      * distance screening: kept units and sigma time against the radius;
      * the two-space GAS restriction (200 orbitals, at most one outer
        electron, handle from factors): sigma time and the product
        kernel's roofline."""
    import numpy as np
    import torch
    import paper_1609_07757_amd as isci
    from isci_inputs import random_vectors, workload
    from isci_inputs.recipes import factors_a, orbital_centres
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    out = {"metric": "extension rows: two-body densities, SIAL propagation, handles from factors, distance screening, GAS",
           "n_gpus": 1, "dtype": "f64", "data": "synthetic (recipe A, seeded)"}
    # two-body densities
    W = workload(a.workload)
    h, eri = W.integrals()
    hd = isci.isci_create(torch.from_numpy(h).to(dev), torch.from_numpy(eri).to(dev), W.norb, 2, 2, W.level, W.tau)
    nv = 4
    c = torch.from_numpy(random_vectors(hd.dim, nv, seed=21)).to(dev)
    d2 = isci.isci_density2(hd, c)
    ms = _events_ms(torch, stream, lambda: isci.isci_density2(hd, c, d2), 5)
    n4 = float(W.norb) ** 4
    nb = nv * 8.0 * (3 * n4 + hd.dim)
    nrm = (c * c).sum(dim=1)
    tr_ab = [float(torch.einsum("pprr->", d2[v, 1]) / nrm[v]) for v in range(nv)]

    def gram_flops(lengths):
        # 2 flops per product of two rows' common prefix, row pairs i <= j:
        # sum over i <= j of min(len_i, len_j), from the lengths sorted downwards
        ls = np.sort(np.asarray(lengths, dtype=np.float64))[::-1]
        return 2.0 * float(np.sum(ls * (np.arange(len(ls)) + 1.0)))
    rs = isci.isci_rowstart(hd)
    _, lev_a = isci.isci_strings(hd, 0)
    _, lev_b = isci.isci_strings(hd, 1)
    le_a = np.array([np.sum(lev_a <= k) for k in range(W.level + 1)])
    len_b = le_a[np.clip(W.level - lev_b, 0, W.level)]
    nn = W.norb * W.norb
    fl = nv * (gram_flops(np.diff(rs)) + gram_flops(len_b) + 2.0 * nn * nn * (nn + 1) / 2.0)
    out["density2"] = {"workload": W.name, "vectors": nv, "ms_per_call": ms, "pairs_ab_from_traces": [min(tr_ab), max(tr_ab)],
                       "roofline": {"bound": "mfma", "kernel": "k_gram_rows (whole call)",
                                    "achieved": fl / (ms * 1e-3) / 1e12, "peak": 78.6, "unit": "TFLOP/s",
                                    "frac": fl / (ms * 1e-3) / 1e12 / 78.6, "algorithmic_flops": fl},
                       "hbm": {"algorithmic_bytes": nb, "achieved_GBps": nb / (ms * 1e-3) / 1e9}}
    del d2
    # SIAL propagation (imaginary time from the reference determinant)
    c1 = torch.zeros(hd.dim, dtype=torch.float64, device=dev)
    c1[0] = 1.0
    s1 = torch.empty_like(c1)
    sig_ms = _events_ms(torch, stream, lambda: isci.isci_sigma(hd, c1, s1, stream=stream), 10)
    isci.isci_propagate(hd, c1.clone(), 0.5, 1, krylov=16)
    torch.cuda.synchronize()

    def prop(steps):
        x = c1.clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        inf = isci.isci_propagate(hd, x, 0.5, steps, krylov=16)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3, inf

    # a call's time is a fixed part (buffers, the final energy) plus a
    # steady part per step: from calls of 5 and 25 steps
    ms5, inf5 = prop(5)
    ms25, info = prop(25)
    per_step = (ms25 - ms5) / 20.0
    calls_per_step = (info["sigma_calls"] - inf5["sigma_calls"]) / 20.0
    out["propagation"] = {"workload": W.name, "dt": 0.5, "krylov_max": 16, "ms_per_step": per_step,
                          "ms_per_call_fixed": ms5 - 5 * per_step, "ms_25_step_call": ms25,
                          "sigma_calls_per_step": calls_per_step, "krylov_last": info["krylov_last"],
                          "energy": info["energy"], "sigma_ms_one_vector": sig_ms,
                          "sigma_share": calls_per_step * sig_ms / per_step}
    del hd
    # handles from factors against dense handles
    Wf = workload(a.rows_factored)
    hf_np, L_np = factors_a(Wf.norb, Wf.box_len, Wf.n_aux, Wf.seed)
    ht = torch.from_numpy(hf_np).to(dev)
    Lt = torch.from_numpy(np.ascontiguousarray(L_np)).to(dev)
    et = torch.from_numpy(Wf.integrals()[1]).to(dev)
    torch.cuda.synchronize()

    def timed_create(fn):
        best = None
        for _ in range(3):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            x = fn()
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            best = dt if best is None else min(best, dt)
        return x, best
    hdn, t_dense = timed_create(lambda: isci.isci_create(ht, et, Wf.norb, 2, 2, Wf.level, Wf.tau))
    hfa, t_fact = timed_create(lambda: isci.isci_create_factored(ht, Lt, Wf.norb, 2, 2, Wf.level, Wf.tau))
    cv = torch.from_numpy(random_vectors(hdn.dim, 2, seed=3)).to(dev)
    sd, sf = isci.isci_sigma(hdn, cv), isci.isci_sigma(hfa, cv)
    # the dense tensor here is the recipe's own assembly (a matrix product),
    # not the factors' ascending-K sums, so the two agree to rounding only
    rel = float((sd - sf).abs().max() / sd.abs().max())
    out["factored"] = {"workload": Wf.name, "naux": Wf.n_aux, "create_dense_s": t_dense, "create_factored_s": t_fact,
                       "bytes_dense_eri": 8.0 * Wf.norb ** 4, "bytes_factors": 8.0 * Wf.n_aux * Wf.norb ** 2,
                       "sigma_max_rel_diff": rel}
    del hdn, hfa, et
    # distance screening
    x = orbital_centres(Wf.norb, Wf.box_len, Wf.n_aux, Wf.seed)
    dist = np.abs(x[:, None] - x[None, :])
    rows = []
    for rmax in (0.0, 6.0, 4.0, 3.0):
        hx = isci.isci_create(ht, torch.from_numpy(Wf.integrals()[1]).to(dev), Wf.norb, 2, 2, Wf.level, Wf.tau,
                              orb_dist=dist if rmax > 0 else None, max_dist=rmax)
        cx = torch.from_numpy(random_vectors(hx.dim, 8, seed=5)).to(dev)
        sx = torch.empty_like(cx)
        ms = _events_ms(torch, stream, lambda: isci.isci_sigma(hx, cx, sx, stream=stream), 10)
        st = isci.isci_get_stats(hx)
        rows.append({"max_dist": rmax if rmax > 0 else None, "kept_units": int(np.sum(st["kept"])),
                     "terms_per_vector": int(np.sum(st["terms"])), "ms_per_step_8_vectors": ms})
        del hx
    out["distance"] = {"workload": Wf.name, "points": rows}
    # two-space GAS restriction (the 200-orbital single-outer-electron
    # workload, its handle built from factors): sigma time of its vectors
    # and the product kernel's share, against the size of the full-CI and
    # excitation-hierarchy spaces of the same orbitals
    Wg = workload("gas1_n200")
    hg_np, Lg_np = factors_a(Wg.norb, Wg.box_len, Wg.n_aux, Wg.seed)
    hg = isci.isci_create_factored(torch.from_numpy(hg_np).to(dev), torch.from_numpy(np.ascontiguousarray(Lg_np)).to(dev),
                                   Wg.norb, 2, 2, Wg.level, Wg.tau, gas_boundary=Wg.gas_boundary)
    cg = torch.from_numpy(random_vectors(hg.dim, Wg.nvec, seed=21)).to(dev)
    sgg = torch.empty_like(cg)
    ms = _events_ms(torch, stream, lambda: isci.isci_sigma(hg, cg, sgg, stream=stream), 20)
    st = isci.isci_get_stats(hg)
    isci.isci_profile(hg, True)
    for _ in range(10):
        isci.isci_sigma(hg, cg, sgg, stream=stream)
    torch.cuda.synchronize()
    prof = isci.isci_profile_read(hg)
    isci.isci_profile(hg, False)
    gm_ms, gm_n = prof.get("k_ab_gemm", (0.0, 1))
    t_ab = int(np.sum(st["terms"][26:42])) + int(np.sum(st["terms"][0:8]))   # one-body units ride in the tiles
    fl = 2.0 * t_ab * Wg.nvec / (gm_n / 10.0)
    out["gas"] = {"workload": Wg.name, "gas_boundary": Wg.gas_boundary, "max_outer_electrons": Wg.level, "dim": hg.dim,
                  "dim_full_ci": math.comb(Wg.norb, 2) ** 2, "nvec": Wg.nvec, "ms_per_step": ms,
                  "sigma_vectors_per_s": Wg.nvec / (ms * 1e-3), "terms_per_vector": int(st["terms_total"]),
                  "roofline": {"bound": "mfma", "kernel": "k_ab_gemm", "avg_launch_ms": gm_ms / gm_n,
                               "achieved": fl / (gm_ms / gm_n * 1e-3) / 1e12, "peak": 78.6, "unit": "TFLOP/s",
                               "frac": fl / (gm_ms / gm_n * 1e-3) / 1e12 / 78.6}}
    del hg
    print(json.dumps(out), flush=True)


def bench_copycal(a):
    """Device-to-device copies of a 512 MiB FP64 buffer: the counters
    FETCH_SIZE / WRITE_SIZE of these dispatches against the known byte
    count give the scale applied to the sigma kernels' counters."""
    import torch
    n = (512 << 20) // 8
    x = torch.empty(n, dtype=torch.float64, device="cuda:0").fill_(1.0)
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"mode": "copycal", "bytes_per_copy": 8 * n, "copies": 3}), flush=True)


def bench_peaks(a):
    """Re-measures the roofline peaks on this GPU: HBM by a 2 GiB device copy
    (bytes read + written per second), FP64 matrix and vector rates by the
    library's issue-rate probes, and a 8192^3 FP64 GEMM through torch
    (rocBLAS) for context.  Prints one JSON line."""
    import torch
    import paper_1609_07757_amd as isci
    dev = torch.device("cuda:0")
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        e0.record(st)
        for _ in range(reps):
            fn()
        e1.record(st)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) * 1e-3 / reps

    n = (2 << 30) // 8
    x = torch.ones(n, dtype=torch.float64, device=dev)
    y = torch.empty_like(x)
    t_copy = timed(lambda: y.copy_(x), 10)
    hbm = 2.0 * 8 * n / t_copy / 1e12
    del x, y
    blocks = 256 * 8
    out = torch.empty(blocks * 256, dtype=torch.float64, device=dev)
    res = {}
    for kind, name, iters in ((0, "fp64_matrix_tflops", 20000), (1, "fp64_vector_tflops", 20000)):
        fl = [0.0]

        def run(kind=kind, iters=iters):
            fl[0] = isci.isci_probe_fp64(kind, iters, blocks, out, st)
        t = timed(run, 3)
        res[name] = fl[0] / t / 1e12
    m = torch.rand(8192, 8192, dtype=torch.float64, device=dev)
    t_mm = timed(lambda: torch.matmul(m, m), 3)
    out_line = {"mode": "peaks", "hbm_copy_tb_s": hbm, **res, "dgemm_8192_tflops": 2.0 * 8192 ** 3 / t_mm / 1e12,
                "published": {"hbm_tb_s": 8.0, "fp64_matrix_tflops": FP64_PEAK_TFLOPS, "fp64_vector_tflops": 78.6}}
    print(json.dumps(out_line), flush=True)


if __name__ == "__main__":
    main()
