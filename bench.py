"""Benchmark of the implicit-solver hot path on one MI355X.

A step is one pseudo-time iteration of the whole path (primitives, residual
with chemistry, diagonal blocks, LU-SGS forward/backward sweeps, consistency
correction and update, norms) over the 512 x 256 polar blunt-body grid with
two-temperature 5-species air at CFL 100 (synthetic free-stream start).
Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# algorithmic bytes per cell-iteration (state read twice and written once,
# geometry read twice, sweep intermediate written and read once)
GEOM_WORDS = 5


def b_alg(m, mode, precision):
    nsol = m.nb if mode == 0 else m.nf + m.ns
    w_sweep = 8 if precision == 0 else 4
    return (3 * m.nv + 2 * GEOM_WORDS) * 8 + 2 * nsol * w_sweep


def run_variant(csi, cfg, m, x, y, fs, q0, mode, kind, precision, steps, warmup):
    import torch
    s = csi.Solver((x, y), m, fs)
    s.set_state(q0)
    s.set_timing(True)
    if warmup:
        s.step(mode, kind, cfg.cfl, warmup, precision=precision, cfl_ramp=100, check_every=max(warmup, 1))
    s.phase_times(reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = s.step(mode, kind, cfg.cfl, steps, precision=precision, cfl_ramp=100, check_every=steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ph = s.phase_times()
    return {"seconds": dt, "iters": st["iters"], "cell_iters_per_s": cfg.ni * cfg.nj * st["iters"] / dt,
            "ms_per_step": 1e3 * dt / max(st["iters"], 1), "phases_ms": ph, "stats": st}


def cpu_baseline(cfg, m, x, y, fs, q0, budget_s=20.0):
    """The oracle on the host cores over a bounded sample: whole c2-size
    iterations (split, CC2) until about budget_s seconds have passed."""
    from oracle import orc
    threads = os.cpu_count() or 1
    o = orc.setup((x, y), m, fs, threads=threads)
    o.set_state(q0)
    t0 = time.perf_counter()
    n = 0
    while True:
        o.step(1, 2, cfg.cfl, 1, ramp=100, it0=n)
        n += 1
        if time.perf_counter() - t0 > budget_s or n >= 50:
            break
    dt = time.perf_counter() - t0
    return {"value": cfg.ni * cfg.nj * n / dt, "unit": "cell-iters/s", "cores": threads, "kind": "oracle",
            "sample": f"{n} split-CC2 FP64 iterations of the {cfg.ni}x{cfg.nj} workload from the free stream"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--config", default="c2")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--variants", default="split64,coupled64,splitmixed")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)

    import torch
    from paper_2403_03440_amd import csi
    from paper_2403_03440_amd import inputs as I

    cfg = I.CONFIGS[args.config]
    m = cfg.mechanism()
    x, y = cfg.grid()
    fs = I.freestream_prims(cfg, m)
    # conservative initial state from the library's own conversion on the device
    s0 = csi.Solver((x, y), m, fs)
    q0 = s0.initial_state(*I.initial_prims(cfg, m))
    del s0
    variants = {"split64": (1, 2, 0), "coupled64": (0, 0, 0), "splitmixed": (1, 2, 1), "coupledmixed": (0, 0, 1)}
    res = {}
    for v in args.variants.split(","):
        mode, kind, prec = variants[v]
        print(f"# running {v}", file=sys.stderr, flush=True)
        res[v] = run_variant(csi, cfg, m, x, y, fs, q0, mode, kind, prec, args.steps, args.warmup)
        res[v]["b_alg"] = b_alg(m, mode, prec)
    head = res.get("split64") or next(iter(res.values()))
    N = cfg.ni * cfg.nj
    # roofline of the dominant phase of the headline variant (event-timed inside the library)
    ph = head["phases_ms"]
    dom = max(ph, key=lambda k: ph[k]["ms"])
    per_iter_ms = ph[dom]["ms"] / max(head["iters"], 1)
    alg_bytes = {"sweeps": 2 * 2 * (m.nf + m.ns) * 8 * N, "cell": (m.nv + m.nv + 1 + (m.nf + m.ns)) * 8 * N}
    traffic_bytes = alg_bytes.get(dom)
    roof = None
    if traffic_bytes is not None:
        ach = traffic_bytes / (per_iter_ms * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": ach, "peak": 8000.0, "unit": "GB/s", "frac": ach / 8000.0,
                "traffic": None, "kernel": dom, "ms_per_launch_group": per_iter_ms}
    out = {
        "metric": "cell-iters/s & time-to-1e-8 residual: split vs coupled, FP64 vs mixed+MLP",
        "value": head["cell_iters_per_s"],
        "unit": "cell-iters/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{cfg.name}: {cfg.ni}x{cfg.nj} polar blunt body, {m.ns}-species air "
                               f"{'2T' if m.two_temp else '1T'}, CFL {cfg.cfl:g}, split FP64 + CC2",
                   "cells": N},
        "variants": {k: {kk: vv for kk, vv in r.items() if kk != "stats"} for k, r in res.items()},
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        print("# cpu baseline", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(cfg, m, x, y, fs, q0)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
