"""Benchmark of the implicit-solver hot path on one MI355X.

A step is one pseudo-time iteration of the whole path: primitives, residual
with chemistry, local time step, diagonal blocks with the source Jacobian, the
LU-SGS forward and backward sweeps, the consistency correction and update, and
the residual norms.  The default workload is the largest single-GPU case: the
2048 x 1024 polar blunt-body grid with a seeded 20-species / 60-reaction
one-temperature mechanism at CFL 1000 from a uniform free stream (synthetic
input; there is no dataset).

Reported per variant (coupled / split, FP64 / mixed, exact / surrogate
species Jacobian block): cell-iterations per second over K timed steps after
W warm-up steps, with per-phase times.  The headline `value` is the split
mixed-precision solver with the surrogate block.  The surrogate network is
trained first on samples of the exact solver's own iterations (sampling and
training times reported separately).

Time to a 1e-8 drop of the density residual from the free stream, with the
same CFL ramp for every variant, is measured on a smaller case (512 x 256,
5-species two-temperature air, CFL 100; `--tol-config`), where every variant
reaches it within seconds, together with the surrogate's amortised total
(sampling + training + solve); `--converge` also runs it on the main workload.
Prints one JSON line.
"""
from __future__ import annotations

import argparse
import dataclasses
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

GEOM_WORDS = 5  # cell volume + four face lengths/normals summarised as one word each
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6   # vector FP64: 256 CUs x 2.4 GHz x 128 flops per clock per CU
VARIANTS = {  # name: (mode, correction kind, precision, species Jacobian 0 exact / 1 surrogate)
    "split64": (1, 2, 0, 0), "coupled64": (0, 0, 0, 0), "splitmixed": (1, 2, 1, 0), "coupledmixed": (0, 0, 1, 0),
    "splitmixed_mlp": (1, 2, 1, 1)}
HEADLINE = "splitmixed_mlp"
KERNEL_SOURCES = {"sweep_fwd": ["csi_group.hpp", "csi_kernels.hpp", "csi_sweep.hpp", "csi_phys.hpp"],
                  "sweep_bwd": ["csi_group.hpp", "csi_kernels.hpp", "csi_sweep.hpp", "csi_phys.hpp"],
                  "block": ["csi_block.hpp", "csi_kernels.hpp", "csi_phys.hpp"],
                  "cell": ["csi_kernels.hpp", "csi_phys.hpp"]}
KERNEL_NAMES = {"sweep_fwd": "k_group_sweep (forward)", "sweep_bwd": "k_group_sweep (backward)",
                "block": "k_block", "cell": "k_cell"}


MECH_TEXT = {"air5": "5-species air", "air11": "11-species ionised air",
             "syn20": "seeded 20-species / 60-reaction mechanism"}


def nsol(m, mode):
    return m.nb if mode == 0 else m.nf + m.ns


def b_alg_iter(m, mode, precision):
    """Algorithmic bytes per cell-iteration of the whole path: state read twice
    and written once, geometry read twice, the sweep intermediate written and
    read once."""
    w = 8 if precision == 0 else 4
    return (3 * m.nv + 2 * GEOM_WORDS) * 8 + 2 * nsol(m, mode) * w


def b_alg_sweep(m, mode, precision):
    """Algorithmic bytes per cell of one sweep launch: the cell's state and
    geometry (from which its diagonal block and face operators follow), the
    incoming right-hand side (b or dQ*) and the outgoing increment."""
    w = 8 if precision == 0 else 4
    return (m.nv + GEOM_WORDS) * 8 + 2 * nsol(m, mode) * w


def chem_flops(m):
    """FP64 flops per cell of the exact chemical source Jacobian: per reaction
    about 40 for the rates (transcendentals counted once) plus a multiply-add
    per entry it adds to the Jacobian (the rows of the species it changes,
    the columns of the species its rate depends on: every species through a
    third body)."""
    import numpy as np
    nu_f, nu_b = np.asarray(m.nu_f), np.asarray(m.nu_b)
    tot = 0
    for r in range(m.nr):
        rows = int(np.count_nonzero(nu_b[r] - nu_f[r]))
        cols = m.ns if m.third[r] else int(np.count_nonzero(nu_f[r] + nu_b[r]))
        tot += 40 + 2 * rows * cols
    return tot


def block_flops(m, mode):
    """Algorithmic FP64 flops per cell of the diagonal-block kernel: the
    chemical source Jacobian and the factorisation (2 n^3 / 3) of the block
    (n = nb coupled, ns split)."""
    n = m.nb if mode == 0 else m.ns
    return chem_flops(m) + 2.0 * n ** 3 / 3.0


def source_hash(kernel):
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kernel]:
        with open(os.path.join(ROOT, "paper_2403_03440_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` from the committed counter summary, if
    that summary was taken on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_hbm_counters.md")
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    hm = re.search(r"source hash:\s*`?([0-9a-f]{16})", txt)
    tm = re.search(r"HBM bytes per launch:\s*([0-9.eE+]+)", txt)
    if not hm or not tm or hm.group(1) != source_hash(kernel):
        return None
    return float(tm.group(1))


JC_READING = -1  # split species block reading (csi_set_species_jacobian); -1 keeps the default
RESIDUAL_SCHEME = 0  # csi_set_residual_scheme: 0 first-order HLLE, 1 MUSCL + Roe


def new_solver(csi, I, cfg, m, x, y, fs, sur=None):
    s = csi.Solver((x, y), m, fs)
    s.set_state(s.initial_state(*I.initial_prims(cfg, m)))
    if JC_READING >= 0:
        s.set_species_jacobian(JC_READING)
    if RESIDUAL_SCHEME:
        s.set_residual_scheme(RESIDUAL_SCHEME)
    if sur is not None:
        s.set_surrogate(sur["params"], sur["scales"])
    return s


def train_surrogate(csi, I, cfg, m, x, y, fs, epochs, snapshots):
    """Samples from the exact split mixed solver's first iterations (every 5th
    iteration, all cells), then training on the GPU; both timed."""
    import torch
    from paper_2403_03440_amd import surrogate as S
    s = new_solver(csi, I, cfg, m, x, y, fs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    xr, jc, its = S.collect(s, (1, 2, 1), cfg.cfl, snapshots * s.N, every=5)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    params, scales, hist = S.train(xr, jc, epochs=epochs, batch=4096, lr=1e-3, seed=cfg.seed + 1,
                                   log=lambda msg: print("# " + msg, file=sys.stderr, flush=True))
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    info = {"samples": int(xr.shape[0]), "collect_iterations": its, "collect_s": t1 - t0, "train_s": t2 - t1,
            "epochs": epochs, "train_loss": hist[-1][1], "val_loss": hist[-1][2], "first_val_loss": hist[0][2],
            "network": f"{m.ns + 3}-64-64-{m.ns * m.ns}, BF16 operands, FP32 accumulation"}
    del s, xr, jc
    return {"params": params, "scales": scales}, info


def throughput(csi, I, cfg, m, x, y, fs, variant, steps, warmup, sur=None):
    import torch
    mode, kind, prec, jac = VARIANTS[variant]
    s = new_solver(csi, I, cfg, m, x, y, fs, sur if jac else None)
    s.set_timing(True)
    if warmup:
        s.step(mode, kind, cfg.cfl, warmup, precision=prec, jac=jac, cfl_ramp=cfg.ramp, check_every=warmup)
    s.phase_times(reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = s.step(mode, kind, cfg.cfl, steps, precision=prec, jac=jac, cfl_ramp=cfg.ramp, check_every=steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ph = s.phase_times()
    n = max(st["iters"], 1)
    out = {"seconds": dt, "iters": st["iters"], "cell_iters_per_s": cfg.ni * cfg.nj * st["iters"] / dt,
           "ms_per_step": 1e3 * dt / n, "phases_ms_per_iter": {k: v["ms_per_iter"] for k, v in ph.items()
                                                                 if isinstance(v, dict)},
           "b_alg_per_cell_iter": b_alg_iter(m, mode, prec)}
    if jac:
        # the dominance check runs only while the surrogate is on: after a stall
        # or divergence switch-off (at global iteration surrogate_off_at; the
        # timed call starts at global iteration `warmup`) every cell takes the
        # exact block
        off = st["surrogate_off_at"]
        n_on = n if off < 0 else min(max(off - warmup, 0), n)
        out["surrogate_accept_frac"] = max(0.0, (n_on * cfg.ni * cfg.nj - st["n_dd_fallback"])
                                       / float(cfg.ni * cfg.nj * n))
        out["surrogate_off_at"] = off
        # a divergence fallback repeats the call's iterations with the exact
        # block: the time then covers both passes
        out["surrogate_diverged"] = st["surrogate_diverged"]
    return out


def converge(csi, I, cfg, m, x, y, fs, variant, tol, max_iter, sur=None):
    import torch
    mode, kind, prec, jac = VARIANTS[variant]
    s = new_solver(csi, I, cfg, m, x, y, fs, sur if jac else None)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = 0
    st = None
    fallback, off_at = 0, None
    while done < max_iter:
        try:
            st = s.step(mode, kind, cfg.cfl, min(1000, max_iter - done), precision=prec, jac=jac,
                        cfl_ramp=cfg.ramp, tol=tol, check_every=50)
        except csi.CsiError as e:
            return {"tol": tol, "converged": False, "iters": done, "seconds": time.perf_counter() - t0,
                    "error": str(e)}
        fallback += st["n_dd_fallback"]
        if st["surrogate_off_at"] >= 0 and off_at is None:
            off_at = st["surrogate_off_at"]
        done += st["iters"]
        print(f"# {variant}: {done} iterations, drop {st['r_last'] / st['r0']:.3e}, "
              f"{time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
        if st["converged"]:
            break
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    qw, qs = s.wall_heat_flux()
    out = {"tol": tol, "converged": bool(st["converged"]), "iters": done, "seconds": dt,
           "drop": st["r_last"] / st["r0"], "q_stag_W_m2": qs, "_state": s.get_state(), "_qw": qw}
    if jac:
        out["surrogate_accept_frac"] = 1.0 - fallback / float(cfg.ni * cfg.nj * max(done, 1))
        out["surrogate_off_at"] = off_at
    return out


def compare_to_fp64(m, res, ref="split64"):
    """Each converged variant's state and wall heat flux against the split
    FP64 run's: per stored variable max|a - b| / max|b| (densities, momenta
    and energies each scaled by their group's largest magnitude), and the wall
    heat flux's largest difference over its largest magnitude."""
    import numpy as np
    r = res.get(ref, {}).get("to_tol", {})
    if "_state" not in r:
        for v in res.values():
            v.get("to_tol", {}).pop("_state", None)
            v.get("to_tol", {}).pop("_qw", None)
        return
    qb, wb = r["_state"], r["_qw"]
    ns = m.ns
    groups = [list(range(ns)), [ns, ns + 1], list(range(ns + 2, qb.shape[0]))]
    scale = np.abs(qb).max(axis=1)
    for g in groups:
        scale[g] = scale[g].max()
    for v in res.values():
        t = v.get("to_tol", {})
        if "_state" in t and t is not r:
            d = np.abs(t["_state"] - qb).max(axis=1) / np.where(scale > 0, scale, 1.0)
            t["vs_split64"] = {"per_variable": [float(e) for e in d],
                               "wall_heat_flux": float(np.abs(t["_qw"] - wb).max() / np.abs(wb).max())}
    for v in res.values():
        v.get("to_tol", {}).pop("_state", None)
        v.get("to_tol", {}).pop("_qw", None)


# the paper's own time per implicit iteration (s) of its species-count study
# (CPU, 10 x 10 x 10 box; a table kept in the paper's source), as context
PAPER_E1 = {16: (6.694e-3, 4.5100e-3), 64: (3.9227e-2, 1.4959e-2), 256: (4.4936e-1, 5.4932e-2),
            1024: (2.8190e1, 2.1695e-1), 4096: (6.5762e2, 8.9015e-1)}


def scaling(csi, I, ns_list, steps, warmup, n_side=16):
    """Species-count study (paper Section 3.1): uniform non-reacting flow in
    a far-field box (n_side x n_side cells, free stream on every side, +-1 %
    seeded density perturbation), seeded synthetic species without
    reactions, one temperature, FP64, on the species-generic kernels at
    every count.  Per species count: ms per implicit iteration of the coupled
    (CI) and split (CS, CC2) forms, that is the diagonal-block assembly and
    inversion and both sweeps (the cell kernel also forms the residual and
    the corrections follow; both are listed), and the CS speed-up 1 - CS/CI
    beside the paper's CPU figures."""
    import numpy as np
    import torch
    x, y = I.box_grid(n_side, n_side, lx=0.01, ly=0.01)
    n = n_side * n_side
    rows = []
    for ns in ns_list:
        m = I.synthetic(ns, 0, 3442)
        Y = np.full(ns, 1.0 / ns)
        fs = (1e-3 * Y, 1000.0, 0.0, 300.0, 300.0)
        rs = fs[0][:, None] * (1.0 + 0.01 * I.uniform_pm1(3442, n))[None, :]
        prims = (np.ascontiguousarray(rs), np.full(n, fs[1]), np.zeros(n), np.full(n, fs[3]), np.full(n, fs[4]))
        row = {"ns": ns}
        for v, (mode, kind) in (("CI", (0, 0)), ("CS", (1, 2))):
            s = csi.Solver((x, y), m, fs, bc_mode=1, generic=True)
            s.set_state(s.initial_state(*prims))
            s.set_timing(True)
            s.step(mode, kind, 10.0, warmup, check_every=warmup)
            s.phase_times(reset=True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            s.step(mode, kind, 10.0, steps, check_every=steps)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            ph = {k: p["ms_per_iter"] for k, p in s.phase_times().items() if isinstance(p, dict)}
            imp = ph["cell"] + ph["block"] + ph["sweep_fwd"] + ph["sweep_bwd"]
            row[v] = {"implicit_ms": imp, "ms_per_iter": 1e3 * dt / steps, "phases": ph}
            print(f"# ns {ns} {v}: implicit {imp:.3f} ms, {1e3 * dt / steps:.3f} ms/it", file=sys.stderr, flush=True)
            del s
            torch.cuda.empty_cache()
        row["cs_speedup_pct"] = 100.0 * (1.0 - row["CS"]["implicit_ms"] / row["CI"]["implicit_ms"])
        if ns in PAPER_E1:
            ci, cs = PAPER_E1[ns]
            row["paper_cpu_s"] = {"CI": ci, "CS": cs, "cs_speedup_pct": 100.0 * (1.0 - cs / ci)}
        rows.append(row)
    fit = {}
    for v in ("CI", "CS"):
        r = [(q["ns"], q[v]["implicit_ms"]) for q in rows]
        if len(r) >= 2:
            fit[v] = float(np.polyfit(np.log([a for a, _ in r]), np.log([b for _, b in r]), 1)[0])
    return {"metric": "implicit iteration time vs species count (non-reacting flow), CI vs CS", "unit": "ms",
            "config": {"workload": f"{n_side}x{n_side} far-field box, uniform non-reacting flow (+-1 % density), "
                                   f"seeded synthetic species without reactions, 1T, FP64, CFL 10, species-generic "
                                   f"kernels, {steps} timed iterations after {warmup}"},
            "rows": rows, "fitted_exponent_implicit": fit}


def residual_ablation(csi, I, config, speeds, max_iter, tol, chunk=2000):
    """The residual scheme as an ablation (the MUSCL (minmod) + Roe residual
    of the paper's cylinder case, Section 3.2, against the default
    first-order HLLE): on the config's grid, mechanism and CFL schedule with
    the free-stream speed replaced, each form (split mixed CC2, coupled FP64)
    from the free stream until the density residual has dropped by tol or
    max_iter iterations have run, checked every chunk iterations.  Per run:
    iterations, seconds (with HIP events per phase on), the drop after each
    chunk, the error that stopped it, if any (a non-physical state), and
    the mean time per iteration of each phase."""
    import torch
    base = I.CONFIGS[config]
    runs = []
    for u in speeds:
        cfg = dataclasses.replace(base, u_inf=u)
        m = cfg.mechanism()
        x, y = cfg.grid()
        fs = I.freestream_prims(cfg, m)
        for scheme, sname in ((1, "muscl_roe"), (0, "hlle")):
            for form, mode, kind, prec in (("split mixed", 1, 2, csi.MIXED), ("coupled FP64", 0, 0, csi.FP64)):
                s = csi.Solver((x, y), m, fs)
                s.set_residual_scheme(scheme)
                s.set_state(s.initial_state(*I.initial_prims(cfg, m)))
                s.set_timing(True)
                run = {"u_inf": u, "residual": sname, "form": form, "drops": [], "error": None}
                done, r0 = 0, None
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                try:
                    while done < max_iter:
                        st = s.step(mode, kind, cfg.cfl, min(chunk, max_iter - done), precision=prec,
                                    cfl_ramp=cfg.ramp if done == 0 else 0, check_every=100)
                        r0 = st["r0"] if r0 is None else r0
                        done += st["iters"]
                        run["drops"].append([done, st["r_last"] / r0])
                        if st["r_last"] / r0 <= tol:
                            break
                except csi.CsiError as e:
                    run["error"] = str(e)
                torch.cuda.synchronize()
                ph = s.phase_times()
                # iterations run, the one that failed included (the timing counts every iteration)
                run["iters"] = max(done, int(ph["iters"]))
                run["seconds"] = time.perf_counter() - t0
                run["phases_ms_per_iter"] = {k: p["ms_per_iter"] for k, p in ph.items() if isinstance(p, dict)}
                print(f"# {sname} u {u:.0f} {form}: {run['iters']} it, drop {run['drops'][-1][1] if run['drops'] else None}, "
                      f"{run['seconds']:.1f} s{', ' + run['error'] if run['error'] else ''}", file=sys.stderr,
                      flush=True)
                runs.append(run)
                del s
                torch.cuda.empty_cache()
    return {"metric": "residual-scheme ablation: density-residual drop against iterations", "unit": "drop",
            "config": {"workload": f"{config} grid, mechanism and CFL schedule with the free-stream speed replaced; "
                                   f"to a {tol:g} drop or {max_iter} iterations"},
            "runs": runs}


def oracle_threads():
    n = len(os.sched_getaffinity(0))
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit():
        n = min(n, int(env))
    return max(n, 1)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            names = [ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")]
        return names[0] if names else "unknown"
    except OSError:
        return "unknown"


def cpu_topology():
    """Sockets, physical cores and logical CPUs of the host (/proc/cpuinfo),
    and the logical CPUs this process may run on."""
    out = {"sockets": None, "physical_cores": None, "logical_cpus": None,
           "logical_cpus_visible": len(os.sched_getaffinity(0))}
    try:
        with open("/proc/cpuinfo") as f:
            txt = f.read()
    except OSError:
        return out
    procs = [blk for blk in txt.split("\n\n") if blk.strip()]
    sockets, cores = set(), set()
    for blk in procs:
        kv = dict((ln.split(":", 1)[0].strip(), ln.split(":", 1)[1].strip()) for ln in blk.splitlines() if ":" in ln)
        sockets.add(kv.get("physical id"))
        cores.add((kv.get("physical id"), kv.get("core id")))
    out["logical_cpus"] = len(procs)
    if None not in sockets:
        out["sockets"] = len(sockets)
    if all(c[1] is not None for c in cores):
        out["physical_cores"] = len(cores)
    return out


def cpu_baseline(I, cfg, m, budget_s=20.0, sample_grid=(128, 64)):
    """The oracle on the host cores over a bounded sample of the workload: the
    same mechanism, free stream and CFL schedule on a coarser grid of the same
    geometry (its cost per cell-iteration does not depend on the grid size),
    whole split-CC2 FP64 iterations from the free stream until about budget_s
    seconds have passed."""
    from oracle import orc
    threads = oracle_threads()
    ni, nj = sample_grid if cfg.ni * cfg.nj > sample_grid[0] * sample_grid[1] else (cfg.ni, cfg.nj)
    scfg = I.Config(cfg.name, ni, nj, cfg.mech, cfg.two_temp, cfg.cfl, cfg.u_inf, ramp=cfg.ramp)
    x, y = scfg.grid()
    fs = I.freestream_prims(scfg, m)

    def run(nthreads, budget, cap):
        o = orc.setup((x, y), m, fs, threads=nthreads)
        o.set_state(o.prim_to_cons(*I.initial_prims(scfg, m)))
        t0 = time.perf_counter()
        n = 0
        while True:
            o.step(1, 2, scfg.cfl, 1, ramp=scfg.ramp, it0=n)
            n += 1
            if time.perf_counter() - t0 > budget or n >= cap:
                break
        return n, time.perf_counter() - t0

    n, dt = run(threads, budget_s, 200)
    out = {"value": ni * nj * n / dt, "unit": "cell-iters/s", "cores": threads, "kind": "oracle",
           "sample": f"first {n} split-CC2 FP64 iterations from the free stream of the same mechanism, flow and "
                     f"CFL schedule on a {ni}x{nj} grid of the same geometry ({dt:.1f} s, {threads} OpenMP "
                     f"threads)",
           "cpu": cpu_model(), **cpu_topology()}
    n1, dt1 = run(1, budget_s / 2, 50)
    out["value_1_thread"] = ni * nj * n1 / dt1
    out["sample_1_thread"] = f"first {n1} of the same iterations on 1 thread ({dt1:.1f} s)"
    return out


def oracle_time_to_tol(csi, I, names, tol, max_iter, window=20, measure_cells=20000):
    """The oracle's time to a tol drop of the density residual (split CC2,
    FP64, from the free stream, on the host cores) beside the GPU's split FP64
    and split mixed runs of the same config.  Configs of at most
    measure_cells cells are run to tol and timed whole ("measured"); larger
    ones are timed over a window of iterations after the CFL ramp and the
    time is the GPU FP64 iteration count times the oracle's seconds per
    iteration over the first `window` iterations ("projected": a full oracle
    run would take hours)."""
    import numpy as np
    import torch
    from oracle import orc
    threads = oracle_threads()
    rows = []
    for name in names:
        cfg = I.CONFIGS[name]
        m = cfg.mechanism()
        x, y = cfg.grid()
        fs = I.freestream_prims(cfg, m)
        N = cfg.ni * cfg.nj
        row = {"config": name, "cells": N, "tol": tol, "oracle_threads": threads}
        gpu_iters = None
        for v, prec in (("gpu_split64", csi.FP64), ("gpu_splitmixed", csi.MIXED)):
            s = new_solver(csi, I, cfg, m, x, y, fs)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st = s.step(1, 2, cfg.cfl, max_iter, precision=prec, cfl_ramp=cfg.ramp, tol=tol, check_every=50)
            torch.cuda.synchronize()
            row[v] = {"iters": st["iters"], "converged": bool(st["converged"]), "seconds": time.perf_counter() - t0}
            if prec == csi.FP64:
                gpu_iters = st["iters"]
            del s
            torch.cuda.empty_cache()
        o = orc.setup((x, y), m, fs, threads=threads)
        o.set_state(o.prim_to_cons(*I.initial_prims(cfg, m)))
        if N <= measure_cells:
            t0 = time.perf_counter()
            done, r0, drop = 0, None, 1.0
            while done < max_iter and drop > tol:
                h = o.step(1, 2, cfg.cfl, 10, ramp=cfg.ramp, it0=done)
                r0 = h[0, 0] if r0 is None else r0
                k = np.nonzero(h[:, 0] / r0 <= tol)[0]
                done += int(k[0]) + 1 if k.size else 10
                drop = h[-1, 0] / r0 if not k.size else h[k[0], 0] / r0
            row["oracle"] = {"kind": "measured", "iters": done, "seconds": time.perf_counter() - t0,
                             "converged": bool(drop <= tol)}
        else:
            # the first `window` iterations from the free stream
            t0 = time.perf_counter()
            o.step(1, 2, cfg.cfl, window, ramp=cfg.ramp)
            spi = (time.perf_counter() - t0) / window
            row["oracle"] = {"kind": "projected", "seconds_per_iter": spi, "window": window,
                             "iters": gpu_iters, "seconds": spi * gpu_iters}
        row["oracle_over_gpu_splitmixed"] = row["oracle"]["seconds"] / row["gpu_splitmixed"]["seconds"]
        print(f"# {name}: oracle {row['oracle']['kind']} {row['oracle']['seconds']:.1f} s, GPU split mixed "
              f"{row['gpu_splitmixed']['seconds']:.2f} s", file=sys.stderr, flush=True)
        rows.append(row)
    return {"metric": "time to a density-residual drop, the oracle (host cores) beside the GPU", "unit": "s",
            "cpu": cpu_model(), **cpu_topology(), "rows": rows}


def copy_probe(gib=1.0, reps=3):
    """A plain device copy of known size, for scaling HBM byte counters."""
    import torch
    n = int(gib * (1 << 30)) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(f"# copy probe: {reps} copies of {4 * n} bytes", file=sys.stderr, flush=True)


def roofline(m, mode, prec, ph, N, workload, accept=0.0):
    """Roofline entry of the headline variant's dominant kernel (the largest
    per-launch time among the block kernel and the two sweeps, one launch
    each per iteration, HIP events on the library's stream).  `accept` is the
    fraction of cell-iterations whose species block came from the surrogate:
    those skip the exact Jacobian, so its flops count only for the rest."""
    cands = {k: ph.get(k, 0.0) for k in ("block", "sweep_fwd", "sweep_bwd") if ph.get(k, 0.0) > 0.0}
    kernel = max(cands, key=cands.get)
    ms = cands[kernel]
    traffic = measured_traffic(kernel, workload)
    if kernel == "block":
        fl = block_flops(m, mode) - accept * chem_flops(m)
        ach = fl * N / (ms * 1e-3) / 1e12
        return {"bound": "alu", "achieved": ach, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": ach / FP64_PEAK_TFLOPS, "traffic": traffic, "kernel": KERNEL_NAMES[kernel],
                "ms_per_launch": ms, "alg_flops_per_cell": fl, "cells_per_launch": N,
                "alg_flops_per_launch": fl * N,
                "surrogate_accept_frac": accept,
                "flops_model": "exact chemical source Jacobian (rates + one multiply-add per Jacobian entry each "
                               "reaction adds) for the cells without an accepted surrogate block + 2 n^3 / 3 "
                               "factorisation of the n x n block, FP64"}
    bytes_launch = b_alg_sweep(m, mode, prec) * N
    ach = bytes_launch / (ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
            "traffic": traffic, "kernel": KERNEL_NAMES[kernel], "ms_per_launch": ms,
            "alg_bytes_per_cell": b_alg_sweep(m, mode, prec), "cells_per_launch": N,
            "alg_bytes_per_launch": bytes_launch}


def workload_text(cfg, m):
    return (f"{cfg.name}: {cfg.ni}x{cfg.nj} polar blunt body, {MECH_TEXT[cfg.mech]} "
            f"{'2T' if m.two_temp else '1T'}, u {cfg.u_inf:g} m/s, CFL {cfg.cfl:g} (ramp over {cfg.ramp} "
            f"iterations), uniform free-stream start")


def tol_leg(csi, I, name, names, tol, max_iter, epochs, snapshots, ramp=0):
    """Every variant from the free stream to the tolerance on one workload,
    the converged states against the split FP64 run's, and the surrogate's
    amortised cost (sampling + training + solve) against the exact block."""
    cfg = I.CONFIGS[name]
    if ramp:
        cfg = dataclasses.replace(cfg, ramp=ramp)
    m = cfg.mechanism()
    x, y = cfg.grid()
    fs = I.freestream_prims(cfg, m)
    sur, info = None, None
    if any(VARIANTS[v][3] for v in names):
        print(f"# {name}: surrogate sampling and training", file=sys.stderr, flush=True)
        sur, info = train_surrogate(csi, I, cfg, m, x, y, fs, epochs, snapshots)
    res = {v: {"to_tol": converge(csi, I, cfg, m, x, y, fs, v, tol, max_iter, sur)} for v in names}
    compare_to_fp64(m, res)
    out = {"workload": workload_text(cfg, m), "cells": cfg.ni * cfg.nj,
           "variants": {v: r["to_tol"] for v, r in res.items()}, "surrogate_training": info}
    t = out["variants"]
    if sur is not None and t.get(HEADLINE, {}).get("converged") and t.get("splitmixed", {}).get("converged"):
        tot = info["collect_s"] + info["train_s"] + t[HEADLINE]["seconds"]
        out["surrogate_amortised"] = {
            "collect_s": info["collect_s"], "train_s": info["train_s"], "solve_s": t[HEADLINE]["seconds"],
            "total_s": tot, "split_mixed_exact_block_s": t["splitmixed"]["seconds"],
            "gain_s": t["splitmixed"]["seconds"] - tot,
            "iterations_vs_exact_block": t[HEADLINE]["iters"] - t["splitmixed"]["iters"]}
    if t.get("coupled64", {}).get("converged") and t.get(HEADLINE, {}).get("converged"):
        out["speedup_time_to_tol_vs_coupled64"] = t["coupled64"]["seconds"] / t[HEADLINE]["seconds"]
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--config", default="c5")
    ap.add_argument("--variants", default="splitmixed_mlp,splitmixed,split64,coupled64,coupledmixed")
    ap.add_argument("--epochs", type=int, default=0, help="surrogate training epochs (0: 20)")
    ap.add_argument("--snapshots", type=int, default=0,
                    help="surrogate training snapshots, all cells each (0: 4 on c5, else 16)")
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--max-iter", type=int, default=12000)
    ap.add_argument("--converge", action="store_true", help="also run every variant to the tolerance on --config")
    ap.add_argument("--tol-config", default="c2", help="workload of the time-to-tolerance legs ('' to skip)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--species-jacobian", type=int, default=-1,
                    help="split species block: 0 fixed T, Tv; 1 fixed velocities and internal energy; "
                         "2 as 1 with Tv held; -1 (default) keeps the default of the temperature model "
                         "(1 in one temperature, 0 in two)")
    ap.add_argument("--ramp", type=int, default=0, help="CFL ramp length in iterations (0: the workload's own)")
    ap.add_argument("--copy-probe", action="store_true", help="also run a 1 GiB device copy (counter scaling)")
    ap.add_argument("--scaling", default="", help="species counts (e.g. 16,64,256,1024,4096): the species-count "
                                                 "study (implicit iteration time of CI and CS in non-reacting flow) "
                                                 "instead of the workload above")
    ap.add_argument("--scaling-grid", type=int, default=16, help="cells per side of the species-count study's box")
    ap.add_argument("--oracle-tol", default="", help="configs (e.g. c1,c2,c4): the oracle's time to --tol "
                    "beside the GPU's (measured up to 20 000 cells, projected from a timed window above)")
    ap.add_argument("--residual", choices=("hlle", "muscl"), default="hlle",
                    help="residual scheme of the throughput and time-to-tolerance legs")
    ap.add_argument("--residual-ablation", default="", help="free-stream speeds (e.g. 2000,5000): MUSCL + Roe "
                    "against HLLE, both forms, on --ablation-config to --tol or --max-iter")
    ap.add_argument("--ablation-config", default="c2", help="workload of --residual-ablation")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this implementation runs on one GPU; --gpus must be 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2403_03440_amd import csi
    from paper_2403_03440_amd import inputs as I

    if args.scaling:
        print(json.dumps(scaling(csi, I, [int(v) for v in args.scaling.split(",")], args.steps, args.warmup,
                                 args.scaling_grid)))
        return
    if args.oracle_tol:
        print(json.dumps(oracle_time_to_tol(csi, I, [v for v in args.oracle_tol.split(",") if v], args.tol,
                                            args.max_iter)))
        return
    if args.residual_ablation:
        print(json.dumps(residual_ablation(csi, I, args.ablation_config,
                                           [float(v) for v in args.residual_ablation.split(",")],
                                           args.max_iter, args.tol)))
        return
    cfg = I.CONFIGS[args.config]
    if args.ramp:
        cfg = dataclasses.replace(cfg, ramp=args.ramp)
    big = cfg.ni * cfg.nj > 1_000_000
    epochs = args.epochs or 20
    snapshots = args.snapshots or (4 if big else 16)
    m = cfg.mechanism()
    x, y = cfg.grid()
    fs = I.freestream_prims(cfg, m)
    N = cfg.ni * cfg.nj
    names = [v for v in args.variants.split(",") if v]
    if HEADLINE not in names:
        names.insert(0, HEADLINE)
    global JC_READING, RESIDUAL_SCHEME
    JC_READING = args.species_jacobian
    RESIDUAL_SCHEME = {"hlle": 0, "muscl": 1}[args.residual]
    sur, sur_info = None, None
    if any(VARIANTS[v][3] for v in names):
        print("# surrogate: sampling and training", file=sys.stderr, flush=True)
        sur, sur_info = train_surrogate(csi, I, cfg, m, x, y, fs, epochs, snapshots)
    res = {}
    for v in names:
        print(f"# throughput {v}", file=sys.stderr, flush=True)
        res[v] = throughput(csi, I, cfg, m, x, y, fs, v, args.steps, args.warmup, sur)
    if args.converge:
        for v in names:
            res[v]["to_tol"] = converge(csi, I, cfg, m, x, y, fs, v, args.tol, args.max_iter, sur)
        compare_to_fp64(m, res)
    if args.copy_probe:
        copy_probe()
    head = res[HEADLINE]
    mode, _, prec, _ = VARIANTS[HEADLINE]
    roof = roofline(m, mode, prec, head["phases_ms_per_iter"], N, cfg.name, head.get("surrogate_accept_frac", 0.0))
    whole = {"alg_GBs": b_alg_iter(m, mode, prec) * head["cell_iters_per_s"] / 1e9}
    whole["frac"] = whole["alg_GBs"] / HBM_PEAK_GBS
    dtype = "f32+f64" if prec == 1 else "f64"
    out = {
        "metric": "cell-iters/s & time-to-1e-8 residual: split vs coupled, FP64 vs mixed+MLP",
        "value": head["cell_iters_per_s"],
        "unit": "cell-iters/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": dtype, "data": "synthetic",
        "config": {"workload": workload_text(cfg, m) + ", headline: split solver, FP32 sweeps and block "
                               "inverses + FP64 residual/chemistry/CC2, species Jacobian block from the BF16 "
                               "surrogate network with exact fallback"
                               + (", MUSCL (minmod) + Roe residual" if RESIDUAL_SCHEME else ""),
                   "cells": N},
        "roofline": roof,
        "whole_iteration_hbm": whole,
        "variants": res,
        "surrogate_training": sur_info,
    }
    if "coupled64" in res:
        out["speedup_vs_coupled64"] = {v: r["cell_iters_per_s"] / res["coupled64"]["cell_iters_per_s"]
                                       for v, r in res.items()}
    if args.tol_config:
        out["time_to_tol"] = tol_leg(csi, I, args.tol_config, names, args.tol, args.max_iter, 20, 16, args.ramp)
    if not args.no_cpu_baseline:
        print("# cpu baseline", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(I, cfg, m)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
