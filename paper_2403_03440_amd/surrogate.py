"""Training pipeline of the species-Jacobian surrogate on the GPU.

Samples (features and exact J_C) are drawn from the method's own iterations:
the exact-Jacobian split solver runs from the given start and every `every`
iterations the library writes the samples of all cells.  The library then
standardises the features and transforms the targets, and trains the network
with its own forward/backward kernels and Adam, over seeded permutations of
the training rows; a held-out tenth of the rows gives the validation loss.
Python only sequences the library calls and owns the tensors.
"""
from __future__ import annotations

import time

import numpy as np

from . import csi
from . import inputs as I


def glorot_params(n_in, n_out, seed):
    """Glorot-uniform initial weights (zero biases) in the packed layout."""
    H = 64
    u = I.uniform_pm1(seed, H * n_in + H + H * H + H + n_out * H + n_out)
    o = 0
    out = []
    for rows, cols, fan_in, fan_out in ((H, n_in, n_in, H), (H, 1, 0, 0), (H, H, H, H), (H, 1, 0, 0),
                                        (n_out, H, H, n_out), (n_out, 1, 0, 0)):
        k = rows * cols
        seg = u[o:o + k] * (np.sqrt(6.0 / (fan_in + fan_out)) if fan_in else 0.0)
        out.append(seg)
        o += k
    return np.concatenate(out).astype(np.float32)


def collect(solver, mode_kind_prec, cfl, n_samples, every=5, cfl_ramp=100, device="cuda"):
    """Run the exact solver, sampling all cells every `every` iterations until
    n_samples rows are stored.  Returns (x_raw, jc) cuda tensors and the
    number of iterations run."""
    import torch
    mode, kind, prec = mode_kind_prec
    m = solver.mech
    N = solver.N
    n_snap = max(1, -(-n_samples // N))
    xr = torch.empty((n_snap * N, m.ns + 3), dtype=torch.float32, device=device)
    jc = torch.empty((n_snap * N, m.ns * m.ns), dtype=torch.float32, device=device)
    its = 0
    for k in range(n_snap):
        st = solver.step(mode, kind, cfl, every, precision=prec, cfl_ramp=cfl_ramp, check_every=every)
        its += st["iters"]
        solver.sample_jacobians(xr[k * N:(k + 1) * N], jc[k * N:(k + 1) * N])
    n = min(n_samples, n_snap * N)
    return xr[:n], jc[:n], its


def train(x_raw, jc, epochs=20, batch=4096, lr=1e-3, seed=3441, holdout=0.1, log=None):
    """Prepare and train; returns params (cuda float32), scales (host), and a
    history of (epoch, train loss, validation loss, seconds)."""
    import torch
    n, n_in = x_raw.shape
    n_out = jc.shape[1]
    net = csi.Mlp(n_in, n_out, batch=batch)
    x, t, scales = net.prepare(x_raw, jc)
    perm = I.permutation(seed, n)
    n_val = max(1, int(holdout * n)) if n > 10 else 0
    val_idx = torch.tensor(perm[:n_val], device=x.device)
    tr = perm[n_val:]
    params = torch.tensor(glorot_params(n_in, n_out, seed + 1), device=x.device)
    m = torch.zeros_like(params)
    v = torch.zeros_like(params)
    hist = []
    step = 0
    t0 = time.perf_counter()
    tr_dev = torch.tensor(tr.astype(np.int64), device=x.device)
    for ep in range(epochs):
        # the seeded permutation of inputs.permutation, sorted on the device
        keys = I.splitmix64(np.uint64(seed + 2 + ep) ^ np.arange(tr.size, dtype=np.uint64))
        keys = torch.from_numpy((keys ^ np.uint64(1 << 63)).view(np.int64)).to(x.device)
        dev_order = tr_dev[torch.argsort(keys, stable=True)].to(torch.int32)
        # the whole epoch in one library call (kernels back to back on the stream)
        tl = net.train_epoch(params, m, v, x, t, dev_order, step, lr=lr)
        nb = -(-tr.size // batch)
        step += nb
        vl = float("nan")
        if n_val:
            vl = 0.0
            for b0 in range(0, n_val, batch):
                idx = val_idx[b0:b0 + batch]
                _, l_ = net.grad(params, x, t, idx)
                vl += l_ * idx.numel()
            vl /= n_val
        torch.cuda.synchronize()
        hist.append((ep, tl, vl, time.perf_counter() - t0))
        if log:
            log(f"epoch {ep}: train {tl:.4e} val {vl:.4e} ({time.perf_counter() - t0:.1f} s, {nb} steps)")
    return params, scales, hist
