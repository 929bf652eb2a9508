"""MLP surrogate of the species source-Jacobian block: plain numpy reference
(TEST INFRASTRUCTURE ONLY: only tests/, __graft_entry__.smoke() and bench.py's
cpu_baseline leg may use anything under oracle/).

The paper's split form (Section 2.3, species block of the implicit operator)
carries J_C = d omega_s / d rho_r at fixed T and Tv in the species diagonal
block.  The surrogate replaces that block by a small network; the paper does
not define one, so the definition below is the reading this implementation
takes (stated with every rounding point so that a GPU implementation with
BF16 operands and FP32 accumulation can be compared against it):

  features   x_raw = (ln T, ln Tv, ln rho, Y_1 .. Y_ns)        (n_in = ns + 3)
  scaling    x = (x_raw - mu) / sigma, sigma := 1 where the sample std < 1e-12
  network    h1 = tanh(W1 x + b1), h2 = tanh(W2 h1 + b2), y = W3 h2 + b3, width 64
  target     t = asinh(tau0 J_C) element-wise, J_C row-major (s, r); tau0 = 1 / the
             geometric mean of the non-zero |J_C| entries of the training set
  output     J_C = sinh(y) / tau0
  loss       mean over samples and outputs of (y - t)^2
  optimiser  Adam (bias-corrected), FP32 master weights

Parameters are one flat vector [W1 (64 x n_in, row-major), b1, W2 (64 x 64),
b2, W3 (n_out x 64), b3].

emulate=True reproduces the BF16 path: x, h1, h2, the three weight matrices
and the back-propagated errors are rounded to bfloat16 (round to nearest even)
before every matrix product; products and sums are exact here and rounded to
FP32 after each sum; biases, tanh, the loss scale and the tanh derivative are
FP32 values.  emulate=False is plain FP64 (for gradient checks).
"""
from __future__ import annotations

import numpy as np

H = 64


def bf16(a):
    """Round to the nearest bfloat16 (ties to even); returns float32 values."""
    f = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) & 0xFFFF0000).astype(np.uint32)
    return r.view(np.float32).reshape(f.shape)


def f32(a):
    return np.asarray(a, dtype=np.float64).astype(np.float32).astype(np.float64)


def n_params(n_in, n_out):
    return H * n_in + H + H * H + H + n_out * H + n_out


def unpack(p, n_in, n_out):
    p = np.asarray(p, dtype=np.float64)
    o = 0
    out = []
    for shape in ((H, n_in), (H,), (H, H), (H,), (n_out, H), (n_out,)):
        k = int(np.prod(shape))
        out.append(p[o:o + k].reshape(shape))
        o += k
    assert o == p.size
    return out


def pack(W1, b1, W2, b2, W3, b3):
    return np.concatenate([np.ravel(a) for a in (W1, b1, W2, b2, W3, b3)])


# ------------------------------------------------------------- data side
def features(T, Tv, rho, Y):
    """x_raw per sample: (ln T, ln Tv, ln rho, Y_1..Y_ns); Y has shape (n, ns)."""
    T, Tv, rho = (np.asarray(a, dtype=np.float64) for a in (T, Tv, rho))
    return np.column_stack([np.log(T), np.log(Tv), np.log(rho), np.asarray(Y, dtype=np.float64)])


def scales(x_raw, J):
    """mu, sigma per feature (population std) and tau0 from a training set."""
    x_raw = np.asarray(x_raw, dtype=np.float64)
    mu = x_raw.mean(axis=0)
    sigma = np.sqrt(((x_raw - mu) ** 2).mean(axis=0))
    sigma = np.where(sigma < 1e-12, 1.0, sigma)
    a = np.abs(np.asarray(J, dtype=np.float64)).ravel()
    a = a[a > 0]
    tau0 = 1.0 / np.exp(np.log(a).mean()) if a.size else 1.0
    return mu, sigma, tau0


def standardise(x_raw, mu, sigma):
    return (np.asarray(x_raw, dtype=np.float64) - mu) / sigma


def target(J, tau0):
    return np.arcsinh(np.asarray(J, dtype=np.float64) * tau0)


def jacobian(y, tau0):
    return np.sinh(np.asarray(y, dtype=np.float64)) / tau0


# ------------------------------------------------------------- network
def forward(p, x, n_out, emulate=False):
    """Network output y (n, n_out) and the activations needed by backward."""
    x = np.asarray(x, dtype=np.float64)
    n_in = x.shape[1]
    W1, b1, W2, b2, W3, b3 = unpack(p, n_in, n_out)
    if emulate:
        W1, W2, W3 = (bf16(w).astype(np.float64) for w in (W1, W2, W3))
        b1, b2, b3 = (f32(b) for b in (b1, b2, b3))
        xb = bf16(x).astype(np.float64)
        h1 = f32(np.tanh(f32(f32(xb @ W1.T) + b1)))
        h1b = bf16(h1).astype(np.float64)
        h2 = f32(np.tanh(f32(f32(h1b @ W2.T) + b2)))
        h2b = bf16(h2).astype(np.float64)
        y = f32(f32(h2b @ W3.T) + b3)
        return y, (xb, h1, h1b, h2, h2b)
    h1 = np.tanh(x @ W1.T + b1)
    h2 = np.tanh(h1 @ W2.T + b2)
    y = h2 @ W3.T + b3
    return y, (x, h1, h1, h2, h2)


def loss_and_grad(p, x, t, emulate=False, n_mean=None):
    """Mean squared error over samples and outputs, and its gradient in the
    packed parameter layout.  n_mean: number of samples the mean divides by
    (default: the rows given)."""
    t = np.asarray(t, dtype=np.float64)
    n, n_out = t.shape
    if n_mean is not None:
        n = n_mean
    n_in = np.asarray(x).shape[1]
    W1, b1, W2, b2, W3, b3 = unpack(p, n_in, n_out)
    y, (xb, h1, h1b, h2, h2b) = forward(p, x, n_out, emulate)
    d = y - t
    loss = float((d * d).sum() / (n * n_out))
    if emulate:
        W2b, W3b = bf16(W2).astype(np.float64), bf16(W3).astype(np.float64)
        g3 = f32(d * f32(2.0 / (n * n_out)))
        g3b = bf16(g3).astype(np.float64)
        g2 = f32(f32(g3b @ W3b) * f32(1.0 - h2 * h2))
        g2b = bf16(g2).astype(np.float64)
        g1 = f32(f32(g2b @ W2b) * f32(1.0 - h1 * h1))
        g1b = bf16(g1).astype(np.float64)
        grads = (f32(g1b.T @ xb), f32(g1.sum(0)), f32(g2b.T @ h1b), f32(g2.sum(0)), f32(g3b.T @ h2b),
                 f32(g3.sum(0)))
        return loss, pack(*grads)
    g3 = d * (2.0 / (n * n_out))
    g2 = (g3 @ W3) * (1.0 - h2 * h2)
    g1 = (g2 @ W2) * (1.0 - h1 * h1)
    return loss, pack(g1.T @ xb, g1.sum(0), g2.T @ h1, g2.sum(0), g3.T @ h2, g3.sum(0))


def adam(p, m, v, g, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One bias-corrected Adam update (step counts from 1); returns new p, m, v."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def init_params(n_in, n_out, u):
    """Glorot-uniform weights from uniform draws u in [-1, 1) (one per
    parameter, in packed order), zero biases."""
    u = np.asarray(u, dtype=np.float64)
    W1, b1, W2, b2, W3, b3 = unpack(u, n_in, n_out)
    lim = lambda fi, fo: np.sqrt(6.0 / (fi + fo))
    return pack(W1 * lim(n_in, H), 0 * b1, W2 * lim(H, H), 0 * b2, W3 * lim(H, n_out), 0 * b3)


def dominance_margin(J, dC, V, M):
    """Per cell, with D_C = dC I - V J written in molar units (row r scaled by
    1/M_r, column c by M_c): min over rows of (D_rr M_r - sum_{c != r} |D_rc|
    M_c) / (|D_rr| M_r), or -1 where a diagonal entry is not positive.  The
    block is strictly row diagonally dominant with a positive diagonal iff
    the margin is positive.  J (n, ns, ns); dC, V (n,); M (ns,)."""
    J = np.asarray(J, dtype=np.float64)
    ns = J.shape[1]
    M = np.asarray(M, dtype=np.float64)
    D = dC[:, None, None] * np.eye(ns)[None] - V[:, None, None] * J
    diag = np.einsum("nii->ni", D)
    off = (np.abs(D) * M[None, None, :]).sum(axis=2) - np.abs(diag) * M[None, :]
    marg = (diag * M[None, :] - off) / (np.abs(diag) * M[None, :] + 1e-300)
    marg = marg.min(axis=1)
    return np.where(np.all(diag > 0, axis=1), marg, -1.0)


def dominant(J, dC, V, M):
    """Acceptance of a surrogate species block (see dominance_margin)."""
    return dominance_margin(J, dC, V, M) > 0


def bf16_tie_distance(v):
    """|v - m| for the bfloat16 rounding midpoint m nearest to each FP32 v."""
    f = np.abs(np.asarray(v, dtype=np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    lo = ((u >> 16) << 16).astype(np.uint32).view(np.float32).astype(np.float64)
    hi = (((u >> 16) + 1) << 16).astype(np.uint32).view(np.float32).astype(np.float64)
    return np.abs(f.astype(np.float64) - 0.5 * (lo + hi))


def near_bf16_tie(v, rel=1e-5):
    """Elements of the FP32 array v within rel*|v| of a bfloat16 rounding
    midpoint: there a sum accumulated in another order may round the other way."""
    f = np.abs(np.asarray(v, dtype=np.float64))
    return bf16_tie_distance(v) <= rel * f + 1e-38


def _bf16_ulp(v):
    """Spacing of bfloat16 numbers at |v| (FP32 input)."""
    f = np.abs(np.asarray(v, dtype=np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    lo = ((u >> 16) << 16).astype(np.uint32).view(np.float32).astype(np.float64)
    hi = (((u >> 16) + 1) << 16).astype(np.uint32).view(np.float32).astype(np.float64)
    return hi - lo


def flip_bound(p, x, n_out, acc_rel=2.5e-7):
    """Per sample and output, a bound on how far y may move when BF16
    roundings of hidden activations lying within FP32 summation noise of a
    rounding midpoint go the other way.  Noise of an activation: acc_rel times
    the sum of |terms| of its pre-activation plus 4 FP32 ulps.  A flip in h1
    moves z2 by at most |W2b| ulp(h1) (|tanh'| <= 1), which may move h2 and its
    own rounding; the bound collects these through |W3b|.  Zero for samples
    without such activations (and inputs away from midpoints)."""
    x = np.asarray(x, dtype=np.float64)
    n_in = x.shape[1]
    W1, b1, W2, b2, W3, b3 = unpack(p, n_in, n_out)
    W1b, W2b, W3b = (bf16(w).astype(np.float64) for w in (W1, W2, W3))
    _, (xb, h1, h1b, h2, h2b) = forward(p, x, n_out, emulate=True)
    s1 = np.abs(xb) @ np.abs(W1b).T + np.abs(f32(b1))
    s2 = np.abs(h1b) @ np.abs(W2b).T + np.abs(f32(b2))
    amb_x = near_bf16_tie(x.astype(np.float32), 1e-6)
    dz1 = (amb_x * _bf16_ulp(x)) @ np.abs(W1b).T                     # input roundings
    amb1 = (bf16_tie_distance(h1) <= acc_rel * s1 + 2.0 ** -22 * np.abs(h1) + dz1) | (dz1 > 0)
    dh1 = amb1 * (_bf16_ulp(h1) + dz1)
    dz2 = dh1 @ np.abs(W2b).T
    amb2 = (bf16_tie_distance(h2) <= acc_rel * s2 + 2.0 ** -22 * np.abs(h2) + dz2) | (dz2 > 0)
    dh2 = amb2 * (_bf16_ulp(h2) + dz2)
    return dh2 @ np.abs(W3b).T


def ambiguous_samples(p, x, n_out, acc_rel=2.5e-7):
    """Samples whose output may move under another FP32 summation order."""
    return np.any(flip_bound(p, x, n_out, acc_rel) > 0, axis=1)
