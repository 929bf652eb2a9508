"""Pins of the surrogate-network oracle (oracle/mlp.py) against library
routines, closed forms and brute force; CPU only."""
import numpy as np
import pytest
import torch

from oracle import mlp
from paper_2403_03440_amd import inputs as I


def _net(n_in, n_out, seed, scale=1.0):
    u = I.uniform_pm1(seed, mlp.n_params(n_in, n_out))
    p = mlp.init_params(n_in, n_out, u) * scale
    # non-zero biases so that every parameter is exercised
    W1, b1, W2, b2, W3, b3 = mlp.unpack(p, n_in, n_out)
    b1[:] = 0.1 * I.uniform_pm1(seed + 1, b1.size)
    b2[:] = 0.1 * I.uniform_pm1(seed + 2, b2.size)
    b3[:] = 0.1 * I.uniform_pm1(seed + 3, b3.size)
    return mlp.pack(W1, b1, W2, b2, W3, b3)


def test_bf16_rounding_known_values():
    e = 2.0 ** -8
    # bfloat16 keeps 7 fraction bits: spacing 2^-7 = 2e on [1, 2); halfway cases go to the even neighbour
    vals = np.array([1.0, 1 + e, 1 + 3 * e, 1 + 2 * e, -1.5, 1 + e + 2.0 ** -20, 0.0, -(1 + 5 * e)], dtype=np.float32)
    want = np.array([1.0, 1.0, 1 + 4 * e, 1 + 2 * e, -1.5, 1 + 2 * e, 0.0, -(1 + 4 * e)], dtype=np.float32)
    assert np.array_equal(mlp.bf16(vals), want)


def test_bf16_matches_torch_conversion():
    x = (I.uniform_pm1(11, 20000) * 10.0 ** (4 * I.uniform_pm1(12, 20000))).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    assert np.array_equal(mlp.bf16(x), ref)


def _torch_forward(p, x, n_out):
    n_in = x.shape[1]
    W1, b1, W2, b2, W3, b3 = (torch.tensor(a, dtype=torch.float64, requires_grad=True)
                              for a in mlp.unpack(p, n_in, n_out))
    X = torch.tensor(x, dtype=torch.float64)
    y = torch.nn.functional.linear(torch.tanh(torch.nn.functional.linear(
        torch.tanh(torch.nn.functional.linear(X, W1, b1)), W2, b2)), W3, b3)
    return y, (W1, b1, W2, b2, W3, b3)


@pytest.mark.parametrize("n_in,n_out", [(8, 25), (14, 121)])
def test_forward_and_gradient_match_torch(n_in, n_out):
    p = _net(n_in, n_out, 5)
    x = I.uniform_pm1(6, 37 * n_in).reshape(37, n_in) * 2.0
    t = I.uniform_pm1(7, 37 * n_out).reshape(37, n_out)
    y, _ = mlp.forward(p, x, n_out)
    yt, params = _torch_forward(p, x, n_out)
    assert np.abs(y - yt.detach().numpy()).max() <= 1e-14 * max(1.0, np.abs(y).max())
    loss, g = mlp.loss_and_grad(p, x, t)
    lt = ((yt - torch.tensor(t)) ** 2).mean()
    lt.backward()
    gt = np.concatenate([a.grad.numpy().ravel() for a in params])
    assert abs(loss - lt.item()) <= 1e-14 * lt.item()
    assert np.abs(g - gt).max() <= 1e-13 * np.abs(gt).max()


def test_gradient_central_differences():
    n_in, n_out = 5, 9
    p = _net(n_in, n_out, 21)
    x = I.uniform_pm1(22, 6 * n_in).reshape(6, n_in)
    t = I.uniform_pm1(23, 6 * n_out).reshape(6, n_out)
    _, g = mlp.loss_and_grad(p, x, t)
    rng = np.random.default_rng(24)
    idx = rng.choice(p.size, 60, replace=False)
    h = 1e-6
    for k in idx:
        pp, pm = p.copy(), p.copy()
        pp[k] += h
        pm[k] -= h
        fd = (mlp.loss_and_grad(pp, x, t)[0] - mlp.loss_and_grad(pm, x, t)[0]) / (2 * h)
        assert abs(fd - g[k]) <= 1e-7 * max(1e-3, np.abs(g).max()), (k, fd, g[k])


def test_emulated_forward_within_bf16_error_bound():
    n_in, n_out = 14, 121
    p = _net(n_in, n_out, 31)
    x = I.uniform_pm1(32, 200 * n_in).reshape(200, n_in) * 2.0
    y64, _ = mlp.forward(p, x, n_out)
    y16, (xb, h1, h1b, h2, h2b) = mlp.forward(p, x, n_out, emulate=True)
    # every bf16 operand carries a relative error <= 2^-9; bound the output error
    # by first-order propagation through the three layers with |tanh'| <= 1
    W1, b1, W2, b2, W3, b3 = mlp.unpack(p, n_in, n_out)
    u = 2.0 ** -9
    a = np.abs(x)
    e1 = (2 * u + 1e-6) * (a @ np.abs(W1).T) + u
    e2 = (2 * u + 1e-6) * (np.abs(h1) @ np.abs(W2).T) + e1 @ np.abs(W2).T + u
    e3 = (2 * u + 1e-6) * (np.abs(h2) @ np.abs(W3).T) + e2 @ np.abs(W3).T
    assert np.all(np.abs(y16 - y64) <= e3)
    assert np.abs(y16 - y64).max() > 0  # the emulation really rounds


def test_emulated_gradient_close_to_fp64():
    n_in, n_out = 14, 121
    p = _net(n_in, n_out, 41)
    x = I.uniform_pm1(42, 256 * n_in).reshape(256, n_in)
    t = I.uniform_pm1(43, 256 * n_out).reshape(256, n_out)
    l64, g64 = mlp.loss_and_grad(p, x, t)
    l16, g16 = mlp.loss_and_grad(p, x, t, emulate=True)
    assert abs(l16 - l64) <= 2e-2 * l64
    assert np.abs(g16 - g64).max() <= 3e-2 * np.abs(g64).max()


def test_adam_matches_torch_and_first_step_closed_form():
    n = 50
    p0 = I.uniform_pm1(51, n)
    grads = [I.uniform_pm1(52 + k, n) * 10.0 ** (-k) for k in range(6)]
    p, m, v = p0.copy(), np.zeros(n), np.zeros(n)
    P = torch.tensor(p0.copy(), requires_grad=True)
    opt = torch.optim.Adam([P], lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    for k, g in enumerate(grads):
        p, m, v = mlp.adam(p, m, v, g, k + 1)
        if k == 0:
            # m_hat = g, v_hat = g^2: every parameter moves by lr g / (|g| + eps)
            assert np.abs(p - (p0 - 1e-3 * g / (np.abs(g) + 1e-8))).max() <= 1e-15
        opt.zero_grad()
        P.grad = torch.tensor(g)
        opt.step()
        assert np.abs(p - P.detach().numpy()).max() <= 1e-15


def test_scales_standardise_and_tau0():
    x = np.column_stack([I.uniform_pm1(61, 1000) * 3 + 7, I.uniform_pm1(62, 1000), np.full(1000, 0.25)])
    J = np.array([[1e-3, 1e3], [0.0, -1.0]])
    mu, sigma, tau0 = mlp.scales(x, J)
    z = mlp.standardise(x, mu, sigma)
    assert np.abs(z[:, :2].mean(0)).max() <= 1e-14
    assert np.abs(np.sqrt((z[:, :2] ** 2).mean(0)) - 1).max() <= 1e-14
    assert sigma[2] == 1.0 and np.all(z[:, 2] == 0.0)      # constant feature: sigma 1
    assert abs(tau0 - 1.0) <= 1e-15                          # geometric mean of 1e-3, 1e3, 1
    J2 = np.array([2.0, 8.0, 0.0, -4.0])
    assert abs(mlp.scales(x, J2)[2] - 0.25) <= 1e-15         # (2 * 8 * 4)^(1/3) = 4
    t = mlp.target(np.array([-3.0, 0.0, 5.0]), 2.0)
    assert np.allclose(mlp.jacobian(t, 2.0), [-3.0, 0.0, 5.0], rtol=1e-15, atol=0)


def test_dominance_cases():
    ns = 2
    M = np.array([1.0, 4.0])
    J = np.zeros((5, ns, ns))
    J[1] = [[0.0, 0.2], [0.0, 0.0]]      # row 0: 1 > 0.2 * 4 / 1 = 0.8 -> dominant
    J[2] = [[0.0, 0.3], [0.0, 0.0]]      # row 0: 1 < 1.2 -> not
    J[3] = [[0.0, 0.0], [3.0, 0.0]]      # row 1: 1 * 4 > 3 * 1 -> dominant
    J[4] = [[2.0, 0.0], [0.0, 0.0]]      # negative diagonal
    dC, V = np.ones(5), np.ones(5)
    assert list(mlp.dominant(J, dC, V, M)) == [True, True, False, True, False]
    marg = mlp.dominance_margin(J, dC, V, M)
    assert abs(marg[1] - 0.2) <= 1e-15 and abs(marg[3] - 0.25) <= 1e-15 and marg[4] == -1.0
    # equal masses: the textbook strict row dominance
    Jt = np.array([[[0.0, 0.5], [0.5, 0.0]], [[0.0, 1.0], [0.0, 0.0]]])
    assert list(mlp.dominant(Jt, np.ones(2), np.ones(2), np.ones(2))) == [True, False]


def test_init_limits():
    n_in, n_out = 14, 121
    p = mlp.init_params(n_in, n_out, np.ones(mlp.n_params(n_in, n_out)))
    W1, b1, W2, b2, W3, b3 = mlp.unpack(p, n_in, n_out)
    assert np.allclose(W1, np.sqrt(6 / 78)) and np.allclose(W3, np.sqrt(6 / 185))
    assert not b1.any() and not b2.any() and not b3.any()


def test_near_tie_detector():
    e = 2.0 ** -8
    v = np.array([1 + e, 1 + e * (1 + 1e-7), 1 + 0.5 * e, -(1 + 3 * e)], dtype=np.float32)
    assert list(mlp.near_bf16_tie(v, 1e-5)) == [True, True, False, True]
