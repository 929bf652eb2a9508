"""GPU parity of the surrogate network's BF16 matrix-core kernels (through the
C-ABI) against the numpy oracle with the same rounding points, and of the
solver-side sampling and inference kernels against the FP64 solver oracle.

A BF16 rounding of an activation that lies within FP32 accumulation noise of a
rounding midpoint may go either way (the matrix cores sum in their own
order); such samples are detected by the oracle itself and held to a looser
bound, all others to 2e-5 of the summed magnitudes."""
import numpy as np
import pytest

from gpu_cases import mech_by_name, normwise, pair, sample_cells
from oracle import mlp
from paper_2403_03440_amd import inputs as I

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    return torch


def _csi():
    from paper_2403_03440_amd import csi
    return csi


def _net(n_in, n_out, seed, bias=0.1):
    p = mlp.init_params(n_in, n_out, I.uniform_pm1(seed, mlp.n_params(n_in, n_out)))
    W1, b1, W2, b2, W3, b3 = mlp.unpack(p, n_in, n_out)
    b1[:] = bias * I.uniform_pm1(seed + 1, b1.size)
    b2[:] = bias * I.uniform_pm1(seed + 2, b2.size)
    b3[:] = bias * I.uniform_pm1(seed + 3, b3.size)
    return mlp.pack(W1, b1, W2, b2, W3, b3).astype(np.float32)


def _dev(a, dtype=None):
    torch = _torch()
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype or torch.float32, device="cuda")


def _output_bound(p, x, n_out):
    """Per-element scale sum_k |W3b[o,k] h2b_k| + |b3_o| of the output sums."""
    W1, b1, W2, b2, W3, b3 = mlp.unpack(p, x.shape[1], n_out)
    _, (xb, h1, h1b, h2, h2b) = mlp.forward(p, x, n_out, emulate=True)
    return np.abs(h2b) @ np.abs(mlp.bf16(W3).astype(np.float64)).T + np.abs(b3)


@pytest.mark.parametrize("n_in,n_out,n", [(14, 121, 1000), (8, 25, 64), (23, 400, 333), (40, 9, 130), (3, 4, 1)])
def test_forward_parity(n_in, n_out, n):
    print(f"forward n_in {n_in} n_out {n_out} n {n}", flush=True)
    csi = _csi()
    p = _net(n_in, n_out, 100 + n_in)
    x = (2.0 * I.uniform_pm1(200 + n_in, n * n_in).reshape(n, n_in)).astype(np.float32)
    net = csi.Mlp(n_in, n_out, batch=256)
    y = net.forward(_dev(p), _dev(x)).cpu().numpy().astype(np.float64)
    yo, _ = mlp.forward(p.astype(np.float64), x.astype(np.float64), n_out, emulate=True)
    fb = mlp.flip_bound(p.astype(np.float64), x.astype(np.float64), n_out)
    scale = _output_bound(p.astype(np.float64), x.astype(np.float64), n_out)
    err = np.abs(y - yo)
    assert (fb.max(axis=1) == 0).mean() >= 0.5 or n < 8
    assert np.all(err <= 2e-5 * scale + fb)


def _emulated_grad_case(n_in, n_out, n_data, batch, seed):
    p = _net(n_in, n_out, seed)
    x = I.uniform_pm1(seed + 10, n_data * n_in).reshape(n_data, n_in).astype(np.float32)
    t = (0.5 * I.uniform_pm1(seed + 11, n_data * n_out).reshape(n_data, n_out)).astype(np.float32)
    idx = (np.arange(batch) * 7 + 3) % n_data
    return p, x, t, idx.astype(np.int32)


@pytest.mark.parametrize("n_in,n_out,batch", [(14, 121, 300), (8, 25, 64), (23, 400, 130), (40, 9, 77)])
def test_gradient_parity(n_in, n_out, batch):
    print(f"grad n_in {n_in} n_out {n_out} batch {batch}", flush=True)
    csi = _csi()
    p, x, t, idx = _emulated_grad_case(n_in, n_out, 500, batch, 300 + n_in)
    net = csi.Mlp(n_in, n_out, batch=batch)
    g, loss = net.grad(_dev(p), _dev(x), _dev(t), _dev(idx, _torch().int32))
    g = g.cpu().numpy().astype(np.float64)
    lo, go = mlp.loss_and_grad(p.astype(np.float64), x[idx].astype(np.float64), t[idx].astype(np.float64),
                               emulate=True)
    assert abs(loss - lo) <= 1e-6 * lo
    parts = [q.astype(np.int64) for q in mlp.unpack(np.arange(go.size), n_in, n_out)]
    for name, sl in zip(("W1", "b1", "W2", "b2", "W3", "b3"), parts):
        k = sl.ravel()
        e = np.abs(g[k] - go[k]).max() / np.abs(go[k]).max()
        assert e <= 1e-3, (name, e)


def test_gradient_skips_out_of_range_rows():
    csi = _csi()
    n_in, n_out = 14, 121
    p, x, t, idx = _emulated_grad_case(n_in, n_out, 100, 70, 41)
    bad = idx.copy()
    bad[5], bad[40] = -1, 100      # outside [0, n_data): skipped
    net = csi.Mlp(n_in, n_out, batch=70)
    g, loss = net.grad(_dev(p), _dev(x), _dev(t), _dev(bad, _torch().int32))
    keep = np.delete(idx, [5, 40])
    # the mean still divides by the nominal batch size
    lo, go = mlp.loss_and_grad(p.astype(np.float64), x[keep].astype(np.float64), t[keep].astype(np.float64),
                               emulate=True, n_mean=70)
    assert abs(loss - lo) <= 1e-6 * lo
    assert np.abs(g.cpu().numpy() - go).max() <= 1e-3 * np.abs(go).max()


def test_adam_step_parity():
    csi = _csi()
    torch = _torch()
    n_in, n_out, batch = 14, 121, 256
    p, x, t, idx = _emulated_grad_case(n_in, n_out, 400, batch, 51)
    npar = p.size
    m0 = (1e-3 * I.uniform_pm1(52, npar)).astype(np.float32)
    v0 = (1e-4 * (1.5 + I.uniform_pm1(53, npar))).astype(np.float32)
    P, M, V = _dev(p), _dev(m0), _dev(v0)
    net = csi.Mlp(n_in, n_out, batch=batch)
    loss = net.train_step(P, M, V, _dev(x), _dev(t), _dev(idx, torch.int32), step=10, lr=1e-3)
    lo, go = mlp.loss_and_grad(p.astype(np.float64), x[idx].astype(np.float64), t[idx].astype(np.float64),
                               emulate=True)
    po, mo, vo = mlp.adam(p.astype(np.float64), m0.astype(np.float64), v0.astype(np.float64), go, 10)
    assert abs(loss - lo) <= 1e-6 * lo
    assert np.abs(P.cpu().numpy() - po).max() <= 1e-6 * np.abs(po).max()
    assert normwise(M.cpu().numpy(), mo).max() <= 1e-5
    assert normwise(V.cpu().numpy(), vo).max() <= 1e-5


def test_training_trajectory_matches_oracle():
    """30 Adam steps on a smooth synthetic regression: the GPU loss history
    follows the emulated oracle's and decreases."""
    csi = _csi()
    torch = _torch()
    n_in, n_out, batch, n_data = 8, 25, 128, 1024
    rng_x = I.uniform_pm1(61, n_data * n_in).reshape(n_data, n_in)
    A = I.uniform_pm1(62, n_in * n_out).reshape(n_in, n_out)
    t = np.tanh(rng_x @ A).astype(np.float32)
    x = rng_x.astype(np.float32)
    p = _net(n_in, n_out, 63)
    P, M, V = _dev(p), _dev(np.zeros_like(p)), _dev(np.zeros_like(p))
    net = csi.Mlp(n_in, n_out, batch=batch)
    po, mo, vo = p.astype(np.float64), np.zeros(p.size), np.zeros(p.size)
    lg, lo = [], []
    for k in range(30):
        idx = ((np.arange(batch) * 13 + 17 * k) % n_data).astype(np.int32)
        lg.append(net.train_step(P, M, V, _dev(x), _dev(t), _dev(idx, torch.int32), step=k + 1, lr=3e-3))
        l_, g_ = mlp.loss_and_grad(po, x[idx].astype(np.float64), t[idx].astype(np.float64), emulate=True)
        po, mo, vo = mlp.adam(po, mo, vo, g_, k + 1, lr=3e-3)
        lo.append(l_)
    lg, lo = np.array(lg), np.array(lo)
    print("loss gpu", lg[[0, 9, 19, 29]], "oracle", lo[[0, 9, 19, 29]])
    assert np.all(np.abs(lg - lo) <= 2e-2 * lo)
    assert lg[-1] < 0.5 * lg[0]


def test_prepare_parity():
    csi = _csi()
    n, n_in, n_out = 5000, 6, 9
    xr = np.column_stack([7 + 2 * I.uniform_pm1(71, n), 8 + I.uniform_pm1(72, n), -5 + I.uniform_pm1(73, n),
                          0.5 + 0.5 * I.uniform_pm1(74, n), np.zeros(n), np.full(n, 0.25)]).astype(np.float32)
    J = (10.0 ** (6 * I.uniform_pm1(75, n * n_out)) * I.uniform_pm1(76, n * n_out)).reshape(n, n_out)
    J[:, 3] = 0.0
    J = J.astype(np.float32)
    net = csi.Mlp(n_in, n_out, batch=64)
    x, t, sc = net.prepare(_dev(xr), _dev(J))
    mu, sigma, tau0 = mlp.scales(xr.astype(np.float64), J.astype(np.float64))
    assert np.abs(sc[:n_in] - mu).max() <= 1e-12 * np.abs(mu).max()
    assert np.abs(sc[n_in:2 * n_in] - sigma).max() <= 1e-12 * np.abs(sigma).max()
    assert abs(sc[-1] - tau0) <= 1e-12 * tau0
    xo = mlp.standardise(xr.astype(np.float64), mu, sigma)
    to = mlp.target(J.astype(np.float64), tau0)
    assert np.abs(x.cpu().numpy() - xo).max() <= 1e-6 * max(1.0, np.abs(xo).max())
    assert np.abs(t.cpu().numpy() - to).max() <= 1e-6 * max(1.0, np.abs(to).max())


def _features_oracle(o, m):
    q = o.get_state()
    rho = q[:m.ns].sum(0)
    T, Tv = o.get("T"), o.get("Tv")
    return mlp.features(T, Tv if m.two_temp else T, rho, (q[:m.ns] / rho).T)


@pytest.mark.parametrize("name", ["air5_2T", "air11_2T", "air5_1T", "syn20_1T", "toy2_1T"])
@pytest.mark.parametrize("reading", [0, 1, 2])
def test_sample_jacobians_parity(name, reading):
    print(f"sample {name} reading {reading}", flush=True)
    torch = _torch()
    m = mech_by_name(name)
    o, s, q0 = pair(m, 32, 24, state="evolved", mech_name=name, iters=40)
    o.set_option("jc_fixed_qf", reading + 1 if reading else 0)
    s.set_species_jacobian(reading)
    o.residual(10.0)
    N = s.N
    xr = torch.empty((N, m.ns + 3), dtype=torch.float32, device="cuda")
    jc = torch.empty((N, m.ns * m.ns), dtype=torch.float32, device="cuda")
    assert s.sample_jacobians(xr, jc) == N
    xo = _features_oracle(o, m)
    # the mass fractions share one scale (trace species fall below FP32's range)
    fg = [[0], [1], [2], list(range(3, m.ns + 3))]
    assert normwise(xr.cpu().numpy().T, xo.T, fg).max() <= 1e-6
    Jo = o.get("JC").transpose(2, 0, 1).reshape(N, -1)       # (s, r) row-major per cell
    Jg = jc.cpu().numpy().astype(np.float64)
    scale = np.abs(Jo).max(axis=1, keepdims=True) + 1e-300
    assert np.all(np.abs(Jg - Jo) <= 1e-6 * scale)
    # seeded subsets of 100 distinct cells (csi.h's definition of the rows)
    subsets = []
    for seed in (7, 3440):
        n = s.sample_jacobians(xr, jc, max_samples=100, seed=seed)
        assert n == 100
        cells = sample_cells(N, 100, seed)
        assert len(set(cells.tolist())) == 100
        subsets.append(set(cells.tolist()))
        Jg100 = jc[:100].cpu().numpy().astype(np.float64)
        assert np.all(np.abs(Jg100 - Jo[cells]) <= 1e-6 * scale[cells])
        assert normwise(xr[:100].cpu().numpy().T, xo[cells].T, fg).max() <= 1e-6
    assert subsets[0] != subsets[1]


def _oracle_scales(o, m):
    """Input / target scales from the oracle's own cells and exact J_C."""
    o.residual(10.0)
    o.implicit_op(1)
    N = o.N
    mu, sigma, tau0 = mlp.scales(_features_oracle(o, m), o.get("JC").transpose(2, 0, 1).reshape(N, -1))
    return np.concatenate([mu, sigma, [tau0]])


def _rejecting_bias(o, m):
    """An output bias that makes V J_C exceed dC by e^10 in the median cell:
    D_C gets a negative diagonal, so every block fails the acceptance test."""
    sc0 = _oracle_scales(o, m)
    return np.arcsinh(np.median(o.get("dC") / o.get("V")) * sc0[-1]) + 10.0


def _install(s, o, m, seed, bias=0.1, b3=None):
    """A random network for the solver's mechanism, with scales from the
    oracle's cells; b3 (optional) replaces the output biases."""
    n_in, n_out = m.ns + 3, m.ns * m.ns
    p = _net(n_in, n_out, seed, bias)
    if b3 is not None:
        W1, b1, W2, b2, W3, b3_ = mlp.unpack(p.astype(np.float64), n_in, n_out)
        b3_[:] = b3
        p = mlp.pack(W1, b1, W2, b2, W3, b3_).astype(np.float32)
    sc = _oracle_scales(o, m)
    P = _dev(p)
    s.set_surrogate(P, sc)
    return p, sc, P


@pytest.mark.parametrize("name", ["air5_2T", "air11_2T", "air5_1T"])
def test_surrogate_inference_parity(name):
    print(f"inference {name}", flush=True)
    csi = _csi()
    m = mech_by_name(name)
    o, s, q0 = pair(m, 32, 24, state="evolved", mech_name=name, iters=40)
    p, sc, P = _install(s, o, m, 81)
    s.set_state(q0)
    s.residual(10.0)
    s.implicit_op(csi.SPLIT, csi.FP64, csi.JAC_SURROGATE)
    Jg = s.get("Jsur").T                                      # (N, ns*ns)
    o.residual(10.0)
    n_in = m.ns + 3
    x = mlp.standardise(_features_oracle(o, m), sc[:n_in], sc[n_in:2 * n_in])
    x32 = x.astype(np.float32).astype(np.float64)
    yo, _ = mlp.forward(p.astype(np.float64), x32, m.ns * m.ns, emulate=True)
    Jo = mlp.jacobian(yo, sc[-1])
    # y differs by at most 2e-5 of its summed scale plus the possible BF16
    # rounding flips; J = sinh(y) / tau0 inherits |dJ| <= cosh(|y| + dy) dy / tau0
    # (+ FP32 rounding of J)
    fb = mlp.flip_bound(p.astype(np.float64), x32, m.ns * m.ns)
    dy = 2e-5 * _output_bound(p.astype(np.float64), x32, m.ns * m.ns) + fb
    bound = np.cosh(np.abs(yo) + dy) * dy / sc[-1] + 2e-7 * np.abs(Jo)
    err = np.abs(Jg - Jo)
    assert (fb.max(axis=1) == 0).mean() >= 0.2
    assert np.all(err <= bound)


@pytest.mark.parametrize("name", ["air5_2T", "air5_1T", "air11_2T"])
def test_surrogate_dominance_selection(name):
    """Per cell the species block comes from the network when the oracle's
    acceptance test (strict row dominance with a positive diagonal, molar
    units) passes on the oracle's own network output, else it is the exact
    block, bitwise."""
    csi = _csi()
    m = mech_by_name(name)
    o, s, q0 = pair(m, 32, 24, state="evolved", mech_name=name, iters=40)
    ns, N = m.ns, s.N
    # output biases that put V J_rr near dC in the median cell (of the oracle's
    # blocks), so that both outcomes of the test occur
    sc0 = _oracle_scales(o, m)
    y0 = np.arcsinh(np.median(o.get("dC") / o.get("V")) * sc0[-1])
    b3 = np.full(ns * ns, y0 - 20.0)
    b3[::ns + 1] = y0 - 1.0
    p, sc, P = _install(s, o, m, 83, bias=0.5, b3=b3)
    res = {}
    for jac in (csi.JAC_EXACT, csi.JAC_SURROGATE):
        s.set_state(q0)
        s.residual(10.0)
        s.implicit_op(csi.SPLIT, csi.FP64, jac)
        res[jac] = s.get("Dinv", csi.SPLIT)[m.nf * m.nf:].T.reshape(N, ns, ns)
    acc_g = np.any(res[csi.JAC_SURROGATE] != res[csi.JAC_EXACT], axis=(1, 2))
    o.set_state(q0)
    o.residual(10.0)
    o.implicit_op(csi.SPLIT)
    dC, V = o.get("dC"), o.get("V")
    n_in = ns + 3
    x32 = mlp.standardise(_features_oracle(o, m), sc[:n_in], sc[n_in:2 * n_in]).astype(np.float32).astype(np.float64)
    yo, _ = mlp.forward(p.astype(np.float64), x32, ns * ns, emulate=True)
    Jo = mlp.jacobian(yo, sc[-1]).reshape(N, ns, ns)
    marg = mlp.dominance_margin(Jo, dC, V, np.array(m.M))
    acc_o = marg > 0
    # decisions within the comparison's noise of the threshold are not compared
    fb = mlp.flip_bound(p.astype(np.float64), x32, ns * ns).max(axis=1)
    clear = (np.abs(marg) > 1e-4) & (fb == 0)
    print(f"{name}: accepted gpu {acc_g.sum()} oracle {acc_o.sum()} of {N}; clear decisions {clear.sum()}")
    assert clear.sum() >= 0.25 * N
    assert np.array_equal(acc_g[clear], acc_o[clear])
    assert 0 < acc_o.sum() < N                       # both outcomes are exercised
    D = dC[:, None, None] * np.eye(ns)[None] - V[:, None, None] * Jo
    for k in np.nonzero(clear & acc_o)[0]:
        Dk = np.linalg.inv(D[k])
        assert np.abs(res[csi.JAC_SURROGATE][k] - Dk).max() <= 1e-4 * np.abs(Dk).max()


def test_surrogate_fallback_everywhere_equals_exact():
    """A network whose blocks never pass the dominance check: every cell falls
    back to the exact block, so the increment is the exact path's, bitwise."""
    csi = _csi()
    m = mech_by_name("air5_2T")
    o, s, q0 = pair(m, 32, 24, state="evolved", mech_name="air5_2T", iters=40)
    _install(s, o, m, 91, b3=_rejecting_bias(o, m))
    for prec in (csi.FP64, csi.MIXED):
        s.set_state(q0)
        s.residual(10.0)
        s.implicit_op(csi.SPLIT, prec, csi.JAC_EXACT)
        d_ex = s.get("dq")
        s.set_state(q0)
        s.residual(10.0)
        s.implicit_op(csi.SPLIT, prec, csi.JAC_SURROGATE)
        assert np.array_equal(s.get("dq"), d_ex)
    s.set_state(q0)
    st = s.step(csi.SPLIT, csi.CC2, 10.0, 3, jac=csi.JAC_SURROGATE)
    assert st["n_dd_fallback"] == 3 * s.N


def test_surrogate_stall_policy_switches_off():
    csi = _csi()
    m = mech_by_name("air5_2T")
    o, s, q0 = pair(m, 32, 24, state="evolved", mech_name="air5_2T", iters=40)
    # blocks that never pass the dominance check keep the run on the exact path
    p, sc, P = _install(s, o, m, 95, b3=_rejecting_bias(o, m))
    # a ratio below any possible residual ratio: "stalled" as soon as the window is full
    s.set_surrogate(P, sc, stall_ratio=1e-30, stall_window=5)
    s.set_state(q0)
    st = s.step(csi.SPLIT, csi.CC2, 10.0, 12, jac=csi.JAC_SURROGATE, check_every=4)
    assert st["surrogate_off_at"] == 5
    s.set_surrogate(P, sc, stall_ratio=1e30, stall_window=5)
    s.set_state(q0)
    st = s.step(csi.SPLIT, csi.CC2, 10.0, 12, jac=csi.JAC_SURROGATE)
    assert st["surrogate_off_at"] == -1


def test_surrogate_argument_errors():
    csi = _csi()
    m = mech_by_name("air5_2T")
    o, s, q0 = pair(m, 8, 6, state="random", T_range=(300.0, 1200.0), speed=800.0)
    s.residual(10.0)
    with pytest.raises(csi.CsiError, match="CSI_ERR_STATE"):
        s.implicit_op(csi.SPLIT, csi.FP64, csi.JAC_SURROGATE)   # nothing installed
    p, sc, P = _install(s, o, m, 97)
    s.residual(10.0)
    with pytest.raises(csi.CsiError, match="CSI_ERR_ARG"):
        s.implicit_op(csi.COUPLED, csi.FP64, csi.JAC_SURROGATE)
    bad = sc.copy()
    bad[m.ns + 3] = 0.0
    with pytest.raises(csi.CsiError, match="CSI_ERR_ARG"):
        s.set_surrogate(P, bad)
    with pytest.raises(csi.CsiError, match="CSI_ERR_ARG"):
        csi.Mlp(65, 10)


def test_trained_surrogate_reaches_the_same_steady_state():
    """Train on the method's own Jacobians (11-species air, 2T), then solve
    with and without the surrogate: the steady state is the root of the exact
    residual either way; report what the network changes in iterations."""
    csi = _csi()
    from paper_2403_03440_amd import surrogate as S
    cfg = I.Config("t4", 32, 24, "air11", 1, 10.0, 5000.0)
    m = cfg.mechanism()
    x, y = cfg.grid()
    fs = I.freestream_prims(cfg, m)
    s = csi.Solver((x, y), m, fs)
    q0 = s.initial_state(*I.initial_prims(cfg, m))
    s.set_state(q0)
    xr, jc, its = S.collect(s, (csi.SPLIT, csi.CC2, csi.MIXED), cfg.cfl, 16 * s.N, every=5)
    params, scales, hist = S.train(xr, jc, epochs=30, batch=1024, lr=3e-3, seed=11)
    print("training", hist[0], hist[-1])
    assert hist[-1][1] < 0.5 * hist[0][1]
    res = {}
    import time
    import torch
    for jac in (csi.JAC_EXACT, csi.JAC_SURROGATE):
        s.set_state(q0)
        if jac == csi.JAC_SURROGATE:
            s.set_surrogate(params, scales)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = s.step(csi.SPLIT, csi.CC2, cfg.cfl, 8000, precision=csi.MIXED, jac=jac, cfl_ramp=100, tol=1e-10,
                    check_every=50)
        torch.cuda.synchronize()
        res[jac] = (st, s.get_state(), s.wall_heat_flux()[1], time.perf_counter() - t0)
        print("jac", jac, "iterations", st["iters"], "converged", st["converged"], "dd fallbacks",
              st["n_dd_fallback"], "off at", st["surrogate_off_at"], f"{res[jac][3]:.3f} s")
    (se, qe, qse, te), (ss, qs, qss, ts) = res[csi.JAC_EXACT], res[csi.JAC_SURROGATE]
    # what the network gains or loses: iterations and solve time against the
    # exact block, and the training time
    print(f"surrogate: {ss['iters'] - se['iters']:+d} iterations, solve {ts - te:+.3f} s, "
          f"training {hist[-1][3]:.3f} s", flush=True)
    assert se["converged"] and ss["converged"]
    # the network was in use: no stall or divergence fallback, and its block
    # passed the dominance check in part of the cell-iterations (about 13 % for
    # 11-species air on this grid, where in molar units about a third of the
    # exact blocks pass it)
    assert ss["surrogate_off_at"] == -1 and ss["surrogate_diverged"] == 0
    assert ss["n_dd_fallback"] <= 0.95 * ss["iters"] * s.N
    assert normwise(qs, qe, [list(range(m.ns)), [m.ns, m.ns + 1], [m.ns + 2], [m.ns + 3]]).max() <= 1e-6
    assert abs(qss - qse) <= 1e-6 * abs(qse)


def test_train_epoch_equals_train_steps():
    """csi_mlp_train_epoch (one call per epoch) takes the same Adam steps as
    csi_mlp_train_step called per batch: the parameters and moments agree
    bitwise, the last batch shorter than the others."""
    torch = _torch()
    csi = _csi()
    n_in, n_out, n_data, batch = 14, 121, 1000, 96
    p, x, t, _ = _emulated_grad_case(n_in, n_out, n_data, batch, 77)
    order = I.permutation(5, n_data)[:700].astype(np.int32)     # 7 full batches and one of 28
    net = csi.Mlp(n_in, n_out, batch=batch)
    xd, td, od = _dev(x), _dev(t), _dev(order, torch.int32)
    pa, ma, va = _dev(p), torch.zeros(p.size, device="cuda"), torch.zeros(p.size, device="cuda")
    pb, mb, vb = _dev(p), torch.zeros(p.size, device="cuda"), torch.zeros(p.size, device="cuda")
    step = 3
    for b0 in range(0, order.size, batch):
        step += 1
        la = net.train_step(pa, ma, va, xd, td, od[b0:b0 + batch], step, lr=2e-3)
    lb = net.train_epoch(pb, mb, vb, xd, td, od, 3, lr=2e-3)
    assert torch.equal(pa, pb) and torch.equal(ma, mb) and torch.equal(va, vb)
    assert la == lb
