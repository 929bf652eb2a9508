"""Pins of the oracle's MUSCL + Roe residual (the second-order scheme of the
paper's cylinder case, Section 3.2, built as the residual ablation).

* Roe flux: consistent (F(q, q) = F(q)); Roe's property holds, so the flux
  of two supersonic states is the upwind state's physical flux, for a
  calorically perfect gas of fixed composition (monatomic species, with and
  without formation energies) and for a real-gas mixture (vibrating
  molecules, a composition jump, two temperatures); a contact discontinuity
  (same pressure and velocity) is upwinded exactly; mirror symmetry
  F(qL, qR, n) = -F(qR, qL, -n).  A wrong eigenvector component, wave
  strength, average or sign breaks one of these, and so does the perfect-gas
  contact energy H - c^2 / beta used for a real gas (an 8 % energy-flux error
  across a hypersonic shock).
* H-correction (the carbuncle cure): a floor eta above every wave speed
  turns the Roe flux into the local Lax-Friedrichs flux with speed eta, the
  species carried by that flux's mass flux; a floor below every wave speed
  changes nothing.  The residual of a state mirrored about the stagnation
  line is mirrored (a neighbour face taken from the wrong side breaks it).
* MUSCL with minmod: linear data reconstruct to the face midpoint, an
  extremum falls back to the cell value, and minmod takes the smaller of two
  same-signed slopes.
* The residual: zero on a uniform free stream; different from the
  first-order HLLE residual on a non-uniform state."""
import dataclasses

import numpy as np
import pytest

from oracle import orc
from paper_2403_03440_amd import inputs as I


def _argon(h_form=0.0):
    """Two identical monatomic species: a calorically perfect gas whatever
    the composition."""
    base = I.air5(0).without_reactions()
    k = list(base.names).index("N")
    idx = [k, k]
    z = np.zeros((0, 2), dtype=np.int32)
    return dataclasses.replace(
        base, names=["A1", "A2"], M=np.full(2, 0.039948), kind=base.kind[idx], theta_v=np.zeros(2),
        theta_r=np.zeros(2), sigma=np.ones(2), g_el=np.ones(2), h_form=np.full(2, h_form), sc=base.sc[idx],
        lt_a=base.lt_a[idx], lt_b=base.lt_b[idx], nu_f=z, nu_b=z, eff=np.zeros((0, 2)), reactions=[])


def _oracle(m):
    o = orc.Oracle()
    x, y = I.box_grid(2, 2)
    o.set_grid(x, y)
    o.set_mechanism(m)
    fs = (np.full(m.ns, 1e-3 / m.ns), 100.0, 0.0, 300.0, 300.0)
    o.set_freestream(*fs)
    return o


def _q(o, m, rho_s, u, v, T, Tv=None):
    rs = np.asarray(rho_s, dtype=float)[:, None]
    return o.prim_to_cons(rs, np.array([u]), np.array([v]), np.array([T]), np.array([Tv or T]))[:, 0]


def _rel(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


@pytest.mark.parametrize("two_temp", [0, 1])
def test_roe_consistency_and_symmetry(two_temp):
    m = I.air5(two_temp)
    o = _oracle(m)
    rng = np.random.default_rng(3)
    for _ in range(5):
        Y = rng.dirichlet(np.ones(m.ns))
        qL = _q(o, m, 0.01 * Y, 800.0, -300.0, 2500.0, 2200.0 if two_temp else None)
        Y2 = rng.dirichlet(np.ones(m.ns))
        qR = _q(o, m, 0.006 * Y2, 200.0, 500.0, 4000.0, 4300.0 if two_temp else None)
        n = np.array([0.6, 0.8])
        assert _rel(o.point_roe(qL, qL, *n), o.point_flux(qL, *n)) <= 1e-14
        assert _rel(o.point_roe(qL, qR, *n), -o.point_roe(qR, qL, *(-n))) <= 1e-14


@pytest.mark.parametrize("h_form", [0.0, 2.5e5])
def test_roe_property_supersonic_perfect_gas(h_form):
    m = _argon(h_form)
    o = _oracle(m)
    n = np.array([0.28, 0.96])
    # both states supersonic towards +n (Mach ~ 3 and ~ 2.2), different composition
    qL = _q(o, m, [2e-3, 1e-3], 1500.0 * n[0] - 100.0 * n[1], 1500.0 * n[1] + 100.0 * n[0], 300.0)
    qR = _q(o, m, [0.4e-3, 2.1e-3], 1300.0 * n[0], 1300.0 * n[1], 420.0)
    F = o.point_roe(qL, qR, *n)
    assert _rel(F, o.point_flux(qL, *n)) <= 1e-12
    # both supersonic towards -n: the right state's flux
    qL2 = _q(o, m, [0.4e-3, 2.1e-3], -1300.0 * n[0], -1300.0 * n[1], 420.0)
    qR2 = _q(o, m, [2e-3, 1e-3], -1500.0 * n[0] + 80.0 * n[1], -1500.0 * n[1] - 80.0 * n[0], 300.0)
    F = o.point_roe(qL2, qR2, *n)
    assert _rel(F, o.point_flux(qR2, *n)) <= 1e-12


@pytest.mark.parametrize("two_temp", [0, 1])
def test_roe_property_supersonic_real_gas(two_temp):
    """The states either side of the shock of the cylinder case: free-stream
    air at 295 K and dissociated air at 7,960 K (T_v 6,500 K), both moving
    along -n (at 5,000 and 1,800 m/s: local Mach numbers about 15 and 1.1),
    then the mirrored pair along +n."""
    m = I.air5(two_temp)
    o = _oracle(m)
    n = np.array([-0.98, 0.195])
    n = n / np.linalg.norm(n)
    Ypre = np.array([0.0, 0.0, 0.0, 0.233, 0.767])
    Ypost = np.array([0.21, 0.07, 0.001, 0.06, 0.659])
    Tv = 6500.0 if two_temp else None
    for sgn in (-1.0, 1.0):
        upost, vpost = sgn * (1800.0 * n[0] - 300.0 * n[1]), sgn * (1800.0 * n[1] + 300.0 * n[0])
        qpost = _q(o, m, 2.8e-3 * Ypost, upost, vpost, 7960.0, Tv)
        qpre = _q(o, m, 1e-3 * Ypre, sgn * 5000.0 * n[0], sgn * 5000.0 * n[1], 295.0)
        F = o.point_roe(qpost, qpre, *n) if sgn < 0 else o.point_roe(qpre, qpost, *n)
        assert _rel(F, o.point_flux(qpre, *n)) <= 1e-12, sgn


@pytest.mark.parametrize("h_form", [0.0, 2.5e5])
def test_roe_contact_exact_perfect_gas(h_form):
    m = _argon(h_form)
    o = _oracle(m)
    n = np.array([1.0, 0.0])
    # same pressure and velocity (subsonic, un > 0), density and composition jump
    p, u, v = 800.0, 120.0, 40.0
    TL, TR = 300.0, 900.0
    R = 8.314462618 / 0.039948
    qL = _q(o, m, [0.7 * p / (R * TL), 0.3 * p / (R * TL)], u, v, TL)
    qR = _q(o, m, [0.2 * p / (R * TR), 0.8 * p / (R * TR)], u, v, TR)
    F = o.point_roe(qL, qR, *n)
    assert _rel(F, o.point_flux(qL, *n)) <= 1e-12
    # a real gas (vibrating molecules, a composition jump) too: the waves at
    # u.n carry the whole jump of rho E
    ma = I.air5(0).without_reactions()
    oa = _oracle(ma)
    YL = np.array([0.2, 0.0, 0.0, 0.0, 0.8])
    YR = np.array([0.05, 0.1, 0.0, 0.3, 0.55])
    RL, RR = np.dot(YL, 8.314462618 / ma.M), np.dot(YR, 8.314462618 / ma.M)
    qaL = _q(oa, ma, YL * p / (RL * 600.0), u, v, 600.0)
    qaR = _q(oa, ma, YR * p / (RR * 3000.0), u, v, 3000.0)
    assert _rel(oa.point_roe(qaL, qaR, *n), oa.point_flux(qaL, *n)) <= 1e-12


def test_muscl_minmod_reconstruction():
    m = I.air5(0).without_reactions()
    o = _oracle(m)
    Y = np.array([0.2, 0.05, 0.05, 0.1, 0.6])
    rho = [1e-3, 1.2e-3, 1.4e-3]
    T = [500.0, 700.0, 900.0]
    u = [100.0, 150.0, 200.0]
    qA, qB, qC = (_q(o, m, rho[k] * Y, u[k], 10.0, T[k]) for k in range(3))
    Tf = o.point_prim(o.point_muscl(qA, qB, qC))[0]
    # linear data: the midpoint between B and C
    assert abs(Tf - 800.0) <= 1e-9 * 800.0
    qf = o.point_muscl(qA, qB, qC)
    assert np.allclose(qf[:m.ns], 1.3e-3 * Y, rtol=1e-13, atol=0.0)
    assert abs(qf[m.ns] / qf[:m.ns].sum() - 175.0) <= 1e-10
    # extremum at B: first order
    qA2 = _q(o, m, rho[0] * Y, u[0], 10.0, 950.0)
    qf = o.point_muscl(qA2, qB, qC)
    assert abs(o.point_prim(qf)[0] - 700.0) <= 1e-9 * 700.0
    # same-signed slopes 50 and 300 (T): minmod takes 50, B + 25
    qA3 = _q(o, m, rho[1] * Y, u[1], 10.0, 650.0)
    qC3 = _q(o, m, rho[1] * Y, u[1], 10.0, 1000.0)
    qf = o.point_muscl(qA3, qB, qC3)
    assert abs(o.point_prim(qf)[0] - 725.0) <= 1e-9 * 725.0


def test_muscl_roe_residual():
    m = I.air5(1).without_reactions()
    x, y = I.polar_grid(12, 8)
    fs = (np.array([0.0, 0.0, 0.0, 0.233e-3, 0.767e-3]), 3000.0, 0.0, 300.0, 300.0)
    o = orc.setup((x, y), m, fs, bc_mode=1)
    n = 96
    q0 = o.prim_to_cons(np.repeat(fs[0][:, None], n, 1), np.full(n, fs[1]), np.zeros(n), np.full(n, fs[3]),
                        np.full(n, fs[4]))
    o.set_option("residual_scheme", 1)
    o.set_state(q0)
    o.residual(5.0)
    R = o.get("R")
    # each row against its convected flux scale |q_k| |u| times a face length
    scale = np.abs(q0).max(axis=1) * 3000.0 * 0.05 + 1e-3 * 3000.0 * 0.05
    assert np.all(np.abs(R).max(axis=1) <= 1e-12 * scale)
    prims = I.random_prims(m, n, 7, T_range=(400.0, 3000.0), speed=800.0, y_floor=0.02)
    q1 = o.prim_to_cons(*prims)
    o.set_state(q1)
    o.residual(5.0)
    R2 = o.get("R")
    o.set_option("residual_scheme", 0)
    o.set_state(q1)
    o.residual(5.0)
    assert np.abs(R2 - o.get("R")).max() > 1e-3 * np.abs(R2).max()


def test_h_correction_limits():
    m = I.air5(1)
    o = _oracle(m)
    n = np.array([0.6, 0.8])
    qL = _q(o, m, [1e-4, 2e-4, 1e-5, 2e-3, 5e-3], 400.0, -200.0, 2500.0, 2000.0)
    qR = _q(o, m, [3e-4, 1e-4, 2e-5, 1e-3, 6e-3], -100.0, 300.0, 3500.0, 3900.0)
    FL, FR = o.point_flux(qL, *n), o.point_flux(qR, *n)
    eta = 1e4  # above |u.n| + c of both states and of their average
    F = o.point_roe(qL, qR, *n, eta=eta)
    ns = m.ns
    lf = 0.5 * (FL + FR) - 0.5 * eta * (qR - qL)
    fm = lf[:ns].sum()
    assert _rel(F[ns:ns + 3], lf[ns:ns + 3]) <= 1e-13
    assert abs(F[:ns].sum() - fm) <= 1e-13 * abs(fm) + 1e-13 * np.abs(lf[:ns]).max()
    up = qL if fm >= 0.0 else qR
    assert np.allclose(F[:ns], fm * up[:ns] / up[:ns].sum(), rtol=1e-13, atol=0.0)
    # a floor below every wave speed: no change
    assert np.array_equal(o.point_roe(qL, qR, *n, eta=1.0), o.point_roe(qL, qR, *n))


def test_muscl_roe_residual_mirror_symmetry():
    m = I.air5(1)
    ni, nj = 12, 8
    x, y = I.polar_grid(ni, nj)
    fs = (np.array([0.0, 0.0, 0.0, 0.233e-3, 0.767e-3]), 3000.0, 0.0, 300.0, 300.0)
    o = orc.setup((x, y), m, fs)
    o.set_option("residual_scheme", 1)
    rs, u, v, T, Tv = I.random_prims(m, ni * nj, 9, T_range=(400.0, 3000.0), speed=800.0, y_floor=0.02)
    # mirror about the stagnation line: cell (i, j) <-> (ni - 1 - i, j), v -> -v
    idx = np.arange(ni * nj).reshape(nj, ni)
    mir = idx[:, ::-1].ravel()
    half = (idx % ni < ni // 2).ravel()
    rs, u, v, T, Tv = (np.where(half, a, a[..., mir]) for a in (rs, u, v, T, Tv))
    v = np.where(half, v, -v[mir])
    assert np.allclose(y[:, ::-1], -y) and np.allclose(x[:, ::-1], x)
    o.set_state(o.prim_to_cons(rs, u, v, T, Tv))
    o.residual(5.0)
    R = o.get("R")
    Rm = R[:, mir].copy()
    Rm[m.ns + 1] *= -1.0
    scale = np.abs(R).max(axis=1, keepdims=True)
    assert np.all(np.abs(R - Rm) <= 1e-11 * scale)
