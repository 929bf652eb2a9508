"""Pins of the oracle's flux-difference off-diagonal operator (the nonlinear
matrix-free form F(Q_N + x) - F(Q_N) of the neighbour term, the alternative
to the linear Jacobian-vector product of the spectral splitting, paper
Section 2.2):

* homogeneity: the inviscid flux of this gas is homogeneous of degree one in
  the conservative state (scaling every density, momentum and energy by
  1 + a keeps the velocity, the temperatures and the mass fractions, and
  scales the pressure), so for x = a Q_N both forms give exactly a F(Q_N);
* consistency: the flux difference differs from the Jacobian-vector product
  by O(|x|^2) (second-order remainder of the Taylor expansion);
* the sweeps with flux differences approach the linear sweeps as the
  right-hand side is scaled down, with a first-order relative remainder
  (which fixes the sign, the face normal and the neighbour the term is
  evaluated at, since the linear sweeps are pinned by the dense solves)."""
import numpy as np
import pytest

from oracle import orc
from paper_2403_03440_amd import inputs as I


def _z_of_q(m, q):
    """coupled unknowns z = (rho, momenta, energies, rho_1..rho_{ns-1})"""
    ns = m.ns
    return np.concatenate([[q[:ns].sum()], q[ns:], q[:ns - 1]])


@pytest.mark.parametrize("two_temp", [0, 1])
@pytest.mark.parametrize("mode", [0, 1])
def test_flux_difference_homogeneity_and_consistency(two_temp, mode):
    m = I.air5(two_temp)
    o = orc.Oracle()
    o.set_mechanism(m)
    q = o.prim_to_cons(*I.random_prims(m, 1, 5, T_range=(3000.0, 6000.0), speed=2500.0, y_floor=0.02))[:, 0]
    nx, ny = 0.6, -0.8
    F = o.point_flux(q, nx, ny)
    ns = m.ns
    if mode == 0:
        zq = _z_of_q(m, q)
        Fz = _z_of_q(m, F)
    else:
        zq = np.concatenate([[q[:ns].sum()], q[ns:]])
        Fz = np.concatenate([[F[:ns].sum()], F[ns:]])
    for a in (0.3, -0.2):
        for fd in (0, 1):
            out = o.point_offdiag(q, nx, ny, mode, fd, a * zq)
            assert np.abs(out - a * Fz).max() <= 1e-12 * np.abs(a * Fz).max(), (fd, a)
    rng = np.random.default_rng(3)
    d = rng.uniform(-1, 1, zq.size) * np.abs(zq) * 0.01
    rem = []
    for eps in (1.0, 0.1, 0.01):
        lin = o.point_offdiag(q, nx, ny, mode, 0, eps * d)
        fdv = o.point_offdiag(q, nx, ny, mode, 1, eps * d)
        rem.append(np.abs(fdv - lin).max() / np.abs(lin).max())
    # relative remainder O(eps): a factor ~10 per decade
    assert 5.0 <= rem[0] / rem[1] <= 20.0 and 5.0 <= rem[1] / rem[2] <= 20.0, rem


@pytest.mark.parametrize("mode", [0, 1])
def test_flux_difference_sweeps_approach_linear_sweeps(mode):
    m = I.air5(1)
    x, y = I.polar_grid(8, 6)
    Y = np.zeros(m.ns)
    Y[m.ns - 1], Y[m.names.index("O2")] = 0.767, 0.233
    fs = (1e-3 * Y, 5000.0, 0.0, 250.0, 250.0)
    o = orc.setup((x, y), m, fs)
    q = o.prim_to_cons(*I.random_prims(m, 48, 9, T_range=(2000.0, 6000.0), speed=2000.0, y_floor=0.02))
    o.set_state(q)
    o.residual(10.0)
    o.implicit_op(mode)
    b = np.random.default_rng(4).uniform(-1, 1, o.get("dq", mode).shape) * 1e-3
    base = o.sweep_rhs(mode, b)
    rem = []
    o.set_option("flux_diff", 1)
    for eps in (1.0, 0.1, 0.01):
        xf = o.sweep_rhs(mode, eps * b)
        rem.append(np.abs(xf - eps * base).max() / np.abs(eps * base).max())
    o.set_option("flux_diff", 0)
    assert rem[0] > 1e-8     # the operators differ at finite increments
    assert 5.0 <= rem[0] / rem[1] <= 20.0 and 5.0 <= rem[1] / rem[2] <= 20.0, rem
