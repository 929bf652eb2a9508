"""Pins of the oracle's wide build (room for 256 species per cell), which the
species-count study (paper Section 3.1: non-reacting flow, implicit step
cost as the number of species grows) checks the species-generic kernels
against.

* The wide build is the same arithmetic as the default build: on a
  five-species case both give bitwise equal residuals and increments.
* Species copies: a mixture in which each species of a base mixture is
  split into identical copies sharing its partial density has the same
  temperature, pressure and flow residual, the copies' residual and split
  increments sum to the base species', and the flow rows of both forms'
  increments equal the base mixture's (to rounding).  A dropped species in a
  loop, a wrong stride in the per-species arrays or a limit that truncates at
  32 species breaks these at 64 and 256 species.
* Free-stream preservation at 256 species on the far-field box: the residual
  of the uniform flow is zero to rounding and so is the increment."""
import numpy as np
import pytest

from oracle import orc
from paper_2403_03440_amd import inputs as I


def _state(o, mech, n, seed):
    prims = I.random_prims(mech, n, seed, T_range=(400.0, 3000.0), speed=600.0, y_floor=0.02)
    return o.prim_to_cons(*prims), prims


def _pair_copies(ns, ni=6, nj=5, bc_mode=0, seed=4):
    base = I.air5(0).without_reactions()
    wide = I.species_copies(base, ns)
    x, y = I.polar_grid(ni, nj)
    fs = (np.array([0.0, 0.0, 0.0, 0.233e-3, 0.767e-3]), 3000.0, 0.0, 250.0, 250.0)
    fsw = (I.split_among_copies(fs[0][:, None], base.ns, ns)[:, 0],) + fs[1:]
    ob = orc.setup((x, y), base, fs, bc_mode=bc_mode)
    ow = orc.setup((x, y), wide, fsw, bc_mode=bc_mode)
    n = ni * nj
    prims = I.random_prims(base, n, seed, T_range=(400.0, 3000.0), speed=600.0, y_floor=0.02)
    qb = ob.prim_to_cons(*prims)
    qw = ow.prim_to_cons(I.split_among_copies(prims[0], base.ns, ns), *prims[1:])
    ob.set_state(qb)
    ow.set_state(qw)
    return base, wide, ob, ow


def _copy_sum(a, base_ns, ns):
    out = np.zeros((base_ns,) + a.shape[1:])
    for k in range(ns):
        out[k % base_ns] += a[k]
    return out


def test_wide_build_equals_default_build():
    m = I.air5(0)
    x, y = I.polar_grid(7, 5)
    fs = (np.array([0.0, 0.0, 0.0, 0.233e-3, 0.767e-3]), 3000.0, 0.0, 250.0, 250.0)
    res = []
    for wide in (False, True):
        o = orc.Oracle(wide=wide)
        o.set_grid(x, y)
        o.set_mechanism(m)
        o.set_freestream(*fs)
        q, _ = _state(o, m, 35, 2)
        o.set_state(q)
        o.residual(10.0)
        o.implicit_op(orc.COUPLED)
        dk = o.get("dq", orc.COUPLED)
        o.implicit_op(orc.SPLIT)
        res.append((o.get("R"), dk, o.get("dq", orc.SPLIT)))
    for a, b in zip(*res):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("ns", [64, 256])
def test_species_copies_leave_the_flow_unchanged(ns):
    base, wide, ob, ow = _pair_copies(ns)
    rb, rw = ob.residual(10.0), ow.residual(10.0)
    for f in ("T", "p", "c", "dtau"):
        assert np.allclose(ow.get(f), ob.get(f), rtol=1e-13, atol=0.0), f
    Rb, Rw = ob.get("R"), ow.get("R")
    nb_, nw = base.ns, wide.ns
    scale = np.abs(Rb).max(axis=1, keepdims=True)
    # flow rows (momenta, energy) and the copies' sums of the species rows
    assert np.all(np.abs(Rw[nw:] - Rb[nb_:]) <= 1e-12 * scale[nb_:])
    dens = np.abs(Rb[:nb_]).max()
    assert np.all(np.abs(_copy_sum(Rw[:nw], nb_, nw) - Rb[:nb_]) <= 1e-12 * dens)
    assert abs(rw[1] - rb[1]) <= 1e-12 * rb[1]
    for mode in (orc.COUPLED, orc.SPLIT):
        ob.implicit_op(mode)
        ow.implicit_op(mode)
        db, dw = ob.get("dq", mode), ow.get("dq", mode)
        sc = np.abs(db[:4]).max(axis=1)
        assert np.all(np.abs(dw[:4] - db[:4]).max(axis=1) <= 1e-11 * sc), mode
        if mode == orc.SPLIT:
            ds = np.abs(db[4:]).max()
            assert np.all(np.abs(_copy_sum(dw[4:], nb_, nw) - db[4:]) <= 1e-11 * ds)


def test_free_stream_preserved_at_256_species():
    m = I.synthetic(256, 0, 3442)
    x, y = I.box_grid(5, 4)
    Y = np.full(m.ns, 1.0 / m.ns)
    fs = (1e-3 * Y, 800.0, 150.0, 600.0, 600.0)
    o = orc.setup((x, y), m, fs, bc_mode=1)
    n = 20
    q = o.prim_to_cons(np.repeat(fs[0][:, None], n, 1), np.full(n, fs[1]), np.full(n, fs[2]), np.full(n, fs[3]),
                       np.full(n, fs[4]))
    o.set_state(q)
    o.residual(10.0)
    R = o.get("R")
    flux_scale = 1e-3 * 800.0 * 0.01  # rho u times a face length
    assert np.abs(R).max() <= 1e-12 * flux_scale
    for mode in (orc.COUPLED, orc.SPLIT):
        o.implicit_op(mode)
        assert np.abs(o.get("dq", mode)).max() <= 1e-12 * np.abs(q).max()
