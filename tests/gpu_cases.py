"""Shared set-up of oracle/HIP pairs for the GPU parity tests."""
import numpy as np

from oracle import orc
from paper_2403_03440_amd import inputs as I


def mech_by_name(name):
    return {
        "air5_1T": lambda: I.air5(0),
        "air5_2T": lambda: I.air5(1),
        "air11_2T": lambda: I.air11(1),
        "air11_1T": lambda: I.air11(0),
        "toy2_1T": lambda: I.toy_dissociation(0),
        "toy3_2T": lambda: I.toy3(1),
        "toy3_1T": lambda: I.toy3(0),
        "syn20_1T": lambda: I.synthetic(20, 60, 3442),
        "syn16_1T": lambda: I.synthetic(16, 40, 3443),
        # 40 reactions: with 60 (seed 3444) the split blocks at CFL 10 are stiff
        # enough that two correct FP64 inversions differ by ~4x the FP64 bar
        "syn32_1T": lambda: I.synthetic(32, 40, 3443),
    }[name]()


def freestream(mech, u=5000.0, T=250.0, rho=1e-3):
    """Major species (the last one, which closes the coupled system) 0.767,
    O2 (or the first other molecule) 0.233."""
    Y = np.zeros(mech.ns)
    names = list(mech.names)
    Y[mech.ns - 1] = 0.767
    if "O2" in names:
        Y[names.index("O2")] = 0.233
    else:
        other = [k for k in range(mech.ns - 1) if mech.kind[k] == I.MOLECULE] or [0]
        Y[other[0]] = 0.233
    return (rho * Y, u, 0.0, T, T)


def oracle_noise(o, q0, mode, cfl, groups, n=3, eps=4e-16, seed=0, levels=None):
    """Sensitivity of the oracle's own increment to rounding-level relative
    perturbations of its input state: the noise floor of the comparison.
    levels: physical-time levels (Q^n, Q^{n-1}) to restore after each
    set_state (dual time stepping)."""
    rng = np.random.default_rng(seed)

    def put(q):
        o.set_state(q)
        if levels is not None:
            o.set_time_levels(*levels)

    put(q0)
    o.residual(cfl)
    o.implicit_op(mode)
    d0 = o.get("dq", mode)
    worst = np.zeros(d0.shape[0])
    for _ in range(n):
        put(q0 * (1.0 + eps * rng.uniform(-1.0, 1.0, q0.shape)))
        o.residual(cfl)
        o.implicit_op(mode)
        worst = np.maximum(worst, normwise(o.get("dq", mode), d0, groups))
    put(q0)
    o.residual(cfl)
    o.implicit_op(mode)
    return worst


def make_pair_evolved(name, ni, nj, iters=40):
    """(mechanism, oracle, HIP solver, state) on an oracle-evolved state."""
    m = mech_by_name(name)
    o, s, q0 = pair(m, ni, nj, state="evolved", mech_name=name, iters=iters)
    return m, o, s, q0


_EVOLVED = {}


def evolved_state(mech_name, mech, ni, nj, iters, u=5000.0, mode=1, kind=2):
    """A physical state with a shock layer and active chemistry: the oracle's
    own iterations from the uniform free stream (CFL ramp 1 -> 10)."""
    key = (mech_name, ni, nj, iters, u)
    if key not in _EVOLVED:
        x, y = I.polar_grid(ni, nj)
        fs = freestream(mech, u=u)
        o = orc.setup((x, y), mech, fs)
        n = ni * nj
        q = o.prim_to_cons(np.repeat(fs[0][:, None], n, 1), np.full(n, fs[1]), np.zeros(n), np.full(n, fs[3]),
                           np.full(n, fs[4]))
        o.set_state(q)
        o.step(mode, kind, 3.0, iters, ramp=iters)
        _EVOLVED[key] = o.get_state()
    return _EVOLVED[key].copy()


def pair(mech, ni, nj, seed=1, state="random", bc_mode=0, grid=None, T_range=(500.0, 9000.0), speed=3000.0,
         mech_name=None, iters=40, u=5000.0):
    """Oracle and HIP solver on the same grid, mechanism, free stream and state.
    state: "random" (seeded primitives), "freestream" (+-1 % density) or
    "evolved" (oracle iterations from the free stream)."""
    from paper_2403_03440_amd import csi
    x, y = grid if grid is not None else I.polar_grid(ni, nj)
    fs = freestream(mech, u=u)
    o = orc.setup((x, y), mech, fs, bc_mode=bc_mode)
    n = ni * nj
    if state == "evolved":
        q0 = evolved_state(mech_name, mech, ni, nj, iters, u=u)
        o.set_state(q0)
        s = csi.Solver((x, y), mech, fs, bc_mode=bc_mode)
        s.set_state(q0)
        return o, s, q0
    if state == "random":
        prims = I.random_prims(mech, n, seed, T_range=T_range, speed=speed, y_floor=0.01)
    else:
        cfg = I.Config("t", ni, nj, "air5", mech.two_temp, 10.0, fs[1], perturb=0.01, seed=seed)
        rs = np.repeat(fs[0][:, None], n, 1) * (1.0 + 0.01 * I.uniform_pm1(seed, n))[None, :]
        prims = (rs, np.full(n, fs[1]), np.zeros(n), np.full(n, fs[3]), np.full(n, fs[4]))
    q0 = o.prim_to_cons(*prims)
    o.set_state(q0)
    s = csi.Solver((x, y), mech, fs, bc_mode=bc_mode)
    s.set_state(q0)
    return o, s, q0


def normwise(a, b, groups=None):
    """max over cells |a - b| / max over cells |b|, per leading variable.
    groups: list of row-index lists sharing units; a row's scale is then the
    largest over its group (rows that are identically zero in the reference,
    e.g. species absent from the free stream, are measured against the
    density scale rather than against their own rounding noise)."""
    a = np.atleast_2d(a)
    b = np.atleast_2d(b)
    scale = np.abs(b).max(axis=-1)
    if groups:
        sc = scale.copy()
        for g in groups:
            sc[g] = scale[g].max()
        scale = sc
    err = np.abs(a - b).max(axis=-1)
    return np.where(scale > 0, err / np.where(scale > 0, scale, 1.0), err)


def groups_state(m):
    """unit groups of the stored variables: densities | momenta | energies"""
    ns = m.ns
    g = [list(range(ns)), [ns, ns + 1], [ns + 2] + ([ns + 3] if m.two_temp else [])]
    return g


def groups_inc(m, mode):
    """unit groups of the increments (coupled z or split layout)"""
    nf = m.nf
    n = m.nb if mode == 0 else nf + m.ns
    dens = [0] + list(range(nf, n))
    return [dens, [1, 2], [3] + ([4] if m.two_temp else [])]


def sample_cells(N, n, seed):
    """The cells of csi_sample_jacobians' rows, from the definition in csi.h:
    every cell in order when n >= N, else row r is cell (b + r a) mod N with
    b = splitmix64(seed) mod N and a the first value coprime with N from
    1 + splitmix64(seed + 1) mod (N - 1) upwards, wrapping within [1, N - 1]."""
    if n >= N:
        return np.arange(N)
    if N <= 1:
        return np.zeros(n, dtype=np.int64)
    mask = (1 << 64) - 1

    def splitmix64(x):
        z = (x + 0x9E3779B97F4A7C15) & mask
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & mask
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & mask
        return z ^ (z >> 31)

    b = splitmix64(seed & mask) % N
    a = 1 + splitmix64((seed + 1) & mask) % (N - 1)
    while np.gcd(a, N) != 1:
        a = a % (N - 1) + 1
    return np.array([(b + r * a) % N for r in range(n)], dtype=np.int64)
