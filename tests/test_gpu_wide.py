"""The species-generic kernels (one temperature, no reactions, any species
count; the configuration of the paper's species-count study, Section 3.1)
through the C-ABI.

* Blocked Gauss-Jordan inverse (csi_block_inverse): permutation and scaled
  permutation matrices invert exactly (their inverse is exact in FP64 and
  the elimination only moves and scales entries); random matrices across
  panel boundaries (n = 1 ... 300) match numpy's inverse to the bound that
  the condition number sets; a singular matrix is reported by index.
* Against the FP64 oracle (wide build) at 64 and 256 species on the
  far-field box and at 64 species on a wall grid: T, p, c, R, dtau, the wall
  heat flux, both forms' increments (1e-12 normwise, or ten times the
  oracle's own rounding sensitivity, as the compiled path's tests), the
  corrected state and a short iteration.
* Against the compiled kernels on the same case (air at 5 and the seeded
  mechanism at 20 species without reactions): the same numbers to 1e-12.
* At the maximum species count (4096): a mixture of identical copies of
  five-species air gives the compiled five-species increments' flow rows and
  species sums (a property that holds at any size)."""
import numpy as np
import pytest

from gpu_cases import groups_inc, groups_state, normwise, oracle_noise
from oracle import orc
from paper_2403_03440_amd import inputs as I

pytestmark = pytest.mark.gpu

TOL64 = 1e-12


def _csi():
    from paper_2403_03440_amd import csi
    return csi


def _dev(a):
    import torch
    return torch.tensor(a, dtype=torch.float64, device="cuda")


# ------------------------------------------------------------ block inverse
@pytest.mark.parametrize("n", [1, 5, 64, 65, 130, 300])
def test_block_inverse_permutations_exact(n):
    csi = _csi()
    rng = np.random.default_rng(n)
    mats = []
    for _ in range(3):
        P = np.eye(n)[rng.permutation(n)]
        D = np.diag(2.0 ** rng.integers(-6, 7, n))
        mats.append(D @ P)
    A = np.stack(mats)
    X = csi.block_inverse(_dev(A)).cpu().numpy()
    for k in range(3):
        assert np.array_equal(X[k], np.linalg.inv(A[k])), k  # exact: entries are powers of two


@pytest.mark.parametrize("n", [1, 7, 63, 64, 65, 129, 300])
def test_block_inverse_random(n):
    csi = _csi()
    rng = np.random.default_rng(100 + n)
    A = rng.standard_normal((4, n, n))
    A[1] += n * np.eye(n)                 # diagonally dominant
    A[2, :, 0] *= 1e-6                     # small leading column: pivoting needed
    X = csi.block_inverse(_dev(A)).cpu().numpy()
    for k in range(4):
        Xr = np.linalg.inv(A[k])
        cond = np.linalg.cond(A[k])
        err = np.linalg.norm(X[k] - Xr) / np.linalg.norm(Xr)
        assert err <= 1e-14 * n * cond, (k, err, cond)


def test_block_inverse_singular_reported():
    csi = _csi()
    rng = np.random.default_rng(9)
    A = rng.standard_normal((3, 70, 70))
    A[1, :, 5] = 0.0
    with pytest.raises(csi.CsiError, match="CSI_ERR_SINGULAR.*matrix 1"):
        csi.block_inverse(_dev(A))


# ---------------------------------------------------------- against oracle
def _pair(ns, ni, nj, bc_mode, seed):
    csi = _csi()
    m = I.synthetic(ns, 0, 3442)
    if bc_mode == 1:
        x, y = I.box_grid(ni, nj, skew=0.2, seed=seed)
    else:
        x, y = I.polar_grid(ni, nj)
    Y = np.full(ns, 1.0 / ns)
    fs = (1e-3 * Y, 1500.0, 200.0, 400.0, 400.0)
    o = orc.setup((x, y), m, fs, bc_mode=bc_mode)
    prims = I.random_prims(m, ni * nj, seed, T_range=(400.0, 3000.0), speed=800.0, y_floor=0.01)
    q0 = o.prim_to_cons(*prims)
    o.set_state(q0)
    s = csi.Solver((x, y), m, fs, bc_mode=bc_mode)
    s.set_state(q0)
    return m, o, s, q0


WIDE_CASES = [(64, 10, 8, 1), (64, 9, 7, 0), (256, 6, 5, 1)]


@pytest.mark.parametrize("ns,ni,nj,bc_mode", WIDE_CASES)
def test_wide_residual_parity(ns, ni, nj, bc_mode):
    print(f"wide residual ns {ns} {ni}x{nj} bc {bc_mode}", flush=True)
    m, o, s, q0 = _pair(ns, ni, nj, bc_mode, seed=11)
    no = o.residual(20.0)
    ng = s.residual(20.0)
    for f in ("T", "p", "c"):
        assert normwise(s.get(f), o.get(f)).max() <= TOL64, f
    assert np.all(normwise(s.get("R"), o.get("R"), groups_state(m)) <= TOL64 * 10)
    assert normwise(s.get("dtau"), o.get("dtau")).max() <= TOL64
    assert abs(ng[1] - no[1]) <= 1e-12 * no[1]
    if bc_mode == 0:
        qg, _ = s.wall_heat_flux()
        qo, _ = o.wall_heat_flux()
        assert normwise(qg, qo).max() <= TOL64


@pytest.mark.parametrize("ns,ni,nj,bc_mode", WIDE_CASES)
@pytest.mark.parametrize("mode", [0, 1])
def test_wide_implicit_op_parity(ns, ni, nj, bc_mode, mode):
    print(f"wide implicit op ns {ns} {ni}x{nj} bc {bc_mode} mode {mode}", flush=True)
    csi = _csi()
    m, o, s, q0 = _pair(ns, ni, nj, bc_mode, seed=13)
    g = groups_inc(m, mode)
    noise = oracle_noise(o, q0, mode, 50.0, g)
    s.residual(50.0)
    s.implicit_op(mode, csi.FP64)
    tol = np.maximum(TOL64, 10.0 * noise)
    assert np.all(tol <= 1e-9), noise
    e_star = normwise(s.get("dqs", mode), o.get("dqs", mode), g)
    e = normwise(s.get("dq", mode), o.get("dq", mode), g)
    print("err", e.max(), "oracle noise", noise.max(), flush=True)
    assert np.all(e_star <= tol), (e_star, noise)
    assert np.all(e <= tol), (e, noise)


@pytest.mark.parametrize("mode,kind", [(0, 0), (1, 1), (1, 2)])
def test_wide_corrections_and_iterations(mode, kind):
    csi = _csi()
    m, o, s, q0 = _pair(64, 9, 7, 0, seed=17)
    # a small step: at larger ones CC2 clips every species of some cells of
    # this random state and the correction is 0/0 there (in both)
    o.residual(0.5)
    s.residual(0.5)
    o.implicit_op(mode)
    s.implicit_op(mode, csi.FP64)
    o.consistency_correct(mode, kind)
    s.consistency_correct(kind)
    assert np.all(normwise(s.get_state(), o.get_state(), groups_state(m)) <= TOL64)
    # iterations from the perturbed free stream (the random state's jumps
    # between neighbouring cells are not a state to iterate from)
    n = 9 * 7
    fs0 = np.full(m.ns, 1e-3 / m.ns)
    rs = fs0[:, None] * (1.0 + 0.01 * I.uniform_pm1(17, n))[None, :]
    q1 = o.prim_to_cons(np.ascontiguousarray(rs), np.full(n, 1500.0), np.full(n, 200.0), np.full(n, 400.0),
                        np.full(n, 400.0))
    o.set_state(q1)
    s.set_state(q1)
    ho = o.step(mode, kind, 5.0, 6)
    st = s.step(mode, kind, 5.0, 6, check_every=6)
    assert st["iters"] == 6
    assert np.all(normwise(s.get_state(), o.get_state(), groups_state(m)) <= 1e-11)
    hg = s.norm_history(6)
    assert np.allclose(hg[:, 1], ho[:, 1], rtol=1e-10, atol=0.0)


# -------------------------------------------------------- against compiled
@pytest.mark.parametrize("name", ["air5", "syn20"])
def test_wide_matches_compiled_kernels(name):
    csi = _csi()
    m = (I.air5(0) if name == "air5" else I.synthetic(20, 60, 3442)).without_reactions()
    x, y = I.polar_grid(20, 14)
    fs = (np.full(m.ns, 1e-3 / m.ns), 3000.0, 0.0, 300.0, 300.0)
    prims = I.random_prims(m, 20 * 14, 21, T_range=(400.0, 4000.0), speed=900.0, y_floor=0.01)
    sc = csi.Solver((x, y), m, fs)
    sw = csi.Solver((x, y), m, fs, generic=True)
    q0 = sc.initial_state(*prims)
    assert np.array_equal(sw.initial_state(*prims), q0)
    for s in (sc, sw):
        s.set_state(q0)
        s.residual(30.0)
    for f in ("T", "p", "c", "dtau"):
        assert normwise(sw.get(f), sc.get(f)).max() <= TOL64, f
    assert np.all(normwise(sw.get("R"), sc.get("R"), groups_state(m)) <= TOL64)
    for mode in (0, 1):
        for s in (sc, sw):
            s.residual(30.0)
            s.implicit_op(mode, csi.FP64)
        e = normwise(sw.get("dq", mode), sc.get("dq", mode), groups_inc(m, mode))
        print(name, "mode", mode, "err", e.max(), flush=True)
        assert np.all(e <= TOL64), e
    # iterations from the perturbed free stream
    n = 20 * 14
    rs = fs[0][:, None] * (1.0 + 0.01 * I.uniform_pm1(5, n))[None, :]
    q1 = sc.initial_state(np.ascontiguousarray(rs), np.full(n, fs[1]), np.zeros(n), np.full(n, fs[3]),
                          np.full(n, fs[4]))
    for mode, kind in ((0, 0), (1, 2)):
        for s in (sc, sw):
            s.set_state(q1)
            s.step(mode, kind, 5.0, 10, check_every=10)
        assert np.all(normwise(sw.get_state(), sc.get_state(), groups_state(m)) <= 1e-11)


# ------------------------------------------------------ maximum species count
def test_species_copies_at_4096():
    csi = _csi()
    base = I.air5(0).without_reactions()
    ns = csi.WIDE_MAX_SPECIES
    wide = I.species_copies(base, ns)
    ni, nj = 7, 5
    x, y = I.polar_grid(ni, nj)
    fsb = (np.array([0.0, 0.0, 0.0, 0.233e-3, 0.767e-3]), 3000.0, 0.0, 250.0, 250.0)
    fsw = (I.split_among_copies(fsb[0][:, None], base.ns, ns)[:, 0],) + fsb[1:]
    prims = I.random_prims(base, ni * nj, 23, T_range=(400.0, 3000.0), speed=600.0, y_floor=0.02)
    sb = csi.Solver((x, y), base, fsb)
    sw = csi.Solver((x, y), wide, fsw)
    qb = sb.initial_state(*prims)
    qw = sw.initial_state(I.split_among_copies(prims[0], base.ns, ns), *prims[1:])
    sb.set_state(qb)
    sw.set_state(qw)
    sb.residual(10.0)
    sw.residual(10.0)
    for f in ("T", "p", "c", "dtau"):
        assert normwise(sw.get(f), sb.get(f)).max() <= 1e-12, f
    Rb, Rw = sb.get("R"), sw.get("R")
    assert np.all(normwise(Rw[ns:], Rb[base.ns:]) <= 1e-11)
    idx = np.arange(ns) % base.ns
    Rsum = np.stack([Rw[:ns][idx == k].sum(0) for k in range(base.ns)])
    assert normwise(Rsum, Rb[:base.ns], [list(range(base.ns))]).max() <= 1e-11
    for mode in (0, 1):
        for s in (sb, sw):
            s.implicit_op(mode, csi.FP64)
        db, dw = sb.get("dq", mode), sw.get("dq", mode)
        e = normwise(dw[:4], db[:4])
        print("mode", mode, "flow rows", e, flush=True)
        assert np.all(e <= 1e-11)
        if mode == 1:
            dsum = np.stack([dw[4:][idx == k].sum(0) for k in range(base.ns)])
            assert normwise(dsum, db[4:], [list(range(base.ns))]).max() <= 1e-11


# ------------------------------------------------------------------ errors
def test_wide_argument_errors():
    csi = _csi()
    x, y = I.box_grid(4, 3)
    m = I.synthetic(40, 0, 3442)
    fs = (np.full(40, 1e-3 / 40), 500.0, 0.0, 300.0, 300.0)
    with pytest.raises(csi.CsiError, match="CSI_ERR_UNSUPPORTED"):
        csi.Solver((x, y), I.synthetic(40, 10, 3442), fs, bc_mode=1)   # reactions above 32 species
    with pytest.raises(csi.CsiError, match="CSI_ERR_UNSUPPORTED"):
        csi.Solver((x, y), m.with_two_temp(1), fs, bc_mode=1)
    big = I.synthetic(csi.WIDE_MAX_SPECIES + 1, 0, 3442)
    with pytest.raises(csi.CsiError, match="CSI_ERR_ARG"):
        csi.Solver((x, y), big, (np.full(big.ns, 1e-6), 500.0, 0.0, 300.0, 300.0), bc_mode=1)
    s = csi.Solver((x, y), m, fs, bc_mode=1)
    s.set_state(s.initial_state(*I.random_prims(m, 12, 3, T_range=(400.0, 900.0), speed=200.0)))
    s.residual(5.0)
    with pytest.raises(csi.CsiError, match="CSI_ERR_UNSUPPORTED"):
        s.implicit_op(csi.SPLIT, csi.MIXED)
    with pytest.raises(csi.CsiError, match="CSI_ERR_UNSUPPORTED"):
        s.set_sweep(1)
    with pytest.raises(csi.CsiError, match="CSI_ERR_UNSUPPORTED"):
        s.set_physical_time(1e-6, 0.5)
    with pytest.raises(csi.CsiError, match="CSI_ERR_UNSUPPORTED"):
        s.set_offdiag(1)
    s.implicit_op(csi.SPLIT, csi.FP64)  # still usable
    with pytest.raises(csi.CsiError, match="CSI_ERR_UNSUPPORTED"):
        s.get("Dinv", csi.SPLIT)
