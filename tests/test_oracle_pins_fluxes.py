"""Pins of the oracle's face fluxes, wall heat flux, vibrational source and
CC1 weights against closed forms that do not come from the oracle:

* the diamond face gradient is exact for linear fields on a skewed (affine)
  grid, so the viscous flux of the constitutive laws (paper Section 2.1:
  Newtonian stress, Fourier conduction in each energy pool, Fick diffusion
  with the mass-conserving correction, the enthalpy carried by diffusion)
  can be written out here from the exact gradients;
* on a straight isothermal wall a linear temperature profile gives the heat
  flux k (T_1 - T_w) / d with d the wall distance of the first cell centre;
* the HLLE flux equals the physical flux of the upwind state for supersonic
  states, the HLL average otherwise, and its species flux is the mass flux
  times the upwind mass fractions;
* the vibrational-energy source is Landau-Teller relaxation with the
  Millikan-White relaxation time (Millikan & White, J. Chem. Phys. 39, 3209,
  1963) plus the energy carried by created species; a 0-D relaxation at fixed
  total energy drives Tv to T monotonically and ends at the one-temperature
  equilibrium of the same energy;
* CC1 (paper Section 2.3, consistence correction) with no species increment
  scales every partial density by the same factor (the weights are the mass
  fractions).

Transport and thermodynamic closures used below are the textbook ones the
oracle's readings name: a power-law mixture viscosity, Eucken conductivities
(15/4 R for atoms, 19/4 R for linear molecules in the translational-rotational
pool, c_v,vib in the vibrational pool), Schmidt-number diffusivities and
harmonic-oscillator vibrational energies."""
import numpy as np
import pytest

from oracle import orc
from paper_2403_03440_amd import inputs as I


# ------------------------------------------------------ textbook closures
def mu_law(m, T):
    return m.mu_ref * (np.asarray(T) / m.T_ref) ** m.mu_exp


def R_s(m):
    return I.R_U / m.M


def e_vib(m, s, T):
    th = m.theta_v[s]
    if m.kind[s] == I.ELECTRON:
        return 1.5 * R_s(m)[s] * T
    if m.kind[s] != I.MOLECULE or th <= 0:
        return 0.0
    return R_s(m)[s] * th / np.expm1(th / T)


def cv_vib(m, s, T):
    th = m.theta_v[s]
    if m.kind[s] == I.ELECTRON:
        return 1.5 * R_s(m)[s]
    if m.kind[s] != I.MOLECULE or th <= 0:
        return 0.0
    x = th / T
    return R_s(m)[s] * x * x * np.exp(x) / np.expm1(x) ** 2


def cv_tr(m, s):
    return {I.ATOM: 1.5, I.MOLECULE: 2.5, I.ELECTRON: 0.0}[int(m.kind[s])] * R_s(m)[s]


def eucken_tr(m, s):
    return {I.ATOM: 15.0 / 4.0, I.MOLECULE: 19.0 / 4.0, I.ELECTRON: 0.0}[int(m.kind[s])] * R_s(m)[s]


def h_species(m, s, T, Tv):
    Tp = Tv if m.kind[s] == I.ELECTRON else T
    return cv_tr(m, s) * T + e_vib(m, s, Tv) + m.h_form[s] / m.M[s] + R_s(m)[s] * Tp


def conductivities(m, T, Tv, Y):
    """(k_tr, k_ve) in two temperatures; (k, 0) with every internal mode in one pool in one temperature."""
    mu = mu_law(m, T)
    ktr = mu * sum(Y[s] * eucken_tr(m, s) for s in range(m.ns))
    kve = mu * sum(Y[s] * cv_vib(m, s, Tv if m.two_temp else T) for s in range(m.ns))
    return (ktr, kve) if m.two_temp else (ktr + kve, 0.0)


# ------------------------------------------------------------------ grids
def affine_grid(ni, nj, dx=1.0e-3, dy=0.8e-3, skew=0.45e-3):
    """Parallelogram cells (non-orthogonal): node (I, J) at (I dx + J skew, J dy);
    the wall J = 0 is the straight line y = 0."""
    J, Ii = np.meshgrid(np.arange(nj + 1, dtype=float), np.arange(ni + 1, dtype=float), indexing="ij")
    return np.ascontiguousarray(Ii * dx + J * skew), np.ascontiguousarray(J * dy)


def centres(x, y):
    xc = 0.25 * (x[:-1, :-1] + x[:-1, 1:] + x[1:, :-1] + x[1:, 1:])
    yc = 0.25 * (y[:-1, :-1] + y[:-1, 1:] + y[1:, :-1] + y[1:, 1:])
    return xc.ravel(), yc.ravel()


def freestream(m):
    Y = np.zeros(m.ns)
    Y[m.names.index("N2")] = 0.767
    Y[m.names.index("O2")] = 0.233
    return (1e-3 * Y, 3000.0, 0.0, 300.0, 300.0)


# -------------------------------------------------------- viscous fluxes
LIN = {"u": (800.0, 3.0e4, -2.0e4), "v": (-300.0, 1.0e4, 2.5e4), "T": (2000.0, 5.0e4, 8.0e4),
       "Tv": (1800.0, -2.0e4, 6.0e4)}


def linear_fields(m, xc, yc):
    f = {k: a + b * xc + c * yc for k, (a, b, c) in LIN.items()}
    if not m.two_temp:
        f["Tv"] = f["T"]
    # mass fractions: a base composition plus gradients that sum to zero
    names = list(m.names)
    Y0 = np.full(m.ns, 0.02)
    Y0[names.index("N2")] = 0.6
    Y0 /= Y0.sum()
    gY = np.zeros((m.ns, 2))
    gY[names.index("O"), :] = (4.0, -3.0)
    gY[names.index("NO"), :] = (-2.0, 5.0)
    gY[names.index("N2"), :] = -gY.sum(0)
    Y = Y0[:, None] + gY[:, :1] * xc[None, :] + gY[:, 1:] * yc[None, :]
    assert Y.min() > 0
    return f, Y, gY


def expected_viscous_flux(m, L, R, nx, ny, f, Y, gY):
    """F_vis . n at the face between cells L and R from the exact gradients
    and the face averages of the cell values (paper Section 2.1)."""
    ns = m.ns
    av = lambda a: 0.5 * (a[L] + a[R])
    gu = LIN["u"][1:]
    gv = LIN["v"][1:]
    gT = LIN["T"][1:]
    gTv = LIN["Tv"][1:] if m.two_temp else gT
    mu = 0.5 * (mu_law(m, f["T"][L]) + mu_law(m, f["T"][R]))
    kl = conductivities(m, f["T"][L], f["Tv"][L], Y[:, L])
    kr = conductivities(m, f["T"][R], f["Tv"][R], Y[:, R])
    k = 0.5 * (kl[0] + kr[0])
    kve = 0.5 * (kl[1] + kr[1])
    div = gu[0] + gv[1]
    txx = mu * (2 * gu[0] - 2.0 / 3.0 * div)
    tyy = mu * (2 * gv[1] - 2.0 / 3.0 * div)
    txy = mu * (gu[1] + gv[0])
    rhoD = mu / m.sc                      # mu and Sc: the face's rho D_s is the mean of the cells' mu/Sc
    Yf = av(Y.T)
    corr = (rhoD[:, None] * gY).sum(0)
    Jn = np.array([(-rhoD[s] * gY[s] + Yf[s] * corr) @ (nx, ny) for s in range(ns)])
    tn = np.array([txx * nx + txy * ny, txy * nx + tyy * ny])
    uf, vf = av(f["u"]), av(f["v"])
    qtr = -k * (gT[0] * nx + gT[1] * ny)
    qve = -kve * (gTv[0] * nx + gTv[1] * ny)
    hf = np.array([0.5 * (h_species(m, s, f["T"][L], f["Tv"][L]) + h_species(m, s, f["T"][R], f["Tv"][R]))
                   for s in range(ns)])
    ef = np.array([0.5 * (e_vib(m, s, f["Tv"][L]) + e_vib(m, s, f["Tv"][R])) for s in range(ns)])
    F = np.zeros(m.nv)
    F[:ns] = Jn
    F[ns] = -tn[0]
    F[ns + 1] = -tn[1]
    F[ns + 2] = -(uf * tn[0] + vf * tn[1]) + qtr + qve + hf @ Jn
    if m.two_temp:
        F[ns + 3] = qve + ef @ Jn
    return F


@pytest.mark.parametrize("two_temp", [0, 1])
def test_viscous_flux_exact_for_linear_fields(two_temp):
    """Interior faces whose diamond has only interior nodes: the oracle's
    viscous flux equals the constitutive laws evaluated with the exact
    gradients of linear u, v, T, Tv and Y fields on a non-orthogonal grid."""
    m = I.air5(two_temp).without_reactions()
    ni, nj = 7, 6
    x, y = affine_grid(ni, nj)
    o = orc.setup((x, y), m, freestream(m), bc_mode=1)
    xc, yc = centres(x, y)
    f, Y, gY = linear_fields(m, xc, yc)
    rho = 0.01
    o.set_state(o.prim_to_cons(rho * Y, f["u"], f["v"], f["T"], f["Tv"]))
    o.residual(1.0)
    FvI = o.get("FvI")
    FvJ = o.get("FvJ")
    # face normals of the affine grid (unit, towards increasing index)
    ti = np.array([0.45e-3, 0.8e-3])
    nI = np.array([ti[1], -ti[0]]) / np.hypot(*ti)
    nJ = np.array([0.0, 1.0])
    checked = 0
    for j in range(1, nj - 1):
        for Iface in range(1, ni):
            L, R = j * ni + Iface - 1, j * ni + Iface
            exp = expected_viscous_flux(m, L, R, nI[0], nI[1], f, Y, gY)
            got = FvI[:, j * (ni + 1) + Iface]
            scale = np.abs(exp).max()
            assert np.allclose(got, exp, rtol=0, atol=1e-11 * scale), (j, Iface, got - exp)
            checked += 1
    for J in range(1, nj):
        for i in range(1, ni - 1):
            L, R = (J - 1) * ni + i, J * ni + i
            exp = expected_viscous_flux(m, L, R, nJ[0], nJ[1], f, Y, gY)
            got = FvJ[:, J * ni + i]
            assert np.allclose(got, exp, rtol=0, atol=1e-11 * np.abs(exp).max()), (J, i, got - exp)
            checked += 1
    assert checked > 40


@pytest.mark.parametrize("two_temp", [0, 1])
def test_wall_heat_flux_linear_profile(two_temp):
    """Straight isothermal wall, skewed cells, T = T_w + a y (and Tv = T_w + b y):
    q_w = k_tr (T_1 - T_w)/d + k_ve (Tv_1 - T_w)/d with the conductivities at
    the wall temperature and the first cell's composition, d = the normal
    distance of the first cell centre from the wall; with u = c y the wall
    shear stress is mu(T_w) c."""
    m = I.air5(two_temp).without_reactions()
    ni, nj = 6, 4
    x, y = affine_grid(ni, nj)
    Tw = 300.0
    o = orc.setup((x, y), m, freestream(m), T_wall=Tw, bc_mode=0)
    xc, yc = centres(x, y)
    a, b = 2.0e6, 1.4e6
    T = Tw + a * yc
    Tv = Tw + b * yc if two_temp else T
    Y = np.zeros((m.ns, xc.size))
    Y[m.names.index("N2")] = 0.7
    Y[m.names.index("O2")] = 0.2
    Y[m.names.index("O")] = 0.1
    shear = 3.0e5                           # Couette profile u = shear * y (no slip at the wall)
    o.set_state(o.prim_to_cons(0.01 * Y, shear * yc, np.zeros_like(xc), T, Tv))
    o.residual(1.0)
    qw, qs = o.wall_heat_flux()
    d = 0.5 * 0.8e-3
    ktr, kve = conductivities(m, Tw, Tw, Y[:, 0])
    expect = ktr * (T[0] - Tw) / d + kve * (Tv[0] - Tw) / d
    assert np.allclose(qw, expect, rtol=1e-12)
    assert abs(qs - expect) <= 1e-12 * expect
    # wall shear stress mu(T_w) du/dy: the x-momentum flux through the wall face (normal +y)
    FvJ = o.get("FvJ")
    assert np.allclose(FvJ[m.ns, :ni], -mu_law(m, Tw) * shear, rtol=1e-12)
    # the distance is the normal one, not the centre-to-face-midpoint distance
    dm = np.hypot(0.5 * 0.45e-3, d)
    assert abs(ktr * (T[0] - Tw) / dm + kve * (Tv[0] - Tw) / dm - expect) > 1e-3 * expect


# ------------------------------------------------------------------- HLLE
def phys_flux(m, rs, u, v, T, Tv, p, rhoE, rhoeve, nx, ny):
    rho = rs.sum()
    un = u * nx + v * ny
    F = np.zeros(m.nv)
    F[:m.ns] = rs * un
    F[m.ns] = rho * u * un + p * nx
    F[m.ns + 1] = rho * v * un + p * ny
    F[m.ns + 2] = (rhoE + p) * un
    if m.two_temp:
        F[m.ns + 3] = rhoeve * un
    return F


def _state(o, m, rs, u, v, T, Tv):
    q = o.prim_to_cons(rs[:, None], np.array([u]), np.array([v]), np.array([T]), np.array([Tv]))[:, 0]
    Tq, Tvq, p, c = o.point_prim(q)
    return q, p, c


@pytest.mark.parametrize("two_temp", [0, 1])
def test_hlle_supersonic_and_subsonic(two_temp):
    m = I.air5(two_temp)
    o = orc.Oracle()
    o.set_mechanism(m)
    nx, ny = 0.6, 0.8
    YL = np.array([0.2, 0.05, 0.03, 0.02, 0.7])
    YR = np.array([0.1, 0.1, 0.1, 0.1, 0.6])
    cases = [
        # (uL, TL, rhoL, uR, TR, rhoR): normal speeds of several sound speeds to
        # either side, then subsonic with a positive and a negative mass flux
        (6000.0, 400.0, 0.01, 5500.0, 500.0, 0.004),
        (-6000.0, 400.0, 0.01, -5800.0, 450.0, 0.004),
        (300.0, 3000.0, 0.01, 150.0, 2500.0, 0.004),
        (-200.0, 3000.0, 0.004, -400.0, 2000.0, 0.01),
    ]
    signs = []
    for k, (uL, TL, rhoL, uR, TR, rhoR) in enumerate(cases):
        rsL, rsR = rhoL * YL, rhoR * YR
        qL, pL, cL = _state(o, m, rsL, uL * nx, uL * ny, TL, 0.9 * TL if two_temp else TL)
        qR, pR, cR = _state(o, m, rsR, uR * nx, uR * ny, TR, 1.1 * TR if two_temp else TR)
        ns = m.ns
        FL = phys_flux(m, rsL, uL * nx, uL * ny, TL, 0, pL, qL[ns + 2], qL[ns + 3] if two_temp else 0, nx, ny)
        FR = phys_flux(m, rsR, uR * nx, uR * ny, TR, 0, pR, qR[ns + 2], qR[ns + 3] if two_temp else 0, nx, ny)
        F = o.point_hlle(qL, qR, nx, ny)
        SL = min(uL - cL, uR - cR)
        SR = max(uL + cL, uR + cR)
        tol = 1e-14 * np.abs(np.r_[FL, FR]).max()
        if SL >= 0:
            assert k == 0
            assert np.allclose(F, FL, rtol=1e-14, atol=tol)
        elif SR <= 0:
            assert k == 1
            assert np.allclose(F, FR, rtol=1e-14, atol=tol)
        else:
            assert k >= 2
            sl, sr = min(SL, 0.0), max(SR, 0.0)
            hll = lambda fl, fr, a, b: (sr * fl - sl * fr + sr * sl * (b - a)) / (sr - sl)
            fmass = hll(FL[:ns].sum(), FR[:ns].sum(), rsL.sum(), rsR.sum())
            for kk in range(ns, ns + 3):
                assert abs(F[kk] - hll(FL[kk], FR[kk], qL[kk], qR[kk])) <= 1e-13 * abs(F[kk]) + tol
            signs.append(np.sign(fmass))
            up_Y, up_q = (YL, qL) if fmass >= 0 else (YR, qR)
            assert np.allclose(F[:ns], fmass * up_Y, rtol=1e-13, atol=tol)
            if two_temp:
                eve_up = up_q[ns + 3] / up_q[:ns].sum()
                assert abs(F[ns + 3] - fmass * eve_up) <= 1e-13 * abs(F[ns + 3]) + tol
    assert signs == [1.0, -1.0]  # one subsonic case of each mass-flux sign


def test_hlle_consistency():
    """F(q, q) = physical flux of q (consistency of the numerical flux)."""
    m = I.air11(1)
    o = orc.Oracle()
    o.set_mechanism(m)
    q = o.prim_to_cons(*I.random_prims(m, 4, seed=31, T_range=(500.0, 9000.0), y_floor=0.01))
    for k in range(4):
        F = o.point_hlle(q[:, k], q[:, k], 0.28, -0.96)
        Fp = o.point_flux(q[:, k], 0.28, -0.96)
        assert np.allclose(F, Fp, rtol=1e-13, atol=1e-13 * np.abs(Fp).max())


# ---------------------------------------------------- vibrational source
ATM = 101325.0


def tau_mw(m, s, T, p):
    """Millikan-White relaxation time (s) for collisions of species s with itself:
    p tau = exp(A (T^-1/3 - B) - 18.42) atm s, A = 1.16e-3 mu^1/2 theta^4/3,
    B = 0.015 mu^1/4, mu the reduced mass in amu."""
    mu = 0.5 * m.M[s] * 1e3
    A = 1.16e-3 * np.sqrt(mu) * m.theta_v[s] ** (4.0 / 3.0)
    B = 0.015 * mu ** 0.25
    return np.exp(A * (T ** (-1.0 / 3.0) - B) - 18.42) / (p / ATM)


def test_omega_ve_landau_teller_millikan_white():
    m = I.air5(1).without_reactions()
    o = orc.Oracle()
    o.set_mechanism(m)
    names = list(m.names)
    for comp in ({"N2": 1.0}, {"N2": 0.7, "O2": 0.2, "O": 0.1}):
        rs = np.zeros(m.ns)
        for n, y in comp.items():
            rs[names.index(n)] = 0.02 * y
        for T, Tv in ((3000.0, 1000.0), (1500.0, 6000.0), (8000.0, 7990.0)):
            om, ov = o.point_production(rs, T, Tv)
            assert np.all(om == 0.0)
            p = sum(rs[s] * R_s(m)[s] * T for s in range(m.ns))
            expect = sum(rs[s] * (e_vib(m, s, T) - e_vib(m, s, Tv)) / tau_mw(m, s, T, p)
                         for s in range(m.ns) if m.kind[s] == I.MOLECULE)
            assert abs(ov - expect) <= 1e-12 * abs(expect)
            assert np.sign(ov) == np.sign(T - Tv)


def test_omega_ve_created_species_term():
    """At T = Tv the relaxation vanishes and omega_ve is the vibrational energy
    carried by the species the reactions create and destroy."""
    m = I.air5(1)
    o = orc.Oracle()
    o.set_mechanism(m)
    rs = np.array([0.2, 0.05, 0.05, 0.05, 0.65]) * 0.01
    for T in (4000.0, 7000.0):
        om, ov = o.point_production(rs, T, T)
        expect = sum(om[s] * e_vib(m, s, T) for s in range(m.ns))
        scale = sum(abs(om[s] * e_vib(m, s, T)) for s in range(m.ns))
        assert abs(ov - expect) <= 1e-13 * scale


def test_vibrational_relaxation_0d():
    """Frozen chemistry, fixed total energy: d(rho e_ve)/dt = omega_ve drives Tv
    to T monotonically (from either side) and ends at the temperature the
    one-temperature model gives for the same total energy."""
    from scipy.integrate import solve_ivp
    m2 = I.air5(1).without_reactions()
    m1 = I.air5(0).without_reactions()
    o2 = orc.Oracle()
    o2.set_mechanism(m2)
    o1 = orc.Oracle()
    o1.set_mechanism(m1)
    ns = m2.ns
    rs = np.array([0.233, 0.0, 0.0, 0.0, 0.767]) * 0.02
    for T0, Tv0 in ((4000.0, 300.0), (900.0, 3000.0)):
        q = o2.prim_to_cons(rs[:, None], np.zeros(1), np.zeros(1), np.array([T0]), np.array([Tv0]))[:, 0]

        def rhs(t, y):
            qq = q.copy()
            qq[ns + 3] = y[0]
            T, Tv, p, c = o2.point_prim(qq)
            return [o2.point_production(rs, T, Tv)[1]]

        T_, Tv_, p0, _ = o2.point_prim(q)
        t_end = 50.0 * tau_mw(m2, ns - 1, min(T0, Tv0), p0)
        sol = solve_ivp(rhs, (0.0, t_end), [q[ns + 3]], method="LSODA", rtol=1e-10, atol=1e-12 * q[ns + 3],
                        dense_output=True)
        assert sol.success
        gaps = []
        for t in np.linspace(0.0, t_end, 200):
            qq = q.copy()
            qq[ns + 3] = sol.sol(t)[0]
            T, Tv, _, _ = o2.point_prim(qq)
            gaps.append(T - Tv)
        gaps = np.array(gaps)
        assert np.all(np.sign(gaps[:-1]) == np.sign(T0 - Tv0)) or np.all(np.abs(gaps[-20:]) < 1e-6 * T0)
        assert np.all(np.diff(np.abs(gaps)) <= 1e-9 * T0)          # monotone approach
        q1 = np.r_[q[:ns + 3]]
        Teq = o1.point_prim(q1)[0]                                 # same total energy, one temperature
        qq = q.copy()
        qq[ns + 3] = sol.y[0, -1]
        T, Tv, _, _ = o2.point_prim(qq)
        assert abs(T - Teq) <= 1e-6 * Teq and abs(Tv - Teq) <= 1e-6 * Teq


# ----------------------------------------------------------------- CC1
@pytest.mark.parametrize("kind", [orc.CC1, orc.CC2])
def test_cc1_weights_are_mass_fractions(kind):
    """No species increment and a total-density increment: CC1 (and CC2)
    leave every mass fraction unchanged and give the flow part's density.
    Weights other than Y_s (e.g. 1/ns, or the increments' own share) would
    change the composition."""
    m = I.air5(0).without_reactions()
    x, y = I.polar_grid(4, 3)
    o = orc.setup((x, y), m, freestream(m))
    rs, u, v, T, Tv = I.random_prims(m, 12, seed=17, T_range=(800.0, 3000.0), y_floor=0.02)
    q0 = o.prim_to_cons(rs, u, v, T, Tv)
    o.set_state(q0)
    o.residual(0.5)
    nsol = m.nf + m.ns
    b = np.zeros((nsol, o.N))
    rng = np.random.default_rng(5)
    b[0] = rng.uniform(0.5, 1.0, o.N) * 1e-3 * np.abs(o.get("DF")[0, 0]) * q0[:m.ns].sum(0)
    dq = o.sweep_rhs(orc.SPLIT, b)
    assert np.all(dq[m.nf:] == 0.0) and np.all(dq[0] != 0.0)
    o.consistency_correct(orc.SPLIT, kind)
    q1 = o.get_state()
    rho0, rho1 = q0[:m.ns].sum(0), q1[:m.ns].sum(0)
    assert np.abs(rho1 / (rho0 + dq[0]) - 1.0).max() <= 4e-16
    assert np.abs(q1[:m.ns] / rho1 - q0[:m.ns] / rho0).max() <= 4e-16
    assert np.abs(dq[0] / rho0).max() > 1e-4    # the density did change


# ------------------------------------ species block at fixed internal energy
@pytest.mark.parametrize("name", ["air5_1T", "syn20_1T", "air5_2T"])
def test_species_jacobian_fixed_internal_energy(name):
    """The split species block's second reading (velocities and the internal
    and vibrational energy densities held, the temperatures following the
    composition) equals the fixed-temperature Jacobian plus the chain rule
    through the energies, written out here: dT/d rho_r = -(e_r - e_ve,r) /
    (rho c_v,tr) and dTv/d rho_r = -e_ve,r / (rho c_v,ve) in two temperatures,
    dT/d rho_r = -e_r / (rho c_v) in one; every derivative of the production
    rates by central differences of the point rates.  The third reading (two
    temperatures: Tv held as well) gives dT/d rho_r = -e_r / (rho c_v,tr)."""
    m = {"air5_1T": lambda: I.air5(0), "syn20_1T": lambda: I.synthetic(20, 60, 3442),
         "air5_2T": lambda: I.air5(1)}[name]()
    x, y = I.polar_grid(4, 3)
    Y = np.zeros(m.ns)
    Y[m.ns - 1], Y[0] = 0.767, 0.233
    o = orc.setup((x, y), m, (1e-3 * Y, 5000.0, 0.0, 250.0, 250.0))
    q = o.prim_to_cons(*I.random_prims(m, 12, 11, T_range=(2500.0, 7000.0), speed=3000.0, y_floor=0.01))
    o.set_state(q)
    JC3s = None
    if m.two_temp:
        o.set_option("jc_fixed_qf", 3)
        o.residual(10.0)
        JC3s = o.get("JC")
    o.set_option("jc_fixed_qf", 2)
    o.residual(10.0)
    JC = o.get("JC")
    T, Tv = o.get("T"), o.get("Tv")
    ns = m.ns
    for p in (0, 5, 11):
        rs = q[:ns, p].copy()
        Tp, Tvp = T[p], Tv[p] if m.two_temp else T[p]
        om = lambda r, t, tv: o.point_production(r, t, tv)[0]
        JT = np.zeros((ns, ns))
        for r in range(ns):
            h = 1e-6 * rs[r]
            dp, dm = rs.copy(), rs.copy()
            dp[r] += h
            dm[r] -= h
            JT[:, r] = (om(dp, Tp, Tvp) - om(dm, Tp, Tvp)) / (2 * h)
        dwdT = (om(rs, Tp * (1 + 1e-7), Tvp) - om(rs, Tp * (1 - 1e-7), Tvp)) / (2e-7 * Tp)
        e, _, cv, _ = o.point_thermo(Tp, Tvp)
        if m.two_temp:
            e0, _, cv0, _ = o.point_thermo(Tp, 1e-3)     # no vibrational energy at Tv -> 0
            eve, cvve = e - e0, cv - cv0
            dT = -(e - eve) / (rs @ cv0)
            dTv = -eve / (rs @ cvve)
            dwdTv = (om(rs, Tp, Tvp * (1 + 1e-7)) - om(rs, Tp, Tvp * (1 - 1e-7))) / (2e-7 * Tvp)
            J = JT + np.outer(dwdT, dT) + np.outer(dwdTv, dTv)
        else:
            J = JT + np.outer(dwdT, -e / (rs @ cv))
        err = np.abs(JC[:, :, p] - J).max() / np.abs(J).max()
        assert err <= 2e-6, (p, err)
        # and the temperature term is not negligible here
        assert np.abs(J - JT).max() >= 1e-3 * np.abs(J).max()
        if m.two_temp:
            JC3 = JC3s[:, :, p]
            J3 = JT + np.outer(dwdT, -e / (rs @ cv0))   # Tv held: T takes all of the added e_r
            assert np.abs(JC3 - J3).max() <= 2e-6 * np.abs(J3).max(), p
