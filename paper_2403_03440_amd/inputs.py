"""Seeded synthetic inputs shared by the HIP path, the tests and the oracle.

This module holds none of the method's arithmetic: it builds grids (node
coordinates), mechanism data tables, the workload configurations and the
initial primitive fields.  Conversion of primitives to conservative variables
is done by each side on its own.

Every physical constant below is ILLUSTRATIVE.  The paper defers its
thermodynamic, transport and kinetic data to other references (Section 2.1);
the values here are round numbers of typical magnitude, chosen for this
synthetic workload and not taken from any published rate or property set.
Parity and speed do not depend on them.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

R_U = 8.314462618
EV_J_PER_MOL = 96485.33212  # 1 eV per particle in J/mol
M_ELECTRON = 5.48579909e-7  # kg/mol

ATOM, MOLECULE, ELECTRON = 0, 1, 2


@dataclasses.dataclass
class Mechanism:
    """Plain species/reaction tables (the C struct of both libraries mirrors it)."""

    names: List[str]
    M: np.ndarray          # kg/mol
    kind: np.ndarray       # 0 atom/atomic ion, 1 linear molecule/ion, 2 electron
    theta_v: np.ndarray    # K
    theta_r: np.ndarray    # K
    sigma: np.ndarray
    g_el: np.ndarray
    h_form: np.ndarray     # J/mol at 0 K
    sc: np.ndarray         # Schmidt numbers
    lt_a: np.ndarray       # Landau-Teller constants (Millikan-White form)
    lt_b: np.ndarray
    A: np.ndarray          # SI
    b: np.ndarray
    theta: np.ndarray      # K
    tctl: np.ndarray       # 0: T, 1: sqrt(T Tv), 2: Tv
    third: np.ndarray
    nu_f: np.ndarray       # [nr, ns]
    nu_b: np.ndarray
    eff: np.ndarray        # [nr, ns]
    two_temp: int = 0
    mu_ref: float = 1.8e-5
    T_ref: float = 300.0
    mu_exp: float = 0.7
    reactions: Optional[List[str]] = None

    @property
    def ns(self) -> int:
        return len(self.names)

    @property
    def nr(self) -> int:
        return len(self.A)

    @property
    def nv(self) -> int:
        return self.ns + 3 + (1 if self.two_temp else 0)

    @property
    def nf(self) -> int:
        return 4 + (1 if self.two_temp else 0)

    @property
    def nb(self) -> int:
        return self.nf + self.ns - 1

    def with_two_temp(self, two_temp: int) -> "Mechanism":
        return dataclasses.replace(self, two_temp=int(two_temp))

    def without_reactions(self) -> "Mechanism":
        z = np.zeros((0, self.ns), dtype=np.int32)
        return dataclasses.replace(
            self, A=np.zeros(0), b=np.zeros(0), theta=np.zeros(0), tctl=np.zeros(0, np.int32),
            third=np.zeros(0, np.int32), nu_f=z, nu_b=z, eff=np.zeros((0, self.ns)), reactions=[])


def species_copies(mech: Mechanism, ns: int) -> Mechanism:
    """A non-reacting mixture of ns species in which species k is an identical
    copy of species k mod mech.ns (same molar mass, modes and transport).
    Giving the copies of a species fractions of its partial density that sum
    to it leaves every mixture property unchanged, so the flow unknowns match
    the base mixture's at any species count."""
    if mech.nr:
        raise ValueError("species_copies: the base mechanism must have no reactions")
    idx = np.arange(ns) % mech.ns
    z = np.zeros((0, ns), dtype=np.int32)
    return dataclasses.replace(
        mech, names=[f"{mech.names[k]}#{i}" for i, k in enumerate(idx)], M=mech.M[idx], kind=mech.kind[idx],
        theta_v=mech.theta_v[idx], theta_r=mech.theta_r[idx], sigma=mech.sigma[idx], g_el=mech.g_el[idx],
        h_form=mech.h_form[idx], sc=mech.sc[idx], lt_a=mech.lt_a[idx], lt_b=mech.lt_b[idx], nu_f=z, nu_b=z,
        eff=np.zeros((0, ns)), reactions=[])


def split_among_copies(rho_s: np.ndarray, base_ns: int, ns: int) -> np.ndarray:
    """Partial densities of the species_copies mixture: each base species'
    density shared equally among its copies (rho_s: [base_ns, n])."""
    idx = np.arange(ns) % base_ns
    counts = np.bincount(idx, minlength=base_ns).astype(np.float64)
    return np.ascontiguousarray(rho_s[idx] / counts[idx][:, None])


# --------------------------------------------------------------- species
def _millikan_white(M_kg: float, theta_v: float):
    """Millikan-White correlation constants a_s, b_s with the species' own reduced mass (amu)."""
    mu = 0.5 * M_kg * 1e3
    return 1.16e-3 * math.sqrt(mu) * theta_v ** (4.0 / 3.0), 0.015 * mu ** 0.25


def _species_table(rows):
    names = [r[0] for r in rows]
    M = np.array([r[1] for r in rows], float)
    kind = np.array([r[2] for r in rows], np.int32)
    tv = np.array([r[3] for r in rows], float)
    tr = np.array([r[4] for r in rows], float)
    sig = np.array([r[5] for r in rows], float)
    g = np.array([r[6] for r in rows], float)
    hf = np.array([r[7] for r in rows], float)
    sc = np.array([r[8] for r in rows], float)
    a = np.zeros(len(rows))
    bb = np.zeros(len(rows))
    for s in range(len(rows)):
        if kind[s] == MOLECULE and tv[s] > 0:
            a[s], bb[s] = _millikan_white(M[s], tv[s])
    return names, M, kind, tv, tr, sig, g, hf, sc, a, bb


# name, M, kind, theta_v, theta_r, sigma, g_el, h_form (0 K, J/mol), Sc  -- illustrative
_AIR_NEUTRAL = [
    ("O2", 31.9988e-3, MOLECULE, 2240.0, 2.08, 2.0, 3.0, 0.0, 0.72),
    ("NO", 30.0061e-3, MOLECULE, 2820.0, 2.45, 1.0, 4.0, 90.0e3, 0.71),
    ("N", 14.0067e-3, ATOM, 0.0, 0.0, 1.0, 4.0, 471.0e3, 0.60),
    ("O", 15.9994e-3, ATOM, 0.0, 0.0, 1.0, 9.0, 247.0e3, 0.62),
]
# N2 closes the coupled system (the ns-th species follows from rho - sum of the
# others), so it is kept last: it is the most abundant species everywhere.
_N2 = [("N2", 28.0134e-3, MOLECULE, 3390.0, 2.88, 2.0, 1.0, 0.0, 0.70)]
_AIR_IONS = [
    ("N2+", 28.0134e-3 - M_ELECTRON, MOLECULE, 3170.0, 2.78, 2.0, 2.0, 15.6 * EV_J_PER_MOL, 0.70),
    ("O2+", 31.9988e-3 - M_ELECTRON, MOLECULE, 2740.0, 2.42, 2.0, 4.0, 12.1 * EV_J_PER_MOL, 0.72),
    ("NO+", 30.0061e-3 - M_ELECTRON, MOLECULE, 3420.0, 2.86, 1.0, 1.0, 90.0e3 + 9.3 * EV_J_PER_MOL, 0.71),
    ("N+", 14.0067e-3 - M_ELECTRON, ATOM, 0.0, 0.0, 1.0, 9.0, 471.0e3 + 14.5 * EV_J_PER_MOL, 0.60),
    ("O+", 15.9994e-3 - M_ELECTRON, ATOM, 0.0, 0.0, 1.0, 4.0, 247.0e3 + 13.6 * EV_J_PER_MOL, 0.62),
    ("e-", M_ELECTRON, ELECTRON, 0.0, 0.0, 1.0, 2.0, 0.0, 0.65),
]


def _reactions(names, hf, rxns):
    """rxns: (lhs dict, rhs dict, A_cgs, b, tctl, third, eff dict or None).
    theta defaults to the 0 K reaction enthalpy / R_u when it is endothermic."""
    ns = len(names)
    idx = {n: k for k, n in enumerate(names)}
    nr = len(rxns)
    nu_f = np.zeros((nr, ns), np.int32)
    nu_b = np.zeros((nr, ns), np.int32)
    eff = np.zeros((nr, ns))
    A = np.zeros(nr)
    b = np.zeros(nr)
    theta = np.zeros(nr)
    tctl = np.zeros(nr, np.int32)
    third = np.zeros(nr, np.int32)
    labels = []
    for r, (lhs, rhs, A_cgs, bb, tc, tb, ef, *th) in enumerate(rxns):
        for n, c in lhs.items():
            nu_f[r, idx[n]] += c
        for n, c in rhs.items():
            nu_b[r, idx[n]] += c
        order = int(nu_f[r].sum()) + (1 if tb else 0)
        A[r] = A_cgs * (1e-6) ** (order - 1)
        b[r] = bb
        tctl[r] = tc
        third[r] = 1 if tb else 0
        if tb:
            eff[r, :] = 1.0
            for n, e in (ef or {}).items():
                eff[r, idx[n]] = e
        dH = float((nu_b[r] - nu_f[r]) @ hf)
        theta[r] = th[0] if th else max(dH, 0.0) / R_U
        labels.append(" + ".join(f"{c if c > 1 else ''}{n}" for n, c in lhs.items()) + " <=> " +
                      " + ".join(f"{c if c > 1 else ''}{n}" for n, c in rhs.items()) + (" (+M)" if tb else ""))
    return A, b, theta, tctl, third, nu_f, nu_b, eff, labels


def air5(two_temp: int = 0) -> Mechanism:
    """5-species air (O2, NO, N, O, N2), 17 reactions: three dissociations with
    five explicit collision partners each and two exchange reactions."""
    names, M, kind, tv, tr, sig, g, hf, sc, a, bb = _species_table(_AIR_NEUTRAL + _N2)
    diss = {"N2": ({"N": 2}, 5.0e21, -1.5), "O2": ({"O": 2}, 2.0e21, -1.5), "NO": ({"N": 1, "O": 1}, 5.0e15, 0.0)}
    rx = []
    for mol, (prod, A0, b0) in diss.items():
        for part in names:
            lhs = {mol: 1}
            lhs[part] = lhs.get(part, 0) + 1
            rhs = dict(prod)
            rhs[part] = rhs.get(part, 0) + 1
            rx.append((lhs, rhs, A0 * (4.0 if part in ("N", "O") else 1.0), b0, 1, False, None))
    rx.append(({"N2": 1, "O": 1}, {"NO": 1, "N": 1}, 6.0e13, 0.0, 0, False, None))
    rx.append(({"NO": 1, "O": 1}, {"O2": 1, "N": 1}, 8.0e9, 1.0, 0, False, None))
    A, b, th, tctl, third, nu_f, nu_b, eff, labels = _reactions(names, hf, rx)
    return Mechanism(names, M, kind, tv, tr, sig, g, hf, sc, a, bb, A, b, th, tctl, third, nu_f, nu_b, eff,
                     two_temp=two_temp, reactions=labels)


def air11(two_temp: int = 1) -> Mechanism:
    """11-species ionised air with 21 reactions: three dissociations with third
    bodies, two exchanges, three associative ionisations, eleven charge
    exchanges and two electron-impact ionisations (the list is this
    workload's own; the paper only names the species)."""
    names, M, kind, tv, tr, sig, g, hf, sc, a, bb = _species_table(_AIR_NEUTRAL + _AIR_IONS + _N2)
    atoms3 = {"N": 3.0, "O": 3.0, "N+": 3.0, "O+": 3.0, "e-": 0.0}
    rx = [
        ({"N2": 1}, {"N": 2}, 5.0e21, -1.5, 1, True, atoms3),
        ({"O2": 1}, {"O": 2}, 2.0e21, -1.5, 1, True, atoms3),
        ({"NO": 1}, {"N": 1, "O": 1}, 5.0e15, 0.0, 1, True, atoms3),
        ({"N2": 1, "O": 1}, {"NO": 1, "N": 1}, 6.0e13, 0.0, 0, False, None),
        ({"NO": 1, "O": 1}, {"O2": 1, "N": 1}, 8.0e9, 1.0, 0, False, None),
        ({"N": 1, "O": 1}, {"NO+": 1, "e-": 1}, 5.0e11, 0.5, 0, False, None),
        ({"N": 2}, {"N2+": 1, "e-": 1}, 2.0e13, 0.0, 0, False, None),
        ({"O": 2}, {"O2+": 1, "e-": 1}, 1.0e12, 0.5, 0, False, None),
        ({"NO+": 1, "O": 1}, {"N+": 1, "O2": 1}, 1.0e12, 0.5, 0, False, None),
        ({"N+": 1, "N2": 1}, {"N2+": 1, "N": 1}, 1.0e12, 0.5, 0, False, None),
        ({"O2+": 1, "N": 1}, {"N+": 1, "O2": 1}, 1.0e13, 0.0, 0, False, None),
        ({"O+": 1, "NO": 1}, {"N+": 1, "O2": 1}, 1.0e12, 0.5, 0, False, None),
        ({"O2+": 1, "N2": 1}, {"N2+": 1, "O2": 1}, 1.0e13, 0.0, 0, False, None),
        ({"O2+": 1, "O": 1}, {"O+": 1, "O2": 1}, 1.0e12, 0.5, 0, False, None),
        ({"NO+": 1, "N": 1}, {"O+": 1, "N2": 1}, 1.0e13, 0.0, 0, False, None),
        ({"NO+": 1, "O2": 1}, {"O2+": 1, "NO": 1}, 1.0e12, 0.5, 0, False, None),
        ({"NO+": 1, "O": 1}, {"O2+": 1, "N": 1}, 1.0e12, 0.5, 0, False, None),
        ({"O+": 1, "N2": 1}, {"N2+": 1, "O": 1}, 1.0e12, 0.5, 0, False, None),
        ({"NO+": 1, "N": 1}, {"N2+": 1, "O": 1}, 1.0e12, 0.5, 0, False, None),
        ({"N": 1, "e-": 1}, {"N+": 1, "e-": 2}, 1.0e25, -2.5, 2, False, None),
        ({"O": 1, "e-": 1}, {"O+": 1, "e-": 2}, 1.0e25, -2.5, 2, False, None),
    ]
    A, b, th, tctl, third, nu_f, nu_b, eff, labels = _reactions(names, hf, rx)
    return Mechanism(names, M, kind, tv, tr, sig, g, hf, sc, a, bb, A, b, th, tctl, third, nu_f, nu_b, eff,
                     two_temp=two_temp, reactions=labels)


def toy_dissociation(two_temp: int = 0) -> Mechanism:
    """A2 + M <=> 2A + M: its equilibrium is the root of a quadratic."""
    rows = [("A2", 28.0e-3, MOLECULE, 3000.0, 2.5, 2.0, 1.0, 0.0, 0.7),
            ("A", 14.0e-3, ATOM, 0.0, 0.0, 1.0, 4.0, 400.0e3, 0.6)]
    names, M, kind, tv, tr, sig, g, hf, sc, a, bb = _species_table(rows)
    rx = [({"A2": 1}, {"A": 2}, 1.0e21, -1.5, 1, True, {"A": 2.0})]
    A, b, th, tctl, third, nu_f, nu_b, eff, labels = _reactions(names, hf, rx)
    return Mechanism(names, M, kind, tv, tr, sig, g, hf, sc, a, bb, A, b, th, tctl, third, nu_f, nu_b, eff,
                     two_temp=two_temp, reactions=labels)


def toy3(two_temp: int = 0) -> Mechanism:
    """3-species / 2-reaction toy: A2 <=> 2A (+M), A2 + A <=> A3 (no third body)."""
    rows = [("A2", 28.0e-3, MOLECULE, 2500.0, 2.0, 2.0, 1.0, 0.0, 0.7),
            ("A", 14.0e-3, ATOM, 0.0, 0.0, 1.0, 2.0, 300.0e3, 0.6),
            ("A3", 42.0e-3, MOLECULE, 1200.0, 0.6, 2.0, 1.0, 150.0e3, 0.8)]
    names, M, kind, tv, tr, sig, g, hf, sc, a, bb = _species_table(rows)
    rx = [({"A2": 1}, {"A": 2}, 3.0e21, -1.5, 1, True, None),
          ({"A2": 1, "A": 1}, {"A3": 1}, 1.0e13, 0.0, 0, False, None, 2000.0)]
    A, b, th, tctl, third, nu_f, nu_b, eff, labels = _reactions(names, hf, rx)
    return Mechanism(names, M, kind, tv, tr, sig, g, hf, sc, a, bb, A, b, th, tctl, third, nu_f, nu_b, eff,
                     two_temp=two_temp, reactions=labels)


def synthetic(ns: int = 20, nr: int = 60, seed: int = 3442) -> Mechanism:
    """Seeded synthetic mechanism: three pseudo-elements, ns species of one to
    three atoms, nr element-balanced reactions (dissociations with a third body
    and atom-transfer exchanges), log10 A ~ U[10, 22] (cm-mol-s),
    b ~ U[-2, 1], theta ~ U[0, 1.2e5] K."""
    rng = np.random.default_rng(seed)
    emass = rng.uniform(10.0, 20.0, 3) * 1e-3
    # compositions: atoms, then diatomics, then triatomics (counts of elements)
    comps = [(1, 0, 0), (0, 1, 0), (0, 0, 1)]
    di = [(2, 0, 0), (0, 2, 0), (0, 0, 2), (1, 1, 0), (1, 0, 1), (0, 1, 1)]
    tri = [(3, 0, 0), (0, 3, 0), (0, 0, 3), (2, 1, 0), (2, 0, 1), (1, 2, 0), (0, 2, 1), (1, 0, 2), (0, 1, 2),
           (1, 1, 1)]
    comps += di
    order = rng.permutation(len(tri))
    for k in order:
        if len(comps) >= ns:
            break
        comps.append(tri[k])
    extra = 0
    while len(comps) < ns:  # isomers: a second species with an existing triatomic composition
        comps.append(tri[order[extra % len(tri)]])
        extra += 1
    comps = comps[:ns]
    hf_atom = rng.uniform(200e3, 500e3, 3)
    rows = []
    for k, c in enumerate(comps):
        nat = sum(c)
        M = float(np.dot(c, emass))
        if nat == 1:
            e = c.index(1)
            rows.append((f"X{k}", M, ATOM, 0.0, 0.0, 1.0, float(rng.integers(1, 6)), float(hf_atom[e]), 0.6))
        else:
            homo = max(c) == nat
            hf = float(np.dot(c, hf_atom)) - (nat - 1) * rng.uniform(300e3, 700e3)
            rows.append((f"X{k}", M, MOLECULE, float(rng.uniform(500.0, 4000.0)), float(rng.uniform(0.5, 3.0)),
                         2.0 if homo else 1.0, float(rng.integers(1, 4)), hf, float(rng.uniform(0.6, 0.8))))
    # the first diatomic (the free stream's major species) closes the coupled
    # system, so it is moved to the end
    major = next(k for k, c in enumerate(comps) if sum(c) == 2)
    order_ = [k for k in range(len(comps)) if k != major] + [major]
    rows = [rows[k] for k in order_]
    comps = [comps[k] for k in order_]
    names, M, kind, tv, tr, sig, g, hf, sc, a, bb = _species_table(rows)
    cidx = {c: k for k, c in enumerate(comps)}
    cand = []
    for k, c in enumerate(comps if nr > 0 else []):  # dissociations A -> B + C
        if sum(c) < 2:
            continue
        for k2, c2 in enumerate(comps):
            rest = tuple(x - y for x, y in zip(c, c2))
            if min(rest) < 0 or sum(rest) == 0 or rest not in cidx or cidx[rest] < k2:
                continue
            cand.append(("d", k, k2, cidx[rest]))
    for k, c in enumerate(comps if nr > 0 else []):  # exchanges X + Y -> X' + Y' moving one atom
        for e in range(3):
            if c[e] == 0 or sum(c) < 2:
                continue
            xp = tuple(c[i] - (1 if i == e else 0) for i in range(3))
            if xp not in cidx:
                continue
            for k2, c2 in enumerate(comps):
                yp = tuple(c2[i] + (1 if i == e else 0) for i in range(3))
                if yp in cidx and k2 != k and cidx[yp] != k:
                    cand.append(("x", k, k2, cidx[xp], cidx[yp]))
    pick = rng.permutation(len(cand))[:nr]
    rx = []
    for p in sorted(pick):
        cd = cand[p]
        logA = rng.uniform(10.0, 22.0)
        bexp = rng.uniform(-2.0, 1.0)
        th = rng.uniform(0.0, 1.2e5)
        th_min = None  # set below from the reaction enthalpy
        if cd[0] == "d":
            lhs = {names[cd[1]]: 1}
            rhs = {}
            for t in (cd[2], cd[3]):
                rhs[names[t]] = rhs.get(names[t], 0) + 1
            rx.append((lhs, rhs, 10.0 ** logA, bexp, 0, True, None, th))
        else:
            lhs = {}
            for t in (cd[1], cd[2]):
                lhs[names[t]] = lhs.get(names[t], 0) + 1
            rhs = {}
            for t in (cd[3], cd[4]):
                rhs[names[t]] = rhs.get(names[t], 0) + 1
            rx.append((lhs, rhs, 10.0 ** logA, bexp, 0, False, None, th))
    A, b, th, tctl, third, nu_f, nu_b, eff, labels = _reactions(names, hf, rx)
    # the forward activation temperature is at least the reaction enthalpy / R_u,
    # so that the backward direction has a non-negative activation energy
    dH = ((nu_b - nu_f) @ hf) / R_U
    th = np.maximum(th, dH)
    return Mechanism(names, M, kind, tv, tr, sig, g, hf, sc, a, bb, A, b, th, tctl, third, nu_f, nu_b, eff,
                     two_temp=0, reactions=labels)


# ------------------------------------------------------------------- grid
def polar_grid(ni: int, nj: int, r_wall: float = 0.1, r_out: float = 0.4, stretch48: float = 1.05):
    """Windward half-annulus theta in [pi/2, 3pi/2] (flow along +x), radial
    geometric stretching q = stretch48 ** (48 / nj).  Returns node arrays
    x, y of shape (nj+1, ni+1), i (theta) fastest."""
    q = stretch48 ** (48.0 / nj)
    J = np.arange(nj + 1, dtype=float)
    r = r_wall + (r_out - r_wall) * (q ** J - 1.0) / (q ** nj - 1.0)
    th = 0.5 * np.pi + np.arange(ni + 1, dtype=float) * np.pi / ni
    x = r[:, None] * np.cos(th)[None, :]
    y = r[:, None] * np.sin(th)[None, :]
    return np.ascontiguousarray(x), np.ascontiguousarray(y)


def box_grid(ni: int, nj: int, lx: float = 0.01, ly: float = 0.01, skew: float = 0.0, seed: int = 0):
    """Small (optionally jittered) quadrilateral grid for unit tests."""
    rng = np.random.default_rng(seed)
    X, Y = np.meshgrid(np.linspace(0, lx, ni + 1), np.linspace(0, ly, nj + 1))
    if skew:
        X = X + skew * lx / ni * rng.uniform(-1, 1, X.shape)
        Y = Y + skew * ly / nj * rng.uniform(-1, 1, Y.shape)
    return np.ascontiguousarray(X), np.ascontiguousarray(Y)


# ------------------------------------------------------------ random numbers
def splitmix64(x: np.ndarray) -> np.ndarray:
    """splitmix64 finaliser (Steele, Lea & Flood 2014) on uint64 inputs."""
    with np.errstate(over="ignore"):
        z = (x.astype(np.uint64) + np.uint64(0x9E3779B97F4A7C15))
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))


def uniform_pm1(seed: int, n: int) -> np.ndarray:
    """xi_p ~ U[-1, 1] from splitmix64(seed XOR p), 53-bit mantissa."""
    z = splitmix64(np.uint64(seed) ^ np.arange(n, dtype=np.uint64))
    u = (z >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)
    return 2.0 * u - 1.0


# ---------------------------------------------------------------- configs
@dataclasses.dataclass
class Config:
    name: str
    ni: int
    nj: int
    mech: str
    two_temp: int
    cfl: float
    u_inf: float
    rho_inf: float = 1e-3
    T_inf: float = 250.0
    T_wall: float = 300.0
    perturb: float = 0.0
    seed: int = 3440
    iters: int = 500
    tol: float = 1e-8
    ramp: int = 100  # iterations over which the CFL number ramps up from 1

    def mechanism(self) -> Mechanism:
        if self.mech == "air5":
            return air5(self.two_temp)
        if self.mech == "air11":
            return air11(self.two_temp)
        if self.mech == "syn20":
            return synthetic(20, 60, 3442)
        raise ValueError(self.mech)

    def freestream_Y(self, mech: Mechanism) -> np.ndarray:
        Y = np.zeros(mech.ns)
        if self.mech == "syn20":
            di = [k for k in range(mech.ns - 1) if mech.kind[k] == MOLECULE and mech.names[k].count("X")][:1]
            Y[mech.ns - 1], Y[di[0]] = 0.767, 0.233
        else:
            Y[mech.names.index("N2")] = 0.767
            Y[mech.names.index("O2")] = 0.233
        return Y

    def grid(self):
        return polar_grid(self.ni, self.nj)


CONFIGS = {
    # 64 x 48, 5-species air, one temperature, CFL 10, 500 iterations, +-1 % density perturbation
    "c1": Config("c1", 64, 48, "air5", 0, 10.0, 5000.0, perturb=0.01, iters=500),
    # 512 x 256, 5-species air, two temperatures, CFL 100, to a 1e-8 residual drop
    "c2": Config("c2", 512, 256, "air5", 1, 100.0, 5000.0, iters=20000),
    # 1024 x 512, 11-species ionised air, two temperatures, 7 km/s
    "c3": Config("c3", 1024, 512, "air11", 1, 100.0, 7000.0, iters=20000, ramp=1000),
    # c2 grid and flow with the 11-species mechanism (surrogate workload)
    "c4": Config("c4", 512, 256, "air11", 1, 100.0, 5000.0, iters=20000),
    # 2048 x 1024, seeded 20-species / 60-reaction mechanism, CFL 1000
    "c5": Config("c5", 2048, 1024, "syn20", 0, 1000.0, 5000.0, iters=20000),
}


def freestream_prims(cfg: Config, mech: Mechanism):
    Y = cfg.freestream_Y(mech)
    return cfg.rho_inf * Y, cfg.u_inf, 0.0, cfg.T_inf, cfg.T_inf


def initial_prims(cfg: Config, mech: Mechanism, ni: Optional[int] = None, nj: Optional[int] = None):
    """Uniform free stream, with the seeded +-perturb density perturbation
    rho_s <- rho_s (1 + perturb xi_p) at fixed u, T, Y when perturb > 0."""
    ni = ni or cfg.ni
    nj = nj or cfg.nj
    n = ni * nj
    rs_inf, u, v, T, Tv = freestream_prims(cfg, mech)
    rs = np.repeat(rs_inf[:, None], n, axis=1)
    if cfg.perturb:
        rs = rs * (1.0 + cfg.perturb * uniform_pm1(cfg.seed, n))[None, :]
    return (np.ascontiguousarray(rs), np.full(n, u), np.full(n, v), np.full(n, T), np.full(n, Tv))


def random_prims(mech: Mechanism, n: int, seed: int, T_range=(300.0, 9000.0), rho_range=(1e-3, 2e-2),
                 speed=3000.0, tv_spread=0.3, y_floor=0.0):
    """Seeded random states within physical bounds (for kernel parity tests)."""
    rng = np.random.default_rng(seed)
    Y = rng.dirichlet(np.ones(mech.ns), size=n).T + y_floor
    if ELECTRON in list(mech.kind):
        e = list(mech.kind).index(ELECTRON)
        ions = [k for k, nm in enumerate(mech.names) if nm.endswith("+")]
        Y[e, :] = 0.0
        # charge neutrality: electrons balance the ions (number densities)
        Y[e, :] = sum(Y[k, :] / mech.M[k] for k in ions) * mech.M[e]
    Y = Y / Y.sum(axis=0, keepdims=True)
    rho = np.exp(rng.uniform(np.log(rho_range[0]), np.log(rho_range[1]), n))
    T = rng.uniform(*T_range, n)
    Tv = T * (1.0 + tv_spread * rng.uniform(-1, 1, n)) if mech.two_temp else T.copy()
    ang = rng.uniform(0, 2 * np.pi, n)
    sp = speed * rng.uniform(0, 1, n)
    return (np.ascontiguousarray(rho[None, :] * Y), sp * np.cos(ang), sp * np.sin(ang), T, Tv)


def permutation(seed: int, n: int) -> np.ndarray:
    """Seeded permutation of 0..n-1: indices ordered by splitmix64(seed XOR i)."""
    keys = splitmix64(np.uint64(seed) ^ np.arange(n, dtype=np.uint64))
    return np.argsort(keys, kind="stable").astype(np.int32)
