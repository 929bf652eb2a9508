"""ctypes wrapper of the oracle library (TEST INFRASTRUCTURE ONLY).

Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg may use
this module.  The oracle shares no code with the HIP path."""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
# the same sources with room for 256 species per cell (the species-count
# study); the default build keeps 32 and with it smaller per-cell records
WIDE_LIB_PATH = os.path.join(HERE, "liboracle_wide.so")
WIDE_MAXS = 256
SOURCES = ["orc.cpp", "orc_mlp.cpp"]

COUPLED, SPLIT = 0, 1
CLOSURE, CC1, CC2 = 0, 1, 2
HYPERPLANE, LEXICOGRAPHIC = 0, 1

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int)


def build(verbose: bool = False) -> str:
    """Compile liboracle.so and liboracle_wide.so with g++ (plain FP64, no
    fused multiply-add contraction)."""
    srcs = [os.path.join(HERE, s) for s in SOURCES if os.path.exists(os.path.join(HERE, s))]
    for path, extra in ((LIB_PATH, []), (WIDE_LIB_PATH, [f"-DORC_MAXS={WIDE_MAXS}"])):
        cmd = ["g++", "-O3", "-std=c++17", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off"] + extra + \
              ["-o", path + ".tmp"] + srcs
        if verbose:
            print(" ".join(cmd))
        subprocess.run(cmd, check=True)
        os.replace(path + ".tmp", path)
    return LIB_PATH


class OrcMechanism(C.Structure):
    _fields_ = [("ns", C.c_int), ("nr", C.c_int), ("two_temp", C.c_int),
                ("M", _dp), ("kind", _ip), ("theta_v", _dp), ("theta_r", _dp), ("sigma", _dp),
                ("g_el", _dp), ("h_form", _dp), ("sc", _dp), ("lt_a", _dp), ("lt_b", _dp),
                ("A", _dp), ("b", _dp), ("theta", _dp), ("tctl", _ip), ("third", _ip),
                ("nu_f", _ip), ("nu_b", _ip), ("eff", _dp),
                ("mu_ref", C.c_double), ("T_ref", C.c_double), ("mu_exp", C.c_double)]


_lib = {}


def lib(wide: bool = False):
    path = WIDE_LIB_PATH if wide else LIB_PATH
    if path not in _lib:
        if not os.path.exists(path):
            build()
        L = C.CDLL(path)
        L.orc_last_error.restype = C.c_char_p
        _lib[path] = L
    return _lib[path]


def _d(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(_dp)


def _i(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(_ip)


class Oracle:
    """One oracle context: grid + mechanism + free stream + state."""

    def __init__(self, threads: int = 0, wide: bool = False):
        """wide: the build with room for up to 256 species (needed above 32)."""
        self.L = lib(wide)
        self.ctx = C.c_void_p()
        self._check(self.L.orc_create(C.byref(self.ctx)))
        if threads:
            self.L.orc_set_threads(self.ctx, threads)
        self._keep = []
        self.mech = None

    def __del__(self):
        try:
            self.L.orc_destroy(self.ctx)
        except Exception:
            pass

    def _check(self, rc):
        if rc != 0:
            msg = self.L.orc_last_error(self.ctx).decode() if getattr(self, "ctx", None) else ""
            raise RuntimeError(f"oracle error {rc}: {msg}")

    def set_physical_time(self, dt, theta=0.0):
        self._check(self.L.orc_set_physical_time(self.ctx, C.c_double(dt), C.c_double(theta)))

    def set_time_levels(self, qn, qnm1):
        a, pa = _d(qn)
        b, pb = _d(qnm1)
        self._check(self.L.orc_set_time_levels(self.ctx, pa, pb))

    def advance_time(self):
        self._check(self.L.orc_advance_time(self.ctx))

    def set_option(self, name, value):
        self._check(self.L.orc_set_option(self.ctx, name.encode(), C.c_double(value)))

    # ---------------------------------------------------------------- setup
    def set_grid(self, x, y, T_wall=300.0, bc_mode=0):
        nj1, ni1 = x.shape
        self.ni, self.nj = ni1 - 1, nj1 - 1
        self.N = self.ni * self.nj
        xa, xp = _d(x)
        ya, yp = _d(y)
        self._check(self.L.orc_set_grid(self.ctx, self.ni, self.nj, xp, yp, C.c_double(T_wall), bc_mode))

    def set_mechanism(self, m):
        keep = []

        def d(a):
            arr, p = _d(a)
            keep.append(arr)
            return p

        def i(a):
            arr, p = _i(a)
            keep.append(arr)
            return p

        s = OrcMechanism(m.ns, m.nr, int(m.two_temp), d(m.M), i(m.kind), d(m.theta_v), d(m.theta_r),
                         d(m.sigma), d(m.g_el), d(m.h_form), d(m.sc), d(m.lt_a), d(m.lt_b),
                         d(m.A if m.nr else [0.0]), d(m.b if m.nr else [0.0]), d(m.theta if m.nr else [0.0]),
                         i(m.tctl if m.nr else [0]), i(m.third if m.nr else [0]),
                         i(np.asarray(m.nu_f).ravel() if m.nr else [0]),
                         i(np.asarray(m.nu_b).ravel() if m.nr else [0]),
                         d(np.asarray(m.eff).ravel() if m.nr else [0.0]),
                         m.mu_ref, m.T_ref, m.mu_exp)
        self._check(self.L.orc_set_mechanism(self.ctx, C.byref(s)))
        self.mech = m

    def set_freestream(self, rho_s, u, v, T, Tv):
        a, p = _d(rho_s)
        self._check(self.L.orc_set_freestream(self.ctx, p, C.c_double(u), C.c_double(v), C.c_double(T),
                                              C.c_double(Tv)))

    def prim_to_cons(self, rho_s, u, v, T, Tv):
        rho_s = np.atleast_2d(rho_s)
        n = rho_s.shape[1]
        q = np.zeros((self.mech.nv, n))
        args = [_d(a) for a in (rho_s, u, v, T, Tv)]
        self._check(self.L.orc_prim_to_cons(self.ctx, n, *[p for _, p in args], q.ctypes.data_as(_dp)))
        return q

    def set_state(self, q):
        a, p = _d(q)
        self._check(self.L.orc_set_state(self.ctx, p))

    def get_state(self):
        q = np.zeros((self.mech.nv, self.N))
        self._check(self.L.orc_get_state(self.ctx, q.ctypes.data_as(_dp)))
        return q

    # ------------------------------------------------------------ algorithm
    def residual(self, cfl):
        nrm = np.zeros(2)
        self._check(self.L.orc_residual(self.ctx, C.c_double(cfl), nrm.ctypes.data_as(_dp)))
        return nrm

    def implicit_op(self, mode, order=HYPERPLANE):
        self._check(self.L.orc_implicit_op(self.ctx, mode, order))

    def nsol(self, mode):
        return self.mech.nb if mode == COUPLED else self.mech.nf + self.mech.ns

    def sweep_rhs(self, mode, b, order=HYPERPLANE):
        x = np.zeros((self.nsol(mode), self.N))
        a, p = _d(b)
        self._check(self.L.orc_sweep_rhs(self.ctx, mode, order, p, x.ctypes.data_as(_dp)))
        return x

    def consistency_correct(self, mode, kind):
        n = C.c_int(0)
        self._check(self.L.orc_consistency_correct(self.ctx, mode, kind, C.byref(n)))
        return n.value

    def sweep_cell(self, mode, fwd, i, j, xs, x=None):
        """One cell of the sweeps with the other cells' values given (see orc.h)."""
        out = np.zeros(self.nsol(mode))
        a, pxs = _d(xs)
        if x is not None:
            b_, px = _d(x)
        else:
            px = None
        self._check(self.L.orc_sweep_cell(self.ctx, mode, int(fwd), i, j, pxs, px, out.ctypes.data_as(_dp)))
        return out

    def step(self, mode, kind, cfl, n_iter, ramp=0, it0=0):
        h = np.zeros((n_iter, 2))
        self._check(self.L.orc_step(self.ctx, mode, kind, C.c_double(cfl), ramp, it0, n_iter,
                                    h.ctypes.data_as(_dp)))
        return h

    def wall_heat_flux(self):
        qw = np.zeros(self.ni)
        qs = C.c_double(0)
        self._check(self.L.orc_wall_heat_flux(self.ctx, qw.ctypes.data_as(_dp), C.byref(qs)))
        return qw, qs.value

    def get(self, name, mode=COUPLED):
        m = self.mech
        N = self.N
        shapes = {"R": (m.nv, N), "dtau": (N,), "V": (N,), "omega": (m.nv, N), "dqs": (self.nsol(mode), N),
                  "dq": (self.nsol(mode), N), "T": (N,), "Tv": (N,), "p": (N,), "c": (N,),
                  "qw": (self.ni,), "dK": (N,), "dF": (N,), "dC": (N,), "JK": (m.nb, m.nb, N),
                  "JC": (m.ns, m.ns, N), "Jve": (m.nf, N), "DK": (m.nb, m.nb, N), "DF": (m.nf, m.nf, N),
                  "DC": (m.ns, m.ns, N), "FvI": (m.nv, (self.ni + 1) * self.nj),
                  "FvJ": (m.nv, self.ni * (self.nj + 1))}
        out = np.zeros(shapes[name])
        self._check(self.L.orc_get(self.ctx, name.encode(), out.ctypes.data_as(_dp)))
        return out

    def dense_operator(self, mode):
        dim = self.N * self.nsol(mode)
        D = np.zeros((dim, dim))
        L = np.zeros((dim, dim))
        U = np.zeros((dim, dim))
        self._check(self.L.orc_dense_operator(self.ctx, mode, D.ctypes.data_as(_dp), L.ctypes.data_as(_dp),
                                              U.ctypes.data_as(_dp)))
        return D, L, U

    # ---------------------------------------------------------------- points
    def point_thermo(self, T, Tv=None):
        ns = self.mech.ns
        e, h, cv, g = (np.zeros(ns) for _ in range(4))
        self._check(self.L.orc_point_thermo(self.ctx, C.c_double(T), C.c_double(T if Tv is None else Tv),
                                            e.ctypes.data_as(_dp), h.ctypes.data_as(_dp),
                                            cv.ctypes.data_as(_dp), g.ctypes.data_as(_dp)))
        return e, h, cv, g

    def point_production(self, rho_s, T, Tv=None):
        om = np.zeros(self.mech.ns)
        ov = C.c_double(0)
        a, p = _d(rho_s)
        self._check(self.L.orc_point_production(self.ctx, p, C.c_double(T), C.c_double(T if Tv is None else Tv),
                                                om.ctypes.data_as(_dp), C.byref(ov)))
        return om, ov.value

    def point_prim(self, q):
        vals = [C.c_double(0) for _ in range(4)]
        a, p = _d(q)
        self._check(self.L.orc_point_prim(self.ctx, p, *[C.byref(v) for v in vals]))
        return tuple(v.value for v in vals)

    def point_flux(self, q, nx, ny):
        F = np.zeros(self.mech.nv)
        a, p = _d(q)
        self._check(self.L.orc_point_flux(self.ctx, p, C.c_double(nx), C.c_double(ny), F.ctypes.data_as(_dp)))
        return F

    def point_hlle(self, qL, qR, nx, ny):
        F = np.zeros(self.mech.nv)
        a, pl = _d(qL)
        b, pr = _d(qR)
        self._check(self.L.orc_point_hlle(self.ctx, pl, pr, C.c_double(nx), C.c_double(ny), F.ctypes.data_as(_dp)))
        return F

    def point_roe(self, qL, qR, nx, ny, eta=0.0):
        F = np.zeros(self.mech.nv)
        a, pl = _d(qL)
        b, pr = _d(qR)
        self._check(self.L.orc_point_roe(self.ctx, pl, pr, C.c_double(nx), C.c_double(ny), C.c_double(eta),
                                         F.ctypes.data_as(_dp)))
        return F

    def point_muscl(self, qA, qB, qC):
        qf = np.zeros(self.mech.nv)
        a, pa = _d(qA)
        b, pb = _d(qB)
        c, pc = _d(qC)
        self._check(self.L.orc_point_muscl(self.ctx, pa, pb, pc, qf.ctypes.data_as(_dp)))
        return qf

    def point_flux_jacobian(self, q, nx, ny):
        nv = self.mech.nv
        A = np.zeros((nv, nv))
        a, p = _d(q)
        self._check(self.L.orc_point_flux_jacobian(self.ctx, p, C.c_double(nx), C.c_double(ny),
                                                   A.ctypes.data_as(_dp)))
        return A

    def point_offdiag(self, q, nx, ny, mode, fd, x):
        n = self.mech.nb if mode == COUPLED else self.mech.nf
        out = np.zeros(n)
        a, p = _d(q)
        b, px = _d(x)
        self._check(self.L.orc_point_offdiag(self.ctx, p, C.c_double(nx), C.c_double(ny), mode, int(fd), px,
                                             out.ctypes.data_as(_dp)))
        return out

    def point_source_jacobian(self, q, which):
        m = self.mech
        n = {0: m.nb * m.nb, 1: m.ns * m.ns, 2: m.nf}[which]
        J = np.zeros(n)
        a, p = _d(q)
        self._check(self.L.orc_point_source_jacobian(self.ctx, p, which, J.ctypes.data_as(_dp)))
        if which == 0:
            return J.reshape(m.nb, m.nb)
        if which == 1:
            return J.reshape(m.ns, m.ns)
        return J


def setup(cfg_or_grid, mech, fs, q0=None, T_wall=300.0, bc_mode=0, threads=0):
    """Convenience: oracle with grid (x, y), mechanism and free stream (rho_s, u, v, T, Tv)."""
    o = Oracle(threads, wide=mech.ns > 32)
    x, y = cfg_or_grid
    o.set_grid(x, y, T_wall, bc_mode)
    o.set_mechanism(mech)
    o.set_freestream(*fs)
    if q0 is not None:
        o.set_state(q0)
    return o
