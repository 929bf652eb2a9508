"""Thin Python binding of libcsi.so (include/csi.h): argument marshalling only.

Device memory (the workspace) and the stream come from PyTorch; every step of
the solver runs in the library's HIP kernels.  There is no fallback: if the
library is missing this module raises.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcsi.so")

COUPLED, SPLIT = 0, 1
FP64, MIXED = 0, 1
CLOSURE, CC1, CC2 = 0, 1, 2
JAC_EXACT, JAC_SURROGATE = 0, 1
ERRORS = {-1: "CSI_ERR_ARG", -2: "CSI_ERR_STATE", -3: "CSI_ERR_HIP", -4: "CSI_ERR_NONFINITE",
          -5: "CSI_ERR_SINGULAR", -6: "CSI_ERR_UNSUPPORTED"}

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int)

EXPORTED = ["csi_create", "csi_destroy", "csi_last_error", "csi_set_grid", "csi_set_mechanism",
            "csi_set_freestream", "csi_workspace_bytes", "csi_bind_workspace", "csi_set_state", "csi_get_state",
            "csi_residual", "csi_implicit_op", "csi_consistency_correct", "csi_step", "csi_wall_heat_flux",
            "csi_get_cells",
            "csi_norm_history", "csi_get_array", "csi_prim_to_cons", "csi_set_timing", "csi_phase_times",
            "csi_set_sweep", "csi_mlp_sizes", "csi_mlp_prepare", "csi_mlp_forward", "csi_mlp_grad",
            "csi_mlp_train_step", "csi_sample_jacobians", "csi_set_surrogate", "csi_mlp_forward_noalloc",
            "csi_set_species_jacobian", "csi_set_physical_time", "csi_advance_time",
            "csi_set_time_levels", "csi_set_offdiag", "csi_mlp_train_epoch", "csi_set_species_generic",
            "csi_block_inverse", "csi_block_inverse_work", "csi_set_residual_scheme"]
WIDE_MAX_SPECIES = 4096
PHASES = ["prim", "faces", "cell", "block", "norms", "sweep_fwd", "sweep_bwd", "update"]


class CsiError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class CsiMechanism(C.Structure):
    _fields_ = [("ns", C.c_int), ("nr", C.c_int), ("two_temp", C.c_int),
                ("M", _dp), ("theta_v", _dp), ("theta_r", _dp), ("sigma", _dp), ("g_el", _dp), ("h_form", _dp),
                ("sc", _dp), ("lt_a", _dp), ("lt_b", _dp), ("kind", _ip), ("A", _dp), ("b", _dp), ("theta", _dp),
                ("tctl", _ip), ("third", _ip), ("nu_f", _ip), ("nu_b", _ip), ("eff", _dp),
                ("mu_ref", C.c_double), ("T_ref", C.c_double), ("mu_exp", C.c_double)]


class StepParams(C.Structure):
    _fields_ = [("mode", C.c_int), ("precision", C.c_int), ("kind", C.c_int), ("jac", C.c_int),
                ("cfl", C.c_double), ("cfl_ramp", C.c_int), ("max_iter", C.c_int), ("tol", C.c_double),
                ("check_every", C.c_int)]


class StepStats(C.Structure):
    _fields_ = [("iters", C.c_int), ("converged", C.c_int), ("it_conv", C.c_int), ("n_clipped", C.c_int),
                ("bad_cell", C.c_int), ("r0", C.c_double), ("r_last", C.c_double),
                ("n_dd_fallback", C.c_longlong), ("surrogate_off_at", C.c_int), ("surrogate_diverged", C.c_int)]


class MlpBatch(C.Structure):
    _fields_ = [("n_in", C.c_int), ("n_out", C.c_int), ("n_data", C.c_int), ("batch", C.c_int),
                ("x", C.c_void_p), ("t", C.c_void_p), ("idx", C.c_void_p), ("params", C.c_void_p),
                ("work", C.c_void_p), ("work_bytes", C.c_size_t)]


class Adam(C.Structure):
    _fields_ = [("lr", C.c_double), ("beta1", C.c_double), ("beta2", C.c_double), ("eps", C.c_double)]


_lib = None


def load():
    """Load libcsi.so; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} not built: run __graft_entry__.build() or "
                              "python paper_2403_03440_amd/build.py")
        _lib = C.CDLL(LIB_PATH)
        _lib.csi_last_error.restype = C.c_char_p
    return _lib


def _d(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(_dp)


def _i(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(_ip)


class Solver:
    """One library context on cuda:`device` with its workspace tensor."""

    def __init__(self, grid, mech, freestream, T_wall: float = 300.0, bc_mode: int = 0, device: int = 0,
                 stream=None, generic: bool = False):
        """generic: the species-generic kernels for any species count (they
        are taken anyway above 32 species)."""
        import torch
        self.torch = torch
        self.L = load()
        self.device = device
        self.dev = torch.device("cuda", device)
        st = stream if stream is not None else torch.cuda.current_stream(self.dev)
        self.stream = st
        self.ctx = C.c_void_p()
        rc = self.L.csi_create(C.byref(self.ctx), device, C.c_void_p(st.cuda_stream))
        if rc:
            raise CsiError(rc, "csi_create")
        x, y = grid
        nj1, ni1 = x.shape
        self.ni, self.nj = ni1 - 1, nj1 - 1
        self.N = self.ni * self.nj
        xa, xp = _d(x)
        ya, yp = _d(y)
        self._check(self.L.csi_set_grid(self.ctx, self.ni, self.nj, xp, yp, C.c_double(T_wall), bc_mode))
        self._check(self.L.csi_set_species_generic(self.ctx, 1 if generic else 0))
        self.set_mechanism(mech)
        self.set_freestream(*freestream)
        nbytes = C.c_size_t(0)
        self._check(self.L.csi_workspace_bytes(self.ctx, C.byref(nbytes)))
        self.ws = torch.empty(nbytes.value, dtype=torch.uint8, device=self.dev)
        self._check(self.L.csi_bind_workspace(self.ctx, C.c_void_p(self.ws.data_ptr()), C.c_size_t(nbytes.value)))
        self.last_mode = None

    def __del__(self):
        try:
            self.L.csi_destroy(self.ctx)
        except Exception:
            pass

    def _check(self, rc):
        if rc != 0:
            raise CsiError(rc, self.L.csi_last_error(self.ctx).decode())

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

        nr = m.nr
        s = CsiMechanism(m.ns, nr, int(m.two_temp), d(m.M), d(m.theta_v), d(m.theta_r), d(m.sigma), d(m.g_el),
                         d(m.h_form), d(m.sc), d(m.lt_a), d(m.lt_b), i(m.kind),
                         d(m.A if nr else [0.0]), d(m.b if nr else [0.0]), d(m.theta if nr else [0.0]),
                         i(m.tctl if nr else [0]), i(m.third if nr else [0]),
                         i(np.asarray(m.nu_f).ravel() if nr else [0]), i(np.asarray(m.nu_b).ravel() if nr else [0]),
                         d(np.asarray(m.eff).ravel() if nr else [0.0]), m.mu_ref, m.T_ref, m.mu_exp)
        self._check(self.L.csi_set_mechanism(self.ctx, C.byref(s)))
        self.mech = m

    def set_freestream(self, rho_s, u, v, T, Tv):
        a, p = _d(rho_s)
        self._check(self.L.csi_set_freestream(self.ctx, p, C.c_double(u), C.c_double(v), C.c_double(T),
                                              C.c_double(Tv)))

    # ------------------------------------------------------------- state
    def set_state(self, q):
        if isinstance(q, np.ndarray):
            a, p = _d(q)
            self._check(self.L.csi_set_state(self.ctx, p, 0))
        else:
            t = q.to(device=self.dev, dtype=self.torch.float64).contiguous()
            self._check(self.L.csi_set_state(self.ctx, C.c_void_p(t.data_ptr()), 1))

    def get_state(self):
        q = np.zeros((self.mech.nv, self.N))
        self._check(self.L.csi_get_state(self.ctx, q.ctypes.data_as(_dp), 0))
        return q

    def get_state_device(self):
        t = self.torch.empty((self.mech.nv, self.N), dtype=self.torch.float64, device=self.dev)
        self._check(self.L.csi_get_state(self.ctx, C.c_void_p(t.data_ptr()), 1))
        return t

    # --------------------------------------------------------- algorithm
    def residual(self, cfl):
        n = np.zeros(2)
        self._check(self.L.csi_residual(self.ctx, C.c_double(cfl), n.ctypes.data_as(_dp)))
        return n

    def implicit_op(self, mode, precision=FP64, jac=JAC_EXACT):
        self._check(self.L.csi_implicit_op(self.ctx, mode, precision, jac))
        self.last_mode = mode

    def consistency_correct(self, kind):
        self._check(self.L.csi_consistency_correct(self.ctx, kind))

    def step(self, mode, kind, cfl, max_iter, precision=FP64, jac=JAC_EXACT, cfl_ramp=0, tol=0.0, check_every=50):
        p = StepParams(mode, precision, kind, jac, cfl, cfl_ramp, max_iter, tol, check_every)
        s = StepStats()
        self._check(self.L.csi_step(self.ctx, C.byref(p), C.byref(s)))
        return {k: getattr(s, k) for k, _ in StepStats._fields_}

    def norm_history(self, n):
        h = np.zeros((n, 2))
        self._check(self.L.csi_norm_history(self.ctx, n, h.ctypes.data_as(_dp)))
        return h

    def wall_heat_flux(self):
        qw = np.zeros(self.ni)
        qs = C.c_double(0)
        self._check(self.L.csi_wall_heat_flux(self.ctx, qw.ctypes.data_as(_dp), C.byref(qs)))
        return qw, qs.value

    def nsol(self, mode):
        return self.mech.nb if mode == COUPLED else self.mech.nf + self.mech.ns

    def get(self, name, mode: Optional[int] = None):
        m = self.mech
        N = self.N
        mode = self.last_mode if mode is None else mode
        shapes = {"R": (m.nv, N), "dtau": (N,), "src": (m.nv, N), "qw": (self.ni,), "T": (N,), "Tv": (N,),
                  "p": (N,), "c": (N,), "Jsur": (m.ns * m.ns, N),
                  "sweep_trace": (2, 2, self.ni, 8)}
        if name in ("b", "dqs", "dq"):
            shape = (self.nsol(mode), N)
        elif name == "Dinv":
            shape = (m.nb * m.nb, N) if mode == COUPLED else (m.nf * m.nf + m.ns * m.ns, N)
        else:
            shape = shapes[name]
        out = np.zeros(shape)
        self._check(self.L.csi_get_array(self.ctx, name.encode(), out.ctypes.data_as(_dp), C.c_size_t(out.size)))
        return out

    def get_cells(self, name, cells, mode: Optional[int] = None):
        """`get(name)` at the listed cells only: [F][len(cells)]."""
        m = self.mech
        mode = self.last_mode if mode is None else mode
        if name == "R":
            F = m.nv
        elif name == "Dinv":
            F = m.nb * m.nb if mode == COUPLED else m.nf * m.nf + m.ns * m.ns
        else:
            F = self.nsol(mode)
        cl = np.ascontiguousarray(np.asarray(cells, dtype=np.int64))
        out = np.zeros((F, cl.size))
        self._check(self.L.csi_get_cells(self.ctx, name.encode(), cl.ctypes.data_as(C.POINTER(C.c_longlong)),
                                         int(cl.size), out.ctypes.data_as(_dp)))
        return out

    def initial_state(self, rho_s, u, v, T, Tv):
        """Conservative variables from primitives with the library's thermodynamics."""
        rho_s = np.atleast_2d(rho_s)
        n = rho_s.shape[1]
        q = np.zeros((self.mech.nv, n))
        args = [_d(a) for a in (rho_s, u, v, T, Tv)]
        self._check(self.L.csi_prim_to_cons(self.ctx, n, *[p for _, p in args], q.ctypes.data_as(_dp)))
        return q

    def set_sweep(self, schedule):
        """0: one launch per i+j hyperplane; 1: persistent group kernels (default)"""
        self._check(self.L.csi_set_sweep(self.ctx, int(schedule)))

    def set_offdiag(self, op):
        """0: linear Jacobian-vector products; 1: flux differences (FP64,
        per-hyperplane schedule)"""
        self._check(self.L.csi_set_offdiag(self.ctx, int(op)))

    def set_timing(self, on=True):
        """1: phase timing with HIP events; 2: also a per-strip sweep trace (get("sweep_trace"))"""
        self._check(self.L.csi_set_timing(self.ctx, int(on)))

    def phase_times(self, reset=False):
        ms = np.zeros(len(PHASES) + 1)
        self._check(self.L.csi_phase_times(self.ctx, ms.ctypes.data_as(_dp), int(reset)))
        n = max(ms[-1], 1.0)
        out = {k: {"ms": float(ms[i]), "ms_per_iter": float(ms[i] / n)} for i, k in enumerate(PHASES)}
        out["iters"] = int(ms[-1])
        return out

    # ---------------------------------------------------------- surrogate
    def sample_jacobians(self, x_raw, jc, max_samples=None, seed=0):
        """Features [n][ns+3] and exact J_C [n][ns*ns] (float32 cuda tensors) of
        every cell of the current state (n = N), or of a seeded subset of
        n = max_samples distinct cells (see csi.h); returns n."""
        n = C.c_int(0)
        ms = self.N if max_samples is None else max_samples
        self._check(self.L.csi_sample_jacobians(self.ctx, ms, C.c_ulonglong(seed), C.c_void_p(x_raw.data_ptr()),
                                                C.c_void_p(jc.data_ptr()), C.byref(n)))
        return n.value


    def set_physical_time(self, dt, theta=0.0):
        """Dual time stepping: physical step dt (0: steady) and theta (0 backward
        Euler, 0.5 second-order backward difference)."""
        self._check(self.L.csi_set_physical_time(self.ctx, C.c_double(dt), C.c_double(theta)))

    def advance_time(self):
        """Q^{n-1} <- Q^n <- Q: start the next physical time step."""
        self._check(self.L.csi_advance_time(self.ctx))

    def set_time_levels(self, qn, qnm1):
        """Time levels Q^n, Q^{n-1} (host float64 [nv][N] each)."""
        a, pa = _d(qn)
        b, pb = _d(qnm1)
        self._check(self.L.csi_set_time_levels(self.ctx, pa, pb, 0))

    def set_residual_scheme(self, scheme):
        """0: first-order HLLE; 1: MUSCL (minmod) + Roe."""
        self._check(self.L.csi_set_residual_scheme(self.ctx, scheme))

    def set_species_jacobian(self, reading):
        """0: split species block at fixed T, Tv; 1: at fixed velocities and
        internal energy densities (temperatures follow the composition)."""
        self._check(self.L.csi_set_species_jacobian(self.ctx, int(reading)))

    def set_surrogate(self, params, scales, stall_ratio=0.98, stall_window=100):
        """Install a network: params float32 cuda tensor, scales (mu, sigma, tau0) host."""
        sa, sp = _d(scales)
        ns = self.mech.ns
        self._check(self.L.csi_set_surrogate(self.ctx, C.c_void_p(params.data_ptr()), sp, ns + 3, ns * ns,
                                             C.c_double(stall_ratio), stall_window))

    def synchronize(self):
        self.torch.cuda.synchronize(self.dev)


def block_inverse(a, device=0, stream=None):
    """In-place inverse of the dense FP64 matrices a[..., n, n] (a contiguous
    cuda tensor) by the library's blocked Gauss-Jordan kernels; returns a."""
    import torch
    L = load()
    if a.dtype != torch.float64 or not a.is_cuda or not a.is_contiguous() or a.dim() < 2 or a.shape[-1] != a.shape[-2]:
        raise ValueError("block_inverse: contiguous cuda float64 tensor of square matrices expected")
    n = a.shape[-1]
    count = a.numel() // (n * n) if n else 0
    dev = torch.device("cuda", device)
    st = stream if stream is not None else torch.cuda.current_stream(dev)
    ctx = C.c_void_p()
    rc = L.csi_create(C.byref(ctx), device, C.c_void_p(st.cuda_stream))
    if rc:
        raise CsiError(rc, "csi_create")
    try:
        wb = C.c_size_t(0)
        rc = L.csi_block_inverse_work(n, count, C.byref(wb))
        if rc:
            raise CsiError(rc, "csi_block_inverse_work")
        work = torch.empty(wb.value, dtype=torch.uint8, device=dev)
        sing = C.c_int(-1)
        rc = L.csi_block_inverse(ctx, n, count, C.c_void_p(a.data_ptr()), C.c_void_p(work.data_ptr()),
                                 C.c_size_t(wb.value), C.byref(sing))
        if rc:
            raise CsiError(rc, L.csi_last_error(ctx).decode())
    finally:
        L.csi_destroy(ctx)
    return a


class Mlp:
    """The surrogate network's kernels (hidden width 64) on one stream: data
    preparation, inference, gradient and Adam training steps.  Tensors are
    cuda tensors owned by the caller; the work buffer is allocated here with
    torch for up to `batch` samples per call."""

    def __init__(self, n_in, n_out, batch=4096, device=0, stream=None):
        import torch
        self.torch = torch
        self.L = load()
        self.n_in, self.n_out, self.batch = n_in, n_out, batch
        self.dev = torch.device("cuda", device)
        st = stream if stream is not None else torch.cuda.current_stream(self.dev)
        self.ctx = C.c_void_p()
        rc = self.L.csi_create(C.byref(self.ctx), device, C.c_void_p(st.cuda_stream))
        if rc:
            raise CsiError(rc, "csi_create")
        npar, wb = C.c_int(0), C.c_size_t(0)
        rc = self.L.csi_mlp_sizes(n_in, n_out, batch, C.byref(npar), C.byref(wb))
        if rc:
            raise CsiError(rc, "csi_mlp_sizes")
        self.n_params = npar.value
        self.work = torch.empty(wb.value, dtype=torch.uint8, device=self.dev)

    def __del__(self):
        try:
            self.L.csi_destroy(self.ctx)
        except Exception:
            pass

    def _check(self, rc):
        if rc != 0:
            raise CsiError(rc, self.L.csi_last_error(self.ctx).decode())

    def _w(self):
        return C.c_void_p(self.work.data_ptr()), C.c_size_t(self.work.numel())

    @staticmethod
    def _p(t):
        return C.c_void_p(t.data_ptr())

    def prepare(self, x_raw, jc):
        """Standardised features, asinh targets and the scales (mu, sigma, tau0)."""
        n = x_raw.shape[0]
        x = self.torch.empty_like(x_raw)
        t = self.torch.empty_like(jc)
        scales = np.zeros(2 * self.n_in + 1)
        self._check(self.L.csi_mlp_prepare(self.ctx, n, self.n_in, self.n_out, self._p(x_raw), self._p(jc),
                                           self._p(x), self._p(t), scales.ctypes.data_as(_dp), *self._w()))
        return x, t, scales

    def forward(self, params, x):
        y = self.torch.empty((x.shape[0], self.n_out), dtype=self.torch.float32, device=self.dev)
        self._check(self.L.csi_mlp_forward(self.ctx, self.n_in, self.n_out, x.shape[0], self._p(params),
                                           self._p(x), self._p(y), *self._w()))
        return y

    def forward_noalloc(self, params, x, y):
        """y[:n] = network(x) through csi_mlp_forward_noalloc: the library's own
        per-GPU scratch instead of this object's work tensor; y is the caller's
        float32 cuda tensor [n][n_out]."""
        self._check(self.L.csi_mlp_forward_noalloc(self.ctx, self.n_in, self.n_out, x.shape[0], self._p(params),
                                                   self._p(x), self._p(y)))
        return y

    def _batch(self, params, x, t, idx):
        w, wb = self._w()
        return MlpBatch(self.n_in, self.n_out, x.shape[0], idx.shape[0], self._p(x).value, self._p(t).value,
                        self._p(idx).value, self._p(params).value, w.value, wb.value)

    def grad(self, params, x, t, idx):
        g = self.torch.empty(self.n_params, dtype=self.torch.float32, device=self.dev)
        loss = C.c_double(0)
        b = self._batch(params, x, t, idx)
        self._check(self.L.csi_mlp_grad(self.ctx, C.byref(b), self._p(g), C.byref(loss)))
        return g, loss.value

    def train_epoch(self, params, m, v, x, t, order, step0, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        """Adam steps over the device row order `order` (int32), self.batch rows
        at a time; returns the last batch's loss."""
        b = self._batch(params, x, t, order[:min(self.batch, order.numel())])
        b.batch = self.batch
        h = Adam(lr, beta1, beta2, eps)
        loss = C.c_double(0)
        self._check(self.L.csi_mlp_train_epoch(self.ctx, C.byref(b), self._p(order), int(order.numel()),
                                               self._p(m), self._p(v), int(step0), C.byref(h), C.byref(loss)))
        return loss.value

    def train_step(self, params, m, v, x, t, idx, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8,
                   want_loss=True):
        b = self._batch(params, x, t, idx)
        h = Adam(lr, beta1, beta2, eps)
        loss = C.c_double(0)
        self._check(self.L.csi_mlp_train_step(self.ctx, C.byref(b), self._p(m), self._p(v), step, C.byref(h),
                                              C.byref(loss) if want_loss else None))
        return loss.value if want_loss else None
