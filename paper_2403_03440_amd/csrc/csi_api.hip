// Host side of the C-ABI (include/csi.h): context, grid metrics, mechanism
// tables, workspace layout inside the caller's device buffer, and the launch
// sequence of each call.  No device memory is allocated here.
#include <climits>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/csi.h"
#include "csi_mech.hpp"
#include "csi_runner.hpp"

using namespace csi;

// per-species-count factories (weak: a build may compile a subset)
__attribute__((weak)) csi::IRunner *csi_make_runner_2(int);
__attribute__((weak)) csi::IRunner *csi_make_runner_3(int);
__attribute__((weak)) csi::IRunner *csi_make_runner_5(int);
__attribute__((weak)) csi::IRunner *csi_make_runner_11(int);
__attribute__((weak)) csi::IRunner *csi_make_runner_20(int);

namespace csi {
IRunner *make_runner(int ns, int nt) {
  switch (ns) {
    case 2: return csi_make_runner_2 ? csi_make_runner_2(nt) : nullptr;
    case 3: return csi_make_runner_3 ? csi_make_runner_3(nt) : nullptr;
    case 5: return csi_make_runner_5 ? csi_make_runner_5(nt) : nullptr;
    case 11: return csi_make_runner_11 ? csi_make_runner_11(nt) : nullptr;
    case 20: return csi_make_runner_20 ? csi_make_runner_20(nt) : nullptr;
    default: return nullptr;
  }
}
}  // namespace csi

struct csi_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string err;
  // grid (host)
  int ni = 0, nj = 0, N = 0, bc_mode = 0;
  double Tw = 300.0;
  std::vector<double> xn, yn, xc, yc, V, fi_nx, fi_ny, fi_S, fj_nx, fj_ny, fj_S;
  // mechanism (host copy of the device table)
  Mech mech;
  int ns = 0, nt = 1;
  IRunner *run = nullptr;
  double qfs[MAXS + 4];
  bool has_grid = false, has_mech = false, has_fs = false, bound = false, has_state = false, has_res = false;
  int last_mode = -1, last_prec = -1;
  bool has_dq = false;
  // workspace
  char *ws = nullptr;
  size_t ws_bytes = 0;
  WS w;
  Geo g;
  long it_global = 0;
  int strip_w = 16;  // sweep schedule: 0 hyperplane launches, 16 / 64 persistent strips
  int pub_every = 4;  // strip progress publication interval (steps)
  // phase timing (HIP events, created on first use)
  bool timing = false;
  std::vector<hipEvent_t> ev;
  double phase_ms[7] = {0, 0, 0, 0, 0, 0, 0};

  int nv() const { return ns + 3 + (nt == 2 ? 1 : 0); }
  int nf() const { return nt == 2 ? 5 : 4; }
  int nb() const { return nf() + ns - 1; }
  int nsplit() const { return nf() + ns; }
  int fail(int code, const std::string &m) { err = m; return code; }
};

namespace {

constexpr int HIST_MAX = 1 << 20;

int hip_check(csi_ctx *c, hipError_t e, const char *what) {
  if (e != hipSuccess) return c->fail(CSI_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
  return CSI_OK;
}

struct Layout {
  size_t off[40];
  size_t total;
};

size_t al(size_t x) { return (x + 255) & ~size_t(255); }

// workspace layout (bytes); order fixed, every block 256-byte aligned
Layout layout(const csi_ctx *c, int nprim) {
  Layout L;
  size_t o = 0;
  int k = 0;
  const size_t N = c->N, NP = size_t(c->ni + 2) * (c->nj + 2), NN = size_t(c->ni + 1) * (c->nj + 1);
  const size_t nfi = size_t(c->ni + 1) * c->nj, nfj = size_t(c->ni) * (c->nj + 1);
  const int nv = c->nv(), nsol = c->nsplit();
  const size_t ndinv = std::max<size_t>(size_t(c->nb()) * c->nb(), 6 + size_t(c->ns) * c->ns);
  const size_t nblk = (N + 255) / 256;
  // per-cell sweep records: cell-major (N) or strip layout (up to the widest strip)
  const StripMap sm = strip_map(c->ni, c->nj, 16), sm64 = strip_map(c->ni, c->nj, 64);
  const size_t A = std::max<size_t>(N, std::max<size_t>(sm.LEN, sm64.LEN));
  const size_t nstrip = std::max(sm.nstrip, sm64.nstrip);
  size_t sizes[] = {
      sizeof(Mech),                       // 0 mech
      N * 8, N * 8, N * 8, NN * 8, NN * 8, // 1-5 V xc yc xn yn
      nfi * 8, nfi * 8, nfi * 8,          // 6-8 fi
      nfj * 8, nfj * 8, nfj * 8,          // 9-11 fj
      size_t(nv) * 8,                     // 12 qfs
      size_t(nv) * N * 8,                 // 13 Q
      size_t(nprim) * NP * 8,             // 14 prim
      size_t(nv) * nfi * 8, size_t(nv) * nfj * 8,      // 15-16 Fi Fj
      size_t(R_N) * nfi * 8, size_t(R_N) * nfj * 8,    // 17-18 Ri Rj
      size_t(nv) * N * 8, N * 8, size_t(nv) * N * 8,   // 19-21 R dtau src
      size_t(c->ni) * 8, 2 * nblk * 8, 2 * 8, 8,       // 22-25 qw part norms r0
      size_t(2) * HIST_MAX * 8,                       // 26 hist
      size_t(nsol) * A * 8, size_t(nsol) * A * 8, size_t(nsol) * A * 8,  // 27-29 b dqs dq
      ndinv * A * 8,                                  // 30 Dinv
      FL_N * 4,                                       // 31 flags
      size_t(6 + 2 * c->ns) * A * 8,                  // 32 strip state records
      size_t(16) * A * 8,                             // 33 strip face records
      size_t(nstrip) * c->nj * nsol * 8,              // 34 strip-boundary pushes
      size_t(2 * nstrip + 2) * 4,                     // 35 strip progress counters and tickets
  };
  for (size_t s : sizes) { L.off[k++] = o; o += al(s); }
  L.total = o;
  return L;
}

void compute_metrics(csi_ctx *c, const double *xn, const double *yn) {
  const int ni = c->ni, nj = c->nj;
  c->xn.assign(xn, xn + size_t(ni + 1) * (nj + 1));
  c->yn.assign(yn, yn + size_t(ni + 1) * (nj + 1));
  auto X = [&](int I, int J) { return c->xn[size_t(J) * (ni + 1) + I]; };
  auto Y = [&](int I, int J) { return c->yn[size_t(J) * (ni + 1) + I]; };
  c->V.assign(c->N, 0.0);
  c->xc.assign(c->N, 0.0);
  c->yc.assign(c->N, 0.0);
  double sgn = 1.0;
  for (int j = 0; j < nj; ++j)
    for (int i = 0; i < ni; ++i) {
      double x0 = X(i, j), y0 = Y(i, j), x1 = X(i + 1, j), y1 = Y(i + 1, j);
      double x2 = X(i + 1, j + 1), y2 = Y(i + 1, j + 1), x3 = X(i, j + 1), y3 = Y(i, j + 1);
      double a = 0.5 * ((x0 * y1 - x1 * y0) + (x1 * y2 - x2 * y1) + (x2 * y3 - x3 * y2) + (x3 * y0 - x0 * y3));
      if (i == 0 && j == 0) sgn = a > 0 ? 1.0 : -1.0;
      size_t p = size_t(j) * ni + i;
      c->V[p] = std::fabs(a);
      c->xc[p] = 0.25 * (x0 + x1 + x2 + x3);
      c->yc[p] = 0.25 * (y0 + y1 + y2 + y3);
    }
  size_t nfi = size_t(ni + 1) * nj, nfj = size_t(ni) * (nj + 1);
  c->fi_nx.assign(nfi, 0); c->fi_ny.assign(nfi, 0); c->fi_S.assign(nfi, 0);
  for (int j = 0; j < nj; ++j)
    for (int I = 0; I <= ni; ++I) {
      double tx = X(I, j + 1) - X(I, j), ty = Y(I, j + 1) - Y(I, j);
      double nx = sgn * ty, ny = -sgn * tx, S = std::sqrt(nx * nx + ny * ny);
      size_t f = size_t(j) * (ni + 1) + I;
      c->fi_S[f] = S; c->fi_nx[f] = nx / S; c->fi_ny[f] = ny / S;
    }
  c->fj_nx.assign(nfj, 0); c->fj_ny.assign(nfj, 0); c->fj_S.assign(nfj, 0);
  for (int J = 0; J <= nj; ++J)
    for (int i = 0; i < ni; ++i) {
      double tx = X(i + 1, J) - X(i, J), ty = Y(i + 1, J) - Y(i, J);
      double nx = -sgn * ty, ny = sgn * tx, S = std::sqrt(nx * nx + ny * ny);
      size_t f = size_t(J) * ni + i;
      c->fj_S[f] = S; c->fj_nx[f] = nx / S; c->fj_ny[f] = ny / S;
    }
}

bool ready(csi_ctx *c) { return c && c->bound && c->has_state; }

int read_flags(csi_ctx *c, int *fl) {
  int rc = hip_check(c, hipMemcpyAsync(fl, c->w.flags, FL_N * sizeof(int), hipMemcpyDeviceToHost, c->stream), "flags");
  if (rc) return rc;
  return hip_check(c, hipStreamSynchronize(c->stream), "sync");
}

int reset_flags(csi_ctx *c) {
  int fl[FL_N] = {INT_MAX, 0, -1, 0, INT_MAX, 0, 0, 0};
  int rc = hip_check(c, hipMemcpyAsync(c->w.flags, fl, sizeof(fl), hipMemcpyHostToDevice, c->stream), "flags");
  if (rc) return rc;
  return hip_check(c, hipStreamSynchronize(c->stream), "sync");
}

}  // namespace

extern "C" {

int csi_create(csi_ctx **ctx, int device, void *hip_stream) {
  if (!ctx) return CSI_ERR_ARG;
  csi_ctx *c = new csi_ctx();
  c->device = device;
  c->stream = reinterpret_cast<hipStream_t>(hip_stream);
  if (hipSetDevice(device) != hipSuccess) { delete c; return CSI_ERR_HIP; }
  *ctx = c;
  return CSI_OK;
}

int csi_destroy(csi_ctx *c) {
  if (!c) return CSI_ERR_ARG;
  for (hipEvent_t e : c->ev) (void)hipEventDestroy(e);
  delete c->run;
  delete c;
  return CSI_OK;
}

const char *csi_last_error(const csi_ctx *c) { return c ? c->err.c_str() : "null context"; }

int csi_set_grid(csi_ctx *c, int ni, int nj, const double *xn, const double *yn, double T_wall, int bc_mode) {
  if (!c) return CSI_ERR_ARG;
  if (ni < 1 || nj < 1 || !xn || !yn || (bc_mode != 0 && bc_mode != 1) || !(T_wall > 0.0) ||
      double(ni) * nj > 2.0e9)
    return c->fail(CSI_ERR_ARG, "set_grid: bad arguments");
  c->ni = ni; c->nj = nj; c->N = ni * nj; c->Tw = T_wall; c->bc_mode = bc_mode;
  compute_metrics(c, xn, yn);
  c->has_grid = true;
  c->bound = false;
  c->has_state = false;
  c->has_res = false;
  return CSI_OK;
}

int csi_set_mechanism(csi_ctx *c, const csi_mechanism *mm) {
  if (!c || !mm) return CSI_ERR_ARG;
  if (mm->ns < 2 || mm->ns > MAXS || mm->nr < 0 || mm->nr > MAXR) return c->fail(CSI_ERR_ARG, "set_mechanism: sizes");
  IRunner *r = make_runner(mm->ns, mm->two_temp ? 2 : 1);
  if (!r) return c->fail(CSI_ERR_UNSUPPORTED, "no kernels compiled for ns = " + std::to_string(mm->ns));
  std::string err;
  if (!build_mech(mm, c->mech, err)) { delete r; return c->fail(CSI_ERR_ARG, "set_mechanism: " + err); }
  delete c->run;
  c->run = r;
  c->ns = mm->ns;
  c->nt = mm->two_temp ? 2 : 1;
  c->strip_w = mm->ns <= 11 ? 64 : 16;  // widest compiled strip (fewest strip boundaries)
  c->has_mech = true;
  c->has_fs = false;
  c->bound = false;
  c->has_state = false;
  c->has_res = false;
  return CSI_OK;
}

int csi_set_freestream(csi_ctx *c, const double *rho_s, double u, double v, double T, double Tv) {
  if (!c || !rho_s) return CSI_ERR_ARG;
  if (!c->has_mech) return c->fail(CSI_ERR_STATE, "set_freestream before set_mechanism");
  if (!(T > 0.0) || (c->nt == 2 && !(Tv > 0.0))) return c->fail(CSI_ERR_ARG, "free-stream temperature");
  (void)c->run->q_from_prim_host(c->mech, rho_s, u, v, T, Tv, c->qfs);
  c->has_fs = true;
  if (c->bound) {
    int rc = hip_check(c, hipMemcpyAsync(c->w.qfs, c->qfs, c->nv() * 8, hipMemcpyHostToDevice, c->stream), "qfs");
    if (rc) return rc;
    return hip_check(c, hipStreamSynchronize(c->stream), "sync");
  }
  return CSI_OK;
}

int csi_workspace_bytes(const csi_ctx *c, size_t *bytes) {
  if (!c || !bytes) return CSI_ERR_ARG;
  if (!c->has_grid || !c->has_mech) return CSI_ERR_STATE;
  *bytes = layout(c, c->run->nprim()).total;
  return CSI_OK;
}

int csi_bind_workspace(csi_ctx *c, void *dev, size_t bytes) {
  if (!c || !dev) return CSI_ERR_ARG;
  if (!c->has_grid || !c->has_mech || !c->has_fs) return c->fail(CSI_ERR_STATE, "bind before grid/mechanism/free stream");
  if (reinterpret_cast<uintptr_t>(dev) % 256) return c->fail(CSI_ERR_ARG, "workspace not 256-byte aligned");
  Layout L = layout(c, c->run->nprim());
  if (bytes < L.total) return c->fail(CSI_ERR_ARG, "workspace too small: need " + std::to_string(L.total));
  char *b = static_cast<char *>(dev);
  c->ws = b;
  c->ws_bytes = bytes;
  WS &w = c->w;
  int k = 0;
  auto D = [&](int idx) { return reinterpret_cast<double *>(b + L.off[idx]); };
  w.mech = reinterpret_cast<Mech *>(b + L.off[k++]);
  w.V = D(1); w.xc = D(2); w.yc = D(3); w.xn = D(4); w.yn = D(5);
  w.fi_nx = D(6); w.fi_ny = D(7); w.fi_S = D(8); w.fj_nx = D(9); w.fj_ny = D(10); w.fj_S = D(11);
  w.qfs = D(12); w.Q = D(13); w.prim = D(14); w.Fi = D(15); w.Fj = D(16); w.Ri = D(17); w.Rj = D(18);
  w.R = D(19); w.dtau = D(20); w.src = D(21); w.qw = D(22); w.part = D(23); w.norms = D(24); w.r0 = D(25);
  w.hist = D(26);
  w.b = b + L.off[27]; w.dqs = b + L.off[28]; w.dq = b + L.off[29]; w.Dinv = b + L.off[30];
  w.flags = reinterpret_cast<int *>(b + L.off[31]);
  w.state = b + L.off[32];
  w.face = b + L.off[33];
  w.bnd = b + L.off[34];
  w.sync = reinterpret_cast<int *>(b + L.off[35]);
  w.strip_w = c->strip_w;
  w.pub_every = c->pub_every;
  w.spin_limit = 4000000;
  w.nblk_cell = (c->N + 255) / 256;
  w.hist_max = HIST_MAX;
  Geo &g = c->g;
  g.ni = c->ni; g.nj = c->nj; g.N = c->N; g.NP = (c->ni + 2) * (c->nj + 2); g.bc_mode = c->bc_mode; g.Tw = c->Tw;
  g.V = w.V; g.xc = w.xc; g.yc = w.yc; g.xn = w.xn; g.yn = w.yn;
  g.fi_nx = w.fi_nx; g.fi_ny = w.fi_ny; g.fi_S = w.fi_S; g.fj_nx = w.fj_nx; g.fj_ny = w.fj_ny; g.fj_S = w.fj_S;
  hipStream_t st = c->stream;
  auto up = [&](double *d, const std::vector<double> &h) {
    return hipMemcpyAsync(d, h.data(), h.size() * 8, hipMemcpyHostToDevice, st);
  };
  hipError_t e = hipMemcpyAsync(w.mech, &c->mech, sizeof(Mech), hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = up(w.V, c->V);
  if (e == hipSuccess) e = up(w.xc, c->xc);
  if (e == hipSuccess) e = up(w.yc, c->yc);
  if (e == hipSuccess) e = up(w.xn, c->xn);
  if (e == hipSuccess) e = up(w.yn, c->yn);
  if (e == hipSuccess) e = up(w.fi_nx, c->fi_nx);
  if (e == hipSuccess) e = up(w.fi_ny, c->fi_ny);
  if (e == hipSuccess) e = up(w.fi_S, c->fi_S);
  if (e == hipSuccess) e = up(w.fj_nx, c->fj_nx);
  if (e == hipSuccess) e = up(w.fj_ny, c->fj_ny);
  if (e == hipSuccess) e = up(w.fj_S, c->fj_S);
  if (e == hipSuccess) e = hipMemcpyAsync(w.qfs, c->qfs, c->nv() * 8, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemsetAsync(w.qw, 0, size_t(c->ni) * 8, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  int rc = hip_check(c, e, "bind_workspace");
  if (rc) return rc;
  c->bound = true;
  c->has_state = false;
  c->has_res = false;
  return reset_flags(c);
}

int csi_set_state(csi_ctx *c, const double *q, int on_device) {
  if (!c || !q) return CSI_ERR_ARG;
  if (!c->bound) return c->fail(CSI_ERR_STATE, "set_state before bind_workspace");
  size_t n = size_t(c->nv()) * c->N * 8;
  int rc = hip_check(c, hipMemcpyAsync(c->w.Q, q, n, on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                                       c->stream), "set_state");
  if (rc) return rc;
  rc = hip_check(c, hipStreamSynchronize(c->stream), "sync");
  if (rc) return rc;
  c->has_state = true;
  c->has_res = false;
  c->has_dq = false;
  c->it_global = 0;
  return reset_flags(c);
}

int csi_get_state(csi_ctx *c, double *q, int on_device) {
  if (!c || !q) return CSI_ERR_ARG;
  if (!ready(c)) return c->fail(CSI_ERR_STATE, "no state");
  size_t n = size_t(c->nv()) * c->N * 8;
  int rc = hip_check(c, hipMemcpyAsync(q, c->w.Q, n, on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                                       c->stream), "get_state");
  if (rc) return rc;
  return hip_check(c, hipStreamSynchronize(c->stream), "sync");
}

int csi_residual(csi_ctx *c, double cfl, double *norms) {
  if (!c) return CSI_ERR_ARG;
  if (!ready(c)) return c->fail(CSI_ERR_STATE, "residual: workspace/state not set");
  if (!(cfl > 0.0)) return c->fail(CSI_ERR_ARG, "cfl must be positive");
  int rc = reset_flags(c);
  if (rc) return rc;
  hipError_t e = c->run->prim(c->g, c->w, c->stream, false);
  if (e == hipSuccess) e = c->run->faces(c->g, c->w, c->stream, false);
  if (e == hipSuccess) e = c->run->cell(c->g, c->w, c->stream, cfl, 0, 0, 1, false);
  if (e == hipSuccess) e = c->run->norms(c->w, c->stream, 0, 0.0, false);
  if ((rc = hip_check(c, e, "residual launch"))) return rc;
  int fl[FL_N];
  if ((rc = read_flags(c, fl))) return rc;
  if (fl[FL_BAD] != INT_MAX) return c->fail(CSI_ERR_NONFINITE, "non-physical state at cell " + std::to_string(fl[FL_BAD]));
  if (norms) {
    rc = hip_check(c, hipMemcpy(norms, c->w.norms, 2 * 8, hipMemcpyDeviceToHost), "norms");
    if (rc) return rc;
  }
  c->has_res = true;
  c->has_dq = false;
  return CSI_OK;
}

int csi_implicit_op(csi_ctx *c, int mode, int precision, int jac) {
  if (!c) return CSI_ERR_ARG;
  if (mode != CSI_COUPLED && mode != CSI_SPLIT) return c->fail(CSI_ERR_ARG, "mode");
  if (precision != CSI_FP64 && precision != CSI_MIXED) return c->fail(CSI_ERR_ARG, "precision");
  if (jac != CSI_JAC_EXACT) return c->fail(CSI_ERR_UNSUPPORTED, "surrogate Jacobian not installed");
  if (!ready(c) || !c->has_res) return c->fail(CSI_ERR_STATE, "implicit_op before residual");
  hipError_t e = c->run->cell(c->g, c->w, c->stream, 0.0, mode, precision, 2, false);
  if (e == hipSuccess) e = c->run->sweeps(c->g, c->w, c->stream, mode, precision, false);
  int rc = hip_check(c, e, "implicit_op launch");
  if (rc) return rc;
  int fl[FL_N];
  if ((rc = read_flags(c, fl))) return rc;
  if (fl[FL_ABORT]) return c->fail(CSI_ERR_HIP, "implicit_op: a sweep wave timed out waiting for its neighbour");
  if (fl[FL_SING] != INT_MAX)
    return c->fail(CSI_ERR_SINGULAR, "singular diagonal block at cell " + std::to_string(fl[FL_SING]));
  c->last_mode = mode;
  c->last_prec = precision;
  c->has_dq = true;
  return CSI_OK;
}

int csi_consistency_correct(csi_ctx *c, int kind) {
  if (!c) return CSI_ERR_ARG;
  if (!ready(c) || !c->has_dq) return c->fail(CSI_ERR_STATE, "consistency_correct before implicit_op");
  if (c->last_mode == CSI_COUPLED && kind != CSI_CLOSURE) return c->fail(CSI_ERR_ARG, "coupled mode uses the closure");
  if (c->last_mode == CSI_SPLIT && kind != CSI_CC1 && kind != CSI_CC2) return c->fail(CSI_ERR_ARG, "split mode uses CC1/CC2");
  hipError_t e = c->run->update(c->g, c->w, c->stream, c->last_mode, c->last_prec, kind, false);
  int rc = hip_check(c, e, "update launch");
  if (rc) return rc;
  int fl[FL_N];
  if ((rc = read_flags(c, fl))) return rc;
  c->has_dq = false;
  c->has_res = false;
  if (fl[FL_BAD] != INT_MAX)
    return c->fail(CSI_ERR_NONFINITE, "non-positive density after update at cell " + std::to_string(fl[FL_BAD]));
  return CSI_OK;
}

int csi_step(csi_ctx *c, const csi_step_params *p, csi_step_stats *s) {
  if (!c || !p) return CSI_ERR_ARG;
  if (!ready(c)) return c->fail(CSI_ERR_STATE, "step: workspace/state not set");
  if ((p->mode != CSI_COUPLED && p->mode != CSI_SPLIT) || (p->precision != CSI_FP64 && p->precision != CSI_MIXED) ||
      !(p->cfl > 0.0) || p->max_iter < 0 || p->cfl_ramp < 0)
    return c->fail(CSI_ERR_ARG, "step: bad parameters");
  if ((p->mode == CSI_COUPLED && p->kind != CSI_CLOSURE) || (p->mode == CSI_SPLIT && p->kind != CSI_CC1 && p->kind != CSI_CC2))
    return c->fail(CSI_ERR_ARG, "step: correction kind does not match mode");
  if (p->jac != CSI_JAC_EXACT) return c->fail(CSI_ERR_UNSUPPORTED, "surrogate Jacobian not installed");
  int rc = reset_flags(c);
  if (rc) return rc;
  int every = p->check_every > 0 ? p->check_every : 50;
  csi_step_stats st{};
  st.bad_cell = -1;
  st.it_conv = -1;
  int fl[FL_N];
  const long it_start = c->it_global;
  for (int it = 0; it < p->max_iter; ++it) {
    long m = c->it_global;
    double cfl = p->cfl_ramp > 0 ? std::pow(p->cfl, double(std::min<long>(m, p->cfl_ramp)) / p->cfl_ramp) : p->cfl;
    hipEvent_t *E = nullptr;
    if (c->timing) {
      size_t slot = size_t(it % every) * 7;
      if (c->ev.size() < slot + 7) {
        size_t old_n = c->ev.size();
        c->ev.resize(size_t(every) * 7 > slot + 7 ? size_t(every) * 7 : slot + 7);
        for (size_t k = old_n; k < c->ev.size(); ++k)
          if ((rc = hip_check(c, hipEventCreate(&c->ev[k]), "event"))) return rc;
      }
      E = &c->ev[slot];
    }
    hipError_t e = hipSuccess;
    if (E) e = hipEventRecord(E[0], c->stream);
    if (e == hipSuccess) e = c->run->prim(c->g, c->w, c->stream, true);
    if (E && e == hipSuccess) e = hipEventRecord(E[1], c->stream);
    if (e == hipSuccess) e = c->run->faces(c->g, c->w, c->stream, true);
    if (E && e == hipSuccess) e = hipEventRecord(E[2], c->stream);
    if (e == hipSuccess) e = c->run->cell(c->g, c->w, c->stream, cfl, p->mode, p->precision, 3, true);
    if (E && e == hipSuccess) e = hipEventRecord(E[3], c->stream);
    if (e == hipSuccess) e = c->run->norms(c->w, c->stream, int(m), p->tol, true);
    if (E && e == hipSuccess) e = hipEventRecord(E[4], c->stream);
    if (e == hipSuccess) e = c->run->sweeps(c->g, c->w, c->stream, p->mode, p->precision, true);
    if (E && e == hipSuccess) e = hipEventRecord(E[5], c->stream);
    if (e == hipSuccess) e = c->run->update(c->g, c->w, c->stream, p->mode, p->precision, p->kind, true);
    if (E && e == hipSuccess) e = hipEventRecord(E[6], c->stream);
    if ((rc = hip_check(c, e, "step launch"))) return rc;
    c->it_global++;
    st.iters = it + 1;
    if ((it + 1) % every == 0 || it + 1 == p->max_iter) {
      if ((rc = read_flags(c, fl))) return rc;
      if (c->timing) {
        int nb_ = (it % every) + 1;
        for (int b = 0; b < nb_; ++b) {
          for (int ph = 0; ph < 6; ++ph) {
            float msf = 0.f;
            if (hipEventElapsedTime(&msf, c->ev[size_t(b) * 7 + ph], c->ev[size_t(b) * 7 + ph + 1]) == hipSuccess)
              c->phase_ms[ph] += msf;
          }
          c->phase_ms[6] += 1.0;
        }
      }
      if (fl[FL_ABORT]) {
        if (s) *s = st;
        return c->fail(CSI_ERR_HIP, "step: a sweep wave timed out waiting for its neighbour strip");
      }
      if (fl[FL_BAD] != INT_MAX || fl[FL_SING] != INT_MAX) {
        st.bad_cell = fl[FL_BAD] != INT_MAX ? fl[FL_BAD] : fl[FL_SING];
        if (s) *s = st;
        return c->fail(fl[FL_BAD] != INT_MAX ? CSI_ERR_NONFINITE : CSI_ERR_SINGULAR,
                       "step: non-physical state or singular block at cell " + std::to_string(st.bad_cell));
      }
      if (fl[FL_DONE]) {
        // the converged iteration's sweeps and update (and everything after
        // it) were skipped on the device: Q is the state whose residual met
        // the tolerance
        st.converged = 1;
        st.it_conv = fl[FL_ITDONE];
        st.iters = int(fl[FL_ITDONE] - it_start);
        c->it_global = fl[FL_ITDONE];
        break;
      }
    }
  }
  if ((rc = read_flags(c, fl))) return rc;
  st.n_clipped = fl[FL_CLIP];
  double nrm[2] = {0, 0}, r0 = 0;
  (void)hipMemcpy(nrm, c->w.norms, 16, hipMemcpyDeviceToHost);
  (void)hipMemcpy(&r0, c->w.r0, 8, hipMemcpyDeviceToHost);
  st.r0 = r0;
  st.r_last = nrm[0];
  if (s) *s = st;
  c->has_res = false;
  c->has_dq = false;
  return CSI_OK;
}

int csi_wall_heat_flux(csi_ctx *c, double *qw, double *q_stag) {
  if (!c) return CSI_ERR_ARG;
  if (!ready(c) || c->bc_mode != 0) return c->fail(CSI_ERR_STATE, "wall heat flux needs a residual on a wall grid");
  std::vector<double> h(c->ni);
  int rc = hip_check(c, hipMemcpy(h.data(), c->w.qw, size_t(c->ni) * 8, hipMemcpyDeviceToHost), "qw");
  if (rc) return rc;
  if (qw) std::memcpy(qw, h.data(), h.size() * 8);
  if (q_stag) {
    int hh = c->ni / 2;
    *q_stag = (c->ni % 2 == 0) ? 0.5 * (h[hh - 1] + h[hh]) : h[hh];
  }
  return CSI_OK;
}

int csi_prim_to_cons(csi_ctx *c, int n, const double *rho_s, const double *u, const double *v, const double *T,
                     const double *Tv, double *q) {
  if (!c || n < 0 || !rho_s || !u || !v || !T || !q) return CSI_ERR_ARG;
  if (!c->has_mech) return c->fail(CSI_ERR_STATE, "prim_to_cons before set_mechanism");
  const int ns = c->ns, nv = c->nv();
  double rs[MAXS], qq[MAXS + 4];
  for (int p = 0; p < n; ++p) {
    for (int s = 0; s < ns; ++s) rs[s] = rho_s[size_t(s) * n + p];
    (void)c->run->q_from_prim_host(c->mech, rs, u[p], v[p], T[p], Tv ? Tv[p] : T[p], qq);
    for (int k = 0; k < nv; ++k) q[size_t(k) * n + p] = qq[k];
  }
  return CSI_OK;
}

int csi_set_sweep(csi_ctx *c, int width, int publish_every) {
  if (!c) return CSI_ERR_ARG;
  if (width != 0 && width != 16 && width != 64) return c->fail(CSI_ERR_ARG, "sweep width must be 0, 16 or 64");
  if (width == 64 && c->ns > 11) return c->fail(CSI_ERR_UNSUPPORTED, "64-column strips are compiled for ns <= 11");
  if (publish_every < 1 || publish_every > 64) return c->fail(CSI_ERR_ARG, "publish interval must be 1..64");
  c->strip_w = width;
  c->w.strip_w = width;
  c->pub_every = publish_every;
  c->w.pub_every = publish_every;
  c->has_res = false;
  c->has_dq = false;
  return CSI_OK;
}

int csi_set_timing(csi_ctx *c, int on) {
  if (!c) return CSI_ERR_ARG;
  c->timing = on != 0;
  return CSI_OK;
}

int csi_phase_times(csi_ctx *c, double *ms, int reset) {
  if (!c) return CSI_ERR_ARG;
  if (ms) std::memcpy(ms, c->phase_ms, sizeof(c->phase_ms));
  if (reset) std::memset(c->phase_ms, 0, sizeof(c->phase_ms));
  return CSI_OK;
}

int csi_norm_history(csi_ctx *c, int n, double *hist) {
  if (!c || !hist || n < 0 || n > HIST_MAX) return CSI_ERR_ARG;
  if (!c->bound) return CSI_ERR_STATE;
  return hip_check(c, hipMemcpy(hist, c->w.hist, size_t(2) * n * 8, hipMemcpyDeviceToHost), "history");
}

int csi_get_array(csi_ctx *c, const char *name, double *out, size_t count) {
  if (!c || !name || !out) return CSI_ERR_ARG;
  if (!c->bound) return c->fail(CSI_ERR_STATE, "not bound");
  std::string n(name);
  const size_t N = c->N;
  const double *src = nullptr;
  const void *rsrc = nullptr;
  size_t cnt = 0;
  size_t NP = size_t(c->ni + 2) * (c->nj + 2);
  int nsol = c->last_mode == CSI_COUPLED ? c->nb() : c->nsplit();
  if (n == "R") { src = c->w.R; cnt = c->nv() * N; }
  else if (n == "dtau") { src = c->w.dtau; cnt = N; }
  else if (n == "src") { src = c->w.src; cnt = c->nv() * N; }
  else if (n == "qw") { src = c->w.qw; cnt = c->ni; }
  else if (n == "b") { rsrc = c->w.b; cnt = nsol * N; }
  else if (n == "dqs") { rsrc = c->w.dqs; cnt = nsol * N; }
  else if (n == "dq") { rsrc = c->w.dq; cnt = nsol * N; }
  else if (n == "Dinv") {
    rsrc = c->w.Dinv;
    cnt = (c->last_mode == CSI_COUPLED ? size_t(c->nb()) * c->nb() : 6 + size_t(c->ns) * c->ns) * N;
  } else if (n == "T" || n == "Tv" || n == "p" || n == "c") {
    int fld = n == "T" ? F_T : n == "Tv" ? F_TV : n == "p" ? F_P : F_C;
    std::vector<double> tmp(NP);
    int rc = hip_check(c, hipMemcpy(tmp.data(), c->w.prim + fld * NP, NP * 8, hipMemcpyDeviceToHost), "get");
    if (rc) return rc;
    if (count < N) return c->fail(CSI_ERR_ARG, "buffer too small");
    for (int j = 0; j < c->nj; ++j)
      for (int i = 0; i < c->ni; ++i) out[size_t(j) * c->ni + i] = tmp[size_t(j + 1) * (c->ni + 2) + i + 1];
    return CSI_OK;
  } else {
    return c->fail(CSI_ERR_ARG, "unknown array " + n);
  }
  if (count < cnt) return c->fail(CSI_ERR_ARG, "buffer too small for " + n);
  if (src) return hip_check(c, hipMemcpy(out, src, cnt * 8, hipMemcpyDeviceToHost), "get");
  // sweep records: cell-major or strip layout, FP64 or FP32
  const size_t rows = cnt / N;
  size_t stride = N;
  StripMap sm{};
  if (c->strip_w > 0) {
    sm = strip_map(c->ni, c->nj, c->strip_w);
    stride = sm.LEN;
  }
  const size_t esz = c->last_prec == CSI_MIXED ? 4 : 8;
  std::vector<char> tmp(rows * stride * esz);
  int rc = hip_check(c, hipMemcpy(tmp.data(), rsrc, tmp.size(), hipMemcpyDeviceToHost), "get");
  if (rc) return rc;
  for (size_t r_ = 0; r_ < rows; ++r_)
    for (int j = 0; j < c->nj; ++j)
      for (int i = 0; i < c->ni; ++i) {
        size_t pos = c->strip_w > 0 ? size_t(strip_pos(sm, i, j)) : size_t(j) * c->ni + i;
        size_t k = r_ * stride + pos;
        out[r_ * N + size_t(j) * c->ni + i] =
            esz == 4 ? double(reinterpret_cast<const float *>(tmp.data())[k]) : reinterpret_cast<const double *>(tmp.data())[k];
      }
  return CSI_OK;
}

}  // extern "C"
