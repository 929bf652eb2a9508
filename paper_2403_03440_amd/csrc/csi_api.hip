// Host side of the C-ABI (include/csi.h): context, grid metrics, mechanism
// tables, workspace layout inside the caller's device buffer, and the launch
// sequence of each call.  No device memory is allocated here.
#include <climits>
#include <cstddef>
#include <mutex>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/csi.h"
#include "csi_mech.hpp"
#include "csi_mlp.hpp"
#include "csi_runner.hpp"

using namespace csi;

// per-(species count, temperature model) factories; weak, so that a build may
// compile a subset (the 16-, 20- and 32-species mechanisms are built for one temperature)
#define CSI_WEAK_FACTORY(ns, nt) __attribute__((weak)) csi::IRunner *csi_make_runner_##ns##_##nt();
CSI_WEAK_FACTORY(2, 1) CSI_WEAK_FACTORY(2, 2) CSI_WEAK_FACTORY(3, 1) CSI_WEAK_FACTORY(3, 2)
CSI_WEAK_FACTORY(5, 1) CSI_WEAK_FACTORY(5, 2) CSI_WEAK_FACTORY(11, 1) CSI_WEAK_FACTORY(11, 2)
CSI_WEAK_FACTORY(16, 1) CSI_WEAK_FACTORY(16, 2) CSI_WEAK_FACTORY(20, 1) CSI_WEAK_FACTORY(20, 2)
CSI_WEAK_FACTORY(32, 1) CSI_WEAK_FACTORY(32, 2)

namespace csi {
IRunner *make_runner(int ns, int nt) {
#define CSI_PICK(n)                                                                  \
  case n:                                                                            \
    if (nt == 1) return csi_make_runner_##n##_1 ? csi_make_runner_##n##_1() : nullptr; \
    return csi_make_runner_##n##_2 ? csi_make_runner_##n##_2() : nullptr;
  switch (ns) {
    CSI_PICK(2)
    CSI_PICK(3)
    CSI_PICK(5)
    CSI_PICK(11)
    CSI_PICK(16)
    CSI_PICK(20)
    CSI_PICK(32)
    default: return nullptr;
  }
#undef CSI_PICK
}
}  // namespace csi

// Device scratch of csi_mlp_forward_noalloc (packed BF16 operands of the
// network), one copy per GPU, held until the process ends.  Host code never
// passes `scratch` itself to a kernel: its device address is taken once per
// device with hipGetSymbolAddress (noalloc_scratch_ptr) and kept in the table.
static __device__ __align__(256) unsigned char scratch[CSI_MLP_NOALLOC_SCRATCH_BYTES];

struct NoallocTable {
  std::mutex mu;
  std::vector<void *> ptr;  // per device ordinal; nullptr until taken
};
NoallocTable &noalloc_table() {
  static NoallocTable t;
  return t;
}

// the device address of `scratch` on `device`, which must be current;
// taken at the first call on that device
hipError_t noalloc_scratch_ptr(int device, void **out) {
  NoallocTable &t = noalloc_table();
  std::lock_guard<std::mutex> lk(t.mu);
  if (device < 0) return hipErrorInvalidDevice;
  if (t.ptr.size() <= size_t(device)) t.ptr.resize(size_t(device) + 1, nullptr);
  if (!t.ptr[device]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    t.ptr[device] = p;
  }
  *out = t.ptr[device];
  return hipSuccess;
}

struct csi_ctx {
  int device = 0;
  void *noalloc = nullptr;  // this device's address of `scratch`
  hipStream_t stream = nullptr;
  // surrogate inference beside the face kernels (created at the first
  // surrogate step; default priority)
  hipStream_t side = nullptr;
  hipEvent_t ev_prim = nullptr, ev_sur = nullptr;
  std::string err;
  // grid (host)
  int ni = 0, nj = 0, N = 0, bc_mode = 0;
  double Tw = 300.0;
  std::vector<double> xn, yn, xc, yc, V, fi_nx, fi_ny, fi_S, fj_nx, fj_ny, fj_S;
  // mechanism (host copy of the device table)
  Mech mech;
  int ns = 0, nt = 1;
  IRunner *run = nullptr;
  std::vector<double> qfs;
  // species-generic kernels (one temperature, no reactions): chosen above 32
  // species, or for every count after csi_set_species_generic(ctx, 1)
  bool wide = false;
  bool want_wide = false;
  bool has_grid = false, has_mech = false, has_fs = false, bound = false, has_state = false, has_res = false;
  int last_mode = -1, last_prec = -1;
  bool has_dq = false;
  bool prim_warm = false;  // the prim array holds temperatures solved since set_state (Newton start points)
  // installed surrogate network (inside the workspace)
  bool has_sur = false;
  double sur_ratio = 0.98;
  int sur_window = 100;
  // workspace
  char *ws = nullptr;
  size_t ws_bytes = 0;
  WS w;
  Geo g;
  long it_global = 0;
  int group_c = 1;  // sweep schedule: 0 hyperplane launches; 1 persistent group kernels
  // phase timing (HIP events, created on first use)
  bool timing = false;
  int trace = 0;                     // per-strip sweep trace (csi_set_timing(ctx, 2))
  long long *trace_buf = nullptr;
  std::vector<hipEvent_t> ev;
  double phase_ms[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};

  // split species block: 0 = J_C at fixed T, Tv; 1 = at fixed velocities,
  // internal and vibrational energy densities (cell kernel flag bit 3); 2 = at
  // fixed velocities, internal energy density and Tv (flag bits 3 and 4)
  int jc_reading = 0;
  // physical time (dual time stepping): the unsteady terms carry
  // pt_a = (1 + theta) / dt and pt_b = theta / dt (both 0: steady)
  double pt_a = 0.0, pt_b = 0.0;
  // off-diagonal operator: 0 linear Jacobian-vector products, 1 flux differences
  int fdiff = 0;
  // residual scheme: 0 first-order HLLE, 1 MUSCL (minmod) + Roe
  int scheme = 0;
  int jc_flag() const { return jc_reading == 0 ? 0 : (jc_reading == 1 ? 8 : 8 | 16); }

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
  size_t off[64];
  size_t total;
};

size_t al(size_t x) { return (x + 255) & ~size_t(255); }

// bytes of the group-schedule arrays of one part (C = 64 / G cells per
// wave): the larger of the two element sizes (the precision can change after
// binding)
struct GroupCap {
  size_t S = 0, x = 0, bnd = 0;
  void merge(const GroupCap &o) { S = std::max(S, o.S); x = std::max(x, o.x); bnd = std::max(bnd, o.bnd); }
};
GroupCap group_cap(int ni, int nj, int part, int ns, int nt) {
  GroupCap r;
  for (int esz = 4; esz <= 8; esz += 4) {
    const RecShape rs = rec_shape(part, ns, nt, esz);
    const GroupMap m = group_map(ni, nj, rs.G);
    GroupCap t;
    t.S = size_t(st_words(rs, long(ni) * nj)) * esz;
    t.x = size_t(m.nblk) * m.Lw * esz;
    t.bnd = size_t(m.nstrip) * nj * rs.G * esz;
    r.merge(t);
  }
  return r;
}

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
  const size_t A = N;
  // group-schedule records, per part (none on the species-generic path,
  // which has neither the group schedule nor the surrogate)
  GroupCap g0, g1;
  MlpDims sd{};
  size_t wtab = 0, gj_perm = 0, gj_xk = 0;
  if (!c->wide) {
    g0 = group_cap(c->ni, c->nj, PART_COUPLED, c->ns, c->nt);
    g0.merge(group_cap(c->ni, c->nj, PART_FLOW, c->ns, c->nt));
    g1 = group_cap(c->ni, c->nj, PART_SPECIES, c->ns, c->nt);
    sd = mlp_dims(c->ns + 3, c->ns * c->ns);
  } else {
    (void)c->run->host_table(&wtab);
    gj_perm = N * size_t(c->nb()) * 4;
    gj_xk = N * size_t(WGJ_SCRATCH_ROWS) * c->nb() * 8;
  }
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
      size_t(nsol) * A * 8, size_t(nsol) * A * 8, size_t(nsol) * A * 8,  // 27-29 b dqs dq (hyperplane schedule)
      ndinv * A * 8,                                  // 30 Dinv (hyperplane schedule)
      FL_N * 4,                                       // 31 flags
      g0.S, g0.x, g0.bnd, g0.bnd, 8,                  // 32-36 group part 0: record staging, dQ, pushes (fwd, bwd), tickets
      g1.S, g1.x, g1.bnd, g1.bnd, 8,                  // 37-41 group part 1
      c->wide ? 0 : size_t(c->ns) * c->ns * N * 4,    // 42 surrogate J_C
      size_t(sd.nslots) * 16,                         // 43 surrogate packed operands
      size_t(sd.np) * 4,                              // 44 surrogate FP32 parameters
      size_t(2 * sd.n_in + 1) * 8,                    // 45 surrogate scales
      size_t(4) * c->ni * TR_N * 8,                   // 46 sweep trace
      size_t(c->ns >= BLOCK_NS_MIN && !c->wide ? hb_fields(c->ns, nv) : 2) * N * 8,  // 47 cell kernel -> block kernel hand-off
      size_t(nv) * N * 8,                             // 48 state at the start of csi_step (surrogate divergence fallback)
      size_t(nv) * N * 8, size_t(nv) * N * 8,         // 49-50 physical-time levels Q^n, Q^{n-1}
      wtab, gj_perm, gj_xk,                           // 51-53 species-generic table and Gauss-Jordan scratch
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
  int fl[FL_N] = {INT_MAX, 0, -1, 0, INT_MAX, 0, -1, 0, 0, 0, 0, 0, 0, 0, 0, 0};
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
  if (noalloc_scratch_ptr(device, &c->noalloc) != hipSuccess) { delete c; return CSI_ERR_HIP; }
  *ctx = c;
  return CSI_OK;
}

int csi_destroy(csi_ctx *c) {
  if (!c) return CSI_ERR_ARG;
  for (hipEvent_t e : c->ev) (void)hipEventDestroy(e);
  if (c->ev_prim) (void)hipEventDestroy(c->ev_prim);
  if (c->ev_sur) (void)hipEventDestroy(c->ev_sur);
  if (c->side) (void)hipStreamDestroy(c->side);
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
  if (mm->ns < 2 || mm->ns > CSI_WIDE_MAX_SPECIES || mm->nr < 0 || mm->nr > MAXR)
    return c->fail(CSI_ERR_ARG, "set_mechanism: sizes");
  const bool wide = c->want_wide || mm->ns > MAXS;
  std::string err;
  IRunner *r = nullptr;
  if (wide) {
    if (mm->nr != 0 || mm->two_temp)
      return c->fail(CSI_ERR_UNSUPPORTED, "the species-generic kernels (ns = " + std::to_string(mm->ns) +
                                              ") take one temperature and no reactions");
    if (c->scheme != 0)
      return c->fail(CSI_ERR_UNSUPPORTED, "the species-generic kernels have the first-order residual only");
    r = make_wide_runner(mm, err);
    if (!r) return c->fail(CSI_ERR_ARG, "set_mechanism: " + err);
    std::memset(&c->mech, 0, sizeof(Mech));  // the generic runner reads its own table
  } else {
    r = make_runner(mm->ns, mm->two_temp ? 2 : 1);
    if (!r)
      return c->fail(CSI_ERR_UNSUPPORTED, "no kernels compiled for ns = " + std::to_string(mm->ns) +
                                              (mm->two_temp ? " with two temperatures" : " with one temperature"));
    if (!build_mech(mm, c->mech, err)) { delete r; return c->fail(CSI_ERR_ARG, "set_mechanism: " + err); }
  }
  delete c->run;
  c->run = r;
  c->wide = wide;
  c->ns = mm->ns;
  c->nt = mm->two_temp ? 2 : 1;
  c->group_c = wide ? 0 : 1;  // persistent group kernels (per-hyperplane launches on the generic path)
  c->has_mech = true;
  // the species block with the temperature following the composition in one
  // temperature; at fixed T, Tv in two (the default readings)
  c->jc_reading = mm->two_temp ? 0 : 1;
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
  c->qfs.assign(c->nv(), 0.0);
  (void)c->run->q_from_prim_host(c->mech, rho_s, u, v, T, Tv, c->qfs.data());
  c->has_fs = true;
  if (c->bound) {
    int rc = hip_check(c, hipMemcpyAsync(c->w.qfs, c->qfs.data(), c->nv() * 8, hipMemcpyHostToDevice, c->stream), "qfs");
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
  for (int q = 0; q < 2; ++q) {
    const int o = 32 + 5 * q;
    GroupBufs &gb = w.grp[q];
    gb.S = b + L.off[o];
    gb.x = b + L.off[o + 1];
    gb.bnd[0] = b + L.off[o + 2];
    gb.bnd[1] = b + L.off[o + 3];
    gb.tickets = reinterpret_cast<int *>(b + L.off[o + 4]);
  }
  w.sur.J = reinterpret_cast<float *>(b + L.off[42]);
  w.sur.P = reinterpret_cast<const u16x8 *>(b + L.off[43]);
  w.sur.p = reinterpret_cast<const float *>(b + L.off[44]);
  w.sur.scales = reinterpret_cast<const double *>(b + L.off[45]);
  c->trace_buf = reinterpret_cast<long long *>(b + L.off[46]);
  w.diag = D(47);
  w.qbak = D(48);
  w.qn = D(49);
  w.qnm1 = D(50);
  w.wtab = D(51);
  w.gj_perm = reinterpret_cast<int *>(b + L.off[52]);
  w.gj_xk = D(53);
  {
    // the compiled table as the streaming kernels read it (views into the
    // device Mech record)
    const char *mb = reinterpret_cast<const char *>(w.mech);
    WMech &v = w.mview;
    v.ns = c->ns;
    v.R = reinterpret_cast<const double *>(mb + offsetof(Mech, R));
    v.cvtr = reinterpret_cast<const double *>(mb + offsetof(Mech, cvtr));
    v.thv = reinterpret_cast<const double *>(mb + offsetof(Mech, thv));
    v.hf = reinterpret_cast<const double *>(mb + offsetof(Mech, hf));
    v.ck = reinterpret_cast<const double *>(mb + offsetof(Mech, ck));
    v.iSc = reinterpret_cast<const double *>(mb + offsetof(Mech, iSc));
    v.kind = reinterpret_cast<const int *>(mb + offsetof(Mech, kind));
    v.mu_ref = c->mech.mu_ref;
    v.T_ref = c->mech.T_ref;
    v.mu_exp = c->mech.mu_exp;
    v.iscmax = 0.0;
    for (int s_ = 0; s_ < c->ns && !c->wide; ++s_) v.iscmax = std::fmax(v.iscmax, c->mech.iSc[s_]);
  }
  w.pt_a = c->pt_a;
  w.pt_b = c->pt_b;
  w.fdiff = c->fdiff;
  w.trace = c->trace > 0 ? c->trace_buf : nullptr;
  c->has_sur = false;
  w.group_c = c->group_c;
  w.spin_limit = 4000000;
  w.nblk_cell = (c->N + 255) / 256;
  w.hist_max = HIST_MAX;
  Geo &g = c->g;
  g.ni = c->ni; g.nj = c->nj; g.N = c->N; g.NP = (c->ni + 2) * (c->nj + 2); g.bc_mode = c->bc_mode; g.Tw = c->Tw;
  g.scheme = c->scheme;
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
  if (e == hipSuccess) e = hipMemcpyAsync(w.qfs, c->qfs.data(), c->nv() * 8, hipMemcpyHostToDevice, st);
  {
    size_t tb = 0;
    const void *tab = c->run->host_table(&tb);
    if (tab && e == hipSuccess) e = hipMemcpyAsync(w.wtab, tab, tb, hipMemcpyHostToDevice, st);
  }
  if (e == hipSuccess) e = hipMemsetAsync(w.qw, 0, size_t(c->ni) * 8, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  int rc = hip_check(c, e, "bind_workspace");
  if (rc) return rc;
  c->bound = true;
  c->has_state = false;
  c->prim_warm = false;
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
  // the physical-time levels start at the state (no unsteady term until csi_advance_time)
  const size_t qb = size_t(c->nv()) * c->N * 8;
  hipError_t e = hipMemcpyAsync(c->w.qn, c->w.Q, qb, hipMemcpyDeviceToDevice, c->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(c->w.qnm1, c->w.Q, qb, hipMemcpyDeviceToDevice, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  rc = hip_check(c, e, "set_state");
  if (rc) return rc;
  c->has_state = true;
  c->has_res = false;
  c->has_dq = false;
  c->prim_warm = false;  // results depend only on the state and the calls since it was set
  c->it_global = 0;
  return reset_flags(c);
}

int csi_set_physical_time(csi_ctx *c, double dt, double theta) {
  if (!c) return CSI_ERR_ARG;
  if (!(dt >= 0.0) || !(theta >= 0.0) || !std::isfinite(dt) || !std::isfinite(theta))
    return c->fail(CSI_ERR_ARG, "set_physical_time: dt and theta must be finite and >= 0");
  if (c->wide && dt > 0.0)
    return c->fail(CSI_ERR_UNSUPPORTED, "physical time on the species-generic kernels: steady only");
  c->pt_a = dt > 0.0 ? (1.0 + theta) / dt : 0.0;
  c->pt_b = dt > 0.0 ? theta / dt : 0.0;
  c->w.pt_a = c->pt_a;
  c->w.pt_b = c->pt_b;
  c->has_res = false;
  c->has_dq = false;
  return CSI_OK;
}

int csi_set_time_levels(csi_ctx *c, const double *qn, const double *qnm1, int on_device) {
  if (!c || !qn || !qnm1) return CSI_ERR_ARG;
  if (!ready(c)) return c->fail(CSI_ERR_STATE, "set_time_levels: workspace/state not set");
  const size_t qb = size_t(c->nv()) * c->N * 8;
  const hipMemcpyKind k = on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  hipError_t e = hipMemcpyAsync(c->w.qn, qn, qb, k, c->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(c->w.qnm1, qnm1, qb, k, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  c->has_res = false;
  c->has_dq = false;
  return hip_check(c, e, "set_time_levels");
}

int csi_advance_time(csi_ctx *c) {
  if (!c) return CSI_ERR_ARG;
  if (!ready(c)) return c->fail(CSI_ERR_STATE, "advance_time: workspace/state not set");
  const size_t qb = size_t(c->nv()) * c->N * 8;
  hipError_t e = hipMemcpyAsync(c->w.qnm1, c->w.qn, qb, hipMemcpyDeviceToDevice, c->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(c->w.qn, c->w.Q, qb, hipMemcpyDeviceToDevice, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  int rc = hip_check(c, e, "advance_time");
  if (rc) return rc;
  c->has_res = false;
  c->has_dq = false;
  c->it_global = 0;  // the next csi_step starts its residual drop and CFL ramp afresh
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
  hipError_t e = c->run->prim(c->g, c->w, c->stream, false, c->prim_warm);
  c->prim_warm = true;
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
  if (jac != CSI_JAC_EXACT && jac != CSI_JAC_SURROGATE) return c->fail(CSI_ERR_ARG, "jac");
  if (jac == CSI_JAC_SURROGATE && mode != CSI_SPLIT) return c->fail(CSI_ERR_ARG, "the surrogate serves the split form");
  if (jac == CSI_JAC_SURROGATE && !c->has_sur) return c->fail(CSI_ERR_STATE, "no surrogate installed");
  if (!ready(c) || !c->has_res) return c->fail(CSI_ERR_STATE, "implicit_op before residual");
  if (c->fdiff && precision != CSI_FP64)
    return c->fail(CSI_ERR_UNSUPPORTED, "flux-difference off-diagonal operator: FP64 sweeps only");
  if (c->wide && precision != CSI_FP64)
    return c->fail(CSI_ERR_UNSUPPORTED, "the species-generic kernels sweep in FP64 only");
  hipError_t e = hipSuccess;
  if (jac == CSI_JAC_SURROGATE) e = c->run->surrogate(c->g, c->w, c->stream, false);
  if (e == hipSuccess) e = c->run->cell(c->g, c->w, c->stream, 0.0, mode, precision, (jac == CSI_JAC_SURROGATE ? 6 : 2) | c->jc_flag(), false);
  if (e == hipSuccess) e = c->run->sweeps(c->g, c->w, c->stream, mode, precision, false);
  int rc = hip_check(c, e, "implicit_op launch");
  if (rc) return rc;
  int fl[FL_N];
  if ((rc = read_flags(c, fl))) return rc;
  if (fl[FL_ABORT]) return c->fail(CSI_ERR_HIP, "implicit_op: a sweep wave timed out waiting for its neighbour");
  if (fl[FL_SING] != INT_MAX)
    return c->fail(CSI_ERR_SINGULAR, "singular diagonal block at cell " + std::to_string(fl[FL_SING]));
  if (fl[FL_BAD] != INT_MAX)
    return c->fail(CSI_ERR_NONFINITE, "flux difference at a non-physical neighbour state (cell " +
                                          std::to_string(fl[FL_BAD]) + ")");
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

// events per timed iteration: boundaries of prim, faces, cell, block, norms, forward sweep, backward sweep,
// update
static constexpr int NEV = 9;

int csi_step(csi_ctx *c, const csi_step_params *p, csi_step_stats *s) {
  if (!c || !p) return CSI_ERR_ARG;
  if (!ready(c)) return c->fail(CSI_ERR_STATE, "step: workspace/state not set");
  if ((p->mode != CSI_COUPLED && p->mode != CSI_SPLIT) || (p->precision != CSI_FP64 && p->precision != CSI_MIXED) ||
      !(p->cfl > 0.0) || p->max_iter < 0 || p->cfl_ramp < 0)
    return c->fail(CSI_ERR_ARG, "step: bad parameters");
  if ((p->mode == CSI_COUPLED && p->kind != CSI_CLOSURE) || (p->mode == CSI_SPLIT && p->kind != CSI_CC1 && p->kind != CSI_CC2))
    return c->fail(CSI_ERR_ARG, "step: correction kind does not match mode");
  if (p->jac != CSI_JAC_EXACT && p->jac != CSI_JAC_SURROGATE) return c->fail(CSI_ERR_ARG, "step: jac");
  const bool sur = p->jac == CSI_JAC_SURROGATE;
  if (sur && p->mode != CSI_SPLIT) return c->fail(CSI_ERR_ARG, "step: the surrogate serves the split form");
  if (sur && !c->has_sur) return c->fail(CSI_ERR_STATE, "step: no surrogate installed");
  if (c->fdiff && p->precision != CSI_FP64)
    return c->fail(CSI_ERR_UNSUPPORTED, "flux-difference off-diagonal operator: FP64 sweeps only");
  if (c->wide && p->precision != CSI_FP64)
    return c->fail(CSI_ERR_UNSUPPORTED, "the species-generic kernels sweep in FP64 only");
  int rc = reset_flags(c);
  if (rc) return rc;
  if (sur && !c->side) {
    hipError_t e = hipSetDevice(c->device);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ev_prim, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ev_sur, hipEventDisableTiming);
    if ((rc = hip_check(c, e, "side stream"))) return rc;
  }
  int every = p->check_every > 0 ? p->check_every : 50;
  csi_step_stats st{};
  st.bad_cell = -1;
  st.it_conv = -1;
  st.surrogate_off_at = -1;
  int fl[FL_N];
  const long it_start = c->it_global;
  // Divergence fallback of the surrogate: the state at the start of the call.
  // If iterations with the surrogate on end in a non-physical state or a zero
  // pivot, that state is restored, the surrogate is switched off from the
  // call's first iteration on, and the iterations are repeated with the exact
  // block (once per call).  A state from a later clean check is not kept: the
  // blocks of a wrong network can spoil the state before any flag shows it.
  const size_t qbytes = size_t(c->nv()) * c->N * 8;
  bool guard = sur;
  const long bak_global = c->it_global;
  const int bak_it = 0;
  if (guard && (rc = hip_check(c, hipMemcpyAsync(c->w.qbak, c->w.Q, qbytes, hipMemcpyDeviceToDevice, c->stream),
                               "state copy")))
    return rc;
  for (int it = 0; it < p->max_iter; ++it) {
    long m = c->it_global;
    double cfl = p->cfl_ramp > 0 ? std::pow(p->cfl, double(std::min<long>(m, p->cfl_ramp)) / p->cfl_ramp) : p->cfl;
    hipEvent_t *E = nullptr;
    if (c->timing) {
      size_t slot = size_t(it % every) * NEV;
      if (c->ev.size() < slot + NEV) {
        size_t old_n = c->ev.size();
        c->ev.resize(size_t(every) * NEV > slot + NEV ? size_t(every) * NEV : slot + NEV);
        for (size_t k = old_n; k < c->ev.size(); ++k)
          if ((rc = hip_check(c, hipEventCreate(&c->ev[k]), "event"))) return rc;
      }
      E = &c->ev[slot];
    }
    hipError_t e = hipSuccess;
    if (E) e = hipEventRecord(E[0], c->stream);
    // the temperature solves start at the previous solve's temperatures once there has been one
    if (e == hipSuccess) e = c->run->prim(c->g, c->w, c->stream, true, c->prim_warm);
    c->prim_warm = true;
    if (E && e == hipSuccess) e = hipEventRecord(E[1], c->stream);
    // the surrogate's inference needs only the primitives: it runs on the side
    // stream while the face kernels run (and the cell kernel, where the
    // diagonal blocks have a kernel of their own); the first kernel that reads
    // its blocks waits for it
    if (sur && e == hipSuccess) e = hipEventRecord(c->ev_prim, c->stream);
    if (sur && e == hipSuccess) e = hipStreamWaitEvent(c->side, c->ev_prim, 0);
    if (sur && e == hipSuccess) e = c->run->surrogate(c->g, c->w, c->side, true);
    if (sur && e == hipSuccess) e = hipEventRecord(c->ev_sur, c->side);
    if (e == hipSuccess) e = c->run->faces(c->g, c->w, c->stream, true);
    if (E && e == hipSuccess) e = hipEventRecord(E[2], c->stream);
    if (e == hipSuccess)
      e = c->run->cell(c->g, c->w, c->stream, cfl, p->mode, p->precision, (sur ? 7 : 3) | c->jc_flag(), true,
                         sur ? c->ev_sur : nullptr, E ? E[3] : nullptr);
    if (E && e == hipSuccess) e = hipEventRecord(E[4], c->stream);
    const StallArgs stall{sur ? c->w.flags + FL_SURR_OFF : nullptr, int(it_start), c->sur_window, c->sur_ratio};
    if (e == hipSuccess) e = c->run->norms(c->w, c->stream, int(m), p->tol, true, stall);
    if (E && e == hipSuccess) e = hipEventRecord(E[5], c->stream);
    if (e == hipSuccess) e = c->run->sweeps(c->g, c->w, c->stream, p->mode, p->precision, true, E ? E[6] : nullptr);
    if (E && e == hipSuccess) e = hipEventRecord(E[7], c->stream);
    if (e == hipSuccess) e = c->run->update(c->g, c->w, c->stream, p->mode, p->precision, p->kind, true);
    if (E && e == hipSuccess) e = hipEventRecord(E[8], c->stream);
    if ((rc = hip_check(c, e, "step launch"))) return rc;
    c->it_global++;
    st.iters = it + 1;
    if ((it + 1) % every == 0 || it + 1 == p->max_iter) {
      if ((rc = read_flags(c, fl))) return rc;
      if (c->timing) {
        int nb_ = (it % every) + 1;
        for (int b = 0; b < nb_; ++b) {
          for (int ph = 0; ph < NEV - 1; ++ph) {
            float msf = 0.f;
            if (hipEventElapsedTime(&msf, c->ev[size_t(b) * NEV + ph], c->ev[size_t(b) * NEV + ph + 1]) == hipSuccess)
              c->phase_ms[ph] += msf;
          }
          c->phase_ms[NEV - 1] += 1.0;
        }
      }
      if (fl[FL_ABORT]) {
        if (s) *s = st;
        return c->fail(CSI_ERR_HIP, "step: a sweep wave timed out waiting for its neighbour strip");
      }
      if ((fl[FL_BAD] != INT_MAX || fl[FL_SING] != INT_MAX) && guard && fl[FL_SURR_OFF] < 0 && !fl[FL_ABORT]) {
        // every flag and counter starts afresh (the discarded iterations'
        // clip and dominance-fallback counts and a stop flag must not carry
        // over), then the surrogate is off from the call's first iteration
        const int off = int(bak_global);
        hipError_t e2 = hipMemcpyAsync(c->w.Q, c->w.qbak, qbytes, hipMemcpyDeviceToDevice, c->stream);
        if ((rc = hip_check(c, e2, "divergence fallback"))) return rc;
        if ((rc = reset_flags(c))) return rc;
        e2 = hipMemcpyAsync(c->w.flags + FL_SURR_OFF, &off, sizeof(int), hipMemcpyHostToDevice, c->stream);
        if (e2 == hipSuccess) e2 = hipStreamSynchronize(c->stream);
        if ((rc = hip_check(c, e2, "divergence fallback"))) return rc;
        c->it_global = bak_global;
        it = bak_it - 1;
        st.surrogate_diverged = 1;
        guard = false;
        continue;
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
  {
    unsigned long long dd;
    std::memcpy(&dd, fl + FL_DDFAIL, sizeof(dd));
    st.n_dd_fallback = (long long)dd;
  }
  st.surrogate_off_at = fl[FL_SURR_OFF];
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

int csi_set_species_jacobian(csi_ctx *c, int reading) {
  if (!c) return CSI_ERR_ARG;
  if (reading < 0 || reading > 2) return c->fail(CSI_ERR_ARG, "set_species_jacobian: reading must be 0, 1 or 2");
  if (!c->has_mech) return c->fail(CSI_ERR_STATE, "set_species_jacobian before set_mechanism");
  c->jc_reading = reading;
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
  std::vector<double> rs(ns), qq(nv);
  for (int p = 0; p < n; ++p) {
    for (int s = 0; s < ns; ++s) rs[s] = rho_s[size_t(s) * n + p];
    (void)c->run->q_from_prim_host(c->mech, rs.data(), u[p], v[p], T[p], Tv ? Tv[p] : T[p], qq.data());
    for (int k = 0; k < nv; ++k) q[size_t(k) * n + p] = qq[k];
  }
  return CSI_OK;
}

int csi_set_sweep(csi_ctx *c, int schedule) {
  if (!c) return CSI_ERR_ARG;
  if (schedule != 0 && schedule != 1) return c->fail(CSI_ERR_ARG, "sweep schedule must be 0 or 1");
  if (c->wide && schedule != 0)
    return c->fail(CSI_ERR_UNSUPPORTED, "the species-generic kernels sweep with per-hyperplane launches only");
  c->group_c = schedule;
  c->w.group_c = schedule;
  c->last_mode = -1;  // the records of the last operator are in the old layout
  c->has_res = false;
  c->has_dq = false;
  return CSI_OK;
}

int csi_set_offdiag(csi_ctx *c, int op) {
  if (!c) return CSI_ERR_ARG;
  if (op != 0 && op != 1) return c->fail(CSI_ERR_ARG, "off-diagonal operator must be 0 or 1");
  if (c->wide && op != 0)
    return c->fail(CSI_ERR_UNSUPPORTED, "the species-generic kernels apply the linear Jacobian-vector product only");
  c->fdiff = op;
  c->w.fdiff = op;
  if (op == 1) return csi_set_sweep(c, 0);  // flux differences run in the per-hyperplane sweeps
  c->has_dq = false;
  return CSI_OK;
}

int csi_set_residual_scheme(csi_ctx *c, int scheme) {
  if (!c) return CSI_ERR_ARG;
  if (scheme != 0 && scheme != 1) return c->fail(CSI_ERR_ARG, "residual scheme must be 0 or 1");
  if (c->wide && scheme != 0)
    return c->fail(CSI_ERR_UNSUPPORTED, "the species-generic kernels have the first-order residual only");
  c->scheme = scheme;
  c->g.scheme = scheme;
  c->has_res = false;
  c->has_dq = false;
  return CSI_OK;
}

int csi_set_species_generic(csi_ctx *c, int on) {
  if (!c) return CSI_ERR_ARG;
  if (on != 0 && on != 1) return c->fail(CSI_ERR_ARG, "set_species_generic: on must be 0 or 1");
  c->want_wide = on != 0;
  return CSI_OK;
}

namespace {

// SplitMix64 (Steele, Lea and Flood's generator, as published by Vigna): one
// step of the sequence from x
unsigned long long splitmix64(unsigned long long x) {
  unsigned long long z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

long long gcd_ll(long long a, long long b) {
  while (b) {
    const long long t = a % b;
    a = b;
    b = t;
  }
  return a;
}

// the seeded subset of csi_sample_jacobians: row r -> cell (b + r a) mod N
// with b = splitmix64(seed) mod N and a the first value coprime with N from
// 1 + splitmix64(seed + 1) mod (N - 1) upwards (wrapping within [1, N - 1])
SampleMap sample_map(unsigned long long seed, int N) {
  if (N <= 1) return SampleMap{1, 0};
  const long long n = N;
  long long b = (long long)(splitmix64(seed) % (unsigned long long)n);
  long long a = 1 + (long long)(splitmix64(seed + 1) % (unsigned long long)(n - 1));
  while (gcd_ll(a, n) != 1) a = a % (n - 1) + 1;
  return SampleMap{a, b};
}

}  // namespace

namespace {
// scratch of csi_block_inverse: row interchanges, pivot rows, singular flag
void block_inverse_layout(int n, int count, size_t off[3], size_t *total) {
  off[0] = 0;
  off[1] = al(size_t(count) * n * 4);
  off[2] = off[1] + al(size_t(count) * WGJ_SCRATCH_ROWS * n * 8);
  *total = off[2] + 256;
}
}  // namespace

int csi_block_inverse_work(int n, int count, size_t *bytes) {
  if (!bytes || n < 1 || n > CSI_WIDE_MAX_SPECIES + 3 || count < 0) return CSI_ERR_ARG;
  size_t off[3];
  block_inverse_layout(n, count, off, bytes);
  return CSI_OK;
}

int csi_block_inverse(csi_ctx *c, int n, int count, double *a, void *work, size_t work_bytes, int *singular) {
  if (!c) return CSI_ERR_ARG;
  if (n < 1 || n > CSI_WIDE_MAX_SPECIES + 3 || count < 0 || (count > 0 && !a))
    return c->fail(CSI_ERR_ARG, "block_inverse: bad arguments");
  size_t off[3], need = 0;
  block_inverse_layout(n, count, off, &need);
  if (!work || reinterpret_cast<uintptr_t>(work) % 256 || work_bytes < need)
    return c->fail(CSI_ERR_ARG, "block_inverse: work buffer missing, not 256-byte aligned or too small");
  if (singular) *singular = -1;
  if (count == 0) return CSI_OK;
  char *w = static_cast<char *>(work);
  int *perm = reinterpret_cast<int *>(w + off[0]);
  double *xk = reinterpret_cast<double *>(w + off[1]);
  int *sing = reinterpret_cast<int *>(w + off[2]);
  const int none = INT_MAX;
  hipError_t e = hipSetDevice(c->device);
  if (e == hipSuccess) e = hipMemcpyAsync(sing, &none, 4, hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) e = wide_invert(a, n, count, perm, xk, sing, nullptr, c->stream);
  int hs = INT_MAX;
  if (e == hipSuccess) e = hipMemcpyAsync(&hs, sing, 4, hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  int rc = hip_check(c, e, "block_inverse");
  if (rc) return rc;
  if (hs != INT_MAX) {
    if (singular) *singular = hs;
    return c->fail(CSI_ERR_SINGULAR, "block_inverse: singular matrix " + std::to_string(hs));
  }
  return CSI_OK;
}

int csi_set_timing(csi_ctx *c, int on) {
  if (!c || on < 0 || on > 2) return CSI_ERR_ARG;
  c->timing = on != 0;
  c->trace = on == 2;
  c->w.trace = c->trace && c->trace_buf ? c->trace_buf : nullptr;
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

}  // extern "C"

namespace {

// Sweep records and results of the last implicit operator, returned cell-major
// as [field][N]: "b" (RHS) and "dqs" / "dq" nsol fields; "Dinv" coupled
// [nb*nb] (row-major D^-1), split [nf*nf + ns*ns] (dense flow inverse, then
// the species inverse).  Reads the cell-major arrays of the hyperplane
// schedule or un-permutes the step-blocked group records.
int get_records(csi_ctx *c, const std::string &n, double *out, size_t count) {
  const size_t N = c->N;
  if (c->wide && n == "Dinv") return c->fail(CSI_ERR_UNSUPPORTED, "Dinv: not kept in this layout by the species-generic kernels");
  const bool coupled = c->last_mode == CSI_COUPLED;
  const int nsol = coupled ? c->nb() : c->nsplit();
  const int nf = c->nf(), ns = c->ns, nb = c->nb();
  const bool dinv = n == "Dinv";
  const size_t F = dinv ? (coupled ? size_t(nb) * nb : size_t(nf) * nf + size_t(ns) * ns) : size_t(nsol);
  if (count < F * N) return c->fail(CSI_ERR_ARG, "buffer too small for " + n);
  const size_t esz = c->last_prec == CSI_MIXED ? 4 : 8;
  auto fetch = [&](const void *src, size_t cnt, std::vector<double> &dst) -> int {
    std::vector<char> tmp(cnt * esz);
    int rc = hip_check(c, hipMemcpy(tmp.data(), src, tmp.size(), hipMemcpyDeviceToHost), "get");
    if (rc) return rc;
    dst.resize(cnt);
    for (size_t k = 0; k < cnt; ++k)
      dst[k] = esz == 4 ? double(reinterpret_cast<const float *>(tmp.data())[k]) : reinterpret_cast<const double *>(tmp.data())[k];
    return CSI_OK;
  };
  std::vector<double> h;
  if (c->group_c == 0) {
    if (!dinv) {
      const void *src = n == "b" ? c->w.b : n == "dqs" ? c->w.dqs : c->w.dq;
      if (int rc = fetch(src, size_t(nsol) * N, h)) return rc;
      std::copy(h.begin(), h.end(), out);
      return CSI_OK;
    }
    const size_t cm = coupled ? size_t(nb) * nb : 6 + size_t(ns) * ns;
    if (int rc = fetch(c->w.Dinv, cm * N, h)) return rc;
    if (coupled) { std::copy(h.begin(), h.end(), out); return CSI_OK; }
    // closed-form flow block (x_k = r_k d0, k < 4; x_4 = (r_4 + sum_k a_k x_k) p) as a dense inverse
    std::fill(out, out + size_t(nf) * nf * N, 0.0);
    for (size_t p = 0; p < N; ++p) {
      const double d0 = h[p];
      for (int r = 0; r < 4; ++r) out[size_t(r * nf + r) * N + p] = d0;
      if (nf == 5) {
        const double piv = h[5 * N + p];
        for (int k = 0; k < 4; ++k) out[size_t(4 * nf + k) * N + p] = h[(1 + k) * N + p] * d0 * piv;
        out[size_t(4 * nf + 4) * N + p] = piv;
      }
    }
    std::copy(h.begin() + 6 * N, h.end(), out + size_t(nf) * nf * N);
    return CSI_OK;
  }
  // group schedule: staging (b, D^-1, dQ*) and the step-blocked dQ
  const int nparts = coupled ? 1 : 2;
  size_t fo = 0;  // first output field of the part
  for (int q = 0; q < nparts; ++q) {
    const RecShape rs = rec_shape(q == 1 ? PART_SPECIES : coupled ? PART_COUPLED : PART_FLOW, ns, c->nt, int(esz));
    const int G = rs.G;
    const GroupMap m = group_map(c->ni, c->nj, G);
    const GroupBufs &gb = c->w.grp[q];
    const bool res = n == "dq";
    if (int rc = fetch(res ? gb.x : gb.S, res ? size_t(m.nblk) * m.Lw : size_t(st_words(rs, long(N))), h)) return rc;
    const int nout = dinv ? G * G : G;
    for (int j = 0; j < c->nj; ++j)
      for (int i = 0; i < c->ni; ++i) {
        int cc;
        const long blk = group_blk(m, i, j, cc);
        const long p = long(j) * c->ni + i;
        for (int f = 0; f < nout; ++f) {
          const int r = dinv ? f / G : f, col = dinv ? f % G : 0;
          const long k = dinv ? st_idx(rs, long(N), 0, rw_d(rs, r, col), p)
                              : n == "b" ? st_idx(rs, long(N), 1, dw_b(r), p)
                                         : n == "dqs" ? st_idx(rs, long(N), 2, dw_b(r), p) : m.res(blk, cc, r);
          out[(fo + f) * N + size_t(p)] = h[size_t(k)];
        }
      }
    fo += nout;
  }
  return CSI_OK;
}

// The same arrays for a list of cells, element by element (out [F][n_cells]):
// full-size runs are checked at sampled cells without copying whole fields.
int get_cells(csi_ctx *c, const std::string &n, const long long *cells, int nc, double *out) {
  const size_t N = c->N;
  if (c->wide && n == "Dinv") return c->fail(CSI_ERR_UNSUPPORTED, "Dinv: not kept in this layout by the species-generic kernels");
  auto elem = [&](const void *base, size_t idx, size_t esz, double &v) -> int {
    if (esz == 8) return hip_check(c, hipMemcpy(&v, static_cast<const char *>(base) + idx * 8, 8, hipMemcpyDeviceToHost), "get");
    float f = 0.f;
    const int rc = hip_check(c, hipMemcpy(&f, static_cast<const char *>(base) + idx * 4, 4, hipMemcpyDeviceToHost), "get");
    v = f;
    return rc;
  };
  if (n == "R") {
    for (int f = 0; f < c->nv(); ++f)
      for (int k = 0; k < nc; ++k)
        if (int rc = elem(c->w.R, size_t(f) * N + size_t(cells[k]), 8, out[size_t(f) * nc + k])) return rc;
    return CSI_OK;
  }
  if (c->last_mode < 0 || c->last_prec < 0) return c->fail(CSI_ERR_STATE, "no implicit operator applied yet");
  const bool coupled = c->last_mode == CSI_COUPLED;
  const int nsol = coupled ? c->nb() : c->nsplit();
  const int nf = c->nf(), ns = c->ns, nb = c->nb();
  const bool dinv = n == "Dinv";
  const size_t esz = c->last_prec == CSI_MIXED ? 4 : 8;
  if (c->group_c == 0) {
    if (!dinv || coupled) {
      const void *src = dinv ? c->w.Dinv : n == "b" ? c->w.b : n == "dqs" ? c->w.dqs : c->w.dq;
      const int F = dinv ? nb * nb : nsol;
      for (int f = 0; f < F; ++f)
        for (int k = 0; k < nc; ++k)
          if (int rc = elem(src, size_t(f) * N + size_t(cells[k]), esz, out[size_t(f) * nc + k])) return rc;
      return CSI_OK;
    }
    // split: the closed-form flow block as a dense inverse, then the species inverse
    for (int k = 0; k < nc; ++k) {
      double h6[6];
      for (int f = 0; f < 6; ++f)
        if (int rc = elem(c->w.Dinv, size_t(f) * N + size_t(cells[k]), esz, h6[f])) return rc;
      for (int f = 0; f < nf * nf; ++f) out[size_t(f) * nc + k] = 0.0;
      for (int r = 0; r < 4; ++r) out[size_t(r * nf + r) * nc + k] = h6[0];
      if (nf == 5) {
        for (int q = 0; q < 4; ++q) out[size_t(4 * nf + q) * nc + k] = h6[1 + q] * h6[0] * h6[5];
        out[size_t(4 * nf + 4) * nc + k] = h6[5];
      }
      for (int f = 0; f < ns * ns; ++f)
        if (int rc = elem(c->w.Dinv, size_t(6 + f) * N + size_t(cells[k]), esz, out[size_t(nf * nf + f) * nc + k]))
          return rc;
    }
    return CSI_OK;
  }
  const int nparts = coupled ? 1 : 2;
  size_t fo = 0;
  for (int q = 0; q < nparts; ++q) {
    const RecShape rs = rec_shape(q == 1 ? PART_SPECIES : coupled ? PART_COUPLED : PART_FLOW, ns, c->nt, int(esz));
    const int G = rs.G;
    const GroupMap m = group_map(c->ni, c->nj, G);
    const GroupBufs &gb = c->w.grp[q];
    const bool res = n == "dq";
    const int nout = dinv ? G * G : G;
    for (int k = 0; k < nc; ++k) {
      const long p = long(cells[k]);
      const int i = int(p % c->ni), j = int(p / c->ni);
      int cc;
      const long blk = group_blk(m, i, j, cc);
      for (int f = 0; f < nout; ++f) {
        const int r = dinv ? f / G : f, col = dinv ? f % G : 0;
        const long idx = dinv ? st_idx(rs, long(N), 0, rw_d(rs, r, col), p)
                              : n == "b" ? st_idx(rs, long(N), 1, dw_b(r), p)
                                         : n == "dqs" ? st_idx(rs, long(N), 2, dw_b(r), p) : m.res(blk, cc, r);
        if (int rc = elem(res ? gb.x : gb.S, size_t(idx), esz, out[(fo + f) * nc + k])) return rc;
      }
    }
    fo += nout;
  }
  return CSI_OK;
}

}  // namespace

extern "C" {

int csi_get_cells(csi_ctx *c, const char *name, const long long *cells, int n_cells, double *out) {
  if (!c || !name || !out || n_cells < 0 || (n_cells > 0 && !cells)) return CSI_ERR_ARG;
  if (!c->bound) return c->fail(CSI_ERR_STATE, "not bound");
  const std::string n(name);
  if (n != "R" && n != "b" && n != "dqs" && n != "dq" && n != "Dinv")
    return c->fail(CSI_ERR_ARG, "get_cells: unknown array " + n);
  for (int k = 0; k < n_cells; ++k)
    if (cells[k] < 0 || cells[k] >= (long long)c->N) return c->fail(CSI_ERR_ARG, "get_cells: cell out of range");
  const int rc = get_cells(c, n, cells, n_cells, out);
  if (rc) return rc;
  return hip_check(c, hipStreamSynchronize(c->stream), "get");
}

int csi_get_array(csi_ctx *c, const char *name, double *out, size_t count) {
  if (!c || !name || !out) return CSI_ERR_ARG;
  if (!c->bound) return c->fail(CSI_ERR_STATE, "not bound");
  std::string n(name);
  const size_t N = c->N;
  const double *src = nullptr;
  size_t cnt = 0;
  size_t NP = size_t(c->ni + 2) * (c->nj + 2);
  if (n == "R") { src = c->w.R; cnt = c->nv() * N; }
  else if (n == "dtau") { src = c->w.dtau; cnt = N; }
  else if (n == "src") { src = c->w.src; cnt = c->nv() * N; }
  else if (n == "qw") { src = c->w.qw; cnt = c->ni; }
  else if (n == "b" || n == "dqs" || n == "dq" || n == "Dinv") {
    if (c->last_mode < 0 || c->last_prec < 0) return c->fail(CSI_ERR_STATE, "no implicit operator applied yet");
    return get_records(c, n, out, count);
  } else if (n == "sweep_trace") {
    if (!c->trace) return c->fail(CSI_ERR_STATE, "sweep trace is off");
    const size_t cntt = size_t(4) * c->ni * TR_N;
    if (count < cntt) return c->fail(CSI_ERR_ARG, "buffer too small for sweep_trace");
    std::vector<long long> tmp(cntt);
    int rc = hip_check(c, hipMemcpy(tmp.data(), c->trace_buf, cntt * 8, hipMemcpyDeviceToHost), "get");
    if (rc) return rc;
    for (size_t k = 0; k < cntt; ++k) out[k] = double(tmp[k]);
    return CSI_OK;
  } else if (n == "Jsur") {
    const size_t cntj = size_t(c->ns) * c->ns * N;
    if (count < cntj) return c->fail(CSI_ERR_ARG, "buffer too small for Jsur");
    std::vector<float> tmp(cntj);
    int rc = hip_check(c, hipMemcpy(tmp.data(), c->w.sur.J, cntj * 4, hipMemcpyDeviceToHost), "get");
    if (rc) return rc;
    const size_t nn = size_t(c->ns) * c->ns;
    if (c->ns >= BLOCK_NS_MIN) {  // stored cell-major for the block kernel
      for (size_t p = 0; p < size_t(N); ++p)
        for (size_t k = 0; k < nn; ++k) out[k * N + p] = tmp[p * nn + k];
    } else {
      for (size_t k = 0; k < cntj; ++k) out[k] = tmp[k];
    }
    return CSI_OK;
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
  return hip_check(c, hipMemcpy(out, src, cnt * 8, hipMemcpyDeviceToHost), "get");
}

// ------------------------------------------------------------ surrogate network
}  // extern "C"

namespace {

struct MlpWork {
  size_t off[7];
  size_t total;
};

// scratch of the network calls: packed operands, gradient partials, loss
// partials, loss, statistics partials, scales
MlpWork mlp_work(const MlpDims &d, int batch) {
  MlpWork W;
  const size_t nblk = (size_t(batch) + 63) / 64;
  size_t sizes[] = {size_t(d.nslots) * 16, nblk * d.np * 4, nblk * 8, 8,
                    size_t(MLP_MAX_IN) * MLP_PREP_BLOCKS * 8, 2 * size_t(MLP_PREP_BLOCKS) * 8,
                    size_t(2 * MLP_MAX_IN + 1) * 8};
  size_t o = 0;
  for (int k = 0; k < 7; ++k) { W.off[k] = o; o += al(sizes[k]); }
  W.total = o;
  return W;
}

bool mlp_ok(int n_in, int n_out) { return n_in >= 1 && n_in <= MLP_MAX_IN && n_out >= 1 && n_out <= MLP_MAX_OUT; }

int mlp_check_work(csi_ctx *c, const MlpDims &d, int batch, const void *work, size_t bytes) {
  if (!work || reinterpret_cast<uintptr_t>(work) % 256) return c->fail(CSI_ERR_ARG, "work buffer missing or not 256-byte aligned");
  if (bytes < mlp_work(d, batch).total) return c->fail(CSI_ERR_ARG, "work buffer too small");
  return CSI_OK;
}

hipError_t mlp_pack(const MlpDims &d, const float *params, void *P, hipStream_t st) {
  hipLaunchKernelGGL(k_mlp_pack, dim3((d.nslots + 255) / 256), dim3(256), 0, st, d, params, static_cast<u16x8 *>(P));
  return hipGetLastError();
}

// gradient partials for one batch, then the ordered reduction (and Adam when m, v are given)
int mlp_grad_adam(csi_ctx *c, const csi_mlp_batch *b, float *grad, float *am, float *av, int step, const csi_adam *h,
                  double *loss) {
  if (!b || !b->x || !b->t || !b->idx || !b->params) return c->fail(CSI_ERR_ARG, "mlp batch: null pointer");
  if (!mlp_ok(b->n_in, b->n_out) || b->batch < 1 || b->n_data < 1) return c->fail(CSI_ERR_ARG, "mlp batch: sizes");
  const MlpDims d = mlp_dims(b->n_in, b->n_out);
  int rc = mlp_check_work(c, d, b->batch, b->work, b->work_bytes);
  if (rc) return rc;
  const MlpWork W = mlp_work(d, b->batch);
  char *w = static_cast<char *>(b->work);
  auto *P = reinterpret_cast<const u16x8 *>(w + W.off[0]);
  auto *part = reinterpret_cast<float *>(w + W.off[1]);
  auto *lpart = reinterpret_cast<double *>(w + W.off[2]);
  auto *ldev = reinterpret_cast<double *>(w + W.off[3]);
  const int nblk = (b->batch + 63) / 64;
  const float scale = float(2.0 / (double(b->batch) * b->n_out));
  hipError_t e = mlp_pack(d, b->params, w + W.off[0], c->stream);
  if (e == hipSuccess) {
    if (d.ks1 == 1)
      hipLaunchKernelGGL(k_mlp_grad<1>, dim3(nblk), dim3(256), 0, c->stream, d, P, b->params, b->x, b->t, b->idx,
                         b->batch, b->n_data, scale, part, lpart);
    else
      hipLaunchKernelGGL(k_mlp_grad<2>, dim3(nblk), dim3(256), 0, c->stream, d, P, b->params, b->x, b->t, b->idx,
                         b->batch, b->n_data, scale, part, lpart);
    e = hipGetLastError();
  }
  if (e == hipSuccess) {
    const double lr = h ? h->lr : 0.0, b1 = h ? h->beta1 : 0.0, b2 = h ? h->beta2 : 0.0, eps = h ? h->eps : 0.0;
    hipLaunchKernelGGL(k_mlp_reduce, dim3((d.np + 255) / 256), dim3(256), 0, c->stream, d.np, nblk, part, lpart,
                       1.0 / (double(b->batch) * b->n_out), ldev, grad, am ? b->params : nullptr, am, av, step, lr, b1,
                       b2, eps);
    e = hipGetLastError();
  }
  if ((rc = hip_check(c, e, "mlp launch"))) return rc;
  if (loss) {
    if ((rc = hip_check(c, hipMemcpyAsync(loss, ldev, 8, hipMemcpyDeviceToHost, c->stream), "loss"))) return rc;
    return hip_check(c, hipStreamSynchronize(c->stream), "sync");
  }
  return CSI_OK;
}

}  // namespace

extern "C" {

int csi_mlp_sizes(int n_in, int n_out, int batch, int *n_params, size_t *work_bytes) {
  if (!mlp_ok(n_in, n_out) || batch < 1) return CSI_ERR_ARG;
  const MlpDims d = mlp_dims(n_in, n_out);
  if (n_params) *n_params = d.np;
  if (work_bytes) *work_bytes = mlp_work(d, batch).total;
  return CSI_OK;
}

int csi_mlp_prepare(csi_ctx *c, int n, int n_in, int n_out, const float *x_raw, const float *jc, float *x, float *t,
                    double *scales_host, void *work, size_t work_bytes) {
  if (!c) return CSI_ERR_ARG;
  if (!mlp_ok(n_in, n_out) || n < 1 || !x_raw || !jc || !x || !t || !scales_host)
    return c->fail(CSI_ERR_ARG, "mlp_prepare: arguments");
  const MlpDims d = mlp_dims(n_in, n_out);
  int rc = mlp_check_work(c, d, 1, work, work_bytes);
  if (rc) return rc;
  const MlpWork W = mlp_work(d, 1);
  char *w = static_cast<char *>(work);
  auto *mpart = reinterpret_cast<double *>(w + W.off[4]);
  auto *jpart = reinterpret_cast<double *>(w + W.off[5]);
  auto *sc = reinterpret_cast<double *>(w + W.off[6]);
  hipStream_t st = c->stream;
  const dim3 gm(MLP_PREP_BLOCKS, n_in);
  hipLaunchKernelGGL(k_prep_moments, gm, dim3(256), 0, st, n, n_in, x_raw, nullptr, mpart);
  hipLaunchKernelGGL(k_prep_logj, dim3(MLP_PREP_BLOCKS), dim3(256), 0, st, long(n) * n_out, jc, jpart);
  hipLaunchKernelGGL(k_prep_finish, dim3(1), dim3(64), 0, st, 0, n, n_in, mpart, jpart, sc);
  hipLaunchKernelGGL(k_prep_moments, gm, dim3(256), 0, st, n, n_in, x_raw, sc, mpart);
  hipLaunchKernelGGL(k_prep_finish, dim3(1), dim3(64), 0, st, 1, n, n_in, mpart, jpart, sc);
  const long tot = long(n) * (n_in > n_out ? n_in : n_out);
  hipLaunchKernelGGL(k_prep_apply, dim3(unsigned((tot + 255) / 256)), dim3(256), 0, st, long(n), n_in, n_out, x_raw, jc,
                     sc, x, t);
  if ((rc = hip_check(c, hipGetLastError(), "mlp_prepare launch"))) return rc;
  if ((rc = hip_check(c, hipMemcpyAsync(scales_host, sc, size_t(2 * n_in + 1) * 8, hipMemcpyDeviceToHost, st), "scales")))
    return rc;
  return hip_check(c, hipStreamSynchronize(st), "sync");
}

// pack the operands into `packed` (d.nslots 16-byte slots), then the forward pass
hipError_t mlp_forward_launch(const MlpDims &d, const float *params, const float *x, int n, float *y, void *packed,
                              hipStream_t st) {
  hipError_t e = mlp_pack(d, params, packed, st);
  auto *P = static_cast<const u16x8 *>(packed);
  const unsigned nb = unsigned((long(n) + 63) / 64);
  if (e == hipSuccess) {
    if (d.ks1 == 1) hipLaunchKernelGGL(k_mlp_forward<1>, dim3(nb), dim3(256), 0, st, d, P, params, x, n, y);
    else hipLaunchKernelGGL(k_mlp_forward<2>, dim3(nb), dim3(256), 0, st, d, P, params, x, n, y);
    e = hipGetLastError();
  }
  return e;
}

int csi_mlp_forward(csi_ctx *c, int n_in, int n_out, int n, const float *params, const float *x, float *y, void *work,
                    size_t work_bytes) {
  if (!c) return CSI_ERR_ARG;
  if (!mlp_ok(n_in, n_out) || n < 1 || !params || !x || !y) return c->fail(CSI_ERR_ARG, "mlp_forward: arguments");
  const MlpDims d = mlp_dims(n_in, n_out);
  int rc = mlp_check_work(c, d, 1, work, work_bytes);
  if (rc) return rc;
  char *w = static_cast<char *>(work);
  const MlpWork W = mlp_work(d, 1);
  return hip_check(c, mlp_forward_launch(d, params, x, n, y, w + W.off[0], c->stream), "mlp_forward launch");
}

int csi_mlp_forward_noalloc(csi_ctx *c, int n_in, int n_out, int n, const float *params, const float *x, float *y) {
  if (!c) return CSI_ERR_ARG;
  if (!mlp_ok(n_in, n_out) || n < 1 || !params || !x || !y)
    return c->fail(CSI_ERR_ARG, "mlp_forward_noalloc: arguments");
  const MlpDims d = mlp_dims(n_in, n_out);
  if (size_t(d.nslots) * 16 > size_t(CSI_MLP_NOALLOC_SCRATCH_BYTES))
    return c->fail(CSI_ERR_ARG, "mlp_forward_noalloc: the packed network needs " + std::to_string(size_t(d.nslots) * 16) +
                                    " bytes of scratch, more than " + std::to_string(CSI_MLP_NOALLOC_SCRATCH_BYTES));
  if (!c->noalloc) return c->fail(CSI_ERR_STATE, "mlp_forward_noalloc: no scratch address for this device");
  return hip_check(c, mlp_forward_launch(d, params, x, n, y, c->noalloc, c->stream), "mlp_forward_noalloc launch");
}

int csi_mlp_grad(csi_ctx *c, const csi_mlp_batch *b, float *grad, double *loss) {
  if (!c) return CSI_ERR_ARG;
  if (!grad) return c->fail(CSI_ERR_ARG, "mlp_grad: null gradient");
  return mlp_grad_adam(c, b, grad, nullptr, nullptr, 0, nullptr, loss);
}

int csi_mlp_train_step(csi_ctx *c, const csi_mlp_batch *b, float *m, float *v, int step, const csi_adam *h,
                       double *loss) {
  if (!c) return CSI_ERR_ARG;
  if (!m || !v || !h || step < 1 || !(h->lr > 0.0) || !(h->beta1 >= 0.0 && h->beta1 < 1.0) ||
      !(h->beta2 >= 0.0 && h->beta2 < 1.0) || !(h->eps > 0.0))
    return c->fail(CSI_ERR_ARG, "mlp_train_step: Adam arguments");
  return mlp_grad_adam(c, b, nullptr, m, v, step, h, loss);
}

int csi_mlp_train_epoch(csi_ctx *c, const csi_mlp_batch *b, const int *order, int n_rows, float *m, float *v,
                        int step0, const csi_adam *h, double *loss) {
  if (!c) return CSI_ERR_ARG;
  if (!b || !order || n_rows < 1 || b->batch < 1 || step0 < 0)
    return c->fail(CSI_ERR_ARG, "mlp_train_epoch: arguments");
  if (!m || !v || !h || !(h->lr > 0.0) || !(h->beta1 >= 0.0 && h->beta1 < 1.0) ||
      !(h->beta2 >= 0.0 && h->beta2 < 1.0) || !(h->eps > 0.0))
    return c->fail(CSI_ERR_ARG, "mlp_train_epoch: Adam arguments");
  // every step's kernels go on the stream back to back; the host waits only
  // for the last batch's loss
  csi_mlp_batch lb = *b;
  int step = step0;
  for (long b0 = 0; b0 < n_rows; b0 += b->batch) {
    const bool last = b0 + b->batch >= n_rows;
    lb.idx = order + b0;
    lb.batch = int(last ? n_rows - b0 : b->batch);
    int rc = mlp_grad_adam(c, &lb, nullptr, m, v, ++step, h, last ? loss : nullptr);
    if (rc) return rc;
  }
  return CSI_OK;
}

int csi_sample_jacobians(csi_ctx *c, int max_samples, unsigned long long seed, float *x_raw, float *jc,
                         int *n_written) {
  if (!c) return CSI_ERR_ARG;
  if (max_samples < 1 || !x_raw || !jc) return c->fail(CSI_ERR_ARG, "sample_jacobians: arguments");
  if (!ready(c)) return c->fail(CSI_ERR_STATE, "sample_jacobians: workspace/state not set");
  if (c->wide) return c->fail(CSI_ERR_UNSUPPORTED, "sample_jacobians: no reactions on the species-generic kernels");
  const int n = max_samples < c->N ? max_samples : c->N;
  const SampleMap sm = n < c->N ? sample_map(seed, c->N) : SampleMap{0, 0};
  int rc = hip_check(c, c->run->sample(c->g, c->w, c->stream, n, x_raw, jc, c->jc_flag(), sm), "sample launch");
  if (rc) return rc;
  int fl[FL_N];
  if ((rc = read_flags(c, fl))) return rc;
  if (fl[FL_BAD] != INT_MAX) return c->fail(CSI_ERR_NONFINITE, "non-physical state at cell " + std::to_string(fl[FL_BAD]));
  if (n_written) *n_written = n;
  c->has_res = false;
  return CSI_OK;
}

int csi_set_surrogate(csi_ctx *c, const float *params, const double *scales, int n_in, int n_out, double stall_ratio,
                      int stall_window) {
  if (!c) return CSI_ERR_ARG;
  if (!c->bound) return c->fail(CSI_ERR_STATE, "set_surrogate before bind_workspace");
  if (c->wide) return c->fail(CSI_ERR_UNSUPPORTED, "set_surrogate: not on the species-generic kernels");
  if (!params || !scales || n_in != c->ns + 3 || n_out != c->ns * c->ns || !(stall_ratio > 0.0) || stall_window < 1)
    return c->fail(CSI_ERR_ARG, "set_surrogate: expects n_in = ns + 3, n_out = ns^2, ratio > 0, window >= 1");
  for (int k = 0; k < 2 * n_in + 1; ++k)
    if (!std::isfinite(scales[k]) || (k >= n_in && !(scales[k] > 0.0)))
      return c->fail(CSI_ERR_ARG, "set_surrogate: scales must be finite with positive sigma and tau0");
  const MlpDims d = mlp_dims(n_in, n_out);
  hipStream_t st = c->stream;
  hipError_t e = hipMemcpyAsync(const_cast<float *>(c->w.sur.p), params, size_t(d.np) * 4, hipMemcpyDeviceToDevice, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(const_cast<double *>(c->w.sur.scales), scales, size_t(2 * n_in + 1) * 8, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = mlp_pack(d, c->w.sur.p, const_cast<u16x8 *>(c->w.sur.P), st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  int rc = hip_check(c, e, "set_surrogate");
  if (rc) return rc;
  c->has_sur = true;
  c->sur_ratio = stall_ratio;
  c->sur_window = stall_window;
  return CSI_OK;
}

}  // extern "C"
