// Launch sequences of the species-generic path (one temperature, no
// reactions, any species count up to CSI_WIDE_MAX_SPECIES), behind the same
// IRunner interface as the compiled runners.
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/csi.h"
#include "csi_runner.hpp"
#include "csi_wide.hpp"

namespace csi {

static_assert(WGJ_B == WGJ_SCRATCH_ROWS, "Gauss-Jordan scratch sized for the panel width");

hipError_t wide_invert(double *W, int n, int count, int *perm, double *XK, int *sing, const int *done,
                       hipStream_t st) {
  if (n <= 0 || count <= 0) return hipSuccess;
  const size_t lds = size_t(n + WGJ_B) * 8;
  const int ct = (n + 63) / 64, cc = (n + 255) / 256;
  for (int kb = 0; kb < n; kb += WGJ_B) {
    hipLaunchKernelGGL(kw_gj_panel, dim3(count), dim3(256), lds, st, W, n, kb, perm, sing, done);
    // the other columns (previous panels' and later ones), if any
    if (kb > 0 || kb + WGJ_B < n) {
      hipLaunchKernelGGL(kw_gj_swap, dim3(count, cc), dim3(256), 0, st, W, n, kb, perm, XK, done);
      hipLaunchKernelGGL(kw_gj_update, dim3(count, ct, ct), dim3(256), 0, st, W, n, kb, XK, done);
    }
  }
  hipLaunchKernelGGL(kw_gj_unpermute, dim3(count, cc), dim3(256), 0, st, W, n, perm, done);
  return hipGetLastError();
}

hipError_t launch_stream_prim(const Geo &g, const WMech &m, const double *Q, const double *qfs, double *prim,
                              int *bad, const int *done, int guess, hipStream_t st) {
  hipLaunchKernelGGL(kw_prim, dim3(nblocks(g.NP)), dim3(256), 0, st, g, m, Q, qfs, prim, bad, done, guess);
  return hipGetLastError();
}

hipError_t launch_stream_faces(const Geo &g, const WMech &m, const double *prim, double *Fi, double *Ri, double *Fj,
                               double *Rj, double *qw, const int *done, hipStream_t st) {
  hipLaunchKernelGGL(kw_face<false>, dim3(nblocks(long(g.ni + 1) * g.nj)), dim3(256), 0, st, g, m, prim, Fi, Ri, qw,
                     done);
  hipLaunchKernelGGL(kw_face<true>, dim3(nblocks(long(g.ni) * (g.nj + 1))), dim3(256), 0, st, g, m, prim, Fj, Rj, qw,
                     done);
  return hipGetLastError();
}

namespace {

// host species table, uploaded at bind: [4 scalars][6 x ns doubles][ns ints]
struct WTable {
  int ns = 0;
  std::vector<char> bytes;
  double *d() { return reinterpret_cast<double *>(bytes.data()); }
  const double *d() const { return reinterpret_cast<const double *>(bytes.data()); }
  const int *kind() const { return reinterpret_cast<const int *>(d() + 4 + 6 * size_t(ns)); }
  double R(int s) const { return d()[4 + s]; }
  double cvtr(int s) const { return d()[4 + ns + s]; }
  double thv(int s) const { return d()[4 + 2 * ns + s]; }
  double hf(int s) const { return d()[4 + 3 * ns + s]; }
};

class WideRunner : public IRunner {
 public:
  explicit WideRunner(WTable t) : T_(std::move(t)), ns_(T_.ns) {}
  int nprim() const override { return WF(ns_).N; }

  const void *host_table(size_t *bytes) const override {
    *bytes = T_.bytes.size();
    return T_.bytes.data();
  }

  hipError_t prim(const Geo &g, const WS &w, hipStream_t st, bool stoppable, bool guess) override {
    return launch_stream_prim(g, mech(w), w.Q, w.qfs, w.prim, w.flags + FL_BAD,
                              stoppable ? w.flags + FL_DONE : nullptr, guess ? 1 : 0, st);
  }

  hipError_t faces(const Geo &g, const WS &w, hipStream_t st, bool stoppable) override {
    return launch_stream_faces(g, mech(w), w.prim, w.Fi, w.Ri, w.Fj, w.Rj, w.qw,
                               stoppable ? w.flags + FL_DONE : nullptr, st);
  }

  hipError_t cell(const Geo &g, const WS &w, hipStream_t st, double cfl, int mode, int prec, int flags,
                  bool stoppable, hipEvent_t sur_ready, hipEvent_t mid) override {
    (void)prec;
    (void)sur_ready;
    const int *done = stoppable ? w.flags + FL_DONE : nullptr;
    const WCellOut o{w.R, w.dtau, w.part, w.diag, static_cast<double *>(w.Dinv), static_cast<double *>(w.b)};
    hipLaunchKernelGGL(kw_cell, dim3(w.nblk_cell), dim3(256), 0, st, g, ns_, w.Fi, w.Fj, w.Ri, w.Rj, cfl, mode,
                       flags, o, done);
    if (mid) {
      const hipError_t e = hipEventRecord(mid, st);
      if (e != hipSuccess) return e;
    }
    if ((flags & 2) && mode == 0) {
      // the coupled block: assembled dense, inverted by blocked Gauss-Jordan
      const int n = ns_ + 3;
      const size_t tot = size_t(n) * n * g.N;
      const int nb = int(std::min<size_t>((tot + 255) / 256, size_t(1) << 20));
      double *W = static_cast<double *>(w.Dinv);
      hipLaunchKernelGGL(kw_ci_assemble, dim3(nb), dim3(256), 0, st, w.diag, g.V, n, g.N, W, done);
      const hipError_t e = wide_invert(W, n, g.N, w.gj_perm, w.gj_xk, w.flags + FL_SING, done, st);
      if (e != hipSuccess) return e;
    }
    return hipGetLastError();
  }

  hipError_t norms(const WS &w, hipStream_t st, int it, double tol, bool stoppable, StallArgs stall) override {
    hipLaunchKernelGGL(k_norms<2>, dim3(1), dim3(256), 0, st, w.part, w.nblk_cell, w.norms,
                       stoppable ? w.hist : nullptr, it, w.hist_max, stoppable ? w.r0 : nullptr, tol,
                       stoppable ? w.flags + FL_DONE : nullptr, w.flags + FL_ITDONE, stall);
    return hipGetLastError();
  }

  hipError_t surrogate(const Geo &, const WS &, hipStream_t, bool) override { return hipErrorNotSupported; }
  hipError_t sample(const Geo &, const WS &, hipStream_t, int, float *, float *, int, SampleMap) override {
    return hipErrorNotSupported;
  }

  hipError_t sweeps(const Geo &g, const WS &w, hipStream_t st, int mode, int prec, bool stoppable,
                    hipEvent_t mid) override {
    (void)prec;
    const int *done = stoppable ? w.flags + FL_DONE : nullptr;
    const WSweep a{w.prim, w.Ri, w.Rj, static_cast<const double *>(w.Dinv), static_cast<const double *>(w.b),
                   static_cast<double *>(w.dqs), static_cast<double *>(w.dq), mode, ns_};
    const int n = mode == 0 ? ns_ + 3 : ns_ + 4;
    const size_t lds = size_t(8 + n) * 8;
    const int nhp = g.ni + g.nj - 1;
    auto cells = [&](int k) {
      const int j0 = k - g.ni + 1 > 0 ? k - g.ni + 1 : 0;
      const int j1 = k < g.nj - 1 ? k : g.nj - 1;
      return j1 - j0 + 1;
    };
    const int nrb = mode == 0 ? (n + WSW_ROWS - 1) / WSW_ROWS : 1;
    for (int k = 0; k < nhp; ++k)
      hipLaunchKernelGGL(kw_sweep<true>, dim3(cells(k), nrb), dim3(256), lds, st, g, a, k, done);
    if (mid) {
      const hipError_t e = hipEventRecord(mid, st);
      if (e != hipSuccess) return e;
    }
    for (int k = nhp - 1; k >= 0; --k)
      hipLaunchKernelGGL(kw_sweep<false>, dim3(cells(k), nrb), dim3(256), lds, st, g, a, k, done);
    return hipGetLastError();
  }

  hipError_t update(const Geo &g, const WS &w, hipStream_t st, int mode, int prec, int kind,
                    bool stoppable) override {
    (void)prec;
    hipLaunchKernelGGL(kw_update, dim3(nblocks(g.N)), dim3(256), 0, st, g, ns_, w.Q,
                       static_cast<const double *>(w.dq), mode, kind, w.flags + FL_CLIP, w.flags + FL_BAD,
                       stoppable ? w.flags + FL_DONE : nullptr);
    return hipGetLastError();
  }

  // as q_from_prim in one temperature, from the host table
  hipError_t q_from_prim_host(const Mech &, const double *rs, double u, double v, double T, double,
                              double *q) override {
    double rho = 0.0, rEi = 0.0;
    const int *kind = T_.kind();
    for (int s = 0; s < ns_; ++s) {
      q[s] = rs[s];
      rho += rs[s];
      const double R = T_.R(s), th = T_.thv(s);
      const double ev = kind[s] == MOLECULE ? evib(R, th, T) : (kind[s] == ELECTRON ? 1.5 * R * T : 0.0);
      rEi += rs[s] * (T_.cvtr(s) * T + ev + T_.hf(s));
    }
    q[ns_] = rho * u;
    q[ns_ + 1] = rho * v;
    q[ns_ + 2] = rEi + 0.5 * rho * (u * u + v * v);
    return hipSuccess;
  }

 private:
  WTable T_;
  int ns_;

  WMech mech(const WS &w) const {
    const int ns = ns_;
    const double *d = w.wtab;
    WMech m;
    m.ns = ns;
    m.mu_ref = T_.d()[0];
    m.T_ref = T_.d()[1];
    m.mu_exp = T_.d()[2];
    m.iscmax = T_.d()[3];
    m.R = d + 4;
    m.cvtr = d + 4 + ns;
    m.thv = d + 4 + 2 * ns;
    m.hf = d + 4 + 3 * ns;
    m.ck = d + 4 + 4 * ns;
    m.iSc = d + 4 + 5 * ns;
    m.kind = reinterpret_cast<const int *>(d + 4 + 6 * size_t(ns));
    return m;
  }
};

}  // namespace

IRunner *make_wide_runner(const csi_mechanism *mm, std::string &err) {
  const int ns = mm->ns;
  WTable t;
  t.ns = ns;
  t.bytes.assign((4 + 6 * size_t(ns)) * 8 + size_t(ns) * 4, 0);
  double *d = t.d();
  int *kind = reinterpret_cast<int *>(d + 4 + 6 * size_t(ns));
  double iscmax = 0.0;
  for (int s = 0; s < ns; ++s) {
    const int kd = mm->kind[s];
    if (kd < 0 || kd > 2 || !(mm->M[s] > 0.0) || !(mm->sc[s] > 0.0)) {
      err = "species " + std::to_string(s);
      return nullptr;
    }
    const double R = RU / mm->M[s];
    d[4 + s] = R;
    d[4 + ns + s] = kd == ATOM ? 1.5 * R : (kd == MOLECULE ? 2.5 * R : 0.0);
    d[4 + 2 * ns + s] = kd == MOLECULE ? mm->theta_v[s] : 0.0;
    d[4 + 3 * ns + s] = mm->h_form[s] / mm->M[s];
    d[4 + 4 * ns + s] = kd == ATOM ? 3.75 * R : (kd == MOLECULE ? 4.75 * R : 0.0);
    d[4 + 5 * ns + s] = 1.0 / mm->sc[s];
    iscmax = std::fmax(iscmax, 1.0 / mm->sc[s]);
    kind[s] = kd;
  }
  d[0] = mm->mu_ref;
  d[1] = mm->T_ref;
  d[2] = mm->mu_exp;
  d[3] = iscmax;
  return new WideRunner(std::move(t));
}

}  // namespace csi
