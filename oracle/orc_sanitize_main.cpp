// TEST INFRASTRUCTURE ONLY: a driver that runs the oracle's C API under the
// address and undefined-behaviour sanitizers (tests/test_oracle_sanitize.py
// builds it with g++ -fsanitize=address,undefined).  It reads a case file
// written by the test: the mechanism tables, the grid nodes, the free stream
// and the state, then runs residuals, both implicit operators in both sweep
// orders, the corrections, a dual-time step, the flux-difference sweeps, the
// wall heat flux and the dense operator, and prints the norms.
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "orc.h"

namespace {

FILE *in;
int geti() {
  int v;
  if (std::fscanf(in, "%d", &v) != 1) { std::fprintf(stderr, "bad case file\n"); std::exit(2); }
  return v;
}
double getd() {
  double v;
  if (std::fscanf(in, "%lf", &v) != 1) { std::fprintf(stderr, "bad case file\n"); std::exit(2); }
  return v;
}
std::vector<double> vd(size_t n) {
  std::vector<double> v(n);
  for (auto &x : v) x = getd();
  return v;
}
std::vector<int> vi(size_t n) {
  std::vector<int> v(n);
  for (auto &x : v) x = geti();
  return v;
}
void check(int rc, const char *what, orc_ctx *c) {
  if (rc != 0) {
    std::fprintf(stderr, "%s failed: %d %s\n", what, rc, orc_last_error(c));
    std::exit(3);
  }
}

}  // namespace

int main(int argc, char **argv) {
  if (argc < 2 || !(in = std::fopen(argv[1], "r"))) return 2;
  const int ns = geti(), nr = geti(), tt = geti();
  auto M = vd(ns);
  auto kind = vi(ns);
  auto thv = vd(ns), thr = vd(ns), sig = vd(ns), gel = vd(ns), hf = vd(ns), sc = vd(ns), la = vd(ns), lb = vd(ns);
  auto A = vd(nr), b = vd(nr), th = vd(nr);
  auto tctl = vi(nr), third = vi(nr), nuf = vi(size_t(nr) * ns), nub = vi(size_t(nr) * ns);
  auto eff = vd(size_t(nr) * ns);
  const double mu_ref = getd(), T_ref = getd(), mu_exp = getd();
  const int ni = geti(), nj = geti();
  auto xn = vd(size_t(ni + 1) * (nj + 1)), yn = vd(size_t(ni + 1) * (nj + 1));
  auto rs = vd(ns);
  const double u = getd(), v = getd(), T = getd(), Tv = getd();
  const int nv = ns + 3 + (tt ? 1 : 0);
  auto q = vd(size_t(nv) * ni * nj);
  std::fclose(in);

  orc_mechanism mm{ns, nr, tt, M.data(), kind.data(), thv.data(), thr.data(), sig.data(), gel.data(), hf.data(),
                   sc.data(), la.data(), lb.data(), A.data(), b.data(), th.data(), tctl.data(), third.data(),
                   nuf.data(), nub.data(), eff.data(), mu_ref, T_ref, mu_exp};
  orc_ctx *c = nullptr;
  check(orc_create(&c), "create", c);
  check(orc_set_grid(c, ni, nj, xn.data(), yn.data(), 300.0, 0), "grid", c);
  check(orc_set_mechanism(c, &mm), "mechanism", c);
  check(orc_set_freestream(c, rs.data(), u, v, T, Tv), "freestream", c);
  check(orc_set_state(c, q.data()), "state", c);
  double nrm[2];
  for (int mode = 0; mode < 2; ++mode)
    for (int order = 0; order < 2; ++order) {
      check(orc_residual(c, 10.0, nrm), "residual", c);
      check(orc_implicit_op(c, mode, order), "implicit_op", c);
    }
  for (int reading = 0; reading < 4; ++reading) {
    check(orc_set_option(c, "jc_fixed_qf", reading), "option", c);
    check(orc_residual(c, 10.0, nrm), "residual", c);
    check(orc_implicit_op(c, 1, 0), "implicit_op", c);
  }
  check(orc_set_option(c, "flux_diff", 1), "option", c);
  for (int mode = 0; mode < 2; ++mode) {
    check(orc_residual(c, 0.01, nrm), "residual", c);  // small increments: the perturbed states stay physical
    check(orc_implicit_op(c, mode, 0), "flux-difference sweeps", c);
  }
  check(orc_set_option(c, "flux_diff", 0), "option", c);
  int nclip = 0;
  check(orc_consistency_correct(c, 1, 2, &nclip), "cc2", c);
  check(orc_set_physical_time(c, 1e-6, 0.5), "physical time", c);
  check(orc_advance_time(c), "advance", c);
  std::vector<double> hist(2 * 3);
  check(orc_step(c, 1, 1, 10.0, 0, 0, 3, hist.data()), "step", c);
  check(orc_step(c, 0, 0, 10.0, 0, 0, 2, hist.data()), "step", c);
  check(orc_set_physical_time(c, 0.0, 0.0), "physical time", c);
  check(orc_residual(c, 10.0, nrm), "residual", c);
  std::vector<double> qw(ni);
  double qs = 0.0;
  check(orc_wall_heat_flux(c, qw.data(), &qs), "wall heat flux", c);
  const int n = ni * nj * (ns + (tt ? 5 : 4) - 1);
  std::vector<double> D(size_t(n) * n), L(size_t(n) * n), U(size_t(n) * n);
  check(orc_dense_operator(c, 0, D.data(), L.data(), U.data()), "dense operator", c);
  std::printf("r_rho %.17g r_E %.17g q_stag %.17g clipped %d\n", nrm[0], nrm[1], qs, nclip);
  orc_destroy(c);
  return 0;
}
