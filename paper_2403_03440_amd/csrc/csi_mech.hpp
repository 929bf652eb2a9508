// Mechanism table construction shared by the host API (and host-side checks).
#pragma once
#include <cmath>
#include <cstring>
#include <string>

#include "../../include/csi.h"
#include "csi_phys.hpp"

namespace csi {

// Copy the caller's tables into the device layout, with the constant parts of
// the Gibbs energies and the per-reaction species lists precomputed.
inline bool build_mech(const csi_mechanism *mm, Mech &m, std::string &err) {
  std::memset(&m, 0, sizeof(Mech));
  const int ns = mm->ns;
  m.ns = ns; m.nr = mm->nr; m.two_temp = mm->two_temp ? 1 : 0; m.e_idx = -1;
  const double kB = 1.380649e-23, hP = 6.62607015e-34, NA = 6.02214076e23, PI = 3.14159265358979323846;
  for (int s = 0; s < ns; ++s) {
    int kd = mm->kind[s];
    if (kd < 0 || kd > 2 || !(mm->M[s] > 0.0)) { err = ("set_mechanism: species"); return false; }
    m.kind[s] = kd;
    if (kd == ELECTRON) m.e_idx = s;
    m.M[s] = mm->M[s];
    m.iM[s] = 1.0 / mm->M[s];
    m.R[s] = RU / mm->M[s];
    m.cvtr[s] = kd == ATOM ? 1.5 * m.R[s] : (kd == MOLECULE ? 2.5 * m.R[s] : 0.0);
    m.thv[s] = kd == MOLECULE ? mm->theta_v[s] : 0.0;
    m.hf[s] = mm->h_form[s] / mm->M[s];
    m.hfm[s] = mm->h_form[s];
    m.ck[s] = kd == ATOM ? 3.75 * m.R[s] : (kd == MOLECULE ? 4.75 * m.R[s] : 0.0);
    m.iSc[s] = 1.0 / mm->sc[s];
    m.lta[s] = mm->lt_a[s];
    m.ltb[s] = mm->lt_b[s];
    double mass = mm->M[s] / NA;
    m.gexp[s] = kd == MOLECULE ? 3.5 : 2.5;
    m.gconst[s] = 1.5 * std::log(2.0 * PI * mass * kB / (hP * hP)) + std::log(kB / 1.0e5) + std::log(mm->g_el[s]);
    if (kd == MOLECULE) m.gconst[s] -= std::log(mm->sigma[s] * mm->theta_r[s]);
  }
  for (int r_ = 0; r_ < mm->nr; ++r_) {
    Reaction &R = m.rx[r_];
    R.lnA = mm->A[r_] > 0.0 ? std::log(mm->A[r_]) : -INFINITY;
    R.b = mm->b[r_];
    R.theta = mm->theta[r_];
    R.tctl = mm->tctl[r_];
    R.third = mm->third[r_] ? 1 : 0;
    R.nreac = R.nprod = R.nnet = R.dnu = 0;
    for (int s = 0; s < ns; ++s) {
      int nf_ = mm->nu_f[r_ * ns + s], nb_ = mm->nu_b[r_ * ns + s];
      if (nf_ < 0 || nb_ < 0) { err = ("negative stoichiometry"); return false; }
      for (int k = 0; k < nf_; ++k) {
        if (R.nreac >= 3) { err = ("more than 3 reactant molecules"); return false; }
        R.reac[R.nreac++] = s;
      }
      for (int k = 0; k < nb_; ++k) {
        if (R.nprod >= 3) { err = ("more than 3 product molecules"); return false; }
        R.prod[R.nprod++] = s;
      }
      m.nuM[r_][s] = mm->M[s] * double(nb_ - nf_);
      if (nb_ != nf_) {
        R.net_s[R.nnet] = s;
        R.net_nu[R.nnet] = nb_ - nf_;
        R.nnet++;
        R.dnu += nb_ - nf_;
      }
      m.eff[r_][s] = mm->eff[r_ * ns + s];
    }
  }
  m.mu_ref = mm->mu_ref; m.T_ref = mm->T_ref; m.mu_exp = mm->mu_exp;
  return true;
}

}  // namespace csi
