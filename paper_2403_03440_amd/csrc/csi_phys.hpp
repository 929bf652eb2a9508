// Device (and host) physics of the implicit solver library: thermodynamics,
// equation of state with its analytic derivatives, finite-rate kinetics with
// analytic source Jacobians, transport.  Templated on the species count NS
// and the temperature model NT (1: one temperature, 2: T and Tv) so that all
// per-cell vectors live in registers.
//
// Model (paper Section 2.1, Eq. (govern) and Eq. (flux); the sub-models the
// paper defers to other references follow the readings in the design notes):
//   e_s(T,Tv) = cvtr_s T + e_ve,s(Tv) + hf_s,  e_ve = harmonic vibration (+ 3/2 R_e Tv for e-)
//   p = sum_heavy rho_s R_s T + rho_e R_e Tv
//   k_f = A Tf^b exp(-theta/Tf),  k_b = A T^b exp(-theta/T) / Kc(T),
//   Kc from the rigid-rotor / harmonic-oscillator Gibbs energies.
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>

#define CSI_HD __host__ __device__ __forceinline__

namespace csi {

constexpr int MAXS = 32;
constexpr int MAXR = 64;
constexpr double RU = 8.314462618;
constexpr double ATM = 101325.0;
constexpr double EPS4 = 4.0 * 2.220446049250313e-16;
constexpr double TV_FLOOR = 50.0;  // lower bound of Tv after an update (positivity of rho e_ve)

enum { ATOM = 0, MOLECULE = 1, ELECTRON = 2 };

struct Reaction {
  double lnA, b, theta;
  int tctl, third, nreac, nprod, dnu, nnet;
  int reac[3], prod[3];      // species per unit stoichiometry (repeats allowed)
  int net_s[6], net_nu[6];   // net stoichiometry nu'' - nu' (non-zero entries)
};

// Mechanism in device memory (read through a uniform pointer).
struct Mech {
  int ns, nr, two_temp, e_idx;   // e_idx: electron species or -1
  double M[MAXS], R[MAXS], cvtr[MAXS], thv[MAXS], hf[MAXS], hfm[MAXS], ck[MAXS], iSc[MAXS];
  double lta[MAXS], ltb[MAXS], gconst[MAXS], gexp[MAXS];
  int kind[MAXS];
  Reaction rx[MAXR];
  double eff[MAXR][MAXS];
  double mu_ref, T_ref, mu_exp;
  double iM[MAXS];          // 1 / M_s
  double nuM[MAXR][MAXS];   // M_s (nu''_rs - nu'_rs): weight of reaction r's rate in omega_s
};

template <int NS, int NT> struct Dims {
  static constexpr int ns = NS;
  static constexpr int nf = (NT == 2) ? 5 : 4;
  static constexpr int nv = NS + 3 + (NT == 2 ? 1 : 0);
  static constexpr int nb = nf + NS - 1;
  static constexpr int nsplit = nf + NS;
};

// ------------------------------------------------------------- thermo
CSI_HD double evib(double R, double th, double T) {
  if (th <= 0.0) return 0.0;
  double em = exp(-th / T);
  return R * th * em / (1.0 - em);
}
CSI_HD double cvvib(double R, double th, double T) {
  if (th <= 0.0) return 0.0;
  double x = th / T, em = exp(-x), d = 1.0 - em;
  return R * x * x * em / (d * d);
}
CSI_HD double eve_s(const Mech &m, int s, double Tv) {
  int k = m.kind[s];
  return k == MOLECULE ? evib(m.R[s], m.thv[s], Tv) : (k == ELECTRON ? 1.5 * m.R[s] * Tv : 0.0);
}
CSI_HD double cvve_s(const Mech &m, int s, double Tv) {
  int k = m.kind[s];
  return k == MOLECULE ? cvvib(m.R[s], m.thv[s], Tv) : (k == ELECTRON ? 1.5 * m.R[s] : 0.0);
}
// e_ve,s and cv_ve,s together, with one exponential (the same operations as
// eve_s and cvve_s, so the same values)
CSI_HD void eve_cvve_s(const Mech &m, int s, double Tv, double &e, double &cv) {
  const int k = m.kind[s];
  if (k == MOLECULE && m.thv[s] > 0.0) {
    const double R = m.R[s], th = m.thv[s];
    const double x = th / Tv, em = exp(-x), d = 1.0 - em;
    e = R * th * em / d;
    cv = R * x * x * em / (d * d);
  } else if (k == ELECTRON) {
    e = 1.5 * m.R[s] * Tv;
    cv = 1.5 * m.R[s];
  } else {
    e = 0.0;
    cv = 0.0;
  }
}
// molar Gibbs energy / (Ru T): hfm/(Ru T) - (gexp ln T + gconst - ln(1 - exp(-thv/T)))
CSI_HD double gRT(const Mech &m, int s, double T, double lnT) {
  double g = m.hfm[s] / (RU * T) - (m.gexp[s] * lnT + m.gconst[s]);
  if (m.kind[s] == MOLECULE && m.thv[s] > 0.0) g += log(1.0 - exp(-m.thv[s] / T));
  return g;
}
// molar enthalpy / (Ru T^2) contribution to d ln Kc / dT:  H/(Ru T^2)
CSI_HD double hRT2(const Mech &m, int s, double T) {
  double h = m.hfm[s] / (RU * T * T) + m.gexp[s] / T;
  if (m.kind[s] == MOLECULE && m.thv[s] > 0.0) {
    double em = exp(-m.thv[s] / T);
    h += m.thv[s] * em / ((1.0 - em) * T * T);
  }
  return h;
}

// Root of an increasing f.  f(x, fv, dv, fa) returns f, f' and the sum of
// the magnitudes of the terms of f: |f| <= 4 eps fa means f vanishes to its
// own rounding, and the iteration stops there, as it does on a step of at
// most 4 ulp of x.
CSI_HD bool root_reached(double fx, double fa) { return fabs(fx) <= 4.0 * 2.220446049250313e-16 * fa; }

// Newton steps kept inside a bisection bracket.
template <class F> CSI_HD bool newton_bracket(F f, double &x, double lo, double hi) {
  double flo, fhi, d, a;
  f(lo, flo, d, a);
  f(hi, fhi, d, a);
  if (!(flo <= 0.0 && fhi >= 0.0)) return false;
  if (!(x > lo && x < hi)) x = 0.5 * (lo + hi);
  for (int it = 0; it < 200; ++it) {
    double fx, dx_, fa;
    f(x, fx, dx_, fa);
    if (fx == 0.0 || root_reached(fx, fa)) return true;
    if (fx < 0.0) lo = x; else hi = x;
    double xn = x - fx / dx_;
    if (!(xn > lo && xn < hi)) xn = 0.5 * (lo + hi);
    double dx = xn - x;
    x = xn;
    if (fabs(dx) <= EPS4 * fabs(x) || hi - lo <= EPS4 * fabs(x)) return true;
  }
  return true;
}

// Newton iteration from a guess already close to the root (at most 4 steps);
// false when it has not converged, so that the caller can bracket instead
template <class F> CSI_HD bool newton_from(F f, double &x) {
  for (int it = 0; it < 4; ++it) {
    double fx, dfx, fa;
    f(x, fx, dfx, fa);
    if (fx == 0.0 || root_reached(fx, fa)) return true;
    if (!(dfx > 0.0)) return false;
    const double xn = x - fx / dfx;
    if (!(xn > 0.0)) return false;
    const double dx = xn - x;
    x = xn;
    if (fabs(dx) <= EPS4 * fabs(x)) return true;
  }
  return false;
}

// Per-cell primitive record
template <int NS, int NT> struct Prim {
  double rho, u, v, T, Tv, p, c, H, eve, rE;
  double Y[NS], rs[NS];
  // EOS derivatives of p w.r.t. stored variables: pr[s] = dp/drho_s,
  // pE = dp/d(rho E), pv = dp/d(rho e_ve); dp/d(rho u) = -pE u, dp/d(rho v) = -pE v
  double pr[NS], pE, pv;
  // temperature derivatives w.r.t. stored variables
  double dT_dr[NS], dT_dE, dT_dv, dTv_dr[NS], dTv_dv;
  double rcv;  // rho cv (1T total, 2T translational-rotational)
  int tvT;     // 1 when Tv follows T (one temperature, or no vibrating species)
};

// q (stored variables) -> primitives and EOS derivatives.  Returns false on a
// non-physical state.  T0, Tv0 > 0: temperatures already solved for this q
// (the Newton iterations then start there).
template <int NS, int NT>
CSI_HD bool prim_from_q(const Mech &m, const double *q, Prim<NS, NT> &P, double T0 = 0.0, double Tv0 = 0.0) {
  double rho = 0.0;
#pragma unroll
  for (int s = 0; s < NS; ++s) { P.rs[s] = q[s]; rho += q[s]; }
  if (!(rho > 0.0)) return false;
  P.rho = rho;
  double irho = 1.0 / rho;
#pragma unroll
  for (int s = 0; s < NS; ++s) P.Y[s] = P.rs[s] / rho;
  P.u = q[NS] / rho;
  P.v = q[NS + 1] / rho;
  P.rE = q[NS + 2];
  double k2 = P.u * P.u + P.v * P.v;
  double ekin = 0.5 * rho * k2;
  (void)irho;
  if (NT == 1) {
    double target = P.rE - ekin;
    auto f = [&](double T, double &fv, double &dv, double &fa) {
      fv = -target;
      dv = 0.0;
      fa = fabs(target);
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        double ev, cv;
        eve_cvve_s(m, s, T, ev, cv);
        const double es = P.rs[s] * (m.cvtr[s] * T + ev + m.hf[s]);
        fv += es;
        fa += fabs(es);
        dv += P.rs[s] * (m.cvtr[s] + cv);
      }
    };
    double T = T0 > 0.0 ? T0 : 1000.0;
    if (!(T0 > 0.0 && newton_from(f, T))) {
      T = T0 > 0.0 ? T0 : 1000.0;  // safeguarded iterations from the guess
      if (!newton_bracket(f, T, 1.0, 1.0e6)) return false;
    }
    P.T = T;
    P.Tv = T;
    P.tvT = 1;
    double rcv = 0.0, rR = 0.0, evs[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      double cv;
      eve_cvve_s(m, s, T, evs[s], cv);
      rcv += P.rs[s] * (m.cvtr[s] + cv);
      rR += P.rs[s] * m.R[s];
    }
    P.rcv = rcv;
    P.p = rR * T;
    double beta = rR / rcv;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      double es = m.cvtr[s] * T + evs[s] + m.hf[s];
      P.dT_dr[s] = (0.5 * k2 - es) / rcv;
      P.pr[s] = m.R[s] * T + rR * P.dT_dr[s];
      P.dTv_dr[s] = P.dT_dr[s];
    }
    P.dT_dE = 1.0 / rcv;
    P.dT_dv = 0.0;
    P.dTv_dv = 0.0;
    P.pE = beta;
    P.pv = 0.0;
    P.eve = 0.0;
  } else {
    double rEve = q[NS + 3];
    double num = P.rE - ekin - rEve, rcv = 0.0;
#pragma unroll
    for (int s = 0; s < NS; ++s) { num -= P.rs[s] * m.hf[s]; rcv += P.rs[s] * m.cvtr[s]; }
    double T = num / rcv;
    if (!(T > 0.0)) return false;
    P.T = T;
    P.rcv = rcv;
    bool has_ve = false;
#pragma unroll
    for (int s = 0; s < NS; ++s)
      if (P.rs[s] > 0.0 && ((m.kind[s] == MOLECULE && m.thv[s] > 0.0) || m.kind[s] == ELECTRON)) has_ve = true;
    double Tv = T;
    if (has_ve) {
      auto f = [&](double t, double &fv, double &dv, double &fa) {
        fv = -rEve;
        dv = 0.0;
        fa = fabs(rEve);
#pragma unroll
        for (int s = 0; s < NS; ++s) {
          double ev, cv;
          eve_cvve_s(m, s, t, ev, cv);
          const double es = P.rs[s] * ev;
          fv += es;
          fa += fabs(es);
          dv += P.rs[s] * cv;
        }
      };
      if (Tv0 > 0.0) Tv = Tv0;
      if (!(Tv0 > 0.0 && newton_from(f, Tv))) {
        Tv = Tv0 > 0.0 ? Tv0 : T;
        if (!newton_bracket(f, Tv, 1.0, 1.0e6)) return false;
      }
    }
    P.Tv = Tv;
    P.tvT = has_ve ? 0 : 1;
    double rRh = 0.0, rRe = 0.0, rcvv = 0.0, evs[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      if (m.kind[s] == ELECTRON) rRe += P.rs[s] * m.R[s];
      else rRh += P.rs[s] * m.R[s];
      double cv;
      eve_cvve_s(m, s, Tv, evs[s], cv);
      rcvv += P.rs[s] * cv;
    }
    P.p = rRh * T + rRe * Tv;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      P.dT_dr[s] = (0.5 * k2 - m.cvtr[s] * T - m.hf[s]) / rcv;
      P.dTv_dr[s] = has_ve ? -evs[s] / rcvv : P.dT_dr[s];
      P.pr[s] = m.R[s] * (m.kind[s] == ELECTRON ? Tv : T) + rRh * P.dT_dr[s] + rRe * P.dTv_dr[s];
    }
    P.dT_dE = 1.0 / rcv;
    P.dT_dv = -1.0 / rcv;
    P.dTv_dv = has_ve ? 1.0 / rcvv : -1.0 / rcv;
    P.pE = rRh / rcv;
    P.pv = -rRh / rcv + rRe * P.dTv_dv;
    P.eve = rEve / rho;
  }
  P.H = (P.rE + P.p) / rho;
  double c2 = P.u * (-P.pE * P.u) + P.v * (-P.pE * P.v) + P.H * P.pE;
#pragma unroll
  for (int s = 0; s < NS; ++s) c2 += P.Y[s] * P.pr[s];
  if (NT == 2) c2 += P.eve * P.pv;
  if (!(c2 > 0.0) || !(P.p > 0.0)) return false;
  P.c = sqrt(c2);
  return true;
}

// primitives -> stored variables
template <int NS, int NT>
CSI_HD void q_from_prim(const Mech &m, const double *rs, double u, double v, double T, double Tv, double *q) {
  if (NT == 1) Tv = T;
  double rho = 0.0, rEi = 0.0, rEve = 0.0;
  for (int s = 0; s < NS; ++s) {
    q[s] = rs[s];
    rho += rs[s];
    rEi += rs[s] * (m.cvtr[s] * T + eve_s(m, s, Tv) + m.hf[s]);
    rEve += rs[s] * eve_s(m, s, Tv);
  }
  q[NS] = rho * u;
  q[NS + 1] = rho * v;
  q[NS + 2] = rEi + 0.5 * rho * (u * u + v * v);
  if (NT == 2) q[NS + 3] = rEve;
}

// ----------------------------------------------------------- transport
struct Transport {
  double mu, k, kve, nuF, nuC, nuK;
};
template <int NS, int NT>
CSI_HD void transport(const Mech &m, const Prim<NS, NT> &P, Transport &t) {
  t.mu = m.mu_ref * exp(m.mu_exp * log(P.T / m.T_ref));
  double ktr = 0.0, kint = 0.0, cvtr = 0.0, cvint = 0.0, iScmax = 0.0;
  double Tint = NT == 2 ? P.Tv : P.T;
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    ktr += P.Y[s] * m.ck[s];
    double cve = cvve_s(m, s, Tint);
    kint += P.Y[s] * cve;
    cvtr += P.Y[s] * m.cvtr[s];
    cvint += P.Y[s] * cve;
    iScmax = fmax(iScmax, m.iSc[s]);
  }
  if (NT == 2) {
    t.k = t.mu * ktr;
    t.kve = t.mu * kint;
    t.nuF = fmax(4.0 * t.mu / (3.0 * P.rho), t.k / (P.rho * cvtr));
  } else {
    t.k = t.mu * (ktr + kint);
    t.kve = 0.0;
    t.nuF = fmax(4.0 * t.mu / (3.0 * P.rho), t.k / (P.rho * (cvtr + cvint)));
  }
  t.nuC = t.mu * iScmax / P.rho;
  t.nuK = fmax(t.nuF, t.nuC);
}

// ------------------------------------------------------------ kinetics
// Production rates omega_s (kg/m^3/s), the vibrational source omega_ve and
// their analytic derivatives at fixed (T, Tv) with respect to rho_s, and with
// respect to T and Tv at fixed rho_s.
template <int NS, int NT> struct Chem {
  double w[NS], dw_dr[NS][NS], dw_dT[NS], dw_dTv[NS];
  double wv, dwv_dr[NS], dwv_dT, dwv_dTv;
};

template <int NS, int NT, bool JAC>
CSI_HD void chemistry(const Mech &m, const double *rs, double T, double Tv, double p,
                                          Chem<NS, NT> &C) {
  double X[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    X[s] = rs[s] / m.M[s];
    C.w[s] = 0.0;
    if (JAC) {
      C.dw_dT[s] = 0.0;
      C.dw_dTv[s] = 0.0;
#pragma unroll
      for (int r = 0; r < NS; ++r) C.dw_dr[s][r] = 0.0;
    }
  }
  if (NT == 1) Tv = T;
  double lnT = log(T), lnTv = log(Tv);
  double gs[NS], hs[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    gs[s] = gRT(m, s, T, lnT);
    if (JAC) hs[s] = hRT2(m, s, T);
  }
  double lnc0 = log(1.0e5 / (RU * T));
  for (int r = 0; r < m.nr; ++r) {
    const Reaction &R = m.rx[r];
    double lnTf = lnT, dTf_dT = 1.0, dTf_dTv = 0.0, Tf = T;
    if (NT == 2 && R.tctl == 1) {
      lnTf = 0.5 * (lnT + lnTv);
      Tf = exp(lnTf);
      dTf_dT = 0.5 * Tf / T;
      dTf_dTv = 0.5 * Tf / Tv;
    } else if (NT == 2 && R.tctl == 2) {
      lnTf = lnTv;
      Tf = Tv;
      dTf_dT = 0.0;
      dTf_dTv = 1.0;
    }
    double kf = exp(R.lnA + R.b * lnTf - R.theta / Tf);
    double lnKc = double(R.dnu) * lnc0, dlnKc = -double(R.dnu) / T;
    for (int e = 0; e < R.nnet; ++e) {
      lnKc -= double(R.net_nu[e]) * gs[R.net_s[e]];
      if (JAC) dlnKc += double(R.net_nu[e]) * hs[R.net_s[e]];
    }
    double kb = exp(R.lnA + R.b * lnT - R.theta / T - lnKc);
    double Pf = 1.0, Pb = 1.0;
    for (int e = 0; e < R.nreac; ++e) Pf *= X[R.reac[e]];
    for (int e = 0; e < R.nprod; ++e) Pb *= X[R.prod[e]];
    double Mc = 1.0;
    if (R.third) {
      Mc = 0.0;
#pragma unroll
      for (int s = 0; s < NS; ++s) Mc += m.eff[r][s] * X[s];
    }
    double net = kf * Pf - kb * Pb;
    double qr = Mc * net;
    // d q / d X_s
    double dq[NS];
    double dqT = 0.0, dqTv = 0.0;
    if (JAC) {
#pragma unroll
      for (int s = 0; s < NS; ++s) dq[s] = R.third ? m.eff[r][s] * net : 0.0;
      for (int e = 0; e < R.nreac; ++e) {
        double lo = 1.0;
        for (int f = 0; f < R.nreac; ++f)
          if (f != e) lo *= X[R.reac[f]];
        int s = R.reac[e];
#pragma unroll
        for (int t = 0; t < NS; ++t)
          if (t == s) dq[t] += Mc * kf * lo;
      }
      for (int e = 0; e < R.nprod; ++e) {
        double lo = 1.0;
        for (int f = 0; f < R.nprod; ++f)
          if (f != e) lo *= X[R.prod[f]];
        int s = R.prod[e];
#pragma unroll
        for (int t = 0; t < NS; ++t)
          if (t == s) dq[t] -= Mc * kb * lo;
      }
      double dkf_dTf = kf * (R.b + R.theta / Tf) / Tf;
      double dkb_dT = kb * ((R.b + R.theta / T) / T - dlnKc);
      dqT = Mc * (dkf_dTf * dTf_dT * Pf - dkb_dT * Pb);
      dqTv = Mc * (dkf_dTf * dTf_dTv * Pf);
    }
    for (int e = 0; e < R.nnet; ++e) {
      int s = R.net_s[e];
      double nu = double(R.net_nu[e]);
#pragma unroll
      for (int t = 0; t < NS; ++t) {
        if (t == s) {
          C.w[t] += m.M[t] * nu * qr;
          if (JAC) {
            C.dw_dT[t] += m.M[t] * nu * dqT;
            C.dw_dTv[t] += m.M[t] * nu * dqTv;
#pragma unroll
            for (int u = 0; u < NS; ++u) C.dw_dr[t][u] += m.M[t] * nu * dq[u] / m.M[u];
          }
        }
      }
    }
  }
  if (NT == 2) {
    // Landau-Teller relaxation with tau_s = exp(a_s (T^-1/3 - b_s) - 18.42) atm / p
    double Tm13 = exp(-lnT / 3.0);
    double pT = 0.0, pTv = 0.0;  // dp/dT, dp/dTv at fixed rho_s
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      if (m.kind[s] == ELECTRON) pTv += rs[s] * m.R[s];
      else pT += rs[s] * m.R[s];
    }
    double wv = 0.0, dT_ = 0.0, dTv_ = 0.0;
    double dr[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) dr[s] = 0.0;
    double lt_sum = 0.0;  // sum rho_s (ev(T)-ev(Tv)) / tau_s, used for the p-derivative
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      if (m.kind[s] == MOLECULE && m.thv[s] > 0.0) {
        double E = exp(18.42 - m.lta[s] * (Tm13 - m.ltb[s]));  // 1/tau = p/ATM * E
        double itau = p / ATM * E;
        double evT = evib(m.R[s], m.thv[s], T), evTv = evib(m.R[s], m.thv[s], Tv);
        double term = rs[s] * (evT - evTv) * itau;
        wv += term;
        lt_sum += term;
        if (JAC) {
          dr[s] += (evT - evTv) * itau;
          // d itau/dT at fixed p: itau * a_s/3 T^-4/3
          dT_ += rs[s] * cvvib(m.R[s], m.thv[s], T) * itau + term * (m.lta[s] / 3.0) * Tm13 / T;
          dTv_ += -rs[s] * cvvib(m.R[s], m.thv[s], Tv) * itau;
        }
      }
    }
    if (JAC) {
      // pressure dependence of 1/tau
#pragma unroll
      for (int s = 0; s < NS; ++s) dr[s] += lt_sum * (m.R[s] * (m.kind[s] == ELECTRON ? Tv : T)) / p;
      dT_ += lt_sum * pT / p;
      dTv_ += lt_sum * pTv / p;
    }
    double ev[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      ev[s] = eve_s(m, s, Tv);
      wv += C.w[s] * ev[s];
    }
    C.wv = wv;
    if (JAC) {
#pragma unroll
      for (int u = 0; u < NS; ++u) {
        double a = dr[u];
#pragma unroll
        for (int s = 0; s < NS; ++s) a += C.dw_dr[s][u] * ev[s];
        C.dwv_dr[u] = a;
      }
      double aT = dT_, aTv = dTv_;
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        aT += C.dw_dT[s] * ev[s];
        aTv += C.dw_dTv[s] * ev[s] + C.w[s] * cvve_s(m, s, Tv);
      }
      C.dwv_dT = aT;
      C.dwv_dTv = aTv;
    }
  } else {
    C.wv = 0.0;
  }
}

// Storage-variable derivatives of T and Tv for column c of
// q = (rho_1..rho_ns, rho u, rho v, rho E, [rho e_ve]).
template <int NS, int NT>
CSI_HD void temp_derivs(const Prim<NS, NT> &P, int c, double &dT, double &dTv) {
  if (c < NS) { dT = P.dT_dr[c]; dTv = P.dTv_dr[c]; }
  else if (c == NS) { dT = -P.u * P.dT_dE; dTv = P.tvT ? dT : 0.0; }
  else if (c == NS + 1) { dT = -P.v * P.dT_dE; dTv = P.tvT ? dT : 0.0; }
  else if (c == NS + 2) { dT = P.dT_dE; dTv = P.tvT ? dT : 0.0; }
  else { dT = P.dT_dv; dTv = P.dTv_dv; }
}

// Temperature derivatives along the direction that adds mass of species r at
// the cell's velocity and internal energy density (rho u, rho v and rho E
// change by u, v and |u|^2 / 2 per unit mass; rho e_ve is held): the split
// species block with the temperatures following the composition.
// hold_tv (two temperatures): the vibrational temperature held as well, rho
// e_ve taking the added mass's e_ve,r(Tv) out of the same internal energy.
template <int NS, int NT>
CSI_HD void temp_derivs_fixed_e(const Mech &m, const Prim<NS, NT> &P, int r, bool hold_tv, double &dT,
                                double &dTv) {
  double a, b;
  const double ke = 0.5 * (P.u * P.u + P.v * P.v);
  temp_derivs<NS, NT>(P, r, dT, dTv);
  if (NT == 2 && hold_tv) {
    const double ev = eve_s(m, r, P.Tv);
    temp_derivs<NS, NT>(P, NS + 3, a, b);
    dT += ev * a;
    dTv += ev * b;
  }
  temp_derivs<NS, NT>(P, NS, a, b);
  dT += P.u * a;
  dTv += P.u * b;
  temp_derivs<NS, NT>(P, NS + 1, a, b);
  dT += P.v * a;
  dTv += P.v * b;
  temp_derivs<NS, NT>(P, NS + 2, a, b);
  dT += ke * a;
  dTv += ke * b;
}

// Coupled source Jacobian dS_z/dz in the coupled unknowns
// z = (rho, m_x, m_y, rhoE, [rhoe_ve], rho_0..rho_{ns-2}) with the last
// species density closed by rho - sum of the others (paper Section 2.1).
// Rows: S_z = (sum_s omega_s, 0, 0, 0, [omega_ve], omega_0..omega_{ns-2}).
template <int NS, int NT>
CSI_HD void coupled_source_jacobian(const Prim<NS, NT> &P, const Chem<NS, NT> &C,
                                    double (&Jz)[Dims<NS, NT>::nb][Dims<NS, NT>::nb]) {
  using D = Dims<NS, NT>;
  constexpr int NV = D::nv, NB = D::nb, NF = D::nf;
  double Jq[NB][NV];  // z-rows x storage columns
#pragma unroll
  for (int c = 0; c < NV; ++c) {
    double dT, dTv;
    temp_derivs<NS, NT>(P, c, dT, dTv);
    double sum = 0.0;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      double v = C.dw_dT[s] * dT + C.dw_dTv[s] * dTv;
      if (c < NS) v += C.dw_dr[s][c < NS ? c : 0];
      if (s < NS - 1) Jq[NF + s][c] = v;
      sum += v;
    }
    Jq[0][c] = sum;
    Jq[1][c] = 0.0;
    Jq[2][c] = 0.0;
    Jq[3][c] = 0.0;
    if (NT == 2) {
      double v = C.dwv_dT * dT + C.dwv_dTv * dTv;
      if (c < NS) v += C.dwv_dr[c < NS ? c : 0];
      Jq[4][c] = v;
    }
  }
#pragma unroll
  for (int r = 0; r < NB; ++r) {
    Jz[r][0] = Jq[r][NS - 1];
    Jz[r][1] = Jq[r][NS];
    Jz[r][2] = Jq[r][NS + 1];
    Jz[r][3] = Jq[r][NS + 2];
    if (NT == 2) Jz[r][4] = Jq[r][NS + 3];
#pragma unroll
    for (int s = 0; s < NS - 1; ++s) Jz[r][NF + s] = Jq[r][s] - Jq[r][NS - 1];
  }
}

// Split flow block source row (two temperatures): d omega_ve / d Q_F at
// frozen mass fractions, Q_F = (rho, m_x, m_y, rhoE, rhoe_ve).
template <int NS, int NT>
CSI_HD void flow_source_row(const Prim<NS, NT> &P, const Chem<NS, NT> &C, double (&dwv)[5]) {
  double a = 0.0;
#pragma unroll
  for (int s = 0; s < NS; ++s) a += P.Y[s] * (C.dwv_dr[s] + C.dwv_dT * P.dT_dr[s] + C.dwv_dTv * P.dTv_dr[s]);
  dwv[0] = a;
#pragma unroll
  for (int c = 1; c < 5; ++c) {
    double dT, dTv;
    temp_derivs<NS, NT>(P, NS - 1 + c, dT, dTv);
    dwv[c] = C.dwv_dT * dT + C.dwv_dTv * dTv;
  }
}

}  // namespace csi
