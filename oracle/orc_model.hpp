// Oracle: TEST INFRASTRUCTURE ONLY. Plain, slow FP64 CPU reference for the
// component-splitting implicit solver. Only tests/, __graft_entry__.smoke() and
// bench.py's cpu_baseline leg may load it. It shares no code with the HIP path.
//
// Physical model (templated on the scalar type so that complex-step
// differentiation gives derivatives exact to rounding):
//   * governing system and constitutive laws: paper Section 2.1,
//     Eq. (govern), Eq. (flux) and the equations for tau, q, q_v, V_s, e_t, e_v, p;
//   * the sub-models the paper defers to other references (thermodynamics,
//     transport, kinetics, vibrational relaxation) use the readings listed in
//     the design notes: rigid-rotor/harmonic-oscillator species with a
//     statistical-mechanics Gibbs energy, mass-action Arrhenius kinetics with
//     thermodynamically consistent backward rates, Park-type sqrt(T Tv)
//     controlling temperature, Landau-Teller relaxation of Millikan-White form,
//     one power-law viscosity with Eucken conductivities and Schmidt-number
//     diffusivities.
#pragma once
#include <cmath>
#include <complex>
#include <type_traits>
#include <utility>
#include <vector>

namespace orc {

using cplx = std::complex<double>;
inline double re(double x) { return x; }
inline double re(const cplx &x) { return x.real(); }

// species limit of the fixed-size per-cell arrays: 32 in the default build,
// larger in the wide build (-DORC_MAXS=256) used for the species-count study
#ifndef ORC_MAXS
#define ORC_MAXS 32
#endif
constexpr int MAXS = ORC_MAXS;
constexpr int MAXV = MAXS + 4;     // stored variables limit
constexpr double Ru = 8.314462618;   // J/(mol K)
constexpr double kB = 1.380649e-23;  // J/K
constexpr double hP = 6.62607015e-34;
constexpr double NA = 6.02214076e23;
constexpr double P_STD = 1.0e5;      // standard-state pressure, Pa
constexpr double ATM = 101325.0;
constexpr double PI = 3.14159265358979323846;

enum { KIND_ATOM = 0, KIND_MOLECULE = 1, KIND_ELECTRON = 2 };

struct Mech {
  int ns = 0, nr = 0, two_temp = 0;
  std::vector<double> M, theta_v, theta_r, sigma, g_el, h_form, sc, lt_a, lt_b;
  std::vector<int> kind;
  std::vector<double> A, b, theta;
  std::vector<int> tctl, third;
  std::vector<int> nu_f, nu_b;   // [nr*ns]
  std::vector<double> eff;       // [nr*ns]
  double mu_ref = 0, T_ref = 0, mu_exp = 0;

  int nv() const { return ns + 3 + (two_temp ? 1 : 0); }
  int nf() const { return 4 + (two_temp ? 1 : 0); }  // flow unknowns of the split form
  int nb() const { return nf() + ns - 1; }           // coupled unknowns
  double R(int s) const { return Ru / M[s]; }
};

// ---------------------------------------------------------------- thermo
// Species energies per unit mass.  Translational-rotational modes at T,
// vibration (and electron translation) at Tv.  In the one-temperature model
// every call passes Tv = T.
inline double cv_tr(const Mech &m, int s) {
  switch (m.kind[s]) {
    case KIND_ATOM: return 1.5 * m.R(s);
    case KIND_MOLECULE: return 2.5 * m.R(s);
    default: return 0.0;
  }
}

// harmonic-oscillator vibrational energy R th/(exp(th/T)-1), written with
// exp(-th/T) so that it stays finite for th/T large.
template <class S> S e_vib(double Rs, double th, const S &T) {
  if (th <= 0.0) return S(0.0);
  S em = std::exp(-th / T);
  return Rs * th * em / (1.0 - em);
}
template <class S> S cv_vib(double Rs, double th, const S &T) {
  if (th <= 0.0) return S(0.0);
  S x = th / T;
  S em = std::exp(-x);
  S d = 1.0 - em;
  return Rs * x * x * em / (d * d);
}

template <class S> S e_ve(const Mech &m, int s, const S &Tv) {
  switch (m.kind[s]) {
    case KIND_MOLECULE: return e_vib(m.R(s), m.theta_v[s], Tv);
    case KIND_ELECTRON: return 1.5 * m.R(s) * Tv;
    default: return S(0.0);
  }
}
template <class S> S cv_ve(const Mech &m, int s, const S &Tv) {
  switch (m.kind[s]) {
    case KIND_MOLECULE: return cv_vib(m.R(s), m.theta_v[s], Tv);
    case KIND_ELECTRON: return S(1.5 * m.R(s));
    default: return S(0.0);
  }
}
inline double hform(const Mech &m, int s) { return m.h_form[s] / m.M[s]; }

// e_s(T, Tv): internal energy per unit mass including the 0 K formation energy.
template <class S> S e_s(const Mech &m, int s, const S &T, const S &Tv) {
  return cv_tr(m, s) * T + e_ve(m, s, Tv) + hform(m, s);
}
// h_s = e_s + p_s/rho_s; the electron partial pressure is taken at Tv.
template <class S> S h_s(const Mech &m, int s, const S &T, const S &Tv) {
  return e_s(m, s, T, Tv) + m.R(s) * (m.kind[s] == KIND_ELECTRON ? Tv : T);
}

// Molar standard Gibbs energy divided by Ru*T, all modes at T, from the
// rigid-rotor / harmonic-oscillator partition function (energies counted from
// the ground state, formation enthalpy at 0 K).
template <class S> S gibbs_RT(const Mech &m, int s, const S &T) {
  double mass = m.M[s] / NA;
  S lnq = 1.5 * std::log(2.0 * PI * mass * kB * T / (hP * hP)) + std::log(kB * T / P_STD) +
          std::log(m.g_el[s]);
  if (m.kind[s] == KIND_MOLECULE) {
    lnq += std::log(T / (m.sigma[s] * m.theta_r[s]));
    if (m.theta_v[s] > 0.0) lnq -= std::log(1.0 - std::exp(-m.theta_v[s] / T));
  }
  return m.h_form[s] / (Ru * T) - lnq;
}

// ---------------------------------------------------------------- state
template <class S> struct Prim {
  S rs[MAXS], Y[MAXS];
  S rho, u, v, T, Tv, p;
};

// Solve f(x) = 0 for an increasing function by Newton steps kept inside a
// bisection bracket; the iteration stops at 4 ulp of x.
template <class F> static bool solve_monotone(F f, double &x, double lo, double hi) {
  double flo = f(lo).first, fhi = f(hi).first;
  if (!(flo <= 0.0 && fhi >= 0.0)) return false;
  if (!(x > lo && x < hi)) x = 0.5 * (lo + hi);
  for (int it = 0; it < 200; ++it) {
    auto fd = f(x);
    if (fd.first == 0.0) return true;
    if (fd.first < 0.0) lo = x; else hi = x;
    double xn = x - fd.first / fd.second;
    if (!(xn > lo && xn < hi)) xn = 0.5 * (lo + hi);
    double dx = xn - x;
    x = xn;
    if (std::fabs(dx) <= 4.0 * 2.220446049250313e-16 * std::fabs(x)) return true;
    if (hi - lo <= 4.0 * 2.220446049250313e-16 * std::fabs(x)) return true;
  }
  return true;
}

// Conservative q = (rho_1..rho_ns, rho u, rho v, rho E, [rho e_ve]) -> primitives.
// 1T: T from the total internal energy by Newton.  2T: T in closed form from
// the translational-rotational energy, Tv by Newton on rho e_ve.
// The complex-valued version first solves on the real parts, then runs a few
// complex Newton steps from that root so that the imaginary parts carry the
// exact derivative of the implicit function.
template <class S> bool recover(const Mech &m, const S *q, Prim<S> &P) {
  const int ns = m.ns;
  S rho = 0.0;
  for (int s = 0; s < ns; ++s) { P.rs[s] = q[s]; rho += q[s]; }
  if (!(re(rho) > 0.0)) return false;
  P.rho = rho;
  for (int s = 0; s < ns; ++s) P.Y[s] = P.rs[s] / rho;
  P.u = q[ns] / rho;
  P.v = q[ns + 1] / rho;
  S rE = q[ns + 2];
  S ekin = 0.5 * rho * (P.u * P.u + P.v * P.v);
  constexpr bool is_c = std::is_same<S, cplx>::value;
  if (!m.two_temp) {
    S target = rE - ekin;
    auto fr = [&](double T) {
      double f = -re(target), d = 0.0;
      for (int s = 0; s < ns; ++s) {
        f += re(P.rs[s]) * re(e_s<double>(m, s, T, T));
        d += re(P.rs[s]) * (cv_tr(m, s) + cv_ve<double>(m, s, T));
      }
      return std::make_pair(f, d);
    };
    double T = 1000.0;
    if (!solve_monotone(fr, T, 1.0, 1.0e6)) return false;
    S Tc = T;
    if (is_c) {
      for (int it = 0; it < 3; ++it) {
        S f = -target, d = 0.0;
        for (int s = 0; s < ns; ++s) {
          f += P.rs[s] * e_s<S>(m, s, Tc, Tc);
          d += P.rs[s] * (cv_tr(m, s) + cv_ve<S>(m, s, Tc));
        }
        Tc = Tc - f / d;
      }
    }
    P.T = Tc;
    P.Tv = Tc;
  } else {
    S rEve = q[ns + 3];
    S num = rE - ekin - rEve, den = 0.0;
    for (int s = 0; s < ns; ++s) { num -= P.rs[s] * hform(m, s); den += P.rs[s] * cv_tr(m, s); }
    P.T = num / den;
    if (!(re(P.T) > 0.0)) return false;
    bool has_ve = false;
    for (int s = 0; s < ns; ++s)
      if ((m.kind[s] == KIND_MOLECULE && m.theta_v[s] > 0.0 && re(P.rs[s]) > 0.0) ||
          (m.kind[s] == KIND_ELECTRON && re(P.rs[s]) > 0.0))
        has_ve = true;
    if (!has_ve) {
      P.Tv = P.T;
    } else {
      auto fr = [&](double Tv) {
        double f = -re(rEve), d = 0.0;
        for (int s = 0; s < ns; ++s) {
          f += re(P.rs[s]) * e_ve<double>(m, s, Tv);
          d += re(P.rs[s]) * cv_ve<double>(m, s, Tv);
        }
        return std::make_pair(f, d);
      };
      double Tv = re(P.T);
      if (!solve_monotone(fr, Tv, 1.0, 1.0e6)) return false;
      S Tvc = Tv;
      if (is_c) {
        for (int it = 0; it < 3; ++it) {
          S f = -rEve, d = 0.0;
          for (int s = 0; s < ns; ++s) {
            f += P.rs[s] * e_ve<S>(m, s, Tvc);
            d += P.rs[s] * cv_ve<S>(m, s, Tvc);
          }
          Tvc = Tvc - f / d;
        }
      }
      P.Tv = Tvc;
    }
  }
  // ideal-gas mixture EOS; electrons at Tv
  S p = 0.0;
  for (int s = 0; s < ns; ++s)
    p += P.rs[s] * m.R(s) * (m.kind[s] == KIND_ELECTRON ? P.Tv : P.T);
  P.p = p;
  return true;
}

// primitives -> conservative (inverse of recover)
template <class S>
void prim_to_cons(const Mech &m, const S *rs, S u, S v, S T, S Tv, S *q) {
  const int ns = m.ns;
  if (!m.two_temp) Tv = T;
  S rho = 0.0, rEi = 0.0, rEve = 0.0;
  for (int s = 0; s < ns; ++s) {
    q[s] = rs[s];
    rho += rs[s];
    rEi += rs[s] * e_s<S>(m, s, T, Tv);
    rEve += rs[s] * e_ve<S>(m, s, Tv);
  }
  q[ns] = rho * u;
  q[ns + 1] = rho * v;
  q[ns + 2] = rEi + 0.5 * rho * (u * u + v * v);
  if (m.two_temp) q[ns + 3] = rEve;
}

// ---------------------------------------------------------------- kinetics
// Mass-action rates (paper Eq. (flux): the source vector S holds omega_s and
// omega_v).  Forward k_f = A Tf^b exp(-theta/Tf) with the controlling
// temperature Tf = T, sqrt(T Tv) or Tv; backward k_b = k_f(T)/Kc(T) with Kc
// from the Gibbs energies above (so omega vanishes at equilibrium).
template <class S>
void production(const Mech &m, const S *rs, const S &T, const S &Tv, S *omega) {
  const int ns = m.ns;
  S X[MAXS];
  for (int s = 0; s < ns; ++s) { X[s] = rs[s] / m.M[s]; omega[s] = 0.0; }
  S lnT = std::log(T);
  S g[MAXS];
  for (int s = 0; s < ns; ++s) g[s] = gibbs_RT<S>(m, s, T);
  S ln_c0 = std::log(P_STD / (Ru * T));
  for (int r = 0; r < m.nr; ++r) {
    if (m.A[r] <= 0.0) continue;
    S Tf = T;
    if (m.two_temp) {
      if (m.tctl[r] == 1) Tf = std::sqrt(T * Tv);
      else if (m.tctl[r] == 2) Tf = Tv;
    }
    S kf = m.A[r] * std::exp(m.b[r] * std::log(Tf) - m.theta[r] / Tf);
    S lnKc = 0.0;
    int dnu = 0;
    for (int s = 0; s < ns; ++s) {
      int nu = m.nu_b[r * ns + s] - m.nu_f[r * ns + s];
      lnKc -= double(nu) * g[s];
      dnu += nu;
    }
    lnKc += double(dnu) * ln_c0;
    S kb = std::exp(std::log(m.A[r]) + m.b[r] * lnT - m.theta[r] / T - lnKc);
    S Pf = 1.0, Pb = 1.0;
    for (int s = 0; s < ns; ++s) {
      for (int k = 0; k < m.nu_f[r * ns + s]; ++k) Pf *= X[s];
      for (int k = 0; k < m.nu_b[r * ns + s]; ++k) Pb *= X[s];
    }
    S Mc = 1.0;
    if (m.third[r]) {
      Mc = 0.0;
      for (int s = 0; s < ns; ++s) Mc += m.eff[r * ns + s] * X[s];
    }
    S qr = Mc * (kf * Pf - kb * Pb);
    for (int s = 0; s < ns; ++s) {
      int nu = m.nu_b[r * ns + s] - m.nu_f[r * ns + s];
      if (nu) omega[s] += m.M[s] * double(nu) * qr;
    }
  }
}

// Vibrational-electronic energy source: Landau-Teller relaxation with a
// Millikan-White-form relaxation time per molecule, plus the energy carried
// by species created or destroyed at Tv (non-preferential).
template <class S>
S omega_ve(const Mech &m, const S *rs, const S &T, const S &Tv, const S &p, const S *omega) {
  S w = 0.0;
  S p_atm = p / ATM;
  S Tm13 = std::exp(-std::log(T) / 3.0);
  for (int s = 0; s < m.ns; ++s) {
    if (m.kind[s] == KIND_MOLECULE && m.theta_v[s] > 0.0) {
      S tau = std::exp(m.lt_a[s] * (Tm13 - m.lt_b[s]) - 18.42) / p_atm;
      w += rs[s] * (e_vib(m.R(s), m.theta_v[s], T) - e_vib(m.R(s), m.theta_v[s], Tv)) / tau;
    }
    w += omega[s] * e_ve<S>(m, s, Tv);
  }
  return w;
}

// ---------------------------------------------------------------- transport
template <class S> S viscosity(const Mech &m, const S &T) {
  return m.mu_ref * std::exp(m.mu_exp * std::log(T / m.T_ref));
}
inline double eucken(const Mech &m, int s) {
  switch (m.kind[s]) {
    case KIND_ATOM: return 3.75 * m.R(s);
    case KIND_MOLECULE: return 4.75 * m.R(s);
    default: return 0.0;
  }
}

}  // namespace orc
