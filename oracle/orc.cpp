// Oracle: TEST INFRASTRUCTURE ONLY (see orc.h).  Plain FP64 CPU reference of
// one pseudo-time iteration of the coupled and the component-split implicit
// solver.  Loops are written in the order the paper states the algorithm;
// derivatives (flux Jacobian-vector products, EOS derivatives, source
// Jacobians) are taken by complex-step differentiation of the plain physical
// functions, so they are exact to rounding and independent of any hand
// derivation.
#include "orc.h"

#include <omp.h>

#include <algorithm>
#include <cstring>
#include <string>
#include <type_traits>
#include <vector>

#include "orc_model.hpp"

using namespace orc;

namespace {

struct CellD {
  double q[MAXV];
  Prim<double> P;
  double c = 0, H = 0, eve = 0;
  double mu = 0, k = 0, kve = 0;
  double rhoD[MAXS], h[MAXS], eves[MAXS];
  double nuF = 0, nuC = 0, nuK = 0;
};

struct Face {
  double F[MAXV];
  double Fv[MAXV] = {};                // viscous part of F (kept for the pins)
  double S = 0, nx = 0, ny = 0;       // length and unit normal (towards increasing index)
  double lam = 0, Uabs = 0;           // |U_f| + c_f and |U_f|
  double lvF = 0, lvC = 0, lvK = 0;   // viscous radii nu_f S_f / V_f (flow, species, coupled)
};

constexpr double CSTEP = 1e-25;     // complex-step size (relative to max(|x|, 1))
constexpr double TV_FLOOR = 50.0;  // lower bound of Tv after an update

}  // namespace

struct orc_ctx {
  std::string err;
  int ni = 0, nj = 0, N = 0, bc_mode = 0;
  double Tw = 300.0;
  std::vector<double> xn, yn, xc, yc, V;
  std::vector<double> fi_nx, fi_ny, fi_S, fj_nx, fj_ny, fj_S;
  bool has_grid = false, has_mech = false, has_fs = false, has_state = false, has_res = false;
  Mech m;
  CellD fs;
  std::vector<double> q;
  std::vector<CellD> cells;  // padded (ni+2)*(nj+2)
  std::vector<Face> fI, fJ;
  std::vector<double> R, dtau, src, dK, dF, dC, JK, JC, Jve, DK, DF, DC, LUK, LUF, LUC;
  std::vector<int> pivK, pivF, pivC;
  std::vector<double> dqs, dq, qw;
  int last_mode = -1;
  // split species block: 0 = d omega / d rho_r at fixed T, Tv; 1 = at fixed
  // momenta and energies (Q_F unchanged), the temperatures following
  int jc_fixed_qf = 0;
  // off-diagonal operator: 0 = linear Jacobian-vector product, 1 = flux
  // difference F(Q_N + x) - F(Q_N) (coupled and flow parts)
  int flux_diff = 0;
  int fd_bad = -1;  // a cell whose neighbour state plus increment was not physical
  // residual scheme: 0 first-order HLLE, 1 MUSCL (minmod) + Roe
  int scheme = 0;
  // dual time stepping: physical time step dt and theta (dt = 0: steady),
  // the time levels Q^n and Q^{n-1}
  double pt_dt = 0.0, pt_theta = 0.0;
  std::vector<double> qn, qnm1;

  int pc(int i, int j) const { return (j + 1) * (ni + 2) + (i + 1); }
  int ci(int i, int j) const { return j * ni + i; }
  int fii(int I, int j) const { return j * (ni + 1) + I; }
  int fji(int i, int J) const { return J * ni + i; }
  double nodex(int I, int J) const { return xn[J * (ni + 1) + I]; }
  double nodey(int I, int J) const { return yn[J * (ni + 1) + I]; }
  int fail(int code, const std::string &msg) { err = msg; return code; }
};

namespace {

// ----------------------------------------------------------- cell state
// physical flux F(q).n (paper Eq. (flux), inviscid part, 2D: w = 0)
template <class S>
void phys_flux(const Mech &m, const S *q, const Prim<S> &P, double nx, double ny, S *F) {
  const int ns = m.ns;
  S un = P.u * nx + P.v * ny;
  for (int s = 0; s < ns; ++s) F[s] = q[s] * un;
  F[ns] = q[ns] * un + P.p * nx;
  F[ns + 1] = q[ns + 1] * un + P.p * ny;
  F[ns + 2] = (q[ns + 2] + P.p) * un;
  if (m.two_temp) F[ns + 3] = q[ns + 3] * un;
}

// frozen sound speed from the EOS derivatives p_q (complex step):
// c^2 = sum_s Y_s p_rho_s + u p_mx + v p_my + H p_rhoE + e_ve p_rhoeve.
double sound_speed(const Mech &m, const double *q, const Prim<double> &P, double H, double eve) {
  const int nv = m.nv(), ns = m.ns;
  double pq[MAXV];
  for (int j = 0; j < nv; ++j) {
    cplx qc[MAXV];
    for (int k = 0; k < nv; ++k) qc[k] = q[k];
    double h = CSTEP * std::max(std::fabs(q[j]), 1.0);
    qc[j] += cplx(0.0, h);
    Prim<cplx> Pc;
    recover<cplx>(m, qc, Pc);
    pq[j] = Pc.p.imag() / h;
  }
  double c2 = 0.0;
  for (int s = 0; s < ns; ++s) c2 += P.Y[s] * pq[s];
  c2 += P.u * pq[ns] + P.v * pq[ns + 1] + H * pq[ns + 2];
  if (m.two_temp) c2 += eve * pq[ns + 3];
  return std::sqrt(c2);
}

bool make_cell(const Mech &m, const double *q, CellD &C) {
  const int nv = m.nv(), ns = m.ns;
  for (int k = 0; k < nv; ++k) C.q[k] = q[k];
  if (!recover<double>(m, q, C.P)) return false;
  const Prim<double> &P = C.P;
  if (!(P.T > 0.0) || !(P.Tv > 0.0) || !(P.p > 0.0)) return false;
  C.H = (q[ns + 2] + P.p) / P.rho;
  C.eve = m.two_temp ? q[ns + 3] / P.rho : 0.0;
  C.c = sound_speed(m, q, P, C.H, C.eve);
  if (!(C.c > 0.0)) return false;
  C.mu = viscosity<double>(m, P.T);
  double ktr = 0.0, kint = 0.0, cvtr = 0.0, cvint = 0.0;
  for (int s = 0; s < ns; ++s) {
    ktr += P.Y[s] * eucken(m, s);
    double cve = cv_ve<double>(m, s, m.two_temp ? P.Tv : P.T);
    kint += P.Y[s] * cve;
    cvtr += P.Y[s] * cv_tr(m, s);
    cvint += P.Y[s] * cve;
  }
  if (m.two_temp) {
    C.k = C.mu * ktr;
    C.kve = C.mu * kint;
    C.nuF = std::max(4.0 * C.mu / (3.0 * P.rho), C.k / (P.rho * cvtr));
  } else {
    C.k = C.mu * (ktr + kint);
    C.kve = 0.0;
    C.nuF = std::max(4.0 * C.mu / (3.0 * P.rho), C.k / (P.rho * (cvtr + cvint)));
  }
  C.nuC = 0.0;
  for (int s = 0; s < ns; ++s) {
    C.rhoD[s] = C.mu / m.sc[s];
    C.nuC = std::max(C.nuC, C.rhoD[s] / P.rho);
    C.h[s] = h_s<double>(m, s, P.T, P.Tv);
    C.eves[s] = e_ve<double>(m, s, P.Tv);
  }
  C.nuK = std::max(C.nuF, C.nuC);
  return true;
}

// mirror ghost about a wall with unit normal n: same scalars, velocity reflected
CellD mirror(const Mech &m, const CellD &P, double nx, double ny) {
  CellD G = P;
  const int ns = m.ns;
  double un = P.P.u * nx + P.P.v * ny;
  G.P.u = P.P.u - 2.0 * un * nx;
  G.P.v = P.P.v - 2.0 * un * ny;
  double mn = P.q[ns] * nx + P.q[ns + 1] * ny;
  G.q[ns] = P.q[ns] - 2.0 * mn * nx;
  G.q[ns + 1] = P.q[ns + 1] - 2.0 * mn * ny;
  return G;
}

// HLLE flux with Davis wave-speed bounds for the mixture equations (total
// mass, momentum, total energy).  The species and vibrational-energy fluxes
// are the HLLE mixture mass flux times the upwind mass fraction / specific
// e_ve (Larrouturou's positivity-preserving construction), so that their
// flux Jacobian has the convective eigenvalue U of the paper's component
// operator.
void hlle(const Mech &m, const CellD &L, const CellD &R, double nx, double ny, double *F) {
  const int ns = m.ns;
  double FL[MAXV], FR[MAXV];
  phys_flux<double>(m, L.q, L.P, nx, ny, FL);
  phys_flux<double>(m, R.q, R.P, nx, ny, FR);
  double unL = L.P.u * nx + L.P.v * ny, unR = R.P.u * nx + R.P.v * ny;
  double SL = std::min(unL - L.c, unR - R.c), SR = std::max(unL + L.c, unR + R.c);
  double sl = std::min(SL, 0.0), sr = std::max(SR, 0.0);
  auto hll = [&](double fl, double fr, double ql, double qr) {
    return (sr * fl - sl * fr + sr * sl * (qr - ql)) / (sr - sl);
  };
  double fmass = hll(L.P.rho * unL, R.P.rho * unR, L.P.rho, R.P.rho);
  const CellD &U = fmass >= 0.0 ? L : R;
  for (int s = 0; s < ns; ++s) F[s] = fmass * U.P.Y[s];
  for (int k = ns; k < ns + 3; ++k) F[k] = hll(FL[k], FR[k], L.q[k], R.q[k]);
  if (m.two_temp) F[ns + 3] = fmass * U.eve;
}

// ------------------------------------------- MUSCL + Roe (residual ablation)
// The second-order residual of the paper's cylinder case (Section 3.2: MUSCL
// reconstruction with the minmod limiter and Roe's approximate Riemann
// solver).  Reconstructed: w = (rho_s, u, v, T, Tv) per cell; at interior
// faces w_face = w_B + 1/2 minmod(w_B - w_A, w_C - w_B) on the side of cell B
// (A beyond B, C across the face); boundary faces first order.  Roe flux for
// the mixture (frozen composition) with the species and e_ve carried by the
// mixture mass flux at the upwind mass fraction / e_ve, as in the HLLE flux.
double minmod(double a, double b) {
  if (!(a * b > 0.0)) return 0.0;
  return std::fabs(a) < std::fabs(b) ? a : b;
}

// dp/d(rho E) at fixed other stored variables (complex step)
double eos_beta(const Mech &m, const double *q) {
  const int nv = m.nv(), ns = m.ns;
  cplx qc[MAXV];
  for (int k = 0; k < nv; ++k) qc[k] = q[k];
  const double h = CSTEP * std::max(std::fabs(q[ns + 2]), 1.0);
  qc[ns + 2] += cplx(0.0, h);
  Prim<cplx> Pc;
  recover<cplx>(m, qc, Pc);
  return Pc.p.imag() / h;
}

bool muscl_state(const Mech &m, const CellD &A, const CellD &B, const CellD &C, CellD &out) {
  const int ns = m.ns;
  auto rec = [&](double a, double b, double cc) { return b + 0.5 * minmod(b - a, cc - b); };
  double rs[MAXS], q[MAXV];
  for (int s = 0; s < ns; ++s) rs[s] = rec(A.P.rs[s], B.P.rs[s], C.P.rs[s]);
  const double u = rec(A.P.u, B.P.u, C.P.u), v = rec(A.P.v, B.P.v, C.P.v);
  const double T = rec(A.P.T, B.P.T, C.P.T);
  const double Tv = m.two_temp ? rec(A.P.Tv, B.P.Tv, C.P.Tv) : T;
  prim_to_cons<double>(m, rs, u, v, T, Tv, q);
  return make_cell(m, q, out);
}

// Roe average with weights w = sqrt(rho_L) / (sqrt(rho_L) + sqrt(rho_R)):
// u, v, H, beta = dp/d(rho E) averaged; the sound speed from
// c^2 = w c_L^2 + (1 - w) c_R^2 + beta w (1 - w) |V_R - V_L|^2 / 2, which is
// Roe's average (gamma - 1)(H - |V|^2/2 - h_f) for a calorically perfect gas
// of fixed composition.  The waves moving at u.n (entropy, composition and
// vibrational energy jumps of a real-gas mixture lumped into one) carry the
// part of the rho E jump the acoustic and shear waves leave: a2 e2 =
// d(rho E) - H dp / c^2 - rho V.dV, so the wave decomposition reproduces the
// jump of every mixture variable and, with the sqrt(rho) averages, the flux
// jump too (Roe's property, for any equation of state); for a calorically
// perfect gas of fixed composition e2 = H - c^2 / beta, Roe's own value.
// Harten's entropy fix (delta = c / 10) on the acoustic waves.  eta: a floor
// on every wave speed (the H-correction below; 0 for none).
void roe(const Mech &m, const CellD &L, const CellD &R, double nx, double ny, double eta, double *F) {
  const int ns = m.ns;
  double FL[MAXV], FR[MAXV];
  phys_flux<double>(m, L.q, L.P, nx, ny, FL);
  phys_flux<double>(m, R.q, R.P, nx, ny, FR);
  const double sL = std::sqrt(L.P.rho), sR = std::sqrt(R.P.rho), w = sL / (sL + sR), wr = 1.0 - w;
  const double u = w * L.P.u + wr * R.P.u, v = w * L.P.v + wr * R.P.v, H = w * L.H + wr * R.H;
  const double beta = w * eos_beta(m, L.q) + wr * eos_beta(m, R.q);
  const double dVx = R.P.u - L.P.u, dVy = R.P.v - L.P.v;
  const double cL2 = L.c * L.c, cR2 = R.c * R.c;
  double c2 = w * cL2 + wr * cR2 + 0.5 * beta * w * wr * (dVx * dVx + dVy * dVy);
  c2 = std::max(c2, 1e-6 * std::min(cL2, cR2));
  const double c = std::sqrt(c2), rho = sL * sR;
  const double un = u * nx + v * ny, ut = -u * ny + v * nx;
  const double unL = L.P.u * nx + L.P.v * ny, unR = R.P.u * nx + R.P.v * ny;
  const double utL = -L.P.u * ny + L.P.v * nx, utR = -R.P.u * ny + R.P.v * nx;
  const double dp = R.P.p - L.P.p, dun = unR - unL, dut = utR - utL, drho = R.P.rho - L.P.rho;
  const double a1 = (dp - rho * c * dun) / (2.0 * c2), a3 = (dp + rho * c * dun) / (2.0 * c2);
  const double a2 = drho - dp / c2, at = rho * dut;
  const double delta = 0.1 * c;
  auto fix = [&](double l) {
    const double a = std::fabs(l);
    return a < delta ? (l * l + delta * delta) / (2.0 * delta) : a;
  };
  const double l1 = std::max(fix(un - c), eta), l2 = std::max(std::fabs(un), eta), l3 = std::max(fix(un + c), eta);
  const double a2e2 = (R.q[ns + 2] - L.q[ns + 2]) - H * dp / c2 - rho * (u * dVx + v * dVy);
  const double D0 = l1 * a1 + l2 * a2 + l3 * a3;
  const double Dx = l1 * a1 * (u - c * nx) + l2 * (a2 * u - at * ny) + l3 * a3 * (u + c * nx);
  const double Dy = l1 * a1 * (v - c * ny) + l2 * (a2 * v + at * nx) + l3 * a3 * (v + c * ny);
  const double DE = l1 * a1 * (H - un * c) + l2 * (a2e2 + at * ut) + l3 * a3 * (H + un * c);
  const double mL = L.P.rho * unL, mR = R.P.rho * unR;
  const double fmass = 0.5 * (mL + mR) - 0.5 * D0;
  const CellD &Up = fmass >= 0.0 ? L : R;
  for (int s = 0; s < ns; ++s) F[s] = fmass * Up.P.Y[s];
  F[ns] = 0.5 * (FL[ns] + FR[ns]) - 0.5 * Dx;
  F[ns + 1] = 0.5 * (FL[ns + 1] + FR[ns + 1]) - 0.5 * Dy;
  F[ns + 2] = 0.5 * (FL[ns + 2] + FR[ns + 2]) - 0.5 * DE;
  if (m.two_temp) F[ns + 3] = fmass * Up.eve;
}

// The H-correction of Sanders, Morano and Druguet against the carbuncle of
// Roe's flux at a shock aligned with the grid: eta of a face is half the
// largest jump of a characteristic speed across it, (|un_R - un_L| +
// |c_R - c_L|) / 2 from the two cells' states, and a face's wave speeds are
// floored by the largest eta among itself and the four faces of the other
// family that share an edge with it.
double eta_face(const CellD &L, const CellD &R, double nx, double ny) {
  const double unL = L.P.u * nx + L.P.v * ny, unR = R.P.u * nx + R.P.v * ny;
  return 0.5 * (std::fabs(unR - unL) + std::fabs(R.c - L.c));
}

struct FaceVals {
  double u, v, Y[MAXS], mu, k, kve, rhoD[MAXS], h[MAXS], eve[MAXS];
};
struct Grad {
  double gu[2], gv[2], gT[2], gTv[2], gY[MAXS][2];
};

// viscous flux F_vis.n (paper Eq. (flux) and the constitutive laws of
// Section 2.1) with the diffusion fluxes corrected to sum to zero.
void viscous_flux(const Mech &m, const FaceVals &f, const Grad &g, double nx, double ny, double *F,
                  double *qcond_n) {
  const int ns = m.ns;
  double div = g.gu[0] + g.gv[1];
  double txx = f.mu * (2.0 * g.gu[0] - 2.0 / 3.0 * div);
  double tyy = f.mu * (2.0 * g.gv[1] - 2.0 / 3.0 * div);
  double txy = f.mu * (g.gu[1] + g.gv[0]);
  double Jc[2] = {0.0, 0.0};
  for (int s = 0; s < ns; ++s) { Jc[0] += f.rhoD[s] * g.gY[s][0]; Jc[1] += f.rhoD[s] * g.gY[s][1]; }
  double Jn[MAXS];
  for (int s = 0; s < ns; ++s) {
    double jx = -f.rhoD[s] * g.gY[s][0] + f.Y[s] * Jc[0];
    double jy = -f.rhoD[s] * g.gY[s][1] + f.Y[s] * Jc[1];
    Jn[s] = jx * nx + jy * ny;
  }
  double tnx = txx * nx + txy * ny, tny = txy * nx + tyy * ny;
  double qtr_n = -f.k * (g.gT[0] * nx + g.gT[1] * ny);
  double qve_n = -f.kve * (g.gTv[0] * nx + g.gTv[1] * ny);
  for (int s = 0; s < ns; ++s) F[s] = Jn[s];
  F[ns] = -tnx;
  F[ns + 1] = -tny;
  double hJ = 0.0, eJ = 0.0;
  for (int s = 0; s < ns; ++s) { hJ += f.h[s] * Jn[s]; eJ += f.eve[s] * Jn[s]; }
  F[ns + 2] = -(f.u * tnx + f.v * tny) + qtr_n + qve_n + hJ;
  if (m.two_temp) F[ns + 3] = qve_n + eJ;
  if (qcond_n) *qcond_n = qtr_n + qve_n;
}

// gradient at a face from the two diagonals of the diamond (L, A, R, B):
// d1.g = phi_R - phi_L, d2.g = phi_B - phi_A (exact for linear fields)
inline void diamond(double d1x, double d1y, double d2x, double d2y, double D1, double D2, double *g) {
  double det = d1x * d2y - d1y * d2x;
  g[0] = (D1 * d2y - D2 * d1y) / det;
  g[1] = (D2 * d1x - D1 * d2x) / det;
}

// LU factorisation with partial pivoting (largest |a|, lowest row on ties)
bool lu_factor(int n, double *a, int *piv) {
  for (int k = 0; k < n; ++k) {
    int p = k;
    double best = std::fabs(a[k * n + k]);
    for (int r = k + 1; r < n; ++r)
      if (std::fabs(a[r * n + k]) > best) { best = std::fabs(a[r * n + k]); p = r; }
    piv[k] = p;
    if (best == 0.0) return false;
    if (p != k)
      for (int c = 0; c < n; ++c) std::swap(a[k * n + c], a[p * n + c]);
    for (int r = k + 1; r < n; ++r) {
      double l = a[r * n + k] / a[k * n + k];
      a[r * n + k] = l;
      for (int c = k + 1; c < n; ++c) a[r * n + c] -= l * a[k * n + c];
    }
  }
  return true;
}
void lu_solve(int n, const double *a, const int *piv, double *x) {
  for (int k = 0; k < n; ++k)
    if (piv[k] != k) std::swap(x[k], x[piv[k]]);
  for (int r = 1; r < n; ++r)
    for (int c = 0; c < r; ++c) x[r] -= a[r * n + c] * x[c];
  for (int r = n - 1; r >= 0; --r) {
    for (int c = r + 1; c < n; ++c) x[r] -= a[r * n + c] * x[c];
    x[r] /= a[r * n + r];
  }
}

// coupled unknowns z <-> stored q (paper Section 2.1: the last species
// density follows from rho - sum of the others)
template <class S> void z_to_q(const Mech &m, const S *z, S *q) {
  const int ns = m.ns, nf = m.nf();
  S last = z[0];
  for (int s = 0; s < ns - 1; ++s) { q[s] = z[nf + s]; last -= z[nf + s]; }
  q[ns - 1] = last;
  q[ns] = z[1];
  q[ns + 1] = z[2];
  q[ns + 2] = z[3];
  if (m.two_temp) q[ns + 3] = z[4];
}
template <class S> void q_to_z(const Mech &m, const S *q, S *z) {
  const int ns = m.ns, nf = m.nf();
  S rho = 0.0;
  for (int s = 0; s < ns; ++s) rho += q[s];
  z[0] = rho;
  z[1] = q[ns];
  z[2] = q[ns + 1];
  z[3] = q[ns + 2];
  if (m.two_temp) z[4] = q[ns + 3];
  for (int s = 0; s < ns - 1; ++s) z[nf + s] = q[s];
}
// a stored-variable vector (flux or residual) expressed in z rows
template <class S> void vec_q_to_z(const Mech &m, const S *v, S *z) { q_to_z<S>(m, v, z); }

// source vector S(q) = (omega_1..omega_ns, 0, 0, 0, [omega_ve])
template <class S> bool source(const Mech &m, const S *q, S *src) {
  Prim<S> P;
  if (!recover<S>(m, q, P)) return false;
  const int ns = m.ns;
  S om[MAXS];
  production<S>(m, P.rs, P.T, P.Tv, om);
  for (int s = 0; s < ns; ++s) src[s] = om[s];
  src[ns] = 0.0;
  src[ns + 1] = 0.0;
  src[ns + 2] = 0.0;
  if (m.two_temp) src[ns + 3] = omega_ve<S>(m, P.rs, P.T, P.Tv, P.p, om);
  return true;
}

inline double step_for(const double *x, int n) {
  double mx = 0.0;
  for (int k = 0; k < n; ++k) mx = std::max(mx, std::fabs(x[k]));
  return mx;
}

// coupled Jacobian-vector product A_N(n) x in z variables, by complex step
void jvp_coupled(const Mech &m, const CellD &C, double nx, double ny, const double *x, double *out) {
  const int nb = m.nb(), nv = m.nv();
  double xm = step_for(x, nb);
  if (xm == 0.0) { for (int k = 0; k < nb; ++k) out[k] = 0.0; return; }
  double h = CSTEP / xm;
  double z[MAXV];
  q_to_z<double>(m, C.q, z);
  cplx zc[MAXV], qc[MAXV], F[MAXV], Fz[MAXV];
  for (int k = 0; k < nb; ++k) zc[k] = cplx(z[k], h * x[k]);
  z_to_q<cplx>(m, zc, qc);
  Prim<cplx> P;
  recover<cplx>(m, qc, P);
  phys_flux<cplx>(m, qc, P, nx, ny, F);
  (void)nv;
  vec_q_to_z<cplx>(m, F, Fz);
  for (int k = 0; k < nb; ++k) out[k] = Fz[k].imag() / h;
}

// flow-part Jacobian-vector product at frozen mass fractions, by complex step
void jvp_flow(const Mech &m, const CellD &C, double nx, double ny, const double *x, double *out) {
  const int nf = m.nf(), ns = m.ns;
  double xm = step_for(x, nf);
  if (xm == 0.0) { for (int k = 0; k < nf; ++k) out[k] = 0.0; return; }
  double h = CSTEP / xm;
  cplx rho(C.P.rho, h * x[0]);
  cplx qc[MAXV], F[MAXV];
  for (int s = 0; s < ns; ++s) qc[s] = C.P.Y[s] * rho;
  qc[ns] = cplx(C.q[ns], h * x[1]);
  qc[ns + 1] = cplx(C.q[ns + 1], h * x[2]);
  qc[ns + 2] = cplx(C.q[ns + 2], h * x[3]);
  if (m.two_temp) qc[ns + 3] = cplx(C.q[ns + 3], h * x[4]);
  Prim<cplx> P;
  recover<cplx>(m, qc, P);
  phys_flux<cplx>(m, qc, P, nx, ny, F);
  cplx mass = 0.0;
  for (int s = 0; s < ns; ++s) mass += F[s];
  out[0] = mass.imag() / h;
  out[1] = F[ns].imag() / h;
  out[2] = F[ns + 1].imag() / h;
  out[3] = F[ns + 2].imag() / h;
  if (m.two_temp) out[4] = F[ns + 3].imag() / h;
}

// flux differences F(Q_N + x).n - F(Q_N).n in the same variables as the
// Jacobian-vector products (the matrix-free alternative of A_N x; false if
// Q_N + x is not a physical state)
bool fdiff_coupled(const Mech &m, const CellD &C, double nx, double ny, const double *x, double *out) {
  const int nb = m.nb();
  double z[MAXV], z1[MAXV], q1[MAXV], F0[MAXV], F1[MAXV], Fz0[MAXV], Fz1[MAXV];
  q_to_z<double>(m, C.q, z);
  for (int k = 0; k < nb; ++k) z1[k] = z[k] + x[k];
  z_to_q<double>(m, z1, q1);
  Prim<double> P1;
  if (!recover<double>(m, q1, P1)) return false;
  phys_flux<double>(m, C.q, C.P, nx, ny, F0);
  phys_flux<double>(m, q1, P1, nx, ny, F1);
  vec_q_to_z<double>(m, F0, Fz0);
  vec_q_to_z<double>(m, F1, Fz1);
  for (int k = 0; k < nb; ++k) out[k] = Fz1[k] - Fz0[k];
  return true;
}

bool fdiff_flow(const Mech &m, const CellD &C, double nx, double ny, const double *x, double *out) {
  const int nf = m.nf(), ns = m.ns;
  double q1[MAXV], F0[MAXV], F1[MAXV];
  const double rho1 = C.P.rho + x[0];
  for (int s = 0; s < ns; ++s) q1[s] = C.P.Y[s] * rho1;
  for (int k = 1; k < nf; ++k) q1[ns + k - 1] = C.q[ns + k - 1] + x[k];
  Prim<double> P1;
  if (!recover<double>(m, q1, P1)) return false;
  phys_flux<double>(m, C.q, C.P, nx, ny, F0);
  phys_flux<double>(m, q1, P1, nx, ny, F1);
  double m0 = 0.0, m1 = 0.0;
  for (int s = 0; s < ns; ++s) { m0 += F0[s]; m1 += F1[s]; }
  out[0] = m1 - m0;
  for (int k = 1; k < nf; ++k) out[k] = F1[ns + k - 1] - F0[ns + k - 1];
  return true;
}

}  // namespace

// ================================================================== API
extern "C" {

int orc_create(orc_ctx **ctx) {
  if (!ctx) return -1;
  *ctx = new orc_ctx();
  return 0;
}
void orc_destroy(orc_ctx *ctx) { delete ctx; }
const char *orc_last_error(const orc_ctx *ctx) { return ctx ? ctx->err.c_str() : "null ctx"; }
int orc_set_threads(orc_ctx *, int n) {
  if (n > 0) omp_set_num_threads(n);
  return 0;
}

int orc_set_option(orc_ctx *c, const char *name, double value) {
  if (!c || !name) return -1;
  const std::string n(name);
  if (n == "jc_fixed_qf") {
    c->jc_fixed_qf = int(value);
    return 0;
  }
  if (n == "flux_diff") {
    c->flux_diff = value != 0.0;
    return 0;
  }
  if (n == "residual_scheme") {
    if (value != 0.0 && value != 1.0) return c->fail(-1, "residual_scheme must be 0 or 1");
    c->scheme = int(value);
    c->has_res = false;
    return 0;
  }
  return c->fail(-1, "unknown option " + n);
}

int orc_set_grid(orc_ctx *c, int ni, int nj, const double *xn, const double *yn, double T_wall,
                 int bc_mode) {
  if (!c || ni < 1 || nj < 1 || !xn || !yn) return -1;
  c->ni = ni; c->nj = nj; c->N = ni * nj; c->Tw = T_wall; c->bc_mode = bc_mode;
  size_t nn = size_t(ni + 1) * (nj + 1);
  c->xn.assign(xn, xn + nn);
  c->yn.assign(yn, yn + nn);
  c->xc.assign(c->N, 0.0); c->yc.assign(c->N, 0.0); c->V.assign(c->N, 0.0);
  double sgn = 0.0;
  for (int j = 0; j < nj; ++j)
    for (int i = 0; i < ni; ++i) {
      double x0 = c->nodex(i, j), y0 = c->nodey(i, j), x1 = c->nodex(i + 1, j), y1 = c->nodey(i + 1, j);
      double x2 = c->nodex(i + 1, j + 1), y2 = c->nodey(i + 1, j + 1), x3 = c->nodex(i, j + 1), y3 = c->nodey(i, j + 1);
      double a = 0.5 * ((x0 * y1 - x1 * y0) + (x1 * y2 - x2 * y1) + (x2 * y3 - x3 * y2) + (x3 * y0 - x0 * y3));
      if (i == 0 && j == 0) sgn = a > 0 ? 1.0 : -1.0;
      if (a * sgn <= 0.0) return c->fail(-1, "grid cell with inconsistent orientation");
      c->V[c->ci(i, j)] = std::fabs(a);
      c->xc[c->ci(i, j)] = 0.25 * (x0 + x1 + x2 + x3);
      c->yc[c->ci(i, j)] = 0.25 * (y0 + y1 + y2 + y3);
    }
  c->fi_nx.assign(size_t(ni + 1) * nj, 0); c->fi_ny = c->fi_nx; c->fi_S = c->fi_nx;
  for (int j = 0; j < nj; ++j)
    for (int I = 0; I <= ni; ++I) {
      double tx = c->nodex(I, j + 1) - c->nodex(I, j), ty = c->nodey(I, j + 1) - c->nodey(I, j);
      double nx = sgn * ty, ny = -sgn * tx, S = std::sqrt(nx * nx + ny * ny);
      c->fi_S[c->fii(I, j)] = S; c->fi_nx[c->fii(I, j)] = nx / S; c->fi_ny[c->fii(I, j)] = ny / S;
    }
  c->fj_nx.assign(size_t(ni) * (nj + 1), 0); c->fj_ny = c->fj_nx; c->fj_S = c->fj_nx;
  for (int J = 0; J <= nj; ++J)
    for (int i = 0; i < ni; ++i) {
      double tx = c->nodex(i + 1, J) - c->nodex(i, J), ty = c->nodey(i + 1, J) - c->nodey(i, J);
      double nx = -sgn * ty, ny = sgn * tx, S = std::sqrt(nx * nx + ny * ny);
      c->fj_S[c->fji(i, J)] = S; c->fj_nx[c->fji(i, J)] = nx / S; c->fj_ny[c->fji(i, J)] = ny / S;
    }
  c->has_grid = true;
  c->has_state = false;
  c->has_res = false;
  return 0;
}

int orc_set_mechanism(orc_ctx *c, const orc_mechanism *mm) {
  if (!c || !mm || mm->ns < 2 || mm->ns > MAXS || mm->nr < 0) return -1;
  Mech &m = c->m;
  int ns = mm->ns, nr = mm->nr;
  m = Mech();
  m.ns = ns; m.nr = nr; m.two_temp = mm->two_temp ? 1 : 0;
  auto cp = [&](const double *p, int n) { return std::vector<double>(p, p + n); };
  m.M = cp(mm->M, ns); m.theta_v = cp(mm->theta_v, ns); m.theta_r = cp(mm->theta_r, ns);
  m.sigma = cp(mm->sigma, ns); m.g_el = cp(mm->g_el, ns); m.h_form = cp(mm->h_form, ns);
  m.sc = cp(mm->sc, ns); m.lt_a = cp(mm->lt_a, ns); m.lt_b = cp(mm->lt_b, ns);
  m.kind.assign(mm->kind, mm->kind + ns);
  if (nr > 0) {
    m.A = cp(mm->A, nr); m.b = cp(mm->b, nr); m.theta = cp(mm->theta, nr);
    m.tctl.assign(mm->tctl, mm->tctl + nr); m.third.assign(mm->third, mm->third + nr);
    m.nu_f.assign(mm->nu_f, mm->nu_f + nr * ns); m.nu_b.assign(mm->nu_b, mm->nu_b + nr * ns);
    m.eff = cp(mm->eff, nr * ns);
  }
  m.mu_ref = mm->mu_ref; m.T_ref = mm->T_ref; m.mu_exp = mm->mu_exp;
  c->has_mech = true;
  // default species-block reading: the temperature following the composition
  // at fixed velocities and internal energy in one temperature, fixed T, Tv in two
  c->jc_fixed_qf = mm->two_temp ? 0 : 2;
  c->has_state = false;
  c->has_fs = false;
  c->has_res = false;
  return 0;
}

int orc_set_freestream(orc_ctx *c, const double *rho_s, double u, double v, double T, double Tv) {
  if (!c || !c->has_mech || !rho_s) return -1;
  double q[MAXV];
  prim_to_cons<double>(c->m, rho_s, u, v, T, Tv, q);
  if (!make_cell(c->m, q, c->fs)) return c->fail(-2, "invalid free stream");
  c->has_fs = true;
  return 0;
}

int orc_prim_to_cons(orc_ctx *c, int n, const double *rho_s, const double *u, const double *v,
                     const double *T, const double *Tv, double *q) {
  if (!c || !c->has_mech) return -1;
  const Mech &m = c->m;
  const int ns = m.ns, nv = m.nv();
  for (int p = 0; p < n; ++p) {
    double rs[MAXS], qq[MAXV];
    for (int s = 0; s < ns; ++s) rs[s] = rho_s[size_t(s) * n + p];
    prim_to_cons<double>(m, rs, u[p], v[p], T[p], Tv ? Tv[p] : T[p], qq);
    for (int k = 0; k < nv; ++k) q[size_t(k) * n + p] = qq[k];
  }
  return 0;
}

int orc_set_state(orc_ctx *c, const double *q) {
  if (!c || !c->has_grid || !c->has_mech || !q) return -1;
  c->q.assign(q, q + size_t(c->m.nv()) * c->N);
  c->qn = c->q;
  c->qnm1 = c->q;
  c->has_state = true;
  c->has_res = false;
  return 0;
}

int orc_set_physical_time(orc_ctx *c, double dt, double theta) {
  if (!c || !(dt >= 0.0) || !(theta >= 0.0)) return -1;
  c->pt_dt = dt;
  c->pt_theta = theta;
  c->has_res = false;
  return 0;
}

int orc_set_time_levels(orc_ctx *c, const double *qn, const double *qnm1) {
  if (!c || !c->has_state || !qn || !qnm1) return -1;
  const size_t n = size_t(c->m.nv()) * c->N;
  c->qn.assign(qn, qn + n);
  c->qnm1.assign(qnm1, qnm1 + n);
  c->has_res = false;
  return 0;
}

int orc_advance_time(orc_ctx *c) {
  if (!c || !c->has_state) return -1;
  c->qnm1 = c->qn;
  c->qn = c->q;
  c->has_res = false;
  return 0;
}
int orc_get_state(orc_ctx *c, double *q) {
  if (!c || !c->has_state) return -1;
  std::copy(c->q.begin(), c->q.end(), q);
  return 0;
}

// ------------------------------------------------------------- residual
int orc_residual(orc_ctx *c, double cfl, double *norms) {
  if (!c || !c->has_state || !c->has_fs) return c ? c->fail(-3, "state/free stream not set") : -1;
  const Mech &m = c->m;
  const int ni = c->ni, nj = c->nj, N = c->N, nv = m.nv(), ns = m.ns, nf = m.nf(), nb = m.nb();
  c->cells.assign(size_t(ni + 2) * (nj + 2), CellD());
  int bad = -1;
  // primitives of the interior cells
#pragma omp parallel for schedule(static)
  for (int p = 0; p < N; ++p) {
    double qq[MAXV];
    for (int k = 0; k < nv; ++k) qq[k] = c->q[size_t(k) * N + p];
    int i = p % ni, j = p / ni;
    if (!make_cell(m, qq, c->cells[c->pc(i, j)])) {
#pragma omp critical
      bad = (bad < 0 || p < bad) ? p : bad;
    }
  }
  if (bad >= 0) return c->fail(-4, "non-physical state at cell " + std::to_string(bad));
  // ghost cells (boundary conditions, explicit)
  for (int i = 0; i < ni; ++i) {
    if (c->bc_mode == 0) {
      int f = c->fji(i, 0);
      c->cells[c->pc(i, -1)] = mirror(m, c->cells[c->pc(i, 0)], c->fj_nx[f], c->fj_ny[f]);
    } else {
      c->cells[c->pc(i, -1)] = c->fs;
    }
    c->cells[c->pc(i, nj)] = c->fs;
  }
  for (int j = -1; j <= nj; ++j) {
    if (c->bc_mode == 0) {
      c->cells[c->pc(-1, j)] = c->cells[c->pc(0, j)];
      c->cells[c->pc(ni, j)] = c->cells[c->pc(ni - 1, j)];
    } else {
      c->cells[c->pc(-1, j)] = c->fs;
      c->cells[c->pc(ni, j)] = c->fs;
    }
  }
  auto cell = [&](int i, int j) -> const CellD & { return c->cells[c->pc(i, j)]; };
  // the H-correction's eta of every face (MUSCL + Roe only)
  std::vector<double> etaI, etaJ;
  if (c->scheme == 1) {
    etaI.assign(size_t(ni + 1) * nj, 0.0);
    etaJ.assign(size_t(ni) * (nj + 1), 0.0);
    for (int j = 0; j < nj; ++j)
      for (int I = 0; I <= ni; ++I)
        etaI[c->fii(I, j)] = eta_face(cell(I - 1, j), cell(I, j), c->fi_nx[c->fii(I, j)], c->fi_ny[c->fii(I, j)]);
    for (int J = 0; J <= nj; ++J)
      for (int i = 0; i < ni; ++i)
        etaJ[c->fji(i, J)] = eta_face(cell(i, J - 1), cell(i, J), c->fj_nx[c->fji(i, J)], c->fj_ny[c->fji(i, J)]);
  }
  auto eta_i = [&](int I, int j) {
    double e = etaI[c->fii(I, j)];
    for (int i = I - 1; i <= I; ++i)
      if (i >= 0 && i < ni) e = std::max(e, std::max(etaJ[c->fji(i, j)], etaJ[c->fji(i, j + 1)]));
    return e;
  };
  auto eta_j = [&](int i, int J) {
    double e = etaJ[c->fji(i, J)];
    for (int j = J - 1; j <= J; ++j)
      if (j >= 0 && j < nj) e = std::max(e, std::max(etaI[c->fii(i, j)], etaI[c->fii(i + 1, j)]));
    return e;
  };
  // node values for the diamond gradients: 0 u, 1 v, 2 T, 3 Tv, 4+s Y_s
  auto cellvar = [&](const CellD &C, int var) -> double {
    switch (var) {
      case 0: return C.P.u;
      case 1: return C.P.v;
      case 2: return C.P.T;
      case 3: return C.P.Tv;
      default: return C.P.Y[var - 4];
    }
  };
  auto nodeval = [&](int I, int J, int var) -> double {
    if (c->bc_mode == 0 && J == 0) {
      if (var <= 1) return 0.0;
      if (var <= 3) return c->Tw;
      return 0.5 * (cellvar(cell(I - 1, 0), var) + cellvar(cell(I, 0), var));
    }
    return 0.25 * (cellvar(cell(I - 1, J - 1), var) + cellvar(cell(I, J - 1), var) +
                   cellvar(cell(I - 1, J), var) + cellvar(cell(I, J), var));
  };
  const int nvar = 4 + ns;
  auto interior_viscous = [&](const CellD &L, const CellD &R, double xL, double yL, double xR, double yR,
                              int IA, int JA, int IB, int JB, double nx, double ny, double *Fv) {
    FaceVals fv;
    fv.u = 0.5 * (L.P.u + R.P.u); fv.v = 0.5 * (L.P.v + R.P.v);
    fv.mu = 0.5 * (L.mu + R.mu); fv.k = 0.5 * (L.k + R.k); fv.kve = 0.5 * (L.kve + R.kve);
    for (int s = 0; s < ns; ++s) {
      fv.Y[s] = 0.5 * (L.P.Y[s] + R.P.Y[s]);
      fv.rhoD[s] = 0.5 * (L.rhoD[s] + R.rhoD[s]);
      fv.h[s] = 0.5 * (L.h[s] + R.h[s]);
      fv.eve[s] = 0.5 * (L.eves[s] + R.eves[s]);
    }
    double d1x = xR - xL, d1y = yR - yL;
    double d2x = c->nodex(IB, JB) - c->nodex(IA, JA), d2y = c->nodey(IB, JB) - c->nodey(IA, JA);
    Grad g;
    for (int var = 0; var < nvar; ++var) {
      double D1 = cellvar(R, var) - cellvar(L, var);
      double D2 = nodeval(IB, JB, var) - nodeval(IA, JA, var);
      double *gg = var == 0 ? g.gu : var == 1 ? g.gv : var == 2 ? g.gT : var == 3 ? g.gTv : g.gY[var - 4];
      diamond(d1x, d1y, d2x, d2y, D1, D2, gg);
    }
    viscous_flux(m, fv, g, nx, ny, Fv, nullptr);
  };
  c->fI.assign(size_t(ni + 1) * nj, Face());
  c->fJ.assign(size_t(ni) * (nj + 1), Face());
  c->qw.assign(ni, 0.0);
  auto radii = [&](Face &F, const CellD &L, const CellD &R, double VL, double VR, bool interior,
                   const CellD &Pin, double Vin) {
    double U = 0.5 * ((L.P.u + R.P.u) * F.nx + (L.P.v + R.P.v) * F.ny);
    F.Uabs = std::fabs(U);
    F.lam = F.Uabs + 0.5 * (L.c + R.c);
    double nF, nC, nK, Vf;
    if (interior) {
      nF = 0.5 * (L.nuF + R.nuF); nC = 0.5 * (L.nuC + R.nuC); nK = 0.5 * (L.nuK + R.nuK);
      Vf = 0.5 * (VL + VR);
    } else {
      nF = Pin.nuF; nC = Pin.nuC; nK = Pin.nuK; Vf = Vin;
    }
    F.lvF = nF * F.S / Vf; F.lvC = nC * F.S / Vf; F.lvK = nK * F.S / Vf;
  };
  // i-faces
#pragma omp parallel for schedule(static)
  for (int idx = 0; idx < (ni + 1) * nj; ++idx) {
    int I = idx % (ni + 1), j = idx / (ni + 1);
    Face &F = c->fI[c->fii(I, j)];
    F.S = c->fi_S[c->fii(I, j)]; F.nx = c->fi_nx[c->fii(I, j)]; F.ny = c->fi_ny[c->fii(I, j)];
    const CellD &L = cell(I - 1, j), &R = cell(I, j);
    bool interior = I > 0 && I < ni;
    if (c->scheme == 1) {
      if (interior) {
        CellD Lf, Rf;
        if (!muscl_state(m, cell(I - 2, j), L, R, Lf) || !muscl_state(m, cell(I + 1, j), R, L, Rf)) {
#pragma omp critical
          bad = (bad < 0 || c->ci(I, j) < bad) ? c->ci(I, j) : bad;
          roe(m, L, R, F.nx, F.ny, eta_i(I, j), F.F);
        } else {
          roe(m, Lf, Rf, F.nx, F.ny, eta_i(I, j), F.F);
        }
      } else {
        roe(m, L, R, F.nx, F.ny, eta_i(I, j), F.F);
      }
    } else {
      hlle(m, L, R, F.nx, F.ny, F.F);
    }
    double VL = interior ? c->V[c->ci(I - 1, j)] : 0.0, VR = interior ? c->V[c->ci(I, j)] : 0.0;
    int pin = I == 0 ? c->ci(0, j) : c->ci(ni - 1, j);
    radii(F, L, R, VL, VR, interior, I == 0 ? cell(0, j) : cell(ni - 1, j), c->V[pin]);
    if (interior) {
      double Fv[MAXV];
      interior_viscous(L, R, c->xc[c->ci(I - 1, j)], c->yc[c->ci(I - 1, j)], c->xc[c->ci(I, j)],
                       c->yc[c->ci(I, j)], I, j, I, j + 1, F.nx, F.ny, Fv);
      for (int k = 0; k < nv; ++k) { F.F[k] += Fv[k]; F.Fv[k] = Fv[k]; }
    }
  }
  // j-faces
#pragma omp parallel for schedule(static)
  for (int idx = 0; idx < ni * (nj + 1); ++idx) {
    int i = idx % ni, J = idx / ni;
    Face &F = c->fJ[c->fji(i, J)];
    F.S = c->fj_S[c->fji(i, J)]; F.nx = c->fj_nx[c->fji(i, J)]; F.ny = c->fj_ny[c->fji(i, J)];
    const CellD &L = cell(i, J - 1), &R = cell(i, J);
    bool interior = J > 0 && J < nj;
    if (c->scheme == 1) {
      if (interior) {
        CellD Lf, Rf;
        if (!muscl_state(m, cell(i, J - 2), L, R, Lf) || !muscl_state(m, cell(i, J + 1), R, L, Rf)) {
#pragma omp critical
          bad = (bad < 0 || c->ci(i, J) < bad) ? c->ci(i, J) : bad;
          roe(m, L, R, F.nx, F.ny, eta_j(i, J), F.F);
        } else {
          roe(m, Lf, Rf, F.nx, F.ny, eta_j(i, J), F.F);
        }
      } else {
        roe(m, L, R, F.nx, F.ny, eta_j(i, J), F.F);
      }
    } else {
      hlle(m, L, R, F.nx, F.ny, F.F);
    }
    double VL = interior ? c->V[c->ci(i, J - 1)] : 0.0, VR = interior ? c->V[c->ci(i, J)] : 0.0;
    int pin = J == 0 ? c->ci(i, 0) : c->ci(i, nj - 1);
    radii(F, L, R, VL, VR, interior, J == 0 ? cell(i, 0) : cell(i, nj - 1), c->V[pin]);
    if (interior) {
      double Fv[MAXV];
      interior_viscous(L, R, c->xc[c->ci(i, J - 1)], c->yc[c->ci(i, J - 1)], c->xc[c->ci(i, J)],
                       c->yc[c->ci(i, J)], i, J, i + 1, J, F.nx, F.ny, Fv);
      for (int k = 0; k < nv; ++k) { F.F[k] += Fv[k]; F.Fv[k] = Fv[k]; }
    } else if (J == 0 && c->bc_mode == 0) {
      // isothermal, no-slip, non-catalytic wall: face values at the wall,
      // normal gradient from the wall value and the first cell centre
      const CellD &P = cell(i, 0);
      FaceVals fv;
      fv.u = 0.0; fv.v = 0.0;
      double muw = viscosity<double>(m, c->Tw);
      double ktr = 0.0, kint = 0.0;
      for (int s = 0; s < ns; ++s) {
        fv.Y[s] = P.P.Y[s]; fv.rhoD[s] = 0.0; fv.h[s] = 0.0; fv.eve[s] = 0.0;
        ktr += P.P.Y[s] * eucken(m, s);
        kint += P.P.Y[s] * cv_ve<double>(m, s, c->Tw);
      }
      fv.mu = muw;
      if (m.two_temp) { fv.k = muw * ktr; fv.kve = muw * kint; }
      else { fv.k = muw * (ktr + kint); fv.kve = 0.0; }
      double xf = 0.5 * (c->nodex(i, 0) + c->nodex(i + 1, 0)), yf = 0.5 * (c->nodey(i, 0) + c->nodey(i + 1, 0));
      double d1x = c->xc[c->ci(i, 0)] - xf, d1y = c->yc[c->ci(i, 0)] - yf;
      double d2x = c->nodex(i + 1, 0) - c->nodex(i, 0), d2y = c->nodey(i + 1, 0) - c->nodey(i, 0);
      Grad g;
      diamond(d1x, d1y, d2x, d2y, P.P.u, 0.0, g.gu);
      diamond(d1x, d1y, d2x, d2y, P.P.v, 0.0, g.gv);
      diamond(d1x, d1y, d2x, d2y, P.P.T - c->Tw, 0.0, g.gT);
      diamond(d1x, d1y, d2x, d2y, P.P.Tv - c->Tw, 0.0, g.gTv);
      for (int s = 0; s < ns; ++s) { g.gY[s][0] = 0.0; g.gY[s][1] = 0.0; }
      double Fv[MAXV], qn;
      viscous_flux(m, fv, g, F.nx, F.ny, Fv, &qn);
      for (int k = 0; k < nv; ++k) { F.F[k] += Fv[k]; F.Fv[k] = Fv[k]; }
      c->qw[i] = -qn;
    }
  }
  if (bad >= 0) return c->fail(-4, "non-physical reconstructed face state next to cell " + std::to_string(bad));
  // cell residual, time step, sources, Jacobians, diagonal blocks
  c->R.assign(size_t(nv) * N, 0.0); c->dtau.assign(N, 0.0); c->src.assign(size_t(nv) * N, 0.0);
  c->dK.assign(N, 0.0); c->dF.assign(N, 0.0); c->dC.assign(N, 0.0);
  c->JK.assign(size_t(nb) * nb * N, 0.0); c->JC.assign(size_t(ns) * ns * N, 0.0);
  c->Jve.assign(size_t(nf) * N, 0.0);
  c->DK.assign(size_t(nb) * nb * N, 0.0); c->DF.assign(size_t(nf) * nf * N, 0.0);
  c->DC.assign(size_t(ns) * ns * N, 0.0);
  c->LUK = c->DK; c->LUF = c->DF; c->LUC = c->DC;
  c->pivK.assign(size_t(nb) * N, 0); c->pivF.assign(size_t(nf) * N, 0); c->pivC.assign(size_t(ns) * N, 0);
  int singular = -1;
#pragma omp parallel for schedule(static)
  for (int p = 0; p < N; ++p) {
    int i = p % ni, j = p / ni;
    const CellD &P = cell(i, j);
    const Face &W = c->fI[c->fii(i, j)], &E = c->fI[c->fii(i + 1, j)];
    const Face &Sf = c->fJ[c->fji(i, j)], &Nf = c->fJ[c->fji(i, j + 1)];
    double Vp = c->V[p];
    double sv[MAXV];
    source<double>(m, P.q, sv);
    // physical-time term of dual time stepping (paper Eq. (linearizedimplicit)):
    // V [(1 + theta)(Q^m - Q^n) - theta (Q^n - Q^{n-1})] / dt joins the residual
    const bool unsteady = c->pt_dt > 0.0;
    for (int k = 0; k < nv; ++k) {
      c->src[size_t(k) * N + p] = sv[k];
      double Rk = E.F[k] * E.S - W.F[k] * W.S + Nf.F[k] * Nf.S - Sf.F[k] * Sf.S - Vp * sv[k];
      if (unsteady) {
        const size_t ix = size_t(k) * N + p;
        Rk += Vp * ((1.0 + c->pt_theta) * (c->q[ix] - c->qn[ix]) - c->pt_theta * (c->qn[ix] - c->qnm1[ix])) /
              c->pt_dt;
      }
      c->R[size_t(k) * N + p] = Rk;
    }
    const Face *fs4[4] = {&W, &E, &Sf, &Nf};
    double slam = 0.0, sU = 0.0, svF = 0.0, svC = 0.0, svK = 0.0;
    for (int f = 0; f < 4; ++f) {
      slam += fs4[f]->lam * fs4[f]->S;
      sU += fs4[f]->Uabs * fs4[f]->S;
      svF += fs4[f]->lvF * fs4[f]->S;
      svC += fs4[f]->lvC * fs4[f]->S;
      svK += fs4[f]->lvK * fs4[f]->S;
    }
    double dt = cfl * Vp / (0.5 * (slam + svK));
    c->dtau[p] = dt;
    // diagonal: V / dtau, plus (1 + theta) V / dt with physical time
    const double Vt = Vp / dt + (unsteady ? (1.0 + c->pt_theta) * Vp / c->pt_dt : 0.0);
    c->dK[p] = Vt + 0.5 * slam + svK;
    c->dF[p] = Vt + 0.5 * slam + svF;
    c->dC[p] = Vt + 0.5 * sU + svC;
    // coupled source Jacobian dS/dz (z = rho, momenta, energies, rho_1..rho_{ns-1})
    double z[MAXV];
    q_to_z<double>(m, P.q, z);
    for (int col = 0; col < nb; ++col) {
      cplx zc[MAXV], qc[MAXV], sc[MAXV], sz[MAXV];
      for (int k = 0; k < nb; ++k) zc[k] = z[k];
      double h = CSTEP * std::max(std::fabs(z[col]), 1.0);
      zc[col] += cplx(0.0, h);
      z_to_q<cplx>(m, zc, qc);
      source<cplx>(m, qc, sc);
      vec_q_to_z<cplx>(m, sc, sz);
      for (int r = 0; r < nb; ++r) c->JK[(size_t(r) * nb + col) * N + p] = sz[r].imag() / h;
    }
    // species block: d omega_s / d rho_r at fixed T, Tv, or with the flow
    // variables (momenta, total and vibrational energy) held fixed
    for (int col = 0; col < ns; ++col) {
      double h = CSTEP * std::max(std::fabs(P.P.rs[col]), 1.0);
      if (c->jc_fixed_qf) {
        cplx qc[MAXV], sc[MAXV];
        for (int k = 0; k < nv; ++k) qc[k] = P.q[k];
        qc[col] += cplx(0.0, h);
        if (c->jc_fixed_qf >= 2) {
          // velocities and the internal energy density held: the added mass
          // carries its momentum and kinetic energy
          qc[ns] += cplx(0.0, h * P.P.u);
          qc[ns + 1] += cplx(0.0, h * P.P.v);
          qc[ns + 2] += cplx(0.0, h * 0.5 * (P.P.u * P.P.u + P.P.v * P.P.v));
        }
        if (c->jc_fixed_qf == 3 && m.two_temp) {
          // and the vibrational temperature held: the vibrational-electronic
          // energy density takes the added mass's e_ve,r(Tv) out of the same
          // internal energy
          qc[ns + 3] += cplx(0.0, h * e_ve<double>(m, col, P.P.Tv));
        }
        source<cplx>(m, qc, sc);
        for (int r = 0; r < ns; ++r) c->JC[(size_t(r) * ns + col) * N + p] = sc[r].imag() / h;
      } else {
        cplx rc[MAXS], om[MAXS];
        for (int s = 0; s < ns; ++s) rc[s] = P.P.rs[s];
        rc[col] += cplx(0.0, h);
        production<cplx>(m, rc, cplx(P.P.T), cplx(P.P.Tv), om);
        for (int r = 0; r < ns; ++r) c->JC[(size_t(r) * ns + col) * N + p] = om[r].imag() / h;
      }
    }
    // flow block source row (two temperatures): d omega_ve / d Q_F at frozen Y
    if (m.two_temp) {
      for (int col = 0; col < nf; ++col) {
        cplx qf[5] = {P.P.rho, P.q[ns], P.q[ns + 1], P.q[ns + 2], P.q[ns + 3]};
        double h = CSTEP * std::max(std::fabs(qf[col].real()), 1.0);
        qf[col] += cplx(0.0, h);
        cplx qc[MAXV], sc[MAXV];
        for (int s = 0; s < ns; ++s) qc[s] = P.P.Y[s] * qf[0];
        qc[ns] = qf[1]; qc[ns + 1] = qf[2]; qc[ns + 2] = qf[3]; qc[ns + 3] = qf[4];
        source<cplx>(m, qc, sc);
        c->Jve[size_t(col) * N + p] = sc[ns + 3].imag() / h;
      }
    }
    // diagonal blocks (paper: I_m = (1/(J dtau)) I - A_S plus the split-radius diagonals)
    bool ok = true;
    {
      thread_local std::vector<double> Abuf;
      Abuf.resize(size_t(nb) * nb);
      double *A = Abuf.data();
      int piv[MAXV];
      for (int r = 0; r < nb; ++r)
        for (int col = 0; col < nb; ++col)
          A[r * nb + col] = (r == col ? c->dK[p] : 0.0) - Vp * c->JK[(size_t(r) * nb + col) * N + p];
      for (int k = 0; k < nb * nb; ++k) c->DK[size_t(k) * N + p] = A[k];
      ok = ok && lu_factor(nb, A, piv);
      for (int k = 0; k < nb * nb; ++k) c->LUK[size_t(k) * N + p] = A[k];
      for (int k = 0; k < nb; ++k) c->pivK[size_t(k) * N + p] = piv[k];
    }
    {
      double A[25];
      int piv[5];
      for (int r = 0; r < nf; ++r)
        for (int col = 0; col < nf; ++col)
          A[r * nf + col] = (r == col ? c->dF[p] : 0.0) -
                            ((m.two_temp && r == nf - 1) ? Vp * c->Jve[size_t(col) * N + p] : 0.0);
      for (int k = 0; k < nf * nf; ++k) c->DF[size_t(k) * N + p] = A[k];
      ok = ok && lu_factor(nf, A, piv);
      for (int k = 0; k < nf * nf; ++k) c->LUF[size_t(k) * N + p] = A[k];
      for (int k = 0; k < nf; ++k) c->pivF[size_t(k) * N + p] = piv[k];
    }
    {
      thread_local std::vector<double> Abuf;
      Abuf.resize(size_t(ns) * ns);
      double *A = Abuf.data();
      int piv[MAXS];
      for (int r = 0; r < ns; ++r)
        for (int col = 0; col < ns; ++col)
          A[r * ns + col] = (r == col ? c->dC[p] : 0.0) - Vp * c->JC[(size_t(r) * ns + col) * N + p];
      for (int k = 0; k < ns * ns; ++k) c->DC[size_t(k) * N + p] = A[k];
      ok = ok && lu_factor(ns, A, piv);
      for (int k = 0; k < ns * ns; ++k) c->LUC[size_t(k) * N + p] = A[k];
      for (int k = 0; k < ns; ++k) c->pivC[size_t(k) * N + p] = piv[k];
    }
    if (!ok) {
#pragma omp critical
      singular = (singular < 0 || p < singular) ? p : singular;
    }
  }
  if (singular >= 0) return c->fail(-5, "singular diagonal block at cell " + std::to_string(singular));
  if (norms) {
    double sr = 0.0, se = 0.0;
    for (int p = 0; p < N; ++p) {
      double rr = 0.0;
      for (int s = 0; s < ns; ++s) rr += c->R[size_t(s) * N + p];
      rr /= c->V[p];
      double re_ = c->R[size_t(ns + 2) * N + p] / c->V[p];
      sr += rr * rr;
      se += re_ * re_;
    }
    norms[0] = std::sqrt(sr);
    norms[1] = std::sqrt(se);
  }
  c->has_res = true;
  return 0;
}

}  // extern "C"

// ---------------------------------------------------------------- sweeps
namespace {

enum Part { P_COUPLED, P_FLOW, P_SPECIES };

// off-diagonal operator O_PN x for the neighbour cell Cn across face F of P,
// with (nx, ny) the outward unit normal of P (paper Section 2.2: spectral
// splitting A+- = (A +- lambda I)/2 and the viscous spectral approximation;
// Section 2.3: flow radius |U|+c, species radius |U| and the scalar species operator)
bool apply_off(const Mech &m, Part part, const Face &F, double nx, double ny, const CellD &Cn,
               const double *x, double *out, bool fdiff) {
  if (part == P_COUPLED) {
    int n = m.nb();
    double a[MAXV];
    if (fdiff) {
      if (!fdiff_coupled(m, Cn, nx, ny, x, a)) return false;
    } else {
      jvp_coupled(m, Cn, nx, ny, x, a);
    }
    for (int k = 0; k < n; ++k) out[k] = 0.5 * F.S * (a[k] - F.lam * x[k]) - F.lvK * F.S * x[k];
  } else if (part == P_FLOW) {
    int n = m.nf();
    double a[MAXV];
    if (fdiff) {
      if (!fdiff_flow(m, Cn, nx, ny, x, a)) return false;
    } else {
      jvp_flow(m, Cn, nx, ny, x, a);
    }
    for (int k = 0; k < n; ++k) out[k] = 0.5 * F.S * (a[k] - F.lam * x[k]) - F.lvF * F.S * x[k];
  } else {
    // species part: the flux difference at unchanged flow variables is
    // exactly (u.n) x, the same as the linear operator
    int n = m.ns;
    double un = Cn.P.u * nx + Cn.P.v * ny;
    double coef = 0.5 * F.S * (un - F.Uabs) - F.lvC * F.S;
    for (int k = 0; k < n; ++k) out[k] = coef * x[k];
  }
  return true;
}

struct PartInfo {
  int n, off;
  const std::vector<double> *LU;
  const std::vector<int> *piv;
};

PartInfo part_info(orc_ctx *c, Part part, int mode) {
  const Mech &m = c->m;
  if (part == P_COUPLED) return {m.nb(), 0, &c->LUK, &c->pivK};
  if (part == P_FLOW) return {m.nf(), 0, &c->LUF, &c->pivF};
  (void)mode;
  return {m.ns, m.nf(), &c->LUC, &c->pivC};
}

void solve_block(orc_ctx *c, const PartInfo &pi, int p, double *x) {
  const int N = c->N, n = pi.n;
  thread_local std::vector<double> Abuf;
  Abuf.resize(size_t(n) * n);
  double *A = Abuf.data();
  int piv[MAXV];
  for (int k = 0; k < n * n; ++k) A[k] = (*pi.LU)[size_t(k) * N + p];
  for (int k = 0; k < n; ++k) piv[k] = (*pi.piv)[size_t(k) * N + p];
  lu_solve(n, A, piv, x);
}

void note_fd_bad(orc_ctx *c, int p) {
#pragma omp critical
  c->fd_bad = (c->fd_bad < 0 || p < c->fd_bad) ? p : c->fd_bad;
}

// forward: (D+L) dQ* = b ; backward: (D+U) dQ = D dQ*  (paper Section 2.2)
void sweep_cell_fwd(orc_ctx *c, Part part, const PartInfo &pi, int i, int j, const std::vector<double> &b,
                    std::vector<double> &xs) {
  const int N = c->N, n = pi.n, off = pi.off;
  const Mech &m = c->m;
  int p = c->ci(i, j);
  double r[MAXV], x[MAXV], o[MAXV];
  for (int k = 0; k < n; ++k) r[k] = b[size_t(off + k) * N + p];
  if (i > 0) {  // west neighbour, face i-face (i, j); outward normal of P is -n
    const Face &F = c->fI[c->fii(i, j)];
    int q = c->ci(i - 1, j);
    for (int k = 0; k < n; ++k) x[k] = xs[size_t(off + k) * N + q];
    if (!apply_off(m, part, F, -F.nx, -F.ny, c->cells[c->pc(i - 1, j)], x, o, c->flux_diff != 0)) note_fd_bad(c, p);
    for (int k = 0; k < n; ++k) r[k] -= o[k];
  }
  if (j > 0) {  // south neighbour
    const Face &F = c->fJ[c->fji(i, j)];
    int q = c->ci(i, j - 1);
    for (int k = 0; k < n; ++k) x[k] = xs[size_t(off + k) * N + q];
    if (!apply_off(m, part, F, -F.nx, -F.ny, c->cells[c->pc(i, j - 1)], x, o, c->flux_diff != 0)) note_fd_bad(c, p);
    for (int k = 0; k < n; ++k) r[k] -= o[k];
  }
  solve_block(c, pi, p, r);
  for (int k = 0; k < n; ++k) xs[size_t(off + k) * N + p] = r[k];
}

void sweep_cell_bwd(orc_ctx *c, Part part, const PartInfo &pi, int i, int j, const std::vector<double> &xs,
                    std::vector<double> &x_out) {
  const int N = c->N, n = pi.n, off = pi.off;
  const Mech &m = c->m;
  int p = c->ci(i, j);
  double r[MAXV], x[MAXV], o[MAXV];
  for (int k = 0; k < n; ++k) r[k] = 0.0;
  if (i < c->ni - 1) {  // east neighbour, face i-face (i+1, j); outward normal +n
    const Face &F = c->fI[c->fii(i + 1, j)];
    int q = c->ci(i + 1, j);
    for (int k = 0; k < n; ++k) x[k] = x_out[size_t(off + k) * N + q];
    if (!apply_off(m, part, F, F.nx, F.ny, c->cells[c->pc(i + 1, j)], x, o, c->flux_diff != 0)) note_fd_bad(c, p);
    for (int k = 0; k < n; ++k) r[k] += o[k];
  }
  if (j < c->nj - 1) {  // north neighbour
    const Face &F = c->fJ[c->fji(i, j + 1)];
    int q = c->ci(i, j + 1);
    for (int k = 0; k < n; ++k) x[k] = x_out[size_t(off + k) * N + q];
    if (!apply_off(m, part, F, F.nx, F.ny, c->cells[c->pc(i, j + 1)], x, o, c->flux_diff != 0)) note_fd_bad(c, p);
    for (int k = 0; k < n; ++k) r[k] += o[k];
  }
  solve_block(c, pi, p, r);
  for (int k = 0; k < n; ++k) x_out[size_t(off + k) * N + p] = xs[size_t(off + k) * N + p] - r[k];
}

void run_sweeps(orc_ctx *c, Part part, int mode, int order, const std::vector<double> &b,
                std::vector<double> &xs, std::vector<double> &x) {
  PartInfo pi = part_info(c, part, mode);
  const int ni = c->ni, nj = c->nj;
  if (order == ORC_LEXICOGRAPHIC) {
    for (int j = 0; j < nj; ++j)
      for (int i = 0; i < ni; ++i) sweep_cell_fwd(c, part, pi, i, j, b, xs);
    for (int j = nj - 1; j >= 0; --j)
      for (int i = ni - 1; i >= 0; --i) sweep_cell_bwd(c, part, pi, i, j, xs, x);
  } else {
    for (int k = 0; k <= ni + nj - 2; ++k) {
      int j0 = std::max(0, k - ni + 1), j1 = std::min(nj - 1, k);
#pragma omp parallel for schedule(static)
      for (int j = j0; j <= j1; ++j) sweep_cell_fwd(c, part, pi, k - j, j, b, xs);
    }
    for (int k = ni + nj - 2; k >= 0; --k) {
      int j0 = std::max(0, k - ni + 1), j1 = std::min(nj - 1, k);
#pragma omp parallel for schedule(static)
      for (int j = j0; j <= j1; ++j) sweep_cell_bwd(c, part, pi, k - j, j, xs, x);
    }
  }
}

int nsol_of(const Mech &m, int mode) { return mode == ORC_COUPLED ? m.nb() : m.nf() + m.ns; }

int sweeps(orc_ctx *c, int mode, int order, const std::vector<double> &b) {
  const int N = c->N, ns_ = nsol_of(c->m, mode);
  c->dqs.assign(size_t(ns_) * N, 0.0);
  c->dq.assign(size_t(ns_) * N, 0.0);
  c->fd_bad = -1;
  if (mode == ORC_COUPLED) {
    run_sweeps(c, P_COUPLED, mode, order, b, c->dqs, c->dq);
  } else {
    // the flow part and the component part are independent (paper Section 2.3)
    run_sweeps(c, P_FLOW, mode, order, b, c->dqs, c->dq);
    run_sweeps(c, P_SPECIES, mode, order, b, c->dqs, c->dq);
  }
  c->last_mode = mode;
  if (c->fd_bad >= 0)
    return c->fail(-4, "flux difference at a non-physical neighbour state (cell " + std::to_string(c->fd_bad) + ")");
  return 0;
}

// the sweeps' right-hand side from the residual: -R in the coupled form's z
// variables, or the flow part (total density, momenta, energies) and the
// species part of the split form
void sweep_rhs_from_residual(orc_ctx *c, int mode, std::vector<double> &b) {
  const Mech &m = c->m;
  const int N = c->N, ns = m.ns, nf = m.nf(), nsol = nsol_of(m, mode);
  b.assign(size_t(nsol) * N, 0.0);
  for (int p = 0; p < N; ++p) {
    double rq[MAXV], rz[MAXV];
    for (int k = 0; k < m.nv(); ++k) rq[k] = c->R[size_t(k) * N + p];
    double sum = 0.0;
    for (int s = 0; s < ns; ++s) sum += rq[s];
    if (mode == ORC_COUPLED) {
      vec_q_to_z<double>(m, rq, rz);
      for (int k = 0; k < nsol; ++k) b[size_t(k) * N + p] = -rz[k];
    } else {
      b[size_t(0) * N + p] = -sum;
      b[size_t(1) * N + p] = -rq[ns];
      b[size_t(2) * N + p] = -rq[ns + 1];
      b[size_t(3) * N + p] = -rq[ns + 2];
      if (m.two_temp) b[size_t(4) * N + p] = -rq[ns + 3];
      for (int s = 0; s < ns; ++s) b[size_t(nf + s) * N + p] = -rq[s];
    }
  }
}

}  // namespace

extern "C" {

int orc_implicit_op(orc_ctx *c, int mode, int order) {
  if (!c || !c->has_res) return c ? c->fail(-3, "residual not computed") : -1;
  std::vector<double> b;
  sweep_rhs_from_residual(c, mode, b);
  return sweeps(c, mode, order, b);
}

int orc_sweep_cell(orc_ctx *c, int mode, int fwd, int i, int j, const double *xs, const double *x, double *out) {
  if (!c || !c->has_res || !xs || !out || (!fwd && !x)) return c ? c->fail(-1, "sweep_cell: arguments") : -1;
  if (i < 0 || i >= c->ni || j < 0 || j >= c->nj) return c->fail(-1, "sweep_cell: cell out of range");
  const int N = c->N, nsol = nsol_of(c->m, mode);
  std::vector<double> b, xsv(xs, xs + size_t(nsol) * N), xv;
  if (fwd) sweep_rhs_from_residual(c, mode, b);
  else xv.assign(x, x + size_t(nsol) * N);
  const Part parts[2] = {mode == ORC_COUPLED ? P_COUPLED : P_FLOW, P_SPECIES};
  c->fd_bad = -1;
  for (int q = 0; q < (mode == ORC_COUPLED ? 1 : 2); ++q) {
    const PartInfo pi = part_info(c, parts[q], mode);
    if (fwd) sweep_cell_fwd(c, parts[q], pi, i, j, b, xsv);
    else sweep_cell_bwd(c, parts[q], pi, i, j, xsv, xv);
  }
  const int p = c->ci(i, j);
  const std::vector<double> &res = fwd ? xsv : xv;
  for (int k = 0; k < nsol; ++k) out[k] = res[size_t(k) * N + p];
  return c->fd_bad >= 0 ? c->fail(-4, "flux difference at a non-physical neighbour state") : 0;
}

int orc_sweep_rhs(orc_ctx *c, int mode, int order, const double *b, double *x) {
  if (!c || !c->has_res) return -1;
  const int nsol = nsol_of(c->m, mode);
  std::vector<double> bb(b, b + size_t(nsol) * c->N);
  int rc = sweeps(c, mode, order, bb);
  if (rc) return rc;
  std::copy(c->dq.begin(), c->dq.end(), x);
  return 0;
}

// paper Section 2.3.3 (consistence correction) and the coupled closure
int orc_consistency_correct(orc_ctx *c, int mode, int kind, int *n_clipped) {
  if (!c || c->last_mode != mode) return c ? c->fail(-3, "implicit_op not run in this mode") : -1;
  const Mech &m = c->m;
  const int N = c->N, ns = m.ns, nf = m.nf();
  int clipped = 0, bad = -1;
  for (int p = 0; p < N; ++p) {
    double rs[MAXS], rho = 0.0;
    for (int s = 0; s < ns; ++s) { rs[s] = c->q[size_t(s) * N + p]; rho += rs[s]; }
    auto dq = [&](int k) { return c->dq[size_t(k) * N + p]; };
    double drho = dq(0);
    double target = rho + drho;
    double nr[MAXS];
    bool clip = false;
    if (mode == ORC_COUPLED) {
      double sum = 0.0;
      for (int s = 0; s < ns - 1; ++s) { nr[s] = rs[s] + dq(nf + s); sum += dq(nf + s); }
      nr[ns - 1] = rs[ns - 1] + (drho - sum);
    } else if (kind == ORC_CC1) {
      double sum = 0.0;
      for (int s = 0; s < ns; ++s) sum += dq(nf + s);
      for (int s = 0; s < ns; ++s) nr[s] = rs[s] + dq(nf + s) + (rs[s] / rho) * (drho - sum);
    } else {
      double sum = 0.0, t[MAXS];
      for (int s = 0; s < ns; ++s) {
        t[s] = std::max(rs[s] + dq(nf + s), 0.0);
        if (rs[s] + dq(nf + s) < 0.0) clip = true;
        sum += t[s];
      }
      for (int s = 0; s < ns; ++s) nr[s] = target * t[s] / sum;
    }
    if (mode == ORC_COUPLED || kind == ORC_CC1) {
      double sum = 0.0;
      for (int s = 0; s < ns; ++s) {
        if (nr[s] < 0.0) { nr[s] = 0.0; clip = true; }
        sum += nr[s];
      }
      if (clip)
        for (int s = 0; s < ns; ++s) nr[s] = nr[s] * (target / sum);
    }
    if (clip) ++clipped;
    if (!(target > 0.0)) bad = (bad < 0) ? p : bad;
    for (int s = 0; s < ns; ++s) c->q[size_t(s) * N + p] = nr[s];
    c->q[size_t(ns) * N + p] += dq(1);
    c->q[size_t(ns + 1) * N + p] += dq(2);
    c->q[size_t(ns + 2) * N + p] += dq(3);
    if (m.two_temp) {
      // positivity of the vibrational-electronic energy: floor at Tv = 50 K
      double eve = c->q[size_t(ns + 3) * N + p] + dq(4), floor_ = 0.0;
      for (int s = 0; s < ns; ++s) floor_ += nr[s] * e_ve<double>(m, s, TV_FLOOR);
      if (eve < floor_) { eve = floor_; if (!clip) ++clipped; }
      c->q[size_t(ns + 3) * N + p] = eve;
    }
  }
  if (n_clipped) *n_clipped = clipped;
  c->has_res = false;
  c->last_mode = -1;
  if (bad >= 0) return c->fail(-4, "non-positive density after update at cell " + std::to_string(bad));
  return 0;
}

// cfl(m) = cfl_target^(min(m, ramp)/ramp): geometric ramp from 1 (ramp = 0: fixed cfl)
int orc_step(orc_ctx *c, int mode, int kind, double cfl_target, int ramp, int it0, int n_iter,
             double *hist) {
  for (int it = 0; it < n_iter; ++it) {
    double nrm[2];
    int m_ = it0 + it;
    double cfl = ramp > 0 ? std::pow(cfl_target, double(std::min(m_, ramp)) / ramp) : cfl_target;
    int rc = orc_residual(c, cfl, nrm);
    if (rc) return rc;
    if (hist) { hist[2 * it] = nrm[0]; hist[2 * it + 1] = nrm[1]; }
    rc = orc_implicit_op(c, mode, ORC_HYPERPLANE);
    if (rc) return rc;
    rc = orc_consistency_correct(c, mode, kind, nullptr);
    if (rc) return rc;
  }
  return 0;
}

int orc_wall_heat_flux(orc_ctx *c, double *qw, double *q_stag) {
  if (!c || !c->has_res || c->bc_mode != 0) return -1;
  if (qw) std::copy(c->qw.begin(), c->qw.end(), qw);
  if (q_stag) {
    int h = c->ni / 2;
    *q_stag = (c->ni % 2 == 0) ? 0.5 * (c->qw[h - 1] + c->qw[h]) : c->qw[h];
  }
  return 0;
}

int orc_get(orc_ctx *c, const char *name, double *out) {
  if (!c || !name || !out) return -1;
  std::string n(name);
  auto put = [&](const std::vector<double> &v) {
    if (v.empty()) return c->fail(-3, "array " + n + " not available");
    std::copy(v.begin(), v.end(), out);
    return 0;
  };
  const int N = c->N;
  if (n == "R") return put(c->R);
  if (n == "dtau") return put(c->dtau);
  if (n == "V") return put(c->V);
  if (n == "omega") return put(c->src);
  if (n == "dqs") return put(c->dqs);
  if (n == "dq") return put(c->dq);
  if (n == "qw") return put(c->qw);
  if (n == "dK") return put(c->dK);
  if (n == "dF") return put(c->dF);
  if (n == "dC") return put(c->dC);
  if (n == "JK") return put(c->JK);
  if (n == "JC") return put(c->JC);
  if (n == "Jve") return put(c->Jve);
  if (n == "DK") return put(c->DK);
  if (n == "DF") return put(c->DF);
  if (n == "DC") return put(c->DC);
  if (n == "FvI" || n == "FvJ") {  // viscous face fluxes [nv][faces] (i faces (ni+1)*nj, j faces ni*(nj+1))
    const std::vector<Face> &fa = n == "FvI" ? c->fI : c->fJ;
    if (fa.empty()) return c->fail(-3, "faces not computed");
    const size_t nfa = fa.size();
    for (int k = 0; k < c->m.nv(); ++k)
      for (size_t f = 0; f < nfa; ++f) out[k * nfa + f] = fa[f].Fv[k];
    return 0;
  }
  if (n == "T" || n == "Tv" || n == "p" || n == "c") {
    if (c->cells.empty()) return c->fail(-3, "primitives not computed");
    for (int p = 0; p < N; ++p) {
      const CellD &C = c->cells[c->pc(p % c->ni, p / c->ni)];
      out[p] = n == "T" ? C.P.T : n == "Tv" ? C.P.Tv : n == "p" ? C.P.p : C.c;
    }
    return 0;
  }
  return c->fail(-1, "unknown array " + n);
}

int orc_dense_operator(orc_ctx *c, int mode, double *D, double *L, double *U) {
  if (!c || !c->has_res) return -1;
  const Mech &m = c->m;
  const int N = c->N, ni = c->ni, nj = c->nj, nsol = nsol_of(m, mode);
  const size_t dim = size_t(N) * nsol;
  std::fill(D, D + dim * dim, 0.0);
  std::fill(L, L + dim * dim, 0.0);
  std::fill(U, U + dim * dim, 0.0);
  std::vector<Part> parts;
  if (mode == ORC_COUPLED) parts = {P_COUPLED}; else parts = {P_FLOW, P_SPECIES};
  for (Part part : parts) {
    PartInfo pi = part_info(c, part, mode);
    const std::vector<double> &Dm = part == P_COUPLED ? c->DK : part == P_FLOW ? c->DF : c->DC;
    const int n = pi.n, off = pi.off;
    for (int j = 0; j < nj; ++j)
      for (int i = 0; i < ni; ++i) {
        int p = c->ci(i, j);
        for (int r = 0; r < n; ++r)
          for (int col = 0; col < n; ++col)
            D[(size_t(p) * nsol + off + r) * dim + size_t(p) * nsol + off + col] = Dm[(size_t(r) * n + col) * N + p];
        struct Nb { int in, jn; const Face *F; double sgn; double *M; };
        Nb nbs[4] = {
            {i - 1, j, &c->fI[c->fii(i, j)], -1.0, L},
            {i, j - 1, &c->fJ[c->fji(i, j)], -1.0, L},
            {i + 1, j, i + 1 <= ni ? &c->fI[c->fii(i + 1, j)] : nullptr, 1.0, U},
            {i, j + 1, j + 1 <= nj ? &c->fJ[c->fji(i, j + 1)] : nullptr, 1.0, U},
        };
        for (auto &nb : nbs) {
          if (nb.in < 0 || nb.jn < 0 || nb.in >= ni || nb.jn >= nj) continue;
          int q = c->ci(nb.in, nb.jn);
          for (int col = 0; col < n; ++col) {
            double e[MAXV] = {0}, o[MAXV];
            e[col] = 1.0;
            (void)apply_off(m, part, *nb.F, nb.sgn * nb.F->nx, nb.sgn * nb.F->ny, c->cells[c->pc(nb.in, nb.jn)], e, o, false);
            for (int r = 0; r < n; ++r)
              nb.M[(size_t(p) * nsol + off + r) * dim + size_t(q) * nsol + off + col] = o[r];
          }
        }
      }
  }
  return 0;
}

// ------------------------------------------------------------ point pins
int orc_point_thermo(orc_ctx *c, double T, double Tv, double *e, double *h, double *cv_total,
                     double *g_RT) {
  if (!c || !c->has_mech) return -1;
  const Mech &m = c->m;
  for (int s = 0; s < m.ns; ++s) {
    if (e) e[s] = e_s<double>(m, s, T, Tv);
    if (h) h[s] = h_s<double>(m, s, T, Tv);
    if (cv_total) cv_total[s] = cv_tr(m, s) + cv_ve<double>(m, s, Tv);
    if (g_RT) g_RT[s] = gibbs_RT<double>(m, s, T);
  }
  return 0;
}

int orc_point_production(orc_ctx *c, const double *rho_s, double T, double Tv, double *omega,
                         double *omega_v) {
  if (!c || !c->has_mech) return -1;
  const Mech &m = c->m;
  double om[MAXS];
  production<double>(m, rho_s, T, Tv, om);
  for (int s = 0; s < m.ns; ++s) omega[s] = om[s];
  if (omega_v) {
    double p = 0.0;
    for (int s = 0; s < m.ns; ++s) p += rho_s[s] * m.R(s) * (m.kind[s] == KIND_ELECTRON ? Tv : T);
    *omega_v = m.two_temp ? omega_ve<double>(m, rho_s, T, Tv, p, om) : 0.0;
  }
  return 0;
}

int orc_point_prim(orc_ctx *c, const double *q, double *T, double *Tv, double *p, double *cs) {
  if (!c || !c->has_mech) return -1;
  CellD C;
  if (!make_cell(c->m, q, C)) return c->fail(-4, "non-physical point state");
  if (T) *T = C.P.T;
  if (Tv) *Tv = C.P.Tv;
  if (p) *p = C.P.p;
  if (cs) *cs = C.c;
  return 0;
}

int orc_point_flux(orc_ctx *c, const double *q, double nx, double ny, double *F) {
  if (!c || !c->has_mech) return -1;
  Prim<double> P;
  if (!recover<double>(c->m, q, P)) return -4;
  phys_flux<double>(c->m, q, P, nx, ny, F);
  return 0;
}

int orc_point_hlle(orc_ctx *c, const double *qL, const double *qR, double nx, double ny, double *F) {
  if (!c || !c->has_mech) return -1;
  CellD L, R;
  if (!make_cell(c->m, qL, L) || !make_cell(c->m, qR, R)) return c->fail(-4, "non-physical point state");
  hlle(c->m, L, R, nx, ny, F);
  return 0;
}

int orc_point_roe(orc_ctx *c, const double *qL, const double *qR, double nx, double ny, double eta, double *F) {
  if (!c || !c->has_mech || !(eta >= 0.0)) return -1;
  CellD L, R;
  if (!make_cell(c->m, qL, L) || !make_cell(c->m, qR, R)) return c->fail(-4, "non-physical point state");
  roe(c->m, L, R, nx, ny, eta, F);
  return 0;
}

int orc_point_muscl(orc_ctx *c, const double *qA, const double *qB, const double *qC, double *qf) {
  if (!c || !c->has_mech) return -1;
  CellD A, B, C, out;
  if (!make_cell(c->m, qA, A) || !make_cell(c->m, qB, B) || !make_cell(c->m, qC, C))
    return c->fail(-4, "non-physical point state");
  if (!muscl_state(c->m, A, B, C, out)) return c->fail(-4, "non-physical reconstructed state");
  for (int k = 0; k < c->m.nv(); ++k) qf[k] = out.q[k];
  return 0;
}

int orc_point_flux_jacobian(orc_ctx *c, const double *q, double nx, double ny, double *A) {
  if (!c || !c->has_mech) return -1;
  const Mech &m = c->m;
  const int nv = m.nv();
  for (int col = 0; col < nv; ++col) {
    cplx qc[MAXV], F[MAXV];
    for (int k = 0; k < nv; ++k) qc[k] = q[k];
    double h = CSTEP * std::max(std::fabs(q[col]), 1.0);
    qc[col] += cplx(0.0, h);
    Prim<cplx> P;
    if (!recover<cplx>(m, qc, P)) return -4;
    phys_flux<cplx>(m, qc, P, nx, ny, F);
    for (int r = 0; r < nv; ++r) A[r * nv + col] = F[r].imag() / h;
  }
  return 0;
}

int orc_point_offdiag(orc_ctx *c, const double *q, double nx, double ny, int mode, int fd, const double *x,
                      double *out) {
  if (!c || !c->has_mech || !q || !x || !out) return -1;
  const Mech &m = c->m;
  CellD C;
  for (int k = 0; k < m.nv(); ++k) C.q[k] = q[k];
  if (!recover<double>(m, C.q, C.P)) return c->fail(-4, "non-physical state");
  if (mode == ORC_COUPLED) {
    if (fd) return fdiff_coupled(m, C, nx, ny, x, out) ? 0 : c->fail(-4, "non-physical perturbed state");
    jvp_coupled(m, C, nx, ny, x, out);
  } else {
    if (fd) return fdiff_flow(m, C, nx, ny, x, out) ? 0 : c->fail(-4, "non-physical perturbed state");
    jvp_flow(m, C, nx, ny, x, out);
  }
  return 0;
}

int orc_point_source_jacobian(orc_ctx *c, const double *q, int which, double *J) {
  if (!c || !c->has_mech) return -1;
  const Mech &m = c->m;
  const int ns = m.ns, nb = m.nb(), nf = m.nf();
  Prim<double> P;
  if (!recover<double>(m, q, P)) return -4;
  if (which == 0) {
    double z[MAXV];
    q_to_z<double>(m, q, z);
    for (int col = 0; col < nb; ++col) {
      cplx zc[MAXV], qc[MAXV], sc[MAXV], sz[MAXV];
      for (int k = 0; k < nb; ++k) zc[k] = z[k];
      double h = CSTEP * std::max(std::fabs(z[col]), 1.0);
      zc[col] += cplx(0.0, h);
      z_to_q<cplx>(m, zc, qc);
      source<cplx>(m, qc, sc);
      vec_q_to_z<cplx>(m, sc, sz);
      for (int r = 0; r < nb; ++r) J[r * nb + col] = sz[r].imag() / h;
    }
  } else if (which == 1) {
    for (int col = 0; col < ns; ++col) {
      cplx rc[MAXS], om[MAXS];
      for (int s = 0; s < ns; ++s) rc[s] = P.rs[s];
      double h = CSTEP * std::max(std::fabs(P.rs[col]), 1.0);
      rc[col] += cplx(0.0, h);
      production<cplx>(m, rc, cplx(P.T), cplx(P.Tv), om);
      for (int r = 0; r < ns; ++r) J[r * ns + col] = om[r].imag() / h;
    }
  } else {
    if (!m.two_temp) return -1;
    for (int col = 0; col < nf; ++col) {
      cplx qf[5] = {P.rho, q[ns], q[ns + 1], q[ns + 2], q[ns + 3]};
      double h = CSTEP * std::max(std::fabs(qf[col].real()), 1.0);
      qf[col] += cplx(0.0, h);
      cplx qc[MAXV], sc[MAXV];
      for (int s = 0; s < ns; ++s) qc[s] = P.Y[s] * qf[0];
      qc[ns] = qf[1]; qc[ns + 1] = qf[2]; qc[ns + 2] = qf[3]; qc[ns + 3] = qf[4];
      source<cplx>(m, qc, sc);
      J[col] = sc[ns + 3].imag() / h;
    }
  }
  return 0;
}

}  // extern "C"
