// HIP kernels of one pseudo-time iteration of the coupled / component-split
// implicit solver for gfx950.  Data are structure-of-arrays in HBM, index
// var*N + j*ni + i (i fastest) so that consecutive lanes touch consecutive
// doubles.  Primitive records carry one ghost layer ((ni+2) x (nj+2)).
#pragma once
#include "csi_phys.hpp"

namespace csi {

// Cells of a training sample: row r holds cell (b + r a) mod n; a = 0: row r
// is cell r.  a is coprime with n, so distinct rows are distinct cells.
struct SampleMap {
  long long a, b;
  __host__ __device__ long operator()(long r, long n) const { return a ? long((b + (long long)r * a) % n) : r; }
};

// ------------------------------------------------------------ workspace view
struct Geo {
  int ni, nj, N, NP, bc_mode;
  int scheme;  // residual: 0 first-order HLLE, 1 MUSCL (minmod) + Roe
  double Tw;
  const double *V, *xc, *yc, *xn, *yn;
  const double *fi_nx, *fi_ny, *fi_S;  // i-faces, index j*(ni+1)+I, normal towards +i
  const double *fj_nx, *fj_ny, *fj_S;  // j-faces, index J*ni+i, normal towards +j
};

// primitive record fields
enum {
  F_RHO = 0, F_U, F_V, F_T, F_TV, F_P, F_C, F_H, F_EVE, F_RE, F_MU, F_K, F_KVE, F_NUF, F_NUC, F_NUK,
  F_PE, F_PV, F_Y0
};
template <int NS> struct PF {
  static constexpr int Y = F_Y0, HS = F_Y0 + NS, EVS = F_Y0 + 2 * NS, PR = F_Y0 + 3 * NS, N = F_Y0 + 4 * NS;
};
// face radius fields
enum { R_LAM = 0, R_UABS, R_LVF, R_LVC, R_LVK, R_N };

// species table read by the streaming (run-time species count) kernels of
// one temperature: device arrays of length ns (the species-generic path's
// own table, or views into a Mech record)
struct WMech {
  int ns;
  const double *R, *cvtr, *thv, *hf, *ck, *iSc;
  const int *kind;
  double mu_ref, T_ref, mu_exp, iscmax;
};

// primitive record fields with a run-time species count (same order as PF)
struct WF {
  int Y, HS, EVS, PR, N;
  __host__ __device__ explicit WF(int ns) : Y(F_Y0), HS(F_Y0 + ns), EVS(F_Y0 + 2 * ns), PR(F_Y0 + 3 * ns),
                                            N(F_Y0 + 4 * ns) {}
};

__device__ __forceinline__ int padc(const Geo &g, int i, int j) { return (j + 1) * (g.ni + 2) + (i + 1); }

// --------------------------------------------------------------- primitives
// One thread per padded cell: interior cells from Q; ghosts by the boundary
// conditions (wall mirror, far-field free stream, zero-gradient outflow) or
// all free stream (bc_mode 1).  guess: the record still holds the previous
// iteration's temperatures, where the Newton iterations start.
template <int NS, int NT>
__global__ void __launch_bounds__(256) k_prim(Geo g, const Mech *__restrict__ mech, const double *__restrict__ Q,
                                              const double *__restrict__ qfs, double *__restrict__ prim,
                                              int *__restrict__ bad, const int *__restrict__ done, int guess) {
  using D = Dims<NS, NT>;
  if (done && *done) return;
  int pc = blockIdx.x * blockDim.x + threadIdx.x;
  if (pc >= g.NP) return;
  const Mech &m = *mech;
  int i = pc % (g.ni + 2) - 1, j = pc / (g.ni + 2) - 1;
  bool interior = i >= 0 && i < g.ni && j >= 0 && j < g.nj;
  int si = i < 0 ? 0 : (i >= g.ni ? g.ni - 1 : i);
  bool use_fs = false, mirror = false;
  if (!interior) {
    if (g.bc_mode == 1) use_fs = true;
    else if (j >= g.nj) use_fs = true;
    else if (j < 0) mirror = true;
  }
  double q[D::nv];
  if (use_fs) {
#pragma unroll
    for (int k = 0; k < D::nv; ++k) q[k] = qfs[k];
  } else {
    int sj = j < 0 ? 0 : j;
    int c = sj * g.ni + si;
#pragma unroll
    for (int k = 0; k < D::nv; ++k) q[k] = Q[size_t(k) * g.N + c];
  }
  Prim<NS, NT> P;
  double T0 = 0.0, Tv0 = 0.0;
  if (guess) {
    T0 = prim[size_t(F_T) * g.NP + pc];
    Tv0 = prim[size_t(F_TV) * g.NP + pc];
  }
  bool ok = prim_from_q<NS, NT>(m, q, P, T0, Tv0);
  if (!ok) {
    if (interior && bad) atomicMin(bad, j * g.ni + i);
    return;
  }
  Transport t;
  transport<NS, NT>(m, P, t);
  if (mirror) {
    int f = si;  // wall face (si, 0)
    double nx = g.fj_nx[f], ny = g.fj_ny[f];
    double un = P.u * nx + P.v * ny;
    P.u = P.u - 2.0 * un * nx;
    P.v = P.v - 2.0 * un * ny;
  }
  const size_t NP = g.NP;
  double *o = prim + pc;
  o[F_RHO * NP] = P.rho; o[F_U * NP] = P.u; o[F_V * NP] = P.v; o[F_T * NP] = P.T; o[F_TV * NP] = P.Tv;
  o[F_P * NP] = P.p; o[F_C * NP] = P.c; o[F_H * NP] = P.H; o[F_EVE * NP] = P.eve; o[F_RE * NP] = P.rE;
  o[F_MU * NP] = t.mu; o[F_K * NP] = t.k; o[F_KVE * NP] = t.kve; o[F_NUF * NP] = t.nuF; o[F_NUC * NP] = t.nuC;
  o[F_NUK * NP] = t.nuK; o[F_PE * NP] = P.pE; o[F_PV * NP] = P.pv;
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    o[(PF<NS>::Y + s) * NP] = P.Y[s];
    o[(PF<NS>::HS + s) * NP] = m.cvtr[s] * P.T + eve_s(m, s, P.Tv) + m.hf[s] + m.R[s] * (m.kind[s] == ELECTRON ? P.Tv : P.T);
    o[(PF<NS>::EVS + s) * NP] = eve_s(m, s, P.Tv);
    o[(PF<NS>::PR + s) * NP] = P.pr[s];
  }
}

// ----------------------------------------------------------------- faces
template <int NS> struct FaceState {
  double rho, u, v, p, c, H, eve, rE, Y[NS];
};
template <int NS>
__device__ __forceinline__ void load_face_state(const double *prim, size_t NP, int pc, FaceState<NS> &s) {
  s.rho = prim[F_RHO * NP + pc]; s.u = prim[F_U * NP + pc]; s.v = prim[F_V * NP + pc];
  s.p = prim[F_P * NP + pc]; s.c = prim[F_C * NP + pc]; s.H = prim[F_H * NP + pc];
  s.eve = prim[F_EVE * NP + pc]; s.rE = prim[F_RE * NP + pc];
#pragma unroll
  for (int k = 0; k < NS; ++k) s.Y[k] = prim[(PF<NS>::Y + k) * NP + pc];
}

// HLLE (Davis bounds) for mass, momentum and total energy; species and e_ve
// carried by the mixture mass flux with upwind mass fraction / e_ve.
template <int NS, int NT>
__device__ __forceinline__ void hlle_flux(const FaceState<NS> &L, const FaceState<NS> &R, double nx, double ny,
                                          double *F) {
  double unL = L.u * nx + L.v * ny, unR = R.u * nx + R.v * ny;
  double SL = fmin(unL - L.c, unR - R.c), SR = fmax(unL + L.c, unR + R.c);
  double sl = fmin(SL, 0.0), sr = fmax(SR, 0.0);
  double id = 1.0 / (sr - sl);
  auto hll = [&](double fl, double fr, double ql, double qr) { return (sr * fl - sl * fr + sr * sl * (qr - ql)) * id; };
  double fm = hll(L.rho * unL, R.rho * unR, L.rho, R.rho);
  const FaceState<NS> &U = fm >= 0.0 ? L : R;
#pragma unroll
  for (int s = 0; s < NS; ++s) F[s] = fm * U.Y[s];
  double mxL = L.rho * L.u, myL = L.rho * L.v, mxR = R.rho * R.u, myR = R.rho * R.v;
  F[NS] = hll(mxL * unL + L.p * nx, mxR * unR + R.p * nx, mxL, mxR);
  F[NS + 1] = hll(myL * unL + L.p * ny, myR * unR + R.p * ny, myL, myR);
  F[NS + 2] = hll((L.rE + L.p) * unL, (R.rE + R.p) * unR, L.rE, R.rE);
  if (NT == 2) F[NS + 3] = fm * U.eve;
}

// ------------------------------------------------ MUSCL (minmod) + Roe
// The second-order residual of the paper's cylinder case (Section 3.2),
// built as an ablation: w = (rho_s, u, v, T, Tv) reconstructed per side at
// interior faces, w_face = w_B + 1/2 minmod(w_B - w_A, w_C - w_B) (A beyond
// the side's cell B, C across the face), boundary faces first order; the Roe
// flux of the mixture at frozen composition, species and e_ve carried by the
// mixture mass flux at the upwind mass fraction / e_ve as in hlle_flux.
__device__ __forceinline__ double minmod(double a, double b) {
  if (!(a * b > 0.0)) return 0.0;
  return fabs(a) < fabs(b) ? a : b;
}

template <int NS> struct RoeState {
  double rho, u, v, p, c, H, rE, eve, beta, Y[NS];
};

template <int NS>
__device__ __forceinline__ void roe_state_cell(const double *prim, size_t NP, int pc, RoeState<NS> &s) {
  s.rho = prim[F_RHO * NP + pc]; s.u = prim[F_U * NP + pc]; s.v = prim[F_V * NP + pc];
  s.p = prim[F_P * NP + pc]; s.c = prim[F_C * NP + pc]; s.H = prim[F_H * NP + pc];
  s.rE = prim[F_RE * NP + pc]; s.eve = prim[F_EVE * NP + pc]; s.beta = prim[F_PE * NP + pc];
#pragma unroll
  for (int k = 0; k < NS; ++k) s.Y[k] = prim[(PF<NS>::Y + k) * NP + pc];
}

// the face state on the side of cell pB (pA beyond it, pC across the face)
template <int NS, int NT>
__device__ __forceinline__ bool roe_state_muscl(const Mech &m, const double *prim, size_t NP, int pA, int pB, int pC,
                                                RoeState<NS> &s) {
  auto rec = [&](double a, double b, double c) { return b + 0.5 * minmod(b - a, c - b); };
  auto fld = [&](int f, int pc) { return prim[size_t(f) * NP + pc]; };
  const double rA = fld(F_RHO, pA), rB = fld(F_RHO, pB), rC = fld(F_RHO, pC);
  double rs[NS];
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    const int f = PF<NS>::Y + k;
    rs[k] = rec(rA * fld(f, pA), rB * fld(f, pB), rC * fld(f, pC));
  }
  const double u = rec(fld(F_U, pA), fld(F_U, pB), fld(F_U, pC));
  const double v = rec(fld(F_V, pA), fld(F_V, pB), fld(F_V, pC));
  const double T = rec(fld(F_T, pA), fld(F_T, pB), fld(F_T, pC));
  const double Tv = NT == 2 ? rec(fld(F_TV, pA), fld(F_TV, pB), fld(F_TV, pC)) : T;
  double q[Dims<NS, NT>::nv];
  q_from_prim<NS, NT>(m, rs, u, v, T, Tv, q);
  Prim<NS, NT> P;
  if (!prim_from_q<NS, NT>(m, q, P, T, Tv)) return false;
  s.rho = P.rho; s.u = P.u; s.v = P.v; s.p = P.p; s.c = P.c; s.H = P.H; s.rE = P.rE; s.eve = P.eve;
  s.beta = P.pE;
#pragma unroll
  for (int k = 0; k < NS; ++k) s.Y[k] = P.Y[k];
  return true;
}

// Roe average with weights w = sqrt(rho_L) / (sqrt(rho_L) + sqrt(rho_R)) of
// u, v, H and beta = dp/d(rho E); c^2 = w c_L^2 + (1 - w) c_R^2 +
// beta w (1 - w) |V_R - V_L|^2 / 2 (Roe's average for a calorically perfect
// gas of fixed composition); the waves at u.n carry the rest of the rho E
// jump, a2 e2 = d(rho E) - H dp / c^2 - rho V.dV, which keeps Roe's property
// for a real-gas mixture (e2 = H - c^2 / beta for a perfect gas); Harten's
// entropy fix (delta = c / 10) on the acoustic waves; eta: the H-correction's
// floor on every wave speed
template <int NS, int NT>
__device__ __forceinline__ void roe_flux(const RoeState<NS> &L, const RoeState<NS> &R, double nx, double ny,
                                         double eta, double *F) {
  const double unL = L.u * nx + L.v * ny, unR = R.u * nx + R.v * ny;
  const double sL = sqrt(L.rho), sR = sqrt(R.rho), w = sL / (sL + sR), wr = 1.0 - w;
  const double u = w * L.u + wr * R.u, v = w * L.v + wr * R.v, H = w * L.H + wr * R.H;
  const double beta = w * L.beta + wr * R.beta;
  const double dVx = R.u - L.u, dVy = R.v - L.v;
  const double cL2 = L.c * L.c, cR2 = R.c * R.c;
  double c2 = w * cL2 + wr * cR2 + 0.5 * beta * w * wr * (dVx * dVx + dVy * dVy);
  c2 = fmax(c2, 1e-6 * fmin(cL2, cR2));
  const double c = sqrt(c2), rho = sL * sR;
  const double un = u * nx + v * ny, ut = -u * ny + v * nx;
  const double utL = -L.u * ny + L.v * nx, utR = -R.u * ny + R.v * nx;
  const double dp = R.p - L.p, dun = unR - unL, dut = utR - utL, drho = R.rho - L.rho;
  const double a1 = (dp - rho * c * dun) / (2.0 * c2), a3 = (dp + rho * c * dun) / (2.0 * c2);
  const double a2 = drho - dp / c2, at = rho * dut;
  const double delta = 0.1 * c;
  auto fix = [&](double l) {
    const double a = fabs(l);
    return a < delta ? (l * l + delta * delta) / (2.0 * delta) : a;
  };
  const double l1 = fmax(fix(un - c), eta), l2 = fmax(fabs(un), eta), l3 = fmax(fix(un + c), eta);
  const double a2e2 = (R.rE - L.rE) - H * dp / c2 - rho * (u * dVx + v * dVy);
  const double D0 = l1 * a1 + l2 * a2 + l3 * a3;
  const double Dx = l1 * a1 * (u - c * nx) + l2 * (a2 * u - at * ny) + l3 * a3 * (u + c * nx);
  const double Dy = l1 * a1 * (v - c * ny) + l2 * (a2 * v + at * nx) + l3 * a3 * (v + c * ny);
  const double DE = l1 * a1 * (H - un * c) + l2 * (a2e2 + at * ut) + l3 * a3 * (H + un * c);
  const double mL = L.rho * unL, mR = R.rho * unR;
  const double fm = 0.5 * (mL + mR) - 0.5 * D0;
  const RoeState<NS> &U = fm >= 0.0 ? L : R;
#pragma unroll
  for (int s = 0; s < NS; ++s) F[s] = fm * U.Y[s];
  F[NS] = 0.5 * ((L.rho * L.u * unL + L.p * nx) + (R.rho * R.u * unR + R.p * nx)) - 0.5 * Dx;
  F[NS + 1] = 0.5 * ((L.rho * L.v * unL + L.p * ny) + (R.rho * R.v * unR + R.p * ny)) - 0.5 * Dy;
  F[NS + 2] = 0.5 * ((L.rE + L.p) * unL + (R.rE + R.p) * unR) - 0.5 * DE;
  if (NT == 2) F[NS + 3] = fm * U.eve;
}

// The H-correction of Sanders, Morano and Druguet against the carbuncle of
// Roe's flux at a shock aligned with the grid: eta of a face is half the
// largest jump of a characteristic speed across it, (|un_R - un_L| +
// |c_R - c_L|) / 2 from the two cells' states, and a face's wave speeds are
// floored by the largest eta among itself and the four faces of the other
// family that share an edge with it.
__device__ __forceinline__ double eta_cells(const double *prim, size_t NP, int pL, int pR, double nx, double ny) {
  const double unL = prim[F_U * NP + pL] * nx + prim[F_V * NP + pL] * ny;
  const double unR = prim[F_U * NP + pR] * nx + prim[F_V * NP + pR] * ny;
  return 0.5 * (fabs(unR - unL) + fabs(prim[F_C * NP + pR] - prim[F_C * NP + pL]));
}

__device__ __forceinline__ double eta_iface(const Geo &g, const double *prim, int I, int j) {
  const size_t NP = g.NP;
  const int f = j * (g.ni + 1) + I;
  double e = eta_cells(prim, NP, padc(g, I - 1, j), padc(g, I, j), g.fi_nx[f], g.fi_ny[f]);
  for (int i = I - 1; i <= I; ++i) {
    if (i < 0 || i >= g.ni) continue;
    for (int J = j; J <= j + 1; ++J)
      e = fmax(e, eta_cells(prim, NP, padc(g, i, J - 1), padc(g, i, J), g.fj_nx[J * g.ni + i], g.fj_ny[J * g.ni + i]));
  }
  return e;
}

__device__ __forceinline__ double eta_jface(const Geo &g, const double *prim, int i, int J) {
  const size_t NP = g.NP;
  const int f = J * g.ni + i;
  double e = eta_cells(prim, NP, padc(g, i, J - 1), padc(g, i, J), g.fj_nx[f], g.fj_ny[f]);
  for (int j = J - 1; j <= J; ++j) {
    if (j < 0 || j >= g.nj) continue;
    for (int I = i; I <= i + 1; ++I) {
      const int fi = j * (g.ni + 1) + I;
      e = fmax(e, eta_cells(prim, NP, padc(g, I - 1, j), padc(g, I, j), g.fi_nx[fi], g.fi_ny[fi]));
    }
  }
  return e;
}

// the inviscid face flux of the MUSCL + Roe scheme; pLL / pRR: the cells
// beyond pL / pR (used at interior faces); false on a non-physical
// reconstructed state (the flux is then the first-order Roe flux)
template <int NS, int NT>
__device__ __forceinline__ bool muscl_roe_flux(const Mech &m, const double *prim, size_t NP, int pLL, int pL, int pR,
                                               int pRR, bool interior, double nx, double ny, double eta, double *F) {
  RoeState<NS> L, R;
  bool ok = true;
  if (interior)
    ok = roe_state_muscl<NS, NT>(m, prim, NP, pLL, pL, pR, L) && roe_state_muscl<NS, NT>(m, prim, NP, pRR, pR, pL, R);
  if (!interior || !ok) {
    roe_state_cell<NS>(prim, NP, pL, L);
    roe_state_cell<NS>(prim, NP, pR, R);
  }
  roe_flux<NS, NT>(L, R, nx, ny, eta, F);
  return ok;
}

// gradient from the two diagonals of the diamond: d1.g = D1, d2.g = D2
__device__ __forceinline__ void diamond_grad(double d1x, double d1y, double d2x, double d2y, double D1, double D2,
                                             double &gx, double &gy) {
  double det = d1x * d2y - d1y * d2x;
  gx = (D1 * d2y - D2 * d1y) / det;
  gy = (D2 * d1x - D1 * d2x) / det;
}

// value of variable var (0 u, 1 v, 2 T, 3 Tv, 4+s Y_s) at grid node (I, J)
template <int NS>
__device__ __forceinline__ double node_value(const Geo &g, const double *prim, int I, int J, int var) {
  const size_t NP = g.NP;
  int fld = var == 0 ? F_U : var == 1 ? F_V : var == 2 ? F_T : var == 3 ? F_TV : PF<NS>::Y + var - 4;
  if (g.bc_mode == 0 && J == 0) {
    if (var <= 1) return 0.0;
    if (var <= 3) return g.Tw;
    return 0.5 * (prim[fld * NP + padc(g, I - 1, 0)] + prim[fld * NP + padc(g, I, 0)]);
  }
  return 0.25 * (prim[fld * NP + padc(g, I - 1, J - 1)] + prim[fld * NP + padc(g, I, J - 1)] +
                 prim[fld * NP + padc(g, I - 1, J)] + prim[fld * NP + padc(g, I, J)]);
}

template <int NS, int NT>
__device__ __forceinline__ double cellvar(const double *prim, size_t NP, int pc, int var) {
  int fld = var == 0 ? F_U : var == 1 ? F_V : var == 2 ? F_T : var == 3 ? F_TV : PF<NS>::Y + var - 4;
  return prim[fld * NP + pc];
}

// Viscous flux F_vis.n at an interior face (paper Section 2.1 constitutive
// laws; diffusion fluxes corrected to sum to zero)
template <int NS, int NT>
__device__ __forceinline__ void viscous_interior(const Geo &g, const Mech &m, const double *prim, int pL, int pR,
                                                 double xL, double yL, double xR, double yR, int IA, int JA, int IB,
                                                 int JB, double nx, double ny, double *F) {
  const size_t NP = g.NP;
  double d1x = xR - xL, d1y = yR - yL;
  int nA = JA * (g.ni + 1) + IA, nB = JB * (g.ni + 1) + IB;
  double d2x = g.xn[nB] - g.xn[nA], d2y = g.yn[nB] - g.yn[nA];
  double gr[4 + NS][2];
#pragma unroll
  for (int var = 0; var < 4 + NS; ++var) {
    double D1 = cellvar<NS, NT>(prim, NP, pR, var) - cellvar<NS, NT>(prim, NP, pL, var);
    double D2 = node_value<NS>(g, prim, IB, JB, var) - node_value<NS>(g, prim, IA, JA, var);
    diamond_grad(d1x, d1y, d2x, d2y, D1, D2, gr[var][0], gr[var][1]);
  }
  auto avg = [&](int fld) { return 0.5 * (prim[fld * NP + pL] + prim[fld * NP + pR]); };
  double mu = avg(F_MU), k = avg(F_K), kve = avg(F_KVE), u = avg(F_U), v = avg(F_V);
  double div = gr[0][0] + gr[1][1];
  double txx = mu * (2.0 * gr[0][0] - 2.0 / 3.0 * div);
  double tyy = mu * (2.0 * gr[1][1] - 2.0 / 3.0 * div);
  double txy = mu * (gr[0][1] + gr[1][0]);
  double muL = prim[F_MU * NP + pL], muR = prim[F_MU * NP + pR];
  double Jcx = 0.0, Jcy = 0.0, rD[NS], Yf[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    rD[s] = 0.5 * (muL * m.iSc[s] + muR * m.iSc[s]);
    Yf[s] = avg(PF<NS>::Y + s);
    Jcx += rD[s] * gr[4 + s][0];
    Jcy += rD[s] * gr[4 + s][1];
  }
  double hJ = 0.0, eJ = 0.0;
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    double jx = -rD[s] * gr[4 + s][0] + Yf[s] * Jcx;
    double jy = -rD[s] * gr[4 + s][1] + Yf[s] * Jcy;
    double jn = jx * nx + jy * ny;
    F[s] = jn;
    hJ += avg(PF<NS>::HS + s) * jn;
    eJ += avg(PF<NS>::EVS + s) * jn;
  }
  double tnx = txx * nx + txy * ny, tny = txy * nx + tyy * ny;
  double qtr = -k * (gr[2][0] * nx + gr[2][1] * ny);
  double qve = -kve * (gr[3][0] * nx + gr[3][1] * ny);
  F[NS] = -tnx;
  F[NS + 1] = -tny;
  F[NS + 2] = -(u * tnx + v * tny) + qtr + qve + hJ;
  if (NT == 2) F[NS + 3] = qve + eJ;
}

template <int NS, int NT>
__device__ __forceinline__ void radii(const Geo &g, const double *prim, int pL, int pR, bool interior, int pIn,
                                      double VL, double VR, double Vin, double nx, double ny, double S, double *rad) {
  const size_t NP = g.NP;
  double U = 0.5 * ((prim[F_U * NP + pL] + prim[F_U * NP + pR]) * nx + (prim[F_V * NP + pL] + prim[F_V * NP + pR]) * ny);
  rad[R_UABS] = fabs(U);
  rad[R_LAM] = fabs(U) + 0.5 * (prim[F_C * NP + pL] + prim[F_C * NP + pR]);
  double nF, nC, nK, Vf;
  if (interior) {
    nF = 0.5 * (prim[F_NUF * NP + pL] + prim[F_NUF * NP + pR]);
    nC = 0.5 * (prim[F_NUC * NP + pL] + prim[F_NUC * NP + pR]);
    nK = 0.5 * (prim[F_NUK * NP + pL] + prim[F_NUK * NP + pR]);
    Vf = 0.5 * (VL + VR);
  } else {
    nF = prim[F_NUF * NP + pIn];
    nC = prim[F_NUC * NP + pIn];
    nK = prim[F_NUK * NP + pIn];
    Vf = Vin;
  }
  rad[R_LVF] = nF * S / Vf;
  rad[R_LVC] = nC * S / Vf;
  rad[R_LVK] = nK * S / Vf;
}

// i-faces: (I, j), I in [0, ni], j in [0, nj); SCH: the residual scheme
// (0 first-order HLLE, 1 MUSCL + Roe)
template <int NS, int NT, int SCH>
__global__ void __launch_bounds__(256) k_face_i(Geo g, const Mech *__restrict__ mech, const double *__restrict__ prim,
                                                double *__restrict__ Fi, double *__restrict__ Ri,
                                                const int *__restrict__ done, int *__restrict__ bad) {
  using D = Dims<NS, NT>;
  if (done && *done) return;
  int f = blockIdx.x * blockDim.x + threadIdx.x;
  int nfc = (g.ni + 1) * g.nj;
  if (f >= nfc) return;
  int I = f % (g.ni + 1), j = f / (g.ni + 1);
  const size_t NP = g.NP;
  int pL = padc(g, I - 1, j), pR = padc(g, I, j);
  double nx = g.fi_nx[f], ny = g.fi_ny[f], S = g.fi_S[f];
  FaceState<NS> L, R;
  load_face_state<NS>(prim, NP, pL, L);
  load_face_state<NS>(prim, NP, pR, R);
  double F[D::nv];
  bool interior = I > 0 && I < g.ni;
  if constexpr (SCH == 1) {
    if (!muscl_roe_flux<NS, NT>(*mech, prim, NP, interior ? padc(g, I - 2, j) : pL, pL, pR,
                                interior ? padc(g, I + 1, j) : pR, interior, nx, ny, eta_iface(g, prim, I, j), F) &&
        bad)
      atomicMin(bad, j * g.ni + (I < g.ni ? I : g.ni - 1));
  } else {
    hlle_flux<NS, NT>(L, R, nx, ny, F);
  }
  double rad[R_N];
  int cin = j * g.ni + (I == 0 ? 0 : g.ni - 1);
  radii<NS, NT>(g, prim, pL, pR, interior, padc(g, I == 0 ? 0 : g.ni - 1, j), interior ? g.V[j * g.ni + I - 1] : 0.0,
                interior ? g.V[j * g.ni + I] : 0.0, g.V[cin], nx, ny, S, rad);
  if (interior) {
    double Fv[D::nv];
    int cL = j * g.ni + I - 1, cR = j * g.ni + I;
    viscous_interior<NS, NT>(g, *mech, prim, pL, pR, g.xc[cL], g.yc[cL], g.xc[cR], g.yc[cR], I, j, I, j + 1, nx, ny, Fv);
#pragma unroll
    for (int k = 0; k < D::nv; ++k) F[k] += Fv[k];
  }
#pragma unroll
  for (int k = 0; k < D::nv; ++k) Fi[size_t(k) * nfc + f] = F[k];
#pragma unroll
  for (int k = 0; k < R_N; ++k) Ri[size_t(k) * nfc + f] = rad[k];
}

// j-faces: (i, J), i in [0, ni), J in [0, nj]; J = 0 is the wall in bc_mode 0
template <int NS, int NT, int SCH>
__global__ void __launch_bounds__(256) k_face_j(Geo g, const Mech *__restrict__ mech, const double *__restrict__ prim,
                                                double *__restrict__ Fj, double *__restrict__ Rj,
                                                double *__restrict__ qw, const int *__restrict__ done,
                                                int *__restrict__ bad) {
  using D = Dims<NS, NT>;
  if (done && *done) return;
  int f = blockIdx.x * blockDim.x + threadIdx.x;
  int nfc = g.ni * (g.nj + 1);
  if (f >= nfc) return;
  const Mech &m = *mech;
  int i = f % g.ni, J = f / g.ni;
  const size_t NP = g.NP;
  int pL = padc(g, i, J - 1), pR = padc(g, i, J);
  double nx = g.fj_nx[f], ny = g.fj_ny[f], S = g.fj_S[f];
  FaceState<NS> L, R;
  load_face_state<NS>(prim, NP, pL, L);
  load_face_state<NS>(prim, NP, pR, R);
  double F[D::nv];
  bool interior = J > 0 && J < g.nj;
  if constexpr (SCH == 1) {
    if (!muscl_roe_flux<NS, NT>(m, prim, NP, interior ? padc(g, i, J - 2) : pL, pL, pR,
                                interior ? padc(g, i, J + 1) : pR, interior, nx, ny, eta_jface(g, prim, i, J), F) &&
        bad)
      atomicMin(bad, (J < g.nj ? J : g.nj - 1) * g.ni + i);
  } else {
    hlle_flux<NS, NT>(L, R, nx, ny, F);
  }
  double rad[R_N];
  int cin = (J == 0 ? 0 : g.nj - 1) * g.ni + i;
  radii<NS, NT>(g, prim, pL, pR, interior, padc(g, i, J == 0 ? 0 : g.nj - 1), interior ? g.V[(J - 1) * g.ni + i] : 0.0,
                interior ? g.V[J * g.ni + i] : 0.0, g.V[cin], nx, ny, S, rad);
  if (interior) {
    double Fv[D::nv];
    int cL = (J - 1) * g.ni + i, cR = J * g.ni + i;
    viscous_interior<NS, NT>(g, m, prim, pL, pR, g.xc[cL], g.yc[cL], g.xc[cR], g.yc[cR], i, J, i + 1, J, nx, ny, Fv);
#pragma unroll
    for (int k = 0; k < D::nv; ++k) F[k] += Fv[k];
  } else if (J == 0 && g.bc_mode == 0) {
    // isothermal no-slip non-catalytic wall: wall values at the face, normal
    // gradient between the face centre and the first cell centre
    int c0 = i;
    double muw = m.mu_ref * exp(m.mu_exp * log(g.Tw / m.T_ref));
    double ktr = 0.0, kint = 0.0;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      double Y = R.Y[s];
      ktr += Y * m.ck[s];
      kint += Y * cvve_s(m, s, g.Tw);
    }
    double kw = NT == 2 ? muw * ktr : muw * (ktr + kint);
    double kvw = NT == 2 ? muw * kint : 0.0;
    int nA = i, nB = i + 1;
    double xf = 0.5 * (g.xn[nA] + g.xn[nB]), yf = 0.5 * (g.yn[nA] + g.yn[nB]);
    double d1x = g.xc[c0] - xf, d1y = g.yc[c0] - yf;
    double d2x = g.xn[nB] - g.xn[nA], d2y = g.yn[nB] - g.yn[nA];
    double gu[2], gv[2], gT[2], gTv[2];
    diamond_grad(d1x, d1y, d2x, d2y, prim[F_U * NP + pR], 0.0, gu[0], gu[1]);
    diamond_grad(d1x, d1y, d2x, d2y, prim[F_V * NP + pR], 0.0, gv[0], gv[1]);
    diamond_grad(d1x, d1y, d2x, d2y, prim[F_T * NP + pR] - g.Tw, 0.0, gT[0], gT[1]);
    diamond_grad(d1x, d1y, d2x, d2y, prim[F_TV * NP + pR] - g.Tw, 0.0, gTv[0], gTv[1]);
    double div = gu[0] + gv[1];
    double txx = muw * (2.0 * gu[0] - 2.0 / 3.0 * div);
    double tyy = muw * (2.0 * gv[1] - 2.0 / 3.0 * div);
    double txy = muw * (gu[1] + gv[0]);
    double tnx = txx * nx + txy * ny, tny = txy * nx + tyy * ny;
    double qtr = -kw * (gT[0] * nx + gT[1] * ny);
    double qve = -kvw * (gTv[0] * nx + gTv[1] * ny);
    F[NS] += -tnx;
    F[NS + 1] += -tny;
    F[NS + 2] += qtr + qve;
    if (NT == 2) F[NS + 3] += qve;
    qw[i] = -(qtr + qve);
  }
#pragma unroll
  for (int k = 0; k < D::nv; ++k) Fj[size_t(k) * nfc + f] = F[k];
#pragma unroll
  for (int k = 0; k < R_N; ++k) Rj[size_t(k) * nfc + f] = rad[k];
}

// ------------------------------------------------------- dense inversion
// In-register Gauss-Jordan inversion with partial pivoting (largest |a|,
// lowest row on ties).  Returns false on a zero pivot.
template <int N>
__device__ __forceinline__ bool invert(double (&a)[N][N], double (&inv)[N][N]) {
#pragma unroll
  for (int r = 0; r < N; ++r)
#pragma unroll
    for (int c = 0; c < N; ++c) inv[r][c] = (r == c) ? 1.0 : 0.0;
#pragma unroll
  for (int k = 0; k < N; ++k) {
    int p = k;
    double best = fabs(a[k][k]);
#pragma unroll
    for (int r = k + 1; r < N; ++r)
      if (fabs(a[r][k]) > best) { best = fabs(a[r][k]); p = r; }
    if (best == 0.0) return false;
    if (p != k) {
#pragma unroll
      for (int r = k + 1; r < N; ++r) {
        if (r == p) {
#pragma unroll
          for (int c = 0; c < N; ++c) {
            double t = a[k][c]; a[k][c] = a[r][c]; a[r][c] = t;
            t = inv[k][c]; inv[k][c] = inv[r][c]; inv[r][c] = t;
          }
        }
      }
    }
    double ip = 1.0 / a[k][k];
#pragma unroll
    for (int c = 0; c < N; ++c) { a[k][c] *= ip; inv[k][c] *= ip; }
#pragma unroll
    for (int r = 0; r < N; ++r) {
      if (r == k) continue;
      double l = a[r][k];
#pragma unroll
      for (int c = 0; c < N; ++c) { a[r][c] -= l * a[k][c]; inv[r][c] -= l * inv[k][c]; }
    }
  }
  return true;
}

// ----------------------------------------------- group-schedule record layout
// The sweeps give each cell a group of G lanes (one per unknown of the swept
// part) and each wavefront a strip of C = 64 / G columns.  The cell kernel
// writes a record per cell and part into a staging array; each sweep step
// gathers the records of the C cells it works on into LDS with 16-byte
// global-to-LDS copies.  A record has three sections (words of RT):
//   common    D^-1 row-major [G][G]; JVP parts also the dp weights w[G] and
//             the coefficients of a, ca[G]
//   forward   RHS b[G]; JVP parts per push face (E, N): g[G], cp[G], then per
//             face (m_x, m_y, u.m); species part per face u.m - c
//   backward  dQ*[G] (written by the forward sweep), then as forward for the
//             faces W, S
// Each section is padded to whole 16-byte granules (GW words); the staging
// array holds the records one after the other (cell p at p (QC + 2 QD) GW),
// so that a sweep step reads each cell's sections as contiguous runs.

// parts of the implicit operator swept by one wavefront
enum { PART_COUPLED = 0, PART_FLOW = 2, PART_SPECIES = 3 };

// From this species count on, the diagonal blocks (source Jacobian, block,
// inverse) are built by k_block with one lane per row; the cell kernel then
// writes only what that kernel reads per cell (field f of cell p at f N + p):
// the scalar diagonals (coupled: dK; split: dF, dC), X_s = rho_s / M_s,
// dT/dq_c and dTv/dq_c over the stored variables, and Y_s.
constexpr int BLOCK_NS_MIN = 5;
constexpr int HB_X = 2;
constexpr int hb_fields(int ns, int nv) { return 2 + 2 * ns + 2 * nv; }

struct RecShape {
  int G, JVP;   // lanes per cell, whether the push is a flux Jacobian-vector product
  int CW, DW;   // words of the common and of each direction section
  int GW;       // words per 16-byte granule
  int QC, QD;   // granules of the common and of each direction section
};
__host__ __device__ constexpr RecShape rec_shape(int part, int ns, int nt, int esz) {
  const int nf = nt == 2 ? 5 : 4, nb = nf + ns - 1;
  const int G = part == PART_COUPLED ? nb : part == PART_FLOW ? nf : ns;
  const int jvp = part != PART_SPECIES;
  const int CW = G * G + (jvp ? 2 * G : 0), DW = G + (jvp ? 4 * G + 6 : 2), GW = 16 / esz;
  return RecShape{G, jvp, CW, DW, GW, (CW + GW - 1) / GW, (DW + GW - 1) / GW};
}
// word offsets: common section
__host__ __device__ constexpr int rw_d(const RecShape &r, int k, int q) { return k * r.G + q; }
__host__ __device__ constexpr int rw_w(const RecShape &r, int q) { return r.G * r.G + q; }
__host__ __device__ constexpr int rw_ca(const RecShape &r, int k) { return r.G * r.G + r.G + k; }
// direction sections (face f = 0, 1: E, N forward; W, S backward)
__host__ __device__ constexpr int dw_b(int k) { return k; }
__host__ __device__ constexpr int dw_g(const RecShape &r, int f, int k) { return r.G + 2 * f * r.G + k; }
__host__ __device__ constexpr int dw_cp(const RecShape &r, int f, int k) { return r.G + (2 * f + 1) * r.G + k; }
__host__ __device__ constexpr int dw_m(const RecShape &r, int f) { return 5 * r.G + 3 * f; }  // m_x, m_y, u.m
__host__ __device__ constexpr int dw_coef(const RecShape &r, int f) { return r.G + f; }      // species
// staging element of word W of section sec (0 common, 1 forward, 2 backward) of cell p
__host__ __device__ constexpr long st_idx(const RecShape &r, long N, int sec, int W, long p) {
  return (p * (r.QC + 2 * r.QD) + (sec == 0 ? 0 : sec == 1 ? r.QC : r.QC + r.QD)) * r.GW + W;
}
__host__ __device__ constexpr long st_words(const RecShape &r, long N) { return long(r.QC + 2 * r.QD) * N * r.GW; }

// strip geometry of one part
struct GroupMap {
  int G, C, NSTEP, nstrip, Lw;
  long nblk;
  // backward results dQ, step-blocked [blk][G C], lane (c, k) at k C + c
  __host__ __device__ long res(long blk, int c, int k) const { return blk * Lw + k * C + c; }
};
__host__ __device__ inline GroupMap group_map(int ni, int nj, int G) {
  GroupMap m;
  m.G = G;
  m.C = 64 / G;
  m.NSTEP = nj + m.C - 1;
  m.nstrip = (ni + m.C - 1) / m.C;
  m.Lw = m.C * G;
  m.nblk = long(m.nstrip) * m.NSTEP;
  return m;
}
// block and column of cell (i, j): block s NSTEP + d, d = j + c
__host__ __device__ inline long group_blk(const GroupMap &m, int i, int j, int &c) {
  const int s = i / m.C;
  c = i - s * m.C;
  return long(s) * m.NSTEP + j + c;
}

// ----------------------------------------------------------- cell kernel
// Residual R = sum_f F_f S_f - V S(Q), local time step, norms partials,
// chemistry and its Jacobian, the diagonal blocks (paper Section 2.2: I_m and
// the split-radius diagonals of Section 2.3) and their inverses, and the RHS.
// mode 0: coupled (nb x nb block in z = rho, momenta, energies, rho_1..rho_{ns-1})
// mode 1: split (flow block in closed form, ns x ns species block)
// Per-cell hand-off from the cell kernel to k_block (fields from HB_X on,
// [field][N]): X_s = rho_s / M_s, dT/dq_c, dTv/dq_c for every stored variable
// (two temperatures only), Y_s.
template <int NS, int NT>
__device__ __forceinline__ void write_handoff(const Mech &m, const double *rs, const Prim<NS, NT> &P, double *diag,
                                              long N, int p) {
  constexpr int NV = Dims<NS, NT>::nv;
  double *hb = diag + size_t(HB_X) * N + p;
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    hb[size_t(s) * N] = rs[s] / m.M[s];
    hb[size_t(NS + 2 * NV + s) * N] = P.Y[s];
  }
#pragma unroll
  for (int c = 0; c < NV; ++c) {
    double dT, dTv;
    temp_derivs<NS, NT>(P, c, dT, dTv);
    hb[size_t(NS + c) * N] = dT;
    if (NT == 2) hb[size_t(NS + NV + c) * N] = dTv;  // one temperature: Tv is T, its row unused
  }
}

// The hand-off alone, for cells 0..n-1 of the state (training samples of the
// block kernel's species Jacobian)
template <int NS, int NT>
__global__ void __launch_bounds__(256) k_handoff(Geo g, const Mech *__restrict__ mech, const double *__restrict__ Q,
                                                 const double *__restrict__ prim, int n, double *__restrict__ diag,
                                                 SampleMap sm) {
  constexpr int NV = Dims<NS, NT>::nv;
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  const int p = int(sm(r, g.N));
  const Mech &m = *mech;
  const size_t NP = g.NP;
  const int pc = padc(g, p % g.ni, p / g.ni);
  double q[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) q[k] = Q[size_t(k) * g.N + p];
  Prim<NS, NT> P;
  prim_from_q<NS, NT>(m, q, P, prim[F_T * NP + pc], prim[F_TV * NP + pc]);
  write_handoff<NS, NT>(m, q, P, diag, g.N, p);
}

struct CellOut {
  double *R, *dtau, *part;     // part: per-block norm partials [2][nblocks]
  void *Dinv;                  // coupled: nb*nb fields; split: DF 6 fields then DC ns*ns fields
  void *b;                     // RHS, nsol fields
  void *gS[2];                 // group schedule: record staging of part 0 (coupled / flow) and 1 (species)
  double *src;                 // optional source vector [nv][N] (debug)
  int *bad;
  int group_c;                 // 0: hyperplane schedule (cell-major records); > 0: group schedule
  double *diag;                // ns >= BLOCK_NS_MIN: [hb_fields][N] hand-off to k_block
  const float *Jsur;           // surrogate J_C [ns * ns][N] (flags bit 4)
  unsigned long long *ddfail;  // count of cells whose surrogate block failed the dominance check
  const int *surr_off;         // >= 0: surrogate switched off (stall), use the exact block
  // dual time stepping: physical-time levels and pt_a = (1 + theta) / dt,
  // pt_b = theta / dt (pt_a = 0: steady)
  const double *qn, *qnm1;
  double pt_a, pt_b;
};

// SRC_BLOCK (one temperature, ns >= BLOCK_NS_MIN, residual and diagonal in
// one pass): the chemical source of R is added by the block kernel from its
// reaction records, so this kernel forms the flux part only
// MODE: the form when fixed at compile time (0 coupled, 1 split), -1: the
// `mode` argument
template <int NS, int NT, typename RT, bool SRC_BLOCK, int MODE = -1>
__global__ void __launch_bounds__(256) k_cell(Geo g, const Mech *__restrict__ mech, const double *__restrict__ Q,
                                              const double *__restrict__ prim, const double *__restrict__ Fi,
                                              const double *__restrict__ Fj, const double *__restrict__ Ri,
                                              const double *__restrict__ Rj, double cfl, int mode, int flags,
                                              CellOut out, const int *__restrict__ done) {
  using D = Dims<NS, NT>;
  if (MODE >= 0) mode = MODE;
  constexpr int NV = D::nv, NB = D::nb, NF = D::nf;
  if (done && *done) return;
  __shared__ double red[2][256];
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  double nr2 = 0.0, ne2 = 0.0;
  if (p < g.N) {
    const Mech &m = *mech;
    const size_t NP = g.NP;
    int i = p % g.ni, j = p / g.ni;
    int pc = padc(g, i, j);
    int nfi = (g.ni + 1) * g.nj, nfj = g.ni * (g.nj + 1);
    int fW = j * (g.ni + 1) + i, fE = fW + 1, fS = j * g.ni + i, fN = fS + g.ni;
    double SW = g.fi_S[fW], SE = g.fi_S[fE], SS = g.fj_S[fS], SN = g.fj_S[fN];
    double Vp = g.V[p];
    double q[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) q[k] = Q[size_t(k) * g.N + p];
    double rs[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) rs[s] = q[s];
    double T = prim[F_T * NP + pc], Tv = prim[F_TV * NP + pc], pp = prim[F_P * NP + pc];
    Chem<NS, NT> C;
    const bool do_res = flags & 1, do_diag = flags & 2;
    // surrogate species block (split form): in 1T the exact J_C is only
    // needed by cells whose surrogate block fails the dominance check; in 2T
    // the flow block's omega_ve row needs the exact derivatives anyway
    constexpr bool BLK = NS >= BLOCK_NS_MIN;
    const bool try_sur = !BLK && do_diag && mode == 1 && (flags & 4) && out.Jsur && *out.surr_off < 0;
    bool have_jac = !BLK && do_diag && !(try_sur && NT == 1);
    if constexpr (SRC_BLOCK) {
#pragma unroll
      for (int s = 0; s < NS; ++s) C.w[s] = 0.0;
    } else {
      if (have_jac) chemistry<NS, NT, true>(m, rs, T, Tv, pp, C);
      else chemistry<NS, NT, false>(m, rs, T, Tv, pp, C);
    }
    double R[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      if (do_res) {
        double sv = k < NS ? C.w[k] : (NT == 2 && k == NS + 3 ? C.wv : 0.0);
        R[k] = Fi[size_t(k) * nfi + fE] * SE - Fi[size_t(k) * nfi + fW] * SW + Fj[size_t(k) * nfj + fN] * SN -
               Fj[size_t(k) * nfj + fS] * SS - Vp * sv;
        // dual time stepping (Section 2.2): the unsteady residual adds
        // V [(1 + theta)(Q - Q^n) - theta (Q^n - Q^{n-1})] / dt
        if (out.pt_a != 0.0) {
          const double qnk = out.qn[size_t(k) * g.N + p], qmk = out.qnm1[size_t(k) * g.N + p];
          R[k] += Vp * (out.pt_a * (q[k] - qnk) - out.pt_b * (qnk - qmk));
        }
        out.R[size_t(k) * g.N + p] = R[k];
        if (out.src) out.src[size_t(k) * g.N + p] = sv;
      } else {
        R[k] = out.R[size_t(k) * g.N + p];
      }
    }
    double slam = Ri[size_t(R_LAM) * nfi + fW] * SW + Ri[size_t(R_LAM) * nfi + fE] * SE +
                  Rj[size_t(R_LAM) * nfj + fS] * SS + Rj[size_t(R_LAM) * nfj + fN] * SN;
    double sU = Ri[size_t(R_UABS) * nfi + fW] * SW + Ri[size_t(R_UABS) * nfi + fE] * SE +
                Rj[size_t(R_UABS) * nfj + fS] * SS + Rj[size_t(R_UABS) * nfj + fN] * SN;
    double svF = Ri[size_t(R_LVF) * nfi + fW] * SW + Ri[size_t(R_LVF) * nfi + fE] * SE +
                 Rj[size_t(R_LVF) * nfj + fS] * SS + Rj[size_t(R_LVF) * nfj + fN] * SN;
    double svC = Ri[size_t(R_LVC) * nfi + fW] * SW + Ri[size_t(R_LVC) * nfi + fE] * SE +
                 Rj[size_t(R_LVC) * nfj + fS] * SS + Rj[size_t(R_LVC) * nfj + fN] * SN;
    double svK = Ri[size_t(R_LVK) * nfi + fW] * SW + Ri[size_t(R_LVK) * nfi + fE] * SE +
                 Rj[size_t(R_LVK) * nfj + fS] * SS + Rj[size_t(R_LVK) * nfj + fN] * SN;
    double dt;
    if (do_res) {
      dt = cfl * Vp / (0.5 * (slam + svK));
      out.dtau[p] = dt;
      double rr = 0.0;
#pragma unroll
      for (int s = 0; s < NS; ++s) rr += R[s];
      rr /= Vp;
      double re_ = R[NS + 2] / Vp;
      nr2 = rr * rr;
      ne2 = re_ * re_;
    } else {
      dt = out.dtau[p];
    }
    if (!do_diag) goto reduce;
    {
    // temperature derivatives w.r.t. stored variables (recomputed from the state)
    Prim<NS, NT> P;
    prim_from_q<NS, NT>(m, q, P, T, Tv);  // T, Tv: k_prim's solution for this q
    if constexpr (BLK) write_handoff<NS, NT>(m, rs, P, out.diag, g.N, p);
    // pseudo-time and physical-time diagonal: V / dtau + (1 + theta) V / dt
    double Vdt = Vp / dt + Vp * out.pt_a;
    // hyperplane schedule: cell-major records (field f at f N + p)
    const bool grp = out.group_c > 0;
    RT *bb = reinterpret_cast<RT *>(out.b);
    RT *Dcm = reinterpret_cast<RT *>(out.Dinv);
    // group schedule: E face = i-face (i+1, j), N face = j-face (i, j+1): outward
    // normals of the receiving neighbours are -n; W face (i, j), S face (i, j): +n
    const double SEh = 0.5 * SE, SNh = 0.5 * SN, SWh = 0.5 * SW, SSh = 0.5 * SS;
    // push fields of a part: normals, then radius coefficient c = S/2 lam + S lam_v
    // push data of a part (q: record array): per face E, N, W, S the outward
    // normal of the receiving cell scaled by S/2 (m), u.m and the radius
    // coefficient c = S/2 lam + S lam_v.  JVP parts (w: dp weights, ca: the
    // coefficient of a): cell fields (m_x, m_y, u.m) and per lane
    //   g_k = [k > 0] u.m - c,  cp_k = (0, m_x, m_y, u.m, 0, ...)_k;
    // species part: u.m - c per face.
    // partc: std::integral_constant of the part, so that the record shape,
    // and with it the per-lane loop below, is known at compile time (the
    // arrays w and ca then stay in registers)
    auto write_push = [&](int q, auto partc, int rv_lam, int rv_vis, const double *w, const double *ca) {
      RT *St = reinterpret_cast<RT *>(out.gS[q]);
      constexpr RecShape S = rec_shape(decltype(partc)::value, NS, NT, sizeof(RT));
      auto put = [&](int sec, int W, double v) { St[st_idx(S, g.N, sec, W, p)] = RT(v); };
      double mx[4], my[4], cf[4], un[4];
      mx[0] = -SEh * g.fi_nx[fE]; my[0] = -SEh * g.fi_ny[fE];
      cf[0] = SEh * Ri[size_t(rv_lam) * nfi + fE] + SE * Ri[size_t(rv_vis) * nfi + fE];
      mx[1] = -SNh * g.fj_nx[fN]; my[1] = -SNh * g.fj_ny[fN];
      cf[1] = SNh * Rj[size_t(rv_lam) * nfj + fN] + SN * Rj[size_t(rv_vis) * nfj + fN];
      mx[2] = SWh * g.fi_nx[fW]; my[2] = SWh * g.fi_ny[fW];
      cf[2] = SWh * Ri[size_t(rv_lam) * nfi + fW] + SW * Ri[size_t(rv_vis) * nfi + fW];
      mx[3] = SSh * g.fj_nx[fS]; my[3] = SSh * g.fj_ny[fS];
      cf[3] = SSh * Rj[size_t(rv_lam) * nfj + fS] + SS * Rj[size_t(rv_vis) * nfj + fS];
#pragma unroll
      for (int f = 0; f < 4; ++f) un[f] = P.u * mx[f] + P.v * my[f];
      // face f of the forward (f < 2) or backward section
      if (!w) {
#pragma unroll
        for (int f = 0; f < 4; ++f) put(1 + f / 2, dw_coef(S, f % 2), un[f] - cf[f]);
        return;
      }
#pragma unroll
      for (int f = 0; f < 4; ++f) {
        put(1 + f / 2, dw_m(S, f % 2), mx[f]);
        put(1 + f / 2, dw_m(S, f % 2) + 1, my[f]);
        put(1 + f / 2, dw_m(S, f % 2) + 2, un[f]);
      }
#pragma unroll
      for (int k = 0; k < S.G; ++k) {
        put(0, rw_w(S, k), w[k]);
        put(0, rw_ca(S, k), ca[k]);
#pragma unroll
        for (int f = 0; f < 4; ++f) {
          const double cp = k == 1 ? mx[f] : k == 2 ? my[f] : k == 3 ? un[f] : 0.0;
          put(1 + f / 2, dw_g(S, f % 2, k), (k > 0 ? un[f] : 0.0) - cf[f]);
          put(1 + f / 2, dw_cp(S, f % 2, k), cp);
        }
      }
    };
    if (mode == 0) {
      // coupled: dS_z/dz, z = (rho, m_x, m_y, rhoE, [rhoe_ve], rho_0..rho_{ns-2})
      // storage derivative of omega_s: dw/dq_j = dw_dr + dw_dT dT/dq_j + dw_dTv dTv/dq_j
      double dK = Vdt + 0.5 * slam + svK;
      double Ai[BLK ? 1 : NB][BLK ? 1 : NB];
      if constexpr (BLK) {
        out.diag[p] = dK;  // k_block assembles and inverts the block
      } else {
        double A[NB][NB];
        {
          double Jz[NB][NB];
          coupled_source_jacobian<NS, NT>(P, C, Jz);
#pragma unroll
          for (int r = 0; r < NB; ++r)
#pragma unroll
            for (int c = 0; c < NB; ++c) A[r][c] = (r == c ? dK : 0.0) - Vp * Jz[r][c];
        }
        bool ok = invert<NB>(A, Ai);
        if (!ok && out.bad) atomicMin(out.bad, p);
      }
      double rsum = 0.0;
#pragma unroll
      for (int s = 0; s < NS; ++s) rsum += R[s];
      double bz[NB];
      bz[0] = -rsum;
      bz[1] = -R[NS];
      bz[2] = -R[NS + 1];
      bz[3] = -R[NS + 2];
      if (NT == 2) bz[4] = -R[NS + 3];
#pragma unroll
      for (int s = 0; s < NS - 1; ++s) bz[NF + s] = -R[s];
      if (!grp) {
#pragma unroll
        for (int r = 0; r < NB; ++r) {
          bb[long(r) * g.N + p] = RT(bz[r]);
          if constexpr (!BLK) {
#pragma unroll
            for (int c = 0; c < NB; ++c) Dcm[long(r * NB + c) * g.N + p] = RT(Ai[r][c]);
          }
        }
      } else {
        constexpr RecShape S = rec_shape(PART_COUPLED, NS, NT, sizeof(RT));
        RT *St = reinterpret_cast<RT *>(out.gS[0]);
        // coefficient of a = dmn - un x_0 in each JVP component, and the dp weights
        double ca[NB], w[NB];
        ca[0] = 0.0; ca[1] = P.u; ca[2] = P.v; ca[3] = P.H;
        if (NT == 2) ca[4] = P.eve;
        w[0] = P.pr[NS - 1]; w[1] = -P.pE * P.u; w[2] = -P.pE * P.v; w[3] = P.pE;
        if (NT == 2) w[4] = P.pv;
#pragma unroll
        for (int s = 0; s < NS - 1; ++s) {
          ca[NF + s] = P.Y[s];
          w[NF + s] = P.pr[s] - P.pr[NS - 1];
        }
#pragma unroll
        for (int r = 0; r < NB; ++r) {
          St[st_idx(S, g.N, 1, dw_b(r), p)] = RT(bz[r]);
          if constexpr (!BLK) {
#pragma unroll
            for (int c = 0; c < NB; ++c) St[st_idx(S, g.N, 0, rw_d(S, r, c), p)] = RT(Ai[r][c]);
          }
        }
        write_push(0, std::integral_constant<int, PART_COUPLED>{}, R_LAM, R_LVK, w, ca);
      }
    } else {
      double dF = Vdt + 0.5 * slam + svF;
      double dC = Vdt + 0.5 * sU + svC;
      // flow block: scalar rows, plus the rho e_ve row -V d omega_ve/dQ_F (frozen Y)
      double df6[6];
      df6[0] = 1.0 / dF;
      for (int k = 1; k < 6; ++k) df6[k] = 0.0;
      if (BLK) {
        out.diag[p] = dF;  // k_block builds both blocks' inverses
        out.diag[g.N + p] = dC;
      } else if (NT == 2) {
        double dwv[5];
        flow_source_row<NS, NT>(P, C, dwv);
        // x4 = (r4 + V sum_{j<4} dwv_j x_j) / (dF - V dwv_4)
        for (int k = 0; k < 4; ++k) df6[1 + k] = Vp * dwv[k];
        double piv = dF - Vp * dwv[4];
        if (piv == 0.0 && out.bad) atomicMin(out.bad, p);
        df6[5] = 1.0 / piv;
      }
      double A[BLK ? 1 : NS][BLK ? 1 : NS], Ai[BLK ? 1 : NS][BLK ? 1 : NS];
      bool use_sur = false, ok = BLK;
      if constexpr (!BLK) {
      if (try_sur) {
        // surrogate J_C, accepted when D_C = dC I - V J_C is strictly row
        // diagonally dominant with a positive diagonal in molar units
        // (rows and columns scaled to concentrations rho_s / M_s):
        //   D_rr M_r > sum_{c != r} |D_rc| M_c
        bool dd = true;
#pragma unroll
        for (int r = 0; r < NS; ++r) {
          double off = 0.0;
#pragma unroll
          for (int c = 0; c < NS; ++c) {
            A[r][c] = (r == c ? dC : 0.0) - Vp * double(out.Jsur[size_t(r * NS + c) * g.N + p]);
            if (c != r) off += fabs(A[r][c]) * m.M[c];
          }
          dd = dd && A[r][r] > 0.0 && A[r][r] * m.M[r] > off;
        }
        if (dd) ok = invert<NS>(A, Ai);
        use_sur = dd && ok;
        if (!use_sur) {
          atomicAdd(out.ddfail, 1ull);
          if (!have_jac) chemistry<NS, NT, true>(m, rs, T, Tv, pp, C);
        }
      }
      if (!use_sur) {
        // flags bit 3: temperatures following the composition at fixed
        // velocities and internal energy densities
        double dTc[NS], dTvc[NS];
#pragma unroll
        for (int c = 0; c < NS; ++c) {
          dTc[c] = 0.0;
          dTvc[c] = 0.0;
          if (flags & 8) temp_derivs_fixed_e<NS, NT>(m, P, c, (flags & 16) != 0, dTc[c], dTvc[c]);
        }
#pragma unroll
        for (int r = 0; r < NS; ++r)
#pragma unroll
          for (int c = 0; c < NS; ++c)
            A[r][c] = (r == c ? dC : 0.0) - Vp * (C.dw_dr[r][c] + C.dw_dT[r] * dTc[c] + C.dw_dTv[r] * dTvc[c]);
        ok = invert<NS>(A, Ai);
      }
      }
      if (!ok && out.bad) atomicMin(out.bad, p);
      double rsum = 0.0;
#pragma unroll
      for (int s = 0; s < NS; ++s) rsum += R[s];
      double bf[NF];
      bf[0] = -rsum;
      bf[1] = -R[NS];
      bf[2] = -R[NS + 1];
      bf[3] = -R[NS + 2];
      if (NT == 2) bf[4] = -R[NS + 3];
      if (!grp) {
        if constexpr (!BLK) {
#pragma unroll
          for (int k = 0; k < 6; ++k) Dcm[long(k) * g.N + p] = RT(df6[k]);
#pragma unroll
          for (int r = 0; r < NS; ++r)
#pragma unroll
            for (int c = 0; c < NS; ++c) Dcm[long(6 + r * NS + c) * g.N + p] = RT(Ai[r][c]);
        }
#pragma unroll
        for (int k = 0; k < NF; ++k) bb[long(k) * g.N + p] = RT(bf[k]);
#pragma unroll
        for (int s = 0; s < NS; ++s) bb[long(NF + s) * g.N + p] = RT(-R[s]);
      } else {
        // flow part: its inverse written as a dense nf x nf block
        {
          constexpr RecShape S = rec_shape(PART_FLOW, NS, NT, sizeof(RT));
          RT *St = reinterpret_cast<RT *>(out.gS[0]);
          double prY = 0.0;
#pragma unroll
          for (int s = 0; s < NS; ++s) prY += P.pr[s] * P.Y[s];
          double ca[NF], w[NF], Df[NF][NF];
          ca[0] = 0.0; ca[1] = P.u; ca[2] = P.v; ca[3] = P.H;
          w[0] = prY; w[1] = -P.pE * P.u; w[2] = -P.pE * P.v; w[3] = P.pE;
#pragma unroll
          for (int r = 0; r < NF; ++r)
#pragma unroll
            for (int c = 0; c < NF; ++c) Df[r][c] = (r == c && r < 4) ? df6[0] : 0.0;
          if (NT == 2) {
            ca[4] = P.eve;
            w[4] = P.pv;
            for (int c = 0; c < 4; ++c) Df[4][c] = df6[1 + c] * df6[0] * df6[5];
            Df[4][4] = df6[5];
          }
#pragma unroll
          for (int r = 0; r < NF; ++r) {
            St[st_idx(S, g.N, 1, dw_b(r), p)] = RT(bf[r]);
            if constexpr (!BLK) {
#pragma unroll
              for (int c = 0; c < NF; ++c) St[st_idx(S, g.N, 0, rw_d(S, r, c), p)] = RT(Df[r][c]);
            }
          }
          write_push(0, std::integral_constant<int, PART_FLOW>{}, R_LAM, R_LVF, w, ca);
        }
        // species part
        {
          constexpr RecShape S = rec_shape(PART_SPECIES, NS, NT, sizeof(RT));
          RT *St = reinterpret_cast<RT *>(out.gS[1]);
#pragma unroll
          for (int r = 0; r < NS; ++r) {
            St[st_idx(S, g.N, 1, dw_b(r), p)] = RT(-R[r]);
            if constexpr (!BLK) {
#pragma unroll
              for (int c = 0; c < NS; ++c) St[st_idx(S, g.N, 0, rw_d(S, r, c), p)] = RT(Ai[r][c]);
            }
          }
          write_push(1, std::integral_constant<int, PART_SPECIES>{}, R_UABS, R_LVC, nullptr, nullptr);
        }
      }
    }
    }
  }
reduce:
  if (!(flags & 1)) return;
  // fixed-order block reduction of the norm partials
  red[0][threadIdx.x] = nr2;
  red[1][threadIdx.x] = ne2;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      red[0][threadIdx.x] += red[0][threadIdx.x + w];
      red[1][threadIdx.x] += red[1][threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out.part[blockIdx.x] = red[0][0];
    out.part[gridDim.x + blockIdx.x] = red[1][0];
  }
}

// Stall policy of the surrogate (surr_off non-null): once `window` iterations
// have run with it since iteration it_on, the first iteration whose density
// residual exceeds `ratio` times the one `window` iterations earlier switches
// it off for the rest of the run (*surr_off = that iteration).
struct StallArgs {
  int *surr_off;
  int it_on, window;
  double ratio;
};

// Final fixed-order reduction of the norm partials (one block); records the
// history and sets the stop flag once r/r0 <= tol.
template <int NS>
__global__ void __launch_bounds__(256) k_norms(const double *__restrict__ part, int nblk, double *__restrict__ norms,
                                               double *__restrict__ hist, int it, int hist_max, double *__restrict__ r0,
                                               double tol, int *__restrict__ done, int *__restrict__ it_done,
                                               StallArgs stall) {
  if (done && *done) return;
  __shared__ double red[2][256];
  double a = 0.0, b = 0.0;
  for (int k = threadIdx.x; k < nblk; k += 256) { a += part[k]; b += part[nblk + k]; }
  red[0][threadIdx.x] = a;
  red[1][threadIdx.x] = b;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      red[0][threadIdx.x] += red[0][threadIdx.x + w];
      red[1][threadIdx.x] += red[1][threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double nr = sqrt(red[0][0]), ne = sqrt(red[1][0]);
    norms[0] = nr;
    norms[1] = ne;
    if (hist && it < hist_max) { hist[2 * it] = nr; hist[2 * it + 1] = ne; }
    if (r0) {
      if (it == 0 || *r0 == 0.0) *r0 = nr;
      if (done && tol > 0.0 && nr <= tol * (*r0)) { *done = 1; if (it_done) *it_done = it; }
    }
    if (stall.surr_off && *stall.surr_off < 0 && hist && it - stall.it_on >= stall.window && it < hist_max &&
        it - stall.window >= 0 && nr > stall.ratio * hist[2 * (it - stall.window)])
      *stall.surr_off = it;
  }
}

}  // namespace csi
