// Species-generic kernels: one temperature, no reactions, any species count
// up to CSI_WIDE_MAX_SPECIES.  This is the configuration of the paper's
// species-count study (Section 3.1, time acceleration test: uniform
// non-reacting flow, the time of one implicit iteration of the coupled and
// component-split forms as the number of species grows).  The species count
// is a run-time value: per-cell vectors live in HBM and LDS instead of
// registers, and the work over species is spread over the threads of a
// workgroup (sweeps, block inversion) or looped by one thread (primitives,
// faces, residual, corrections).  Equations, field layouts and operation
// order follow the compiled kernels, so both give the same numbers to
// rounding where both apply.
//
// Coupled form: the dense (nb x nb) diagonal block is assembled per cell and
// inverted by a blocked Gauss-Jordan elimination (panels of WGJ_B columns,
// partial pivoting); the sweeps apply the inverse as a dense product.  With
// no reactions its content is (V/dtau + radii) I, but the coupled method
// treats it as the general block it is in reacting or two-temperature flow,
// and that is what its cost measures.  Split form: the flow block is the
// scalar diagonal and the species block (V/dtau + species radii) I minus V
// times a zero source Jacobian, both applied as scalars.
#pragma once
#include "csi_kernels.hpp"

namespace csi {

constexpr int WGJ_B = 64;  // Gauss-Jordan panel width

// e_ve,s and cv_ve,s at T (the same operations as eve_cvve_s)
__device__ __forceinline__ void w_eve_cv(const WMech &m, int s, double T, double &e, double &cv) {
  const int k = m.kind[s];
  if (k == MOLECULE && m.thv[s] > 0.0) {
    const double R = m.R[s], th = m.thv[s];
    const double x = th / T, em = exp(-x), d = 1.0 - em;
    e = R * th * em / d;
    cv = R * x * x * em / (d * d);
  } else if (k == ELECTRON) {
    e = 1.5 * m.R[s] * T;
    cv = 1.5 * m.R[s];
  } else {
    e = 0.0;
    cv = 0.0;
  }
}
__device__ __forceinline__ double w_eve(const WMech &m, int s, double T) {
  const int k = m.kind[s];
  return k == MOLECULE ? evib(m.R[s], m.thv[s], T) : (k == ELECTRON ? 1.5 * m.R[s] * T : 0.0);
}
__device__ __forceinline__ double w_cvve(const WMech &m, int s, double T) {
  const int k = m.kind[s];
  return k == MOLECULE ? cvvib(m.R[s], m.thv[s], T) : (k == ELECTRON ? 1.5 * m.R[s] : 0.0);
}

// -------------------------------------------------------------- reductions
// sum over the 256 threads of a workgroup (every thread gets the result);
// sh: 8 doubles of LDS
__device__ __forceinline__ double wg_sum(double v, double *sh) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[w] = v;
  __syncthreads();
  return (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

// --------------------------------------------------------------- primitives
// One thread per padded cell, as k_prim (ghosts: wall mirror, far field,
// zero-gradient outflow, or all far field in bc_mode 1).
__global__ void __launch_bounds__(256) kw_prim(Geo g, WMech m, const double *__restrict__ Q,
                                               const double *__restrict__ qfs, double *__restrict__ prim,
                                               int *__restrict__ bad, const int *__restrict__ done, int guess) {
  if (done && *done) return;
  const int pc = blockIdx.x * blockDim.x + threadIdx.x;
  if (pc >= g.NP) return;
  const int ns = m.ns;
  const WF PFw(ns);
  const int i = pc % (g.ni + 2) - 1, j = pc / (g.ni + 2) - 1;
  const bool interior = i >= 0 && i < g.ni && j >= 0 && j < g.nj;
  const int si = i < 0 ? 0 : (i >= g.ni ? g.ni - 1 : i);
  bool use_fs = false, mirror = false;
  if (!interior) {
    if (g.bc_mode == 1) use_fs = true;
    else if (j >= g.nj) use_fs = true;
    else if (j < 0) mirror = true;
  }
  const double *src;
  size_t str;
  if (use_fs) {
    src = qfs;
    str = 1;
  } else {
    const int sj = j < 0 ? 0 : j;
    src = Q + size_t(sj) * g.ni + si;
    str = size_t(g.N);
  }
  auto qk = [&](int k) { return src[size_t(k) * str]; };
  double rho = 0.0;
  for (int s = 0; s < ns; ++s) rho += qk(s);
  if (!(rho > 0.0)) {
    if (interior && bad) atomicMin(bad, j * g.ni + i);
    return;
  }
  double u = qk(ns) / rho, v = qk(ns + 1) / rho;
  const double rE = qk(ns + 2);
  const double k2 = u * u + v * v;
  const double ekin = 0.5 * rho * k2;
  const double target = rE - ekin;
  auto f = [&](double T, double &fv, double &dv, double &fa) {
    fv = -target;
    dv = 0.0;
    fa = fabs(target);
    for (int s = 0; s < ns; ++s) {
      const double rs = qk(s);
      double ev, cv;
      w_eve_cv(m, s, T, ev, cv);
      const double es = rs * (m.cvtr[s] * T + ev + m.hf[s]);
      fv += es;
      fa += fabs(es);
      dv += rs * (m.cvtr[s] + cv);
    }
  };
  const double T0 = guess ? prim[size_t(F_T) * g.NP + pc] : 0.0;
  double T = T0 > 0.0 ? T0 : 1000.0;
  if (!(T0 > 0.0 && newton_from(f, T))) {
    T = T0 > 0.0 ? T0 : 1000.0;
    if (!newton_bracket(f, T, 1.0, 1.0e6)) {
      if (interior && bad) atomicMin(bad, j * g.ni + i);
      return;
    }
  }
  double rcv = 0.0, rR = 0.0;
  for (int s = 0; s < ns; ++s) {
    const double rs = qk(s);
    double ev, cv;
    w_eve_cv(m, s, T, ev, cv);
    rcv += rs * (m.cvtr[s] + cv);
    rR += rs * m.R[s];
  }
  const double p = rR * T, beta = rR / rcv;
  const double H = (rE + p) / rho;
  double c2 = u * (-beta * u) + v * (-beta * v) + H * beta;
  // transport sums and the per-species fields
  double ktr = 0.0, kint = 0.0, cvtr = 0.0, cvint = 0.0;
  const size_t NP = g.NP;
  double *o = prim + pc;
  for (int s = 0; s < ns; ++s) {
    const double rs = qk(s);
    const double Y = rs / rho;
    double ev, cv;
    w_eve_cv(m, s, T, ev, cv);
    const double es = m.cvtr[s] * T + ev + m.hf[s];
    const double dT_dr = (0.5 * k2 - es) / rcv;
    const double pr = m.R[s] * T + rR * dT_dr;
    c2 += Y * pr;
    ktr += Y * m.ck[s];
    const double cve = w_cvve(m, s, T);
    kint += Y * cve;
    cvtr += Y * m.cvtr[s];
    cvint += Y * cve;
    const double eve = w_eve(m, s, T);
    o[size_t(PFw.Y + s) * NP] = Y;
    o[size_t(PFw.HS + s) * NP] = m.cvtr[s] * T + eve + m.hf[s] + m.R[s] * T;
    o[size_t(PFw.EVS + s) * NP] = eve;
    o[size_t(PFw.PR + s) * NP] = pr;
  }
  if (!(c2 > 0.0) || !(p > 0.0)) {
    if (interior && bad) atomicMin(bad, j * g.ni + i);
    return;
  }
  const double mu = m.mu_ref * exp(m.mu_exp * log(T / m.T_ref));
  const double kc = mu * (ktr + kint);
  const double nuF = fmax(4.0 * mu / (3.0 * rho), kc / (rho * (cvtr + cvint)));
  const double nuC = mu * m.iscmax / rho;
  if (mirror) {
    const int fw = si;  // wall face (si, 0)
    const double nx = g.fj_nx[fw], ny = g.fj_ny[fw];
    const double un = u * nx + v * ny;
    u = u - 2.0 * un * nx;
    v = v - 2.0 * un * ny;
  }
  o[F_RHO * NP] = rho; o[F_U * NP] = u; o[F_V * NP] = v; o[F_T * NP] = T; o[F_TV * NP] = T;
  o[F_P * NP] = p; o[F_C * NP] = sqrt(c2); o[F_H * NP] = H; o[F_EVE * NP] = 0.0; o[F_RE * NP] = rE;
  o[F_MU * NP] = mu; o[F_K * NP] = kc; o[F_KVE * NP] = 0.0; o[F_NUF * NP] = nuF; o[F_NUC * NP] = nuC;
  o[F_NUK * NP] = fmax(nuF, nuC); o[F_PE * NP] = beta; o[F_PV * NP] = 0.0;
}

// -------------------------------------------------------------------- faces
// value of a primitive field at grid node (I, J) (as node_value)
__device__ __forceinline__ double w_node(const Geo &g, const double *prim, int I, int J, int fld, int wall_kind) {
  const size_t NP = g.NP;
  if (g.bc_mode == 0 && J == 0) {
    if (wall_kind == 1) return 0.0;   // velocity
    if (wall_kind == 2) return g.Tw;  // temperature
    return 0.5 * (prim[fld * NP + padc(g, I - 1, 0)] + prim[fld * NP + padc(g, I, 0)]);
  }
  return 0.25 * (prim[fld * NP + padc(g, I - 1, J - 1)] + prim[fld * NP + padc(g, I, J - 1)] +
                 prim[fld * NP + padc(g, I - 1, J)] + prim[fld * NP + padc(g, I, J)]);
}

// One thread per face (JF: j-faces), as k_face_i / k_face_j: HLLE with
// upwinded species, face radii, viscous flux at interior faces, isothermal
// no-slip wall at J = 0 in bc_mode 0.
template <bool JF>
__global__ void __launch_bounds__(256) kw_face(Geo g, WMech m, const double *__restrict__ prim, double *__restrict__ Fo,
                                               double *__restrict__ Ro, double *__restrict__ qw,
                                               const int *__restrict__ done) {
  if (done && *done) return;
  const int ns = m.ns;
  const WF PFw(ns);
  const int nfc = JF ? g.ni * (g.nj + 1) : (g.ni + 1) * g.nj;
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= nfc) return;
  const size_t NP = g.NP;
  int pL, pR, cL = 0, cR = 0, cin, pIn, IA, JA, IB, JB;
  bool interior;
  double nx, ny, S;
  if (!JF) {
    const int I = f % (g.ni + 1), j = f / (g.ni + 1);
    pL = padc(g, I - 1, j);
    pR = padc(g, I, j);
    nx = g.fi_nx[f]; ny = g.fi_ny[f]; S = g.fi_S[f];
    interior = I > 0 && I < g.ni;
    cin = j * g.ni + (I == 0 ? 0 : g.ni - 1);
    pIn = padc(g, I == 0 ? 0 : g.ni - 1, j);
    if (interior) { cL = j * g.ni + I - 1; cR = j * g.ni + I; }
    IA = I; JA = j; IB = I; JB = j + 1;
  } else {
    const int i = f % g.ni, J = f / g.ni;
    pL = padc(g, i, J - 1);
    pR = padc(g, i, J);
    nx = g.fj_nx[f]; ny = g.fj_ny[f]; S = g.fj_S[f];
    interior = J > 0 && J < g.nj;
    cin = (J == 0 ? 0 : g.nj - 1) * g.ni + i;
    pIn = padc(g, i, J == 0 ? 0 : g.nj - 1);
    if (interior) { cL = (J - 1) * g.ni + i; cR = J * g.ni + i; }
    IA = i; JA = J; IB = i + 1; JB = J;
  }
  auto P = [&](int fld, int pc) { return prim[size_t(fld) * NP + pc]; };
  // HLLE (Davis bounds)
  const double rL = P(F_RHO, pL), uL = P(F_U, pL), vL = P(F_V, pL), prL = P(F_P, pL), cLs = P(F_C, pL), EL = P(F_RE, pL);
  const double rR = P(F_RHO, pR), uR = P(F_U, pR), vR = P(F_V, pR), prR = P(F_P, pR), cRs = P(F_C, pR), ER = P(F_RE, pR);
  const double unL = uL * nx + vL * ny, unR = uR * nx + vR * ny;
  const double SL = fmin(unL - cLs, unR - cRs), SR = fmax(unL + cLs, unR + cRs);
  const double sl = fmin(SL, 0.0), sr = fmax(SR, 0.0);
  const double id = 1.0 / (sr - sl);
  auto hll = [&](double fl, double fr, double ql, double qr) { return (sr * fl - sl * fr + sr * sl * (qr - ql)) * id; };
  const double fm = hll(rL * unL, rR * unR, rL, rR);
  const int pU = fm >= 0.0 ? pL : pR;
  const double mxL = rL * uL, myL = rL * vL, mxR = rR * uR, myR = rR * vR;
  double F0 = hll(mxL * unL + prL * nx, mxR * unR + prR * nx, mxL, mxR);
  double F1 = hll(myL * unL + prL * ny, myR * unR + prR * ny, myL, myR);
  double F2 = hll((EL + prL) * unL, (ER + prR) * unR, EL, ER);
  // face radii
  {
    const double U = 0.5 * ((P(F_U, pL) + P(F_U, pR)) * nx + (P(F_V, pL) + P(F_V, pR)) * ny);
    double nF, nC, nK, Vf;
    if (interior) {
      nF = 0.5 * (P(F_NUF, pL) + P(F_NUF, pR));
      nC = 0.5 * (P(F_NUC, pL) + P(F_NUC, pR));
      nK = 0.5 * (P(F_NUK, pL) + P(F_NUK, pR));
      Vf = 0.5 * (g.V[cL] + g.V[cR]);
    } else {
      nF = P(F_NUF, pIn);
      nC = P(F_NUC, pIn);
      nK = P(F_NUK, pIn);
      Vf = g.V[cin];
    }
    Ro[size_t(R_UABS) * nfc + f] = fabs(U);
    Ro[size_t(R_LAM) * nfc + f] = fabs(U) + 0.5 * (P(F_C, pL) + P(F_C, pR));
    Ro[size_t(R_LVF) * nfc + f] = nF * S / Vf;
    Ro[size_t(R_LVC) * nfc + f] = nC * S / Vf;
    Ro[size_t(R_LVK) * nfc + f] = nK * S / Vf;
  }
  if (interior) {
    // diamond gradients (cell centres L, R and nodes A, B)
    const double d1x = g.xc[cR] - g.xc[cL], d1y = g.yc[cR] - g.yc[cL];
    const int nA = JA * (g.ni + 1) + IA, nB = JB * (g.ni + 1) + IB;
    const double d2x = g.xn[nB] - g.xn[nA], d2y = g.yn[nB] - g.yn[nA];
    auto grad = [&](int fld, int wall_kind, double &gx, double &gy) {
      const double D1 = P(fld, pR) - P(fld, pL);
      const double D2 = w_node(g, prim, IB, JB, fld, wall_kind) - w_node(g, prim, IA, JA, fld, wall_kind);
      diamond_grad(d1x, d1y, d2x, d2y, D1, D2, gx, gy);
    };
    double gu[2], gv[2], gT[2], gTv[2];
    grad(F_U, 1, gu[0], gu[1]);
    grad(F_V, 1, gv[0], gv[1]);
    grad(F_T, 2, gT[0], gT[1]);
    grad(F_TV, 2, gTv[0], gTv[1]);
    auto avg = [&](int fld) { return 0.5 * (P(fld, pL) + P(fld, pR)); };
    const double mu = avg(F_MU), k = avg(F_K), kve = avg(F_KVE), u = avg(F_U), v = avg(F_V);
    const double div = gu[0] + gv[1];
    const double txx = mu * (2.0 * gu[0] - 2.0 / 3.0 * div);
    const double tyy = mu * (2.0 * gv[1] - 2.0 / 3.0 * div);
    const double txy = mu * (gu[1] + gv[0]);
    const double muL = P(F_MU, pL), muR = P(F_MU, pR);
    double Jcx = 0.0, Jcy = 0.0;
    for (int s = 0; s < ns; ++s) {
      const double rD = 0.5 * (muL * m.iSc[s] + muR * m.iSc[s]);
      double gx, gy;
      grad(PFw.Y + s, 0, gx, gy);
      Jcx += rD * gx;
      Jcy += rD * gy;
    }
    double hJ = 0.0;
    for (int s = 0; s < ns; ++s) {
      const double rD = 0.5 * (muL * m.iSc[s] + muR * m.iSc[s]);
      double gx, gy;
      grad(PFw.Y + s, 0, gx, gy);
      const double Yf = avg(PFw.Y + s);
      const double jx = -rD * gx + Yf * Jcx;
      const double jy = -rD * gy + Yf * Jcy;
      const double jn = jx * nx + jy * ny;
      Fo[size_t(s) * nfc + f] = fm * P(PFw.Y + s, pU) + jn;
      hJ += avg(PFw.HS + s) * jn;
    }
    const double tnx = txx * nx + txy * ny, tny = txy * nx + tyy * ny;
    const double qtr = -k * (gT[0] * nx + gT[1] * ny);
    const double qve = -kve * (gTv[0] * nx + gTv[1] * ny);
    F0 += -tnx;
    F1 += -tny;
    F2 += -(u * tnx + v * tny) + qtr + qve + hJ;
  } else {
    for (int s = 0; s < ns; ++s) Fo[size_t(s) * nfc + f] = fm * P(PFw.Y + s, pU);
    if (JF && f < g.ni && g.bc_mode == 0) {
      // isothermal no-slip non-catalytic wall (face (i, 0))
      const int i = f, c0 = i;
      const double muw = m.mu_ref * exp(m.mu_exp * log(g.Tw / m.T_ref));
      double ktr = 0.0, kint = 0.0;
      for (int s = 0; s < ns; ++s) {
        const double Y = P(PFw.Y + s, pR);
        ktr += Y * m.ck[s];
        kint += Y * w_cvve(m, s, g.Tw);
      }
      const double kw = muw * (ktr + kint);
      const double kvw = 0.0;
      const int nA = i, nB = i + 1;
      const double xf = 0.5 * (g.xn[nA] + g.xn[nB]), yf = 0.5 * (g.yn[nA] + g.yn[nB]);
      const double d1x = g.xc[c0] - xf, d1y = g.yc[c0] - yf;
      const double d2x = g.xn[nB] - g.xn[nA], d2y = g.yn[nB] - g.yn[nA];
      double gu[2], gv[2], gT[2], gTv[2];
      diamond_grad(d1x, d1y, d2x, d2y, P(F_U, pR), 0.0, gu[0], gu[1]);
      diamond_grad(d1x, d1y, d2x, d2y, P(F_V, pR), 0.0, gv[0], gv[1]);
      diamond_grad(d1x, d1y, d2x, d2y, P(F_T, pR) - g.Tw, 0.0, gT[0], gT[1]);
      diamond_grad(d1x, d1y, d2x, d2y, P(F_TV, pR) - g.Tw, 0.0, gTv[0], gTv[1]);
      const double div = gu[0] + gv[1];
      const double txx = muw * (2.0 * gu[0] - 2.0 / 3.0 * div);
      const double tyy = muw * (2.0 * gv[1] - 2.0 / 3.0 * div);
      const double txy = muw * (gu[1] + gv[0]);
      const double tnx = txx * nx + txy * ny, tny = txy * nx + tyy * ny;
      const double qtr = -kw * (gT[0] * nx + gT[1] * ny);
      const double qve = -kvw * (gTv[0] * nx + gTv[1] * ny);
      F0 += -tnx;
      F1 += -tny;
      F2 += qtr + qve;
      qw[i] = -(qtr + qve);
    }
  }
  Fo[size_t(ns) * nfc + f] = F0;
  Fo[size_t(ns + 1) * nfc + f] = F1;
  Fo[size_t(ns + 2) * nfc + f] = F2;
}

// --------------------------------------------------------------------- cell
struct WCellOut {
  double *R, *dtau, *part;
  double *diag;   // coupled: dK per cell (the block assembly reads it)
  double *Dinv;   // split: [2][N] = 1/dF, 1/dC
  double *b;      // right-hand side [nsol][N]
};

// One thread per cell, as k_cell: flags bit 0 the residual, its norms and
// dtau; bit 1 the diagonal terms and the right-hand side of mode.
__global__ void __launch_bounds__(256) kw_cell(Geo g, int ns, const double *__restrict__ Fi,
                                               const double *__restrict__ Fj, const double *__restrict__ Ri,
                                               const double *__restrict__ Rj, double cfl, int mode, int flags,
                                               WCellOut out, const int *__restrict__ done) {
  if (done && *done) return;
  __shared__ double red[2][256];
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  double nr2 = 0.0, ne2 = 0.0;
  if (p < g.N) {
    const int nv = ns + 3;
    const int i = p % g.ni, j = p / g.ni;
    const int nfi = (g.ni + 1) * g.nj, nfj = g.ni * (g.nj + 1);
    const int fW = j * (g.ni + 1) + i, fE = fW + 1, fS = j * g.ni + i, fN = fS + g.ni;
    const double SW = g.fi_S[fW], SE = g.fi_S[fE], SS = g.fj_S[fS], SN = g.fj_S[fN];
    const double Vp = g.V[p];
    const bool do_res = flags & 1, do_diag = flags & 2;
    // R = sum of the face fluxes (no source without reactions)
    auto Rk = [&](int k) {
      return Fi[size_t(k) * nfi + fE] * SE - Fi[size_t(k) * nfi + fW] * SW + Fj[size_t(k) * nfj + fN] * SN -
             Fj[size_t(k) * nfj + fS] * SS - Vp * 0.0;
    };
    double rsum = 0.0;
    if (do_res) {
      for (int k = 0; k < nv; ++k) {
        const double r = Rk(k);
        out.R[size_t(k) * g.N + p] = r;
        if (k < ns) rsum += r;
      }
    } else {
      for (int s = 0; s < ns; ++s) rsum += out.R[size_t(s) * g.N + p];
    }
    auto face_sum = [&](int fld) {
      return Ri[size_t(fld) * nfi + fW] * SW + Ri[size_t(fld) * nfi + fE] * SE + Rj[size_t(fld) * nfj + fS] * SS +
             Rj[size_t(fld) * nfj + fN] * SN;
    };
    const double slam = face_sum(R_LAM), sU = face_sum(R_UABS), svF = face_sum(R_LVF), svC = face_sum(R_LVC),
                 svK = face_sum(R_LVK);
    double dt;
    if (do_res) {
      dt = cfl * Vp / (0.5 * (slam + svK));
      out.dtau[p] = dt;
      const double rr = rsum / Vp;
      const double re_ = out.R[size_t(ns + 2) * g.N + p] / Vp;
      nr2 = rr * rr;
      ne2 = re_ * re_;
    } else {
      dt = out.dtau[p];
    }
    if (do_diag) {
      const double Vdt = Vp / dt + Vp * 0.0;
      auto Rg = [&](int k) { return out.R[size_t(k) * g.N + p]; };
      if (mode == 0) {
        out.diag[p] = Vdt + 0.5 * slam + svK;
        // z = (rho, m_x, m_y, rhoE, rho_0..rho_{ns-2})
        out.b[p] = -rsum;
        out.b[size_t(g.N) + p] = -Rg(ns);
        out.b[size_t(2) * g.N + p] = -Rg(ns + 1);
        out.b[size_t(3) * g.N + p] = -Rg(ns + 2);
        for (int s = 0; s < ns - 1; ++s) out.b[size_t(4 + s) * g.N + p] = -Rg(s);
      } else {
        const double dF = Vdt + 0.5 * slam + svF;
        const double dC = Vdt + 0.5 * sU + svC;
        out.Dinv[p] = 1.0 / dF;
        out.Dinv[size_t(g.N) + p] = 1.0 / (dC - Vp * 0.0);
        out.b[p] = -rsum;
        out.b[size_t(g.N) + p] = -Rg(ns);
        out.b[size_t(2) * g.N + p] = -Rg(ns + 1);
        out.b[size_t(3) * g.N + p] = -Rg(ns + 2);
        for (int s = 0; s < ns; ++s) out.b[size_t(4 + s) * g.N + p] = -Rg(s);
      }
    }
  }
  if (!(flags & 1)) return;
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

// ------------------------------------------------- coupled block and inverse
// Dense coupled block per cell, cell-major [N][n][n] row-major: the pseudo-
// and physical-time diagonal and the radii, minus V times the source
// Jacobian (zero without reactions in one temperature).
__global__ void __launch_bounds__(256) kw_ci_assemble(const double *__restrict__ diag, const double *__restrict__ V,
                                                      int n, int N, double *__restrict__ W,
                                                      const int *__restrict__ done) {
  if (done && *done) return;
  const size_t nn = size_t(n) * n, tot = nn * N;
  for (size_t e = size_t(blockIdx.x) * blockDim.x + threadIdx.x; e < tot; e += size_t(gridDim.x) * blockDim.x) {
    const size_t p = e / nn, rc = e % nn;
    const size_t r = rc / n, c = rc % n;
    W[e] = (r == c ? diag[p] : 0.0) - V[p] * 0.0;
  }
}

// Blocked in-place Gauss-Jordan inversion with partial pivoting (largest
// |a| in the pivot column among the rows not yet used, lowest row on ties),
// one matrix per cell.  Per panel of nbk = min(WGJ_B, n - kb) columns:
//  (1) kw_gj_panel: the nbk elimination steps on the panel's columns (all
//      rows); the panel then holds, in the final row order, the inverse of
//      the pivot block (pivot rows) and minus the other rows times it;
//  (2) kw_gj_swap: the panel's row interchanges on every other column, and
//      a copy of the pivot rows there (XK);
//  (3) kw_gj_update: every other column x += T XK with T the panel minus
//      the identity on the pivot rows (the nbk steps at once);
// then kw_gj_unpermute: the column interchanges of the inverse.
__global__ void __launch_bounds__(256) kw_gj_panel(double *__restrict__ W, int n, int kb, int *__restrict__ perm,
                                                   int *__restrict__ sing, const int *__restrict__ done) {
  if (done && *done) return;
  extern __shared__ double wsh[];
  double *colk = wsh;                // [n]
  double *prow = wsh + n;            // [WGJ_B]
  __shared__ double bv[4];
  __shared__ int bi[4];
  const int p = blockIdx.x, tid = threadIdx.x;
  // update mapping: lane jj owns panel column jj, wave rg rows rg, rg + 4, ...
  const int jj = tid & 63, rg = tid >> 6;
  double *A = W + size_t(p) * n * n;
  const int nbk = min(WGJ_B, n - kb);
  constexpr int U = 8;  // rows per thread with their loads in flight together
  for (int jk = 0; jk < nbk; ++jk) {
    const int k = kb + jk;
    // pivot: largest |a| in column k among rows k..n-1, lowest row on ties
    double best = -1.0;
    int bidx = n;
    for (int r = k + tid; r < n; r += 256) {
      const double a = fabs(A[size_t(r) * n + k]);
      if (a > best) { best = a; bidx = r; }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const double ob = __shfl_xor(best, o, 64);
      const int oi = __shfl_xor(bidx, o, 64);
      if (ob > best || (ob == best && oi < bidx)) { best = ob; bidx = oi; }
    }
    if ((tid & 63) == 0) { bv[tid >> 6] = best; bi[tid >> 6] = bidx; }
    __syncthreads();
    best = bv[0];
    bidx = bi[0];
#pragma unroll
    for (int w = 1; w < 4; ++w)
      if (bv[w] > best || (bv[w] == best && bi[w] < bidx)) { best = bv[w]; bidx = bi[w]; }
    // (a column without a comparable entry, NaN throughout, keeps row k and
    // is reported singular)
    const int piv = bidx < n ? bidx : k;
    if (tid == 0) {
      perm[size_t(p) * n + k] = piv;
      if (!(best > 0.0) && sing) atomicMin(sing, p);
    }
    // interchange rows k and piv on the panel's columns
    if (piv != k && tid < nbk) {
      const double t = A[size_t(k) * n + kb + tid];
      A[size_t(k) * n + kb + tid] = A[size_t(piv) * n + kb + tid];
      A[size_t(piv) * n + kb + tid] = t;
    }
    __syncthreads();
    for (int r = tid; r < n; r += 256) colk[r] = A[size_t(r) * n + k];
    if (tid < nbk) prow[tid] = A[size_t(k) * n + kb + tid];
    __syncthreads();
    // the scaled pivot row replaces row k; every other row r takes
    // a_rc - a_rk (a_kc / a_kk), column k becoming -a_rk / a_kk
    if (jj < nbk) {
      const double ip = 1.0 / colk[k];
      const double prs = jj == jk ? ip : prow[jj] * ip;
      double *col = A + kb + jj;
      for (int r0 = rg; r0 < n; r0 += 4 * U) {
        double v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int r = r0 + 4 * u;
          v[u] = r < n ? col[size_t(r) * n] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int r = r0 + 4 * u;
          if (r < n) col[size_t(r) * n] = r == k ? prs : (jj == jk ? 0.0 : v[u]) - colk[r] * prs;
        }
      }
    }
    __syncthreads();
  }
}

// grid (cells, ceil(n / 256)): one thread per column outside the panel
__global__ void __launch_bounds__(256) kw_gj_swap(double *__restrict__ W, int n, int kb, const int *__restrict__ perm,
                                                  double *__restrict__ XK, const int *__restrict__ done) {
  if (done && *done) return;
  const int c = blockIdx.y * blockDim.x + threadIdx.x, p = blockIdx.x;
  const int nbk = min(WGJ_B, n - kb);
  if (c >= n || (c >= kb && c < kb + nbk)) return;
  double *A = W + size_t(p) * n * n;
  const int *pm = perm + size_t(p) * n;
  for (int jk = 0; jk < nbk; ++jk) {
    const int k = kb + jk, piv = pm[k];
    if (piv != k) {
      const double t = A[size_t(k) * n + c];
      A[size_t(k) * n + c] = A[size_t(piv) * n + c];
      A[size_t(piv) * n + c] = t;
    }
  }
  for (int jk = 0; jk < nbk; ++jk) XK[(size_t(p) * WGJ_B + jk) * n + c] = A[size_t(kb + jk) * n + c];
}

// grid (cells, ceil(n / 64) column tiles, ceil(n / 64) row tiles); 16 x 16
// threads, each with a 4 x 4 block of a 64 x 64 tile (rows ty + 16 a,
// columns tx + 16 b); the panel's columns taken WGJ_K at a time through LDS
constexpr int WGJ_K = 32;
__global__ void __launch_bounds__(256) kw_gj_update(double *__restrict__ W, int n, int kb,
                                                    const double *__restrict__ XK, const int *__restrict__ done) {
  if (done && *done) return;
  __shared__ double Ts[64][WGJ_K + 1];
  __shared__ double Xs[WGJ_K][64 + 1];
  const int p = blockIdx.x, c0 = blockIdx.y * 64, r0 = blockIdx.z * 64;
  const int nbk = min(WGJ_B, n - kb);
  // a tile wholly inside the panel has nothing to do
  if (c0 >= kb && c0 + 64 <= kb + nbk) return;
  double *A = W + size_t(p) * n * n;
  const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
  double acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
  for (int j0 = 0; j0 < nbk; j0 += WGJ_K) {
    const int kc = min(WGJ_K, nbk - j0);
    for (int e = tid; e < 64 * WGJ_K; e += 256) {
      const int rr = e / WGJ_K, jj = e - rr * WGJ_K;
      const int r = r0 + rr, col = j0 + jj;
      double t = 0.0;
      if (r < n && jj < kc) t = A[size_t(r) * n + kb + col] - (r == kb + col ? 1.0 : 0.0);
      Ts[rr][jj] = t;
    }
    for (int e = tid; e < WGJ_K * 64; e += 256) {
      const int jj = e >> 6, cc = e & 63;
      const int c = c0 + cc;
      Xs[jj][cc] = (jj < kc && c < n) ? XK[(size_t(p) * WGJ_B + j0 + jj) * n + c] : 0.0;
    }
    __syncthreads();
    for (int jj = 0; jj < kc; ++jj) {
      double tv[4], xv[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) tv[a] = Ts[ty + 16 * a][jj];
#pragma unroll
      for (int b = 0; b < 4; ++b) xv[b] = Xs[jj][tx + 16 * b];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = fma(tv[a], xv[b], acc[a][b]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const int r = r0 + ty + 16 * a;
    if (r >= n) continue;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int c = c0 + tx + 16 * b;
      if (c >= n || (c >= kb && c < kb + nbk)) continue;
      A[size_t(r) * n + c] += acc[a][b];
    }
  }
}

// grid (cells, ceil(n / 256)): one thread per row; the inverse's columns
// take the row interchanges in reverse order
__global__ void __launch_bounds__(256) kw_gj_unpermute(double *__restrict__ W, int n, const int *__restrict__ perm,
                                                       const int *__restrict__ done) {
  if (done && *done) return;
  const int r = blockIdx.y * blockDim.x + threadIdx.x, p = blockIdx.x;
  if (r >= n) return;
  double *A = W + size_t(p) * n * n + size_t(r) * n;
  const int *pm = perm + size_t(p) * n;
  for (int k = n - 1; k >= 0; --k) {
    const int piv = pm[k];
    if (piv != k) {
      const double t = A[k];
      A[k] = A[piv];
      A[piv] = t;
    }
  }
}

// ------------------------------------------------------------------- sweeps
struct WSweep {
  const double *prim, *Ri, *Rj;
  const double *Dinv;  // coupled: [N][nb][nb]; split: [2][N]
  const double *b;
  double *xs, *x;
  int mode, ns;
};

// r += sg * O_PN x_N (matrix-free off-diagonal term of neighbour N through
// face f, outward normal sgn_n n), as off_accumulate with the linear
// Jacobian-vector product; r in LDS, components spread over the threads
__device__ __forceinline__ void w_off(const Geo &g, const WSweep &a, int pcN, int cN, bool iface, int f, double sgn_n,
                                      double sg, const double *__restrict__ X, double *r, double *sh) {
  const int ns = a.ns, tid = threadIdx.x;
  const WF PFw(ns);
  const size_t NP = g.NP;
  const int nfc = iface ? (g.ni + 1) * g.nj : g.ni * (g.nj + 1);
  const double *Rr = iface ? a.Ri : a.Rj;
  const double nx = sgn_n * (iface ? g.fi_nx[f] : g.fj_nx[f]);
  const double ny = sgn_n * (iface ? g.fi_ny[f] : g.fj_ny[f]);
  const double S = iface ? g.fi_S[f] : g.fj_S[f];
  const double lam = Rr[size_t(R_LAM) * nfc + f];
  const double u = a.prim[F_U * NP + pcN], v = a.prim[F_V * NP + pcN], H = a.prim[F_H * NP + pcN];
  const double pE = a.prim[F_PE * NP + pcN];
  const double x0 = X[cN], x1 = X[size_t(g.N) + cN], x2 = X[size_t(2) * g.N + cN], x3 = X[size_t(3) * g.N + cN];
  const double un = u * nx + v * ny, dmn = x1 * nx + x2 * ny, am = dmn - un * x0;
  if (a.mode == 0) {
    // z = (rho, m_x, m_y, rhoE, rho_0..rho_{ns-2}); rho_{ns-1} = rho - sum
    double s1 = 0.0, s2 = 0.0;
    for (int k = tid; k < ns - 1; k += 256) {
      const double xk = X[size_t(4 + k) * g.N + cN];
      s1 += xk;
      s2 += a.prim[size_t(PFw.PR + k) * NP + pcN] * xk;
    }
    s1 = wg_sum(s1, sh);
    s2 = wg_sum(s2, sh);
    const double last = x0 - s1;
    const double dp = pE * (x3 - u * x1 - v * x2) + s2 + a.prim[size_t(PFw.PR + ns - 1) * NP + pcN] * last;
    const double lv = Rr[size_t(R_LVK) * nfc + f];
    auto acc = [&](int k, double o, double xk) { r[k] += sg * (0.5 * S * (o - lam * xk) - lv * S * xk); };
    if (tid == 0) {
      acc(0, dmn, x0);
      acc(1, un * x1 + u * am + nx * dp, x1);
      acc(2, un * x2 + v * am + ny * dp, x2);
      acc(3, un * (x3 + dp) + H * am, x3);
    }
    for (int k = tid; k < ns - 1; k += 256) {
      const double xk = X[size_t(4 + k) * g.N + cN];
      acc(4 + k, un * xk + a.prim[size_t(PFw.Y + k) * NP + pcN] * am, xk);
    }
  } else {
    // flow part at frozen mass fractions, species part as a scalar
    double prY = 0.0;
    for (int k = tid; k < ns; k += 256)
      prY += a.prim[size_t(PFw.PR + k) * NP + pcN] * a.prim[size_t(PFw.Y + k) * NP + pcN];
    prY = wg_sum(prY, sh);
    const double dp = prY * x0 + pE * (x3 - u * x1 - v * x2);
    const double lvF = Rr[size_t(R_LVF) * nfc + f];
    auto acc = [&](int k, double o, double xk) { r[k] += sg * (0.5 * S * (o - lam * xk) - lvF * S * xk); };
    if (tid == 0) {
      acc(0, dmn, x0);
      acc(1, un * x1 + u * am + nx * dp, x1);
      acc(2, un * x2 + v * am + ny * dp, x2);
      acc(3, un * (x3 + dp) + H * am, x3);
    }
    const double coef = 0.5 * S * (un - Rr[size_t(R_UABS) * nfc + f]) - Rr[size_t(R_LVC) * nfc + f] * S;
    for (int k = tid; k < ns; k += 256) r[4 + k] += sg * coef * X[size_t(4 + k) * g.N + cN];
  }
  __syncthreads();
}

// rows of the coupled inverse per workgroup of the sweep: a cell's dense
// product is spread over ceil(n / WSW_ROWS) workgroups, each of which forms
// the (cheap, O(ns)) right-hand side itself
constexpr int WSW_ROWS = 64;

// rows [r0, r1) of x = D^-1 r (coupled: dense product, one wave per row;
// split: scalars)
__device__ __forceinline__ void w_apply_dinv(const Geo &g, const WSweep &a, int p, int n, int r0, int r1,
                                             const double *r, double *xo, bool bwd, const double *xs) {
  const int tid = threadIdx.x;
  if (a.mode == 0) {
    const double *Dp = a.Dinv + size_t(p) * n * n;
    const int lane = tid & 63, w = tid >> 6;
    for (int row = r0 + w; row < r1; row += 4) {
      const double *Dr = Dp + size_t(row) * n;
      double acc = 0.0;
      for (int c = lane; c < n; c += 64) acc += Dr[c] * r[c];
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
      if (lane == 0) {
        const size_t at = size_t(row) * g.N + p;
        xo[at] = bwd ? xs[at] - acc : acc;
      }
    }
  } else {
    const double dF = a.Dinv[p], dC = a.Dinv[size_t(g.N) + p];
    for (int k = r0 + tid; k < r1; k += 256) {
      const double v = r[k] * (k < 4 ? dF : dC);
      const size_t at = size_t(k) * g.N + p;
      xo[at] = bwd ? xs[at] - v : v;
    }
  }
}

// one hyperplane i + j = k: blockIdx.x the cell on the hyperplane,
// blockIdx.y its block of WSW_ROWS rows (coupled; split: one block, all rows)
template <bool FWD>
__global__ void __launch_bounds__(256) kw_sweep(Geo g, WSweep a, int k, const int *__restrict__ done) {
  if (done && *done) return;
  extern __shared__ double wsh[];
  double *r = wsh + 8;  // wsh[0..8): reduction scratch
  const int j0 = k - g.ni + 1 > 0 ? k - g.ni + 1 : 0;
  const int j = j0 + blockIdx.x;
  const int i = k - j;
  const int p = j * g.ni + i;
  const int n = a.mode == 0 ? a.ns + 3 : a.ns + 4;
  const int r0 = a.mode == 0 ? blockIdx.y * WSW_ROWS : 0;
  const int r1 = a.mode == 0 ? min(n, r0 + WSW_ROWS) : n;
  for (int q = threadIdx.x; q < n; q += 256) r[q] = FWD ? a.b[size_t(q) * g.N + p] : 0.0;
  __syncthreads();
  if (FWD) {
    if (i > 0) w_off(g, a, padc(g, i - 1, j), p - 1, true, j * (g.ni + 1) + i, -1.0, -1.0, a.xs, r, wsh);
    if (j > 0) w_off(g, a, padc(g, i, j - 1), p - g.ni, false, j * g.ni + i, -1.0, -1.0, a.xs, r, wsh);
    w_apply_dinv(g, a, p, n, r0, r1, r, a.xs, false, nullptr);
  } else {
    if (i < g.ni - 1) w_off(g, a, padc(g, i + 1, j), p + 1, true, j * (g.ni + 1) + i + 1, 1.0, 1.0, a.x, r, wsh);
    if (j < g.nj - 1) w_off(g, a, padc(g, i, j + 1), p + g.ni, false, (j + 1) * g.ni + i, 1.0, 1.0, a.x, r, wsh);
    w_apply_dinv(g, a, p, n, r0, r1, r, a.x, true, a.xs);
  }
}

// -------------------------------------------------------------- corrections
// One thread per cell, as k_update in one temperature: coupled closure,
// split CC1 / CC2, clipping of negative partial densities.
__global__ void __launch_bounds__(256) kw_update(Geo g, int ns, double *__restrict__ Q, const double *__restrict__ dq,
                                                 int mode, int kind, int *__restrict__ nclip, int *__restrict__ bad,
                                                 const int *__restrict__ done) {
  if (done && *done) return;
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= g.N) return;
  auto IX = [&](int k) { return dq[size_t(k) * g.N + p]; };
  auto QS = [&](int s) -> double & { return Q[size_t(s) * g.N + p]; };
  double rho = 0.0;
  for (int s = 0; s < ns; ++s) rho += QS(s);
  const double drho = IX(0);
  const double target = rho + drho;
  bool clip = false;
  // new partial densities, written in place (each depends only on its own
  // old value and on sums taken before the loop that writes)
  if (mode == 0) {
    double sum = 0.0;
    for (int s = 0; s < ns - 1; ++s) sum += IX(4 + s);
    for (int s = 0; s < ns - 1; ++s) QS(s) = QS(s) + IX(4 + s);
    QS(ns - 1) = QS(ns - 1) + (drho - sum);
  } else if (kind == 1) {
    double sum = 0.0;
    for (int s = 0; s < ns; ++s) sum += IX(4 + s);
    for (int s = 0; s < ns; ++s) {
      const double rs = QS(s);
      QS(s) = rs + IX(4 + s) + (rs / rho) * (drho - sum);
    }
  } else {
    double sum = 0.0;
    for (int s = 0; s < ns; ++s) {
      const double v = QS(s) + IX(4 + s);
      if (v < 0.0) clip = true;
      sum += v > 0.0 ? v : 0.0;
    }
    for (int s = 0; s < ns; ++s) {
      const double v = QS(s) + IX(4 + s);
      QS(s) = target * (v > 0.0 ? v : 0.0) / sum;
    }
  }
  if (mode == 0 || kind == 1) {
    double sum = 0.0;
    for (int s = 0; s < ns; ++s) {
      if (QS(s) < 0.0) { QS(s) = 0.0; clip = true; }
      sum += QS(s);
    }
    if (clip)
      for (int s = 0; s < ns; ++s) QS(s) = QS(s) * (target / sum);
  }
  if (clip && nclip) atomicAdd(nclip, 1);
  if (!(target > 0.0) && bad) atomicMin(bad, p);
  Q[size_t(ns) * g.N + p] += IX(1);
  Q[size_t(ns + 1) * g.N + p] += IX(2);
  Q[size_t(ns + 2) * g.N + p] += IX(3);
}

}  // namespace csi
