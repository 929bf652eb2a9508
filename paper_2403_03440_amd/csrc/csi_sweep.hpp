// LU-SGS sweeps (paper Section 2.2: forward (D+L) dQ* = RHS, backward
// (D+U) dQ = D dQ*) with the off-diagonal blocks applied matrix-free:
//   O_PN x = 1/2 S_f [A_N(n) x - lambda_f x] - lambda^v_f S_f x
// (spectral splitting A+- = (A +- lambda I)/2 and the viscous spectral
// approximation), with the paper's Section 2.3 radii for the split parts:
// flow |U|+c at frozen mass fractions, species |U| as a scalar times a vector.
// RT is the arithmetic type of the sweeps (double, or float in the mixed mode).
#pragma once
#include "csi_kernels.hpp"

namespace csi {

// neighbour data needed by the Jacobian-vector products
template <int NS, typename RT> struct NbState {
  RT u, v, H, eve, pE, pv, Y[NS], pr[NS];
};
template <int NS, int NT, typename RT, int PART>
__device__ __forceinline__ void load_nb(const double *prim, size_t NP, int pc, NbState<NS, RT> &s) {
  s.u = RT(prim[F_U * NP + pc]);
  s.v = RT(prim[F_V * NP + pc]);
  if (PART != 2) {
    s.H = RT(prim[F_H * NP + pc]);
    s.eve = RT(prim[F_EVE * NP + pc]);
    s.pE = RT(prim[F_PE * NP + pc]);
    s.pv = RT(prim[F_PV * NP + pc]);
#pragma unroll
    for (int k = 0; k < NS; ++k) {
      s.Y[k] = RT(prim[(PF<NS>::Y + k) * NP + pc]);
      s.pr[k] = RT(prim[(PF<NS>::PR + k) * NP + pc]);
    }
  }
}

// analytic Jacobian-vector product of the physical flux F(q).n
// coupled: x in z = (rho, m_x, m_y, rhoE, [rhoe_ve], rho_0..rho_{ns-2})
template <int NS, int NT, typename RT>
__device__ __forceinline__ void jvp_coupled(const NbState<NS, RT> &s, RT nx, RT ny, const RT *x, RT *o) {
  using D = Dims<NS, NT>;
  constexpr int NF = D::nf;
  RT dr[NS];
  RT last = x[0];
#pragma unroll
  for (int k = 0; k < NS - 1; ++k) { dr[k] = x[NF + k]; last -= x[NF + k]; }
  dr[NS - 1] = last;
  RT dp = s.pE * (x[3] - s.u * x[1] - s.v * x[2]);
  if (NT == 2) dp += s.pv * x[4];
#pragma unroll
  for (int k = 0; k < NS; ++k) dp += s.pr[k] * dr[k];
  RT un = s.u * nx + s.v * ny;
  RT dmn = x[1] * nx + x[2] * ny;
  RT a = dmn - un * x[0];
  o[0] = dmn;
  o[1] = un * x[1] + s.u * a + nx * dp;
  o[2] = un * x[2] + s.v * a + ny * dp;
  o[3] = un * (x[3] + dp) + s.H * a;
  if (NT == 2) o[4] = un * x[4] + s.eve * a;
#pragma unroll
  for (int k = 0; k < NS - 1; ++k) o[NF + k] = un * dr[k] + s.Y[k] * a;
}

// flow part at frozen mass fractions: x = (rho, m_x, m_y, rhoE, [rhoe_ve])
template <int NS, int NT, typename RT>
__device__ __forceinline__ void jvp_flow(const NbState<NS, RT> &s, RT nx, RT ny, const RT *x, RT *o) {
  RT prY = RT(0);
#pragma unroll
  for (int k = 0; k < NS; ++k) prY += s.pr[k] * s.Y[k];
  RT dp = prY * x[0] + s.pE * (x[3] - s.u * x[1] - s.v * x[2]);
  if (NT == 2) dp += s.pv * x[4];
  RT un = s.u * nx + s.v * ny;
  RT dmn = x[1] * nx + x[2] * ny;
  RT a = dmn - un * x[0];
  o[0] = dmn;
  o[1] = un * x[1] + s.u * a + nx * dp;
  o[2] = un * x[2] + s.v * a + ny * dp;
  o[3] = un * (x[3] + dp) + s.H * a;
  if (NT == 2) o[4] = un * x[4] + s.eve * a;
}

struct SweepArgs {
  const double *prim, *Ri, *Rj;
  const void *Dinv, *b;
  void *xs, *x;
  int mode;
  // flux-difference off-diagonal operator (FP64 sweeps): the state, the
  // mechanism, and the flag receiving the first cell whose neighbour state
  // plus increment is not physical (null: linear Jacobian-vector products)
  const double *Q;
  const Mech *mech;
  int *bad;
};

// physical flux F(q).n of a state in the coupled unknowns' rows
// (sum_s rho_s u_n, rho u u_n + p n_x, rho v u_n + p n_y, (rho E + p) u_n,
// [rho e_ve u_n], rho_s u_n for s < ns - 1); flow part: the first nf rows
template <int NS, int NT>
__device__ __forceinline__ void flux_z(const double *q, double rho, double u, double v, double p, double nx,
                                       double ny, double *f) {
  using D = Dims<NS, NT>;
  constexpr int NF = D::nf;
  const double un = u * nx + v * ny;
  f[0] = rho * un;
  f[1] = q[NS] * un + p * nx;
  f[2] = q[NS + 1] * un + p * ny;
  f[3] = (q[NS + 2] + p) * un;
  if (NT == 2) f[4] = q[NS + 3] * un;
#pragma unroll
  for (int k = 0; k < NS - 1; ++k) f[NF + k] = q[k] * un;
}

// Flux difference F(Q_N + x).n - F(Q_N).n, the nonlinear matrix-free
// alternative to A_N(n) x: coupled (x in z) or flow part (x in Q_F at frozen
// mass fractions).  False if Q_N + x is not a physical state.
template <int NS, int NT>
__device__ __forceinline__ bool flux_difference(const Geo &g, const SweepArgs &a, int pcN, int cN, int mode,
                                                double nx, double ny, const double *x, double *o) {
  using D = Dims<NS, NT>;
  constexpr int NV = D::nv, NF = D::nf;
  const Mech &m = *a.mech;
  const size_t NP = g.NP;
  double q0[NV], q1[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) q0[k] = a.Q[size_t(k) * g.N + cN];
  double rho0 = 0.0;
#pragma unroll
  for (int s = 0; s < NS; ++s) rho0 += q0[s];
  if (mode == 0) {
    double last = x[0];
#pragma unroll
    for (int s = 0; s < NS - 1; ++s) {
      q1[s] = q0[s] + x[NF + s];
      last -= x[NF + s];
    }
    q1[NS - 1] = q0[NS - 1] + last;
  } else {
    const double f = (rho0 + x[0]) / rho0;
#pragma unroll
    for (int s = 0; s < NS; ++s) q1[s] = q0[s] * f;
  }
#pragma unroll
  for (int k = 0; k < NF - 1; ++k) q1[NS + k] = q0[NS + k] + x[1 + k];
  Prim<NS, NT> P1;
  if (!prim_from_q<NS, NT>(m, q1, P1, a.prim[F_T * NP + pcN], a.prim[F_TV * NP + pcN])) return false;
  double f0[D::nb], f1[D::nb];
  flux_z<NS, NT>(q0, rho0, a.prim[F_U * NP + pcN], a.prim[F_V * NP + pcN], a.prim[F_P * NP + pcN], nx, ny, f0);
  flux_z<NS, NT>(q1, P1.rho, P1.u, P1.v, P1.p, nx, ny, f1);
  const int n = mode == 0 ? D::nb : NF;
#pragma unroll
  for (int k = 0; k < D::nb; ++k)
    if (k < n) o[k] = f1[k] - f0[k];
  return true;
}

// apply O_PN to the neighbour increment(s) and accumulate with sign sg into r
template <int NS, int NT, typename RT>
__device__ __forceinline__ void off_accumulate(const Geo &g, const SweepArgs &a, int pcN, int cN, bool iface, int f,
                                               RT sgn_n, RT sg, const RT *X, RT *r) {
  using D = Dims<NS, NT>;
  constexpr int NB = D::nb, NF = D::nf;
  const size_t NP = g.NP;
  int nfc = iface ? (g.ni + 1) * g.nj : g.ni * (g.nj + 1);
  const double *Rr = iface ? a.Ri : a.Rj;
  RT nx = sgn_n * RT(iface ? g.fi_nx[f] : g.fj_nx[f]);
  RT ny = sgn_n * RT(iface ? g.fi_ny[f] : g.fj_ny[f]);
  RT S = RT(iface ? g.fi_S[f] : g.fj_S[f]);
  RT lam = RT(Rr[size_t(R_LAM) * nfc + f]);
  RT half = RT(0.5);
  if (a.mode == 0) {
    NbState<NS, RT> s;
    load_nb<NS, NT, RT, 0>(a.prim, NP, pcN, s);
    RT x[NB], o[NB];
#pragma unroll
    for (int k = 0; k < NB; ++k) x[k] = X[size_t(k) * g.N + cN];
    if constexpr (sizeof(RT) == 8) {
      if (a.mech) {
        if (!flux_difference<NS, NT>(g, a, pcN, cN, 0, nx, ny, x, o)) {
          atomicMin(a.bad, cN);
#pragma unroll
          for (int k = 0; k < NB; ++k) o[k] = 0.0;
        }
      } else {
        jvp_coupled<NS, NT, RT>(s, nx, ny, x, o);
      }
    } else {
      jvp_coupled<NS, NT, RT>(s, nx, ny, x, o);
    }
    RT lv = RT(Rr[size_t(R_LVK) * nfc + f]);
#pragma unroll
    for (int k = 0; k < NB; ++k) r[k] += sg * (half * S * (o[k] - lam * x[k]) - lv * S * x[k]);
  } else {
    NbState<NS, RT> s;
    load_nb<NS, NT, RT, 1>(a.prim, NP, pcN, s);
    RT x[NF], o[D::nb];
#pragma unroll
    for (int k = 0; k < NF; ++k) x[k] = X[size_t(k) * g.N + cN];
    if constexpr (sizeof(RT) == 8) {
      if (a.mech) {
        if (!flux_difference<NS, NT>(g, a, pcN, cN, 1, nx, ny, x, o)) {
          atomicMin(a.bad, cN);
#pragma unroll
          for (int k = 0; k < NF; ++k) o[k] = 0.0;
        }
      } else {
        jvp_flow<NS, NT, RT>(s, nx, ny, x, o);
      }
    } else {
      jvp_flow<NS, NT, RT>(s, nx, ny, x, o);
    }
    RT lvF = RT(Rr[size_t(R_LVF) * nfc + f]);
#pragma unroll
    for (int k = 0; k < NF; ++k) r[k] += sg * (half * S * (o[k] - lam * x[k]) - lvF * S * x[k]);
    RT un = s.u * nx + s.v * ny;
    RT coef = half * S * (un - RT(Rr[size_t(R_UABS) * nfc + f])) - RT(Rr[size_t(R_LVC) * nfc + f]) * S;
#pragma unroll
    for (int k = 0; k < NS; ++k) r[NF + k] += sg * coef * X[size_t(NF + k) * g.N + cN];
  }
}

// x = D^-1 r  (coupled dense inverse; split: closed-form flow block + dense species inverse)
template <int NS, int NT, typename RT>
__device__ __forceinline__ void apply_dinv(const Geo &g, const SweepArgs &a, int p, const RT *r, RT *x) {
  using D = Dims<NS, NT>;
  constexpr int NB = D::nb, NF = D::nf;
  const RT *Di = reinterpret_cast<const RT *>(a.Dinv);
  if (a.mode == 0) {
#pragma unroll
    for (int rr = 0; rr < NB; ++rr) {
      RT acc = RT(0);
#pragma unroll
      for (int c = 0; c < NB; ++c) acc += Di[size_t(rr * NB + c) * g.N + p] * r[c];
      x[rr] = acc;
    }
  } else {
    const RT *DF = Di;
    const RT *DC = Di + size_t(6) * g.N;
    RT d0 = DF[p];
#pragma unroll
    for (int k = 0; k < 4; ++k) x[k] = r[k] * d0;
    if (NT == 2) {
      RT acc = r[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) acc += DF[size_t(1 + k) * g.N + p] * x[k];
      x[4] = acc * DF[size_t(5) * g.N + p];
    }
#pragma unroll
    for (int rr = 0; rr < NS; ++rr) {
      RT acc = RT(0);
#pragma unroll
      for (int c = 0; c < NS; ++c) acc += DC[size_t(rr * NS + c) * g.N + p] * r[NF + c];
      x[NF + rr] = acc;
    }
  }
}

// one hyperplane i + j = k of the forward sweep
template <int NS, int NT, typename RT>
__global__ void __launch_bounds__(256) k_sweep_fwd_hp(Geo g, SweepArgs a, int k, const int *__restrict__ done) {
  using D = Dims<NS, NT>;
  constexpr int NSOL = D::nsplit;
  if (done && *done) return;
  int j0 = k - g.ni + 1 > 0 ? k - g.ni + 1 : 0;
  int j = j0 + blockIdx.x * blockDim.x + threadIdx.x;
  int j1 = k < g.nj - 1 ? k : g.nj - 1;
  if (j > j1) return;
  int i = k - j;
  int p = j * g.ni + i;
  int n = a.mode == 0 ? D::nb : NSOL;
  const RT *b = reinterpret_cast<const RT *>(a.b);
  RT *xs = reinterpret_cast<RT *>(a.xs);
  RT r[NSOL];
#pragma unroll
  for (int q = 0; q < NSOL; ++q) r[q] = q < n ? b[size_t(q) * g.N + p] : RT(0);
  if (i > 0) off_accumulate<NS, NT, RT>(g, a, padc(g, i - 1, j), p - 1, true, j * (g.ni + 1) + i, RT(-1), RT(-1), xs, r);
  if (j > 0) off_accumulate<NS, NT, RT>(g, a, padc(g, i, j - 1), p - g.ni, false, j * g.ni + i, RT(-1), RT(-1), xs, r);
  RT x[NSOL];
  apply_dinv<NS, NT, RT>(g, a, p, r, x);
#pragma unroll
  for (int q = 0; q < NSOL; ++q)
    if (q < n) xs[size_t(q) * g.N + p] = x[q];
}

// one hyperplane i + j = k of the backward sweep
template <int NS, int NT, typename RT>
__global__ void __launch_bounds__(256) k_sweep_bwd_hp(Geo g, SweepArgs a, int k, const int *__restrict__ done) {
  using D = Dims<NS, NT>;
  constexpr int NSOL = D::nsplit;
  if (done && *done) return;
  int j0 = k - g.ni + 1 > 0 ? k - g.ni + 1 : 0;
  int j = j0 + blockIdx.x * blockDim.x + threadIdx.x;
  int j1 = k < g.nj - 1 ? k : g.nj - 1;
  if (j > j1) return;
  int i = k - j;
  int p = j * g.ni + i;
  int n = a.mode == 0 ? D::nb : NSOL;
  const RT *xs = reinterpret_cast<const RT *>(a.xs);
  RT *xo = reinterpret_cast<RT *>(a.x);
  RT r[NSOL];
#pragma unroll
  for (int q = 0; q < NSOL; ++q) r[q] = RT(0);
  if (i < g.ni - 1)
    off_accumulate<NS, NT, RT>(g, a, padc(g, i + 1, j), p + 1, true, j * (g.ni + 1) + i + 1, RT(1), RT(1), xo, r);
  if (j < g.nj - 1)
    off_accumulate<NS, NT, RT>(g, a, padc(g, i, j + 1), p + g.ni, false, (j + 1) * g.ni + i, RT(1), RT(1), xo, r);
  RT x[NSOL];
  apply_dinv<NS, NT, RT>(g, a, p, r, x);
#pragma unroll
  for (int q = 0; q < NSOL; ++q)
    if (q < n) xo[size_t(q) * g.N + p] = xs[size_t(q) * g.N + p] - x[q];
}

// ------------------------------------------------------------ corrections
// where k_update finds the increment dQ: C[0] == 0: cell-major array; else
// the group-schedule results of part 0 (coupled / flow, C[0] cells per wave)
// and part 1 (species, C[1])
struct IncView {
  const void *x[2];
  int C[2];
};

// coupled closure rho_ns = rho - sum_{s<ns} rho_s; split CC1 (increment
// normalisation with W_s = rho_s/rho) or CC2 (mass-fraction normalisation),
// paper Section 2.3 "Consistence correction"; negative partial densities are
// clipped (CC2 before normalising; closure and CC1 after, with renormalisation).
template <int NS, int NT, typename RT>
__global__ void __launch_bounds__(256) k_update(Geo g, const Mech *__restrict__ mech, double *__restrict__ Q,
                                                const void *__restrict__ dqv, int mode,
                                                int kind, int *__restrict__ nclip, int *__restrict__ bad,
                                                const int *__restrict__ done, IncView iv) {
  using D = Dims<NS, NT>;
  constexpr int NF = D::nf;
  if (done && *done) return;
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= g.N) return;
  const RT *dq = reinterpret_cast<const RT *>(dqv);
  // component k of the increment: cell-major (hyperplane schedule), or the
  // step-blocked results of the group schedule (part 0: the first G0
  // unknowns; part 1: the species of the split form)
  const int i = p % g.ni, j = p / g.ni;
  const int G0 = mode == 0 ? D::nb : NF;
  GroupMap m0{}, m1{};
  long b0 = 0, b1 = 0;
  int c0 = 0, c1 = 0;
  if (iv.C[0] > 0) {
    m0 = group_map(g.ni, g.nj, G0);
    b0 = group_blk(m0, i, j, c0);
    if (mode != 0) {
      m1 = group_map(g.ni, g.nj, NS);
      b1 = group_blk(m1, i, j, c1);
    }
  }
  const RT *x0 = reinterpret_cast<const RT *>(iv.x[0]), *x1 = reinterpret_cast<const RT *>(iv.x[1]);
  auto IX = [&](int k) -> RT {
    if (iv.C[0] == 0) return dq[long(k) * g.N + p];
    if (k < G0) return x0[m0.res(b0, c0, k)];
    return x1[m1.res(b1, c1, k - G0)];
  };
  double rs[NS], rho = 0.0;
#pragma unroll
  for (int s = 0; s < NS; ++s) { rs[s] = Q[size_t(s) * g.N + p]; rho += rs[s]; }
  double drho = double(IX(0));
  double target = rho + drho;
  double nr[NS];
  bool clip = false;
  if (mode == 0) {
    double sum = 0.0;
#pragma unroll
    for (int s = 0; s < NS - 1; ++s) {
      double d = double(IX(NF + s));
      nr[s] = rs[s] + d;
      sum += d;
    }
    nr[NS - 1] = rs[NS - 1] + (drho - sum);
  } else if (kind == 1) {
    double sum = 0.0;
#pragma unroll
    for (int s = 0; s < NS; ++s) sum += double(IX(NF + s));
#pragma unroll
    for (int s = 0; s < NS; ++s) nr[s] = rs[s] + double(IX(NF + s)) + (rs[s] / rho) * (drho - sum);
  } else {
    double t[NS], sum = 0.0;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      double v = rs[s] + double(IX(NF + s));
      if (v < 0.0) clip = true;
      t[s] = v > 0.0 ? v : 0.0;
      sum += t[s];
    }
#pragma unroll
    for (int s = 0; s < NS; ++s) nr[s] = target * t[s] / sum;
  }
  if (mode == 0 || kind == 1) {
    double sum = 0.0;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      if (nr[s] < 0.0) { nr[s] = 0.0; clip = true; }
      sum += nr[s];
    }
    if (clip) {
#pragma unroll
      for (int s = 0; s < NS; ++s) nr[s] = nr[s] * (target / sum);
    }
  }
  if (clip && nclip) atomicAdd(nclip, 1);
  if (!(target > 0.0) && bad) atomicMin(bad, p);
#pragma unroll
  for (int s = 0; s < NS; ++s) Q[size_t(s) * g.N + p] = nr[s];
  Q[size_t(NS) * g.N + p] += double(IX(1));
  Q[size_t(NS + 1) * g.N + p] += double(IX(2));
  Q[size_t(NS + 2) * g.N + p] += double(IX(3));
  if (NT == 2) {
    // positivity of the vibrational-electronic energy: floor at Tv = TV_FLOOR
    double eve = Q[size_t(NS + 3) * g.N + p] + double(IX(4)), fl = 0.0;
#pragma unroll
    for (int s = 0; s < NS; ++s) fl += nr[s] * eve_s(*mech, s, TV_FLOOR);
    if (eve < fl) {
      eve = fl;
      if (!clip && nclip) atomicAdd(nclip, 1);
    }
    Q[size_t(NS + 3) * g.N + p] = eve;
  }
}

}  // namespace csi
