// Diagonal blocks with many species: one group of G lanes per cell.
//
// The diagonal block of the implicit operator (paper Section 2.2: V/dtau plus
// the spectral radii, minus V times the chemical source Jacobian; Section 2.3
// for the split parts) is ns x ns (split species part) or nb x nb (coupled).
// Held by one thread, its FP64 source Jacobian, the block and the inverse do
// not fit in registers once ns is large.  Here each cell is owned by a group
// of G lanes and lane k owns row k:
//   * the chemistry row: lane k accumulates d omega_t / d rho_u (all u) and
//     d omega_t / dT, dTv of its own species t over all reactions (the
//     reaction rates are evaluated by every lane of the group);
//   * sums over species (the total-density row of the coupled block, the
//     vibrational-energy source terms) are column sums through LDS;
//   * the block row, then a Gauss-Jordan inversion with partial pivoting
//     across the group: per column the group picks its pivot row (largest
//     magnitude, lowest lane on ties), the pivot lane publishes its scaled row
//     in LDS and every other lane eliminates;
//   * the lane whose row became pivot r writes row r of the inverse.
// Used for ns >= BLOCK_NS_MIN; the cell kernel writes the right-hand sides, push data
// and the scalar diagonals (V/dtau + radii) that this kernel reads.
#pragma once
#include "csi_kernels.hpp"

namespace csi {

// Row t of the species production Jacobian at fixed (T, Tv) (t < 0: none):
// w = omega_t, row[u] = d omega_t / d rho_u, dT, dTv = d omega_t / dT, dTv.
// The same kinetics as `chemistry`, accumulated for one species.
template <int NS, int NT>
__device__ __forceinline__ void chem_row(const Mech &m, const double *rs, double T, double Tv, double p, int t,
                                         double &w, double (&row)[NS], double &dT, double &dTv) {
  double X[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    X[s] = rs[s] / m.M[s];
    row[s] = 0.0;
  }
  w = dT = dTv = 0.0;
  if (NT == 1) Tv = T;
  const double lnT = log(T), lnTv = log(Tv);
  const double Mt = t >= 0 ? m.M[t] : 0.0;
  const double lnc0 = log(1.0e5 / (RU * T));
  for (int r = 0; r < m.nr; ++r) {
    const Reaction &R = m.rx[r];
    // this species' net stoichiometric coefficient in reaction r
    double nu = 0.0;
    for (int e = 0; e < R.nnet; ++e) nu += R.net_s[e] == t ? double(R.net_nu[e]) : 0.0;
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
    const double kf = exp(R.lnA + R.b * lnTf - R.theta / Tf);
    double lnKc = double(R.dnu) * lnc0, dlnKc = -double(R.dnu) / T;
    for (int e = 0; e < R.nnet; ++e) {
      const int s = R.net_s[e];
      lnKc -= double(R.net_nu[e]) * gRT(m, s, T, lnT);
      dlnKc += double(R.net_nu[e]) * hRT2(m, s, T);
    }
    const double kb = exp(R.lnA + R.b * lnT - R.theta / T - lnKc);
    double Pf = 1.0, Pb = 1.0;
    for (int e = 0; e < R.nreac; ++e) Pf *= X[R.reac[e]];
    for (int e = 0; e < R.nprod; ++e) Pb *= X[R.prod[e]];
    double Mc = 1.0;
    if (R.third) {
      Mc = 0.0;
#pragma unroll
      for (int s = 0; s < NS; ++s) Mc += m.eff[r][s] * X[s];
    }
    const double net = kf * Pf - kb * Pb;
    // d q / d X_s, scaled by M_t nu / M_s below
    double dq[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) dq[s] = R.third ? m.eff[r][s] * net : 0.0;
    for (int e = 0; e < R.nreac; ++e) {
      double lo = 1.0;
      for (int f = 0; f < R.nreac; ++f)
        if (f != e) lo *= X[R.reac[f]];
      dq[R.reac[e]] += Mc * kf * lo;
    }
    for (int e = 0; e < R.nprod; ++e) {
      double lo = 1.0;
      for (int f = 0; f < R.nprod; ++f)
        if (f != e) lo *= X[R.prod[f]];
      dq[R.prod[e]] -= Mc * kb * lo;
    }
    const double dkf_dTf = kf * (R.b + R.theta / Tf) / Tf;
    const double dkb_dT = kb * ((R.b + R.theta / T) / T - dlnKc);
    const double a = Mt * nu;
    w += a * Mc * net;
    dT += a * Mc * (dkf_dTf * dTf_dT * Pf - dkb_dT * Pb);
    dTv += a * Mc * (dkf_dTf * dTf_dTv * Pf);
#pragma unroll
    for (int u = 0; u < NS; ++u) row[u] += a * dq[u] / m.M[u];
  }
}

// Landau-Teller part of omega_ve (same model as `chemistry`): its value and its
// derivatives with respect to rho_u, T and Tv.
template <int NS>
__device__ __forceinline__ void lt_relax(const Mech &m, const double *rs, double T, double Tv, double p, double &wv,
                                         double (&dr)[NS], double &dT_, double &dTv_) {
  const double Tm13 = exp(-log(T) / 3.0);
  double pT = 0.0, pTv = 0.0;
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    if (m.kind[s] == ELECTRON) pTv += rs[s] * m.R[s];
    else pT += rs[s] * m.R[s];
    dr[s] = 0.0;
  }
  wv = dT_ = dTv_ = 0.0;
  double lt_sum = 0.0;
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    if (m.kind[s] == MOLECULE && m.thv[s] > 0.0) {
      const double E = exp(18.42 - m.lta[s] * (Tm13 - m.ltb[s]));
      const double itau = p / ATM * E;
      const double evT = evib(m.R[s], m.thv[s], T), evTv = evib(m.R[s], m.thv[s], Tv);
      const double term = rs[s] * (evT - evTv) * itau;
      wv += term;
      lt_sum += term;
      dr[s] += (evT - evTv) * itau;
      dT_ += rs[s] * cvvib(m.R[s], m.thv[s], T) * itau + term * (m.lta[s] / 3.0) * Tm13 / T;
      dTv_ += -rs[s] * cvvib(m.R[s], m.thv[s], Tv) * itau;
    }
  }
#pragma unroll
  for (int s = 0; s < NS; ++s) dr[s] += lt_sum * (m.R[s] * (m.kind[s] == ELECTRON ? Tv : T)) / p;
  dT_ += lt_sum * pT / p;
  dTv_ += lt_sum * pTv / p;
}

struct BlockOut {
  void *gS[2];                 // group schedule: record staging of part 0 (coupled / flow), 1 (species)
  void *Dinv;                  // hyperplane schedule: cell-major inverses (layout as the cell kernel's)
  int group_c;                 // 0: hyperplane schedule; > 0: group schedule
  const double *diag;          // [2][N] from the cell kernel: split dF, dC; coupled dK
  const float *Jsur;           // surrogate J_C [ns * ns][N]
  unsigned long long *ddfail;  // cells whose surrogate block failed the dominance check
  const int *surr_off;         // >= 0: surrogate switched off
  int *bad;                    // first singular cell
};

template <int NS, int NT, int MODE> struct BlockDims {
  static constexpr int NF = NT == 2 ? 5 : 4, NB = NF + NS - 1, NV = NS + 3 + (NT == 2 ? 1 : 0);
  static constexpr int G = MODE == 0 ? NB : NS, C = 64 / G;
  // LDS per group: column-sum buffer [G][NS], scalars (4G), vector results (2 NS)
  static constexpr int BUF = G * NS + 4 * G + 2 * NS;
};

// Exchange point between the lanes of one wave through LDS: stores made before
// it are seen by loads after it.  The LDS operations of a wave complete in
// order; the fences keep the compiler from moving memory operations across it
// and the (convergent) wave barrier from duplicating or merging the code
// around it.  Every lane of the wave passes it together (no divergent code
// between two exchange points communicates).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}
// v as held by lane `src` of the wave (modulo 64; every lane active)
__device__ __forceinline__ double lane_read(double v, int src) {
  const long long u = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_ds_bpermute(src << 2, int(u & 0xffffffffll));
  const int hi = __builtin_amdgcn_ds_bpermute(src << 2, int(u >> 32));
  return __builtin_bit_cast(double, (long long)(unsigned(lo)) | ((long long)hi << 32));
}

// sum over the group of each lane's vector v[NS]; every lane receives the sums.
// Lane k < NS sums column k; the lanes beyond repeat column NS - 1 (G <= 2 NS).
template <int NS, int G>
__device__ __forceinline__ void group_colsum(double *buf, int k, const double (&v)[NS], double (&s)[NS]) {
  static_assert(G <= 2 * NS, "column-sum lanes");
#pragma unroll
  for (int u = 0; u < NS; ++u) buf[k * NS + u] = v[u];
  wave_sync();
  const int kk = k < NS ? k : NS - 1;
  double acc = 0.0;
  for (int j = 0; j < G; ++j) acc += buf[j * NS + kk];
  wave_sync();
  double *res = buf + G * NS + 4 * G;
  res[kk] = acc;
  wave_sync();
#pragma unroll
  for (int u = 0; u < NS; ++u) s[u] = res[u];
  wave_sync();
}
// sums over the group of four scalars per lane; every lane receives them
template <int NS, int G>
__device__ __forceinline__ void group_sum4(double *buf, int k, const double (&v)[4], double (&s)[4]) {
  double *sb = buf + G * NS;
#pragma unroll
  for (int j = 0; j < 4; ++j) sb[k * 4 + j] = v[j];
  wave_sync();
#pragma unroll
  for (int j = 0; j < 4; ++j) s[j] = 0.0;
  for (int l = 0; l < G; ++l)
#pragma unroll
    for (int j = 0; j < 4; ++j) s[j] += sb[l * 4 + j];
  wave_sync();
}

// Gauss-Jordan inversion with partial pivoting of the G x G matrix whose row k
// is A (lane base + k); on return Inv holds row `pos` of the inverse.  Per
// column the group takes as pivot the unused row of largest magnitude (lowest
// lane on ties; a NaN entry counts as zero) and every lane reads the scaled
// pivot row from the pivot lane's registers.  Every lane ends with a distinct
// pos in [0, G); false on a zero pivot (the group agrees).
template <int G>
__device__ __forceinline__ bool group_invert(int k, int base, double (&A)[G], double (&Inv)[G], int &pos) {
#pragma unroll
  for (int c = 0; c < G; ++c) Inv[c] = c == k ? 1.0 : 0.0;
  pos = -1;
  bool ok = true;
#pragma unroll
  for (int kc = 0; kc < G; ++kc) {
    const double a = fabs(A[kc]);
    const double cand = pos >= 0 ? -1.0 : (a >= 0.0 ? a : 0.0);
    int piv = 0;
    double best = -2.0;
    for (int j = 0; j < G; ++j) {
      const double v = lane_read(cand, base + j);
      if (v > best) {
        best = v;
        piv = j;
      }
    }
    if (!(best > 0.0)) ok = false;
    const bool me = k == piv;
    if (me) pos = kc;
    const double f = A[kc], ip = 1.0 / f;
    const int src = base + piv;
#pragma unroll
    for (int c = 0; c < G; ++c) {
      const double ra = lane_read(A[c] * ip, src), ri = lane_read(Inv[c] * ip, src);
      A[c] = me ? ra : A[c] - f * ra;
      Inv[c] = me ? ri : Inv[c] - f * ri;
    }
  }
  return ok;
}

// One group of G lanes per cell, two waves per block.  MODE 0: coupled block
// (G = nb; lane 0 carries the last species' chemistry row, which only enters
// the total-density row; lanes 1..4 have no species row); MODE 1: split
// species block (G = ns) and the flow block's inverse (lanes k < nf).
template <int NS, int NT, typename RT, int MODE>
__global__ void __launch_bounds__(128) k_block(Geo g, const Mech *__restrict__ mech, const double *__restrict__ Q,
                                               const double *__restrict__ prim, int flags, BlockOut out,
                                               const int *__restrict__ done) {
  using BD = BlockDims<NS, NT, MODE>;
  constexpr int G = BD::G, C = BD::C, NF = BD::NF, NB = BD::NB, NV = BD::NV;
  __shared__ double sh[2][C + 1][BD::BUF];
  if (done && *done) return;
  const Mech &m = *mech;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int grp = lane / G, k = lane - grp * G;
  double *buf = sh[wave][grp < C ? grp : C];  // idle lanes work in a buffer of their own
  const long cell = (long(blockIdx.x) * 2 + wave) * C + grp;
  const bool real = grp < C && cell < g.N;
  const int p = int(real ? cell : 0);
  const int i = p % g.ni, j = p / g.ni;
  const int pc = padc(g, i, j);
  const size_t NP = g.NP;
  double q[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) q[v] = Q[size_t(v) * g.N + p];
  const double T = prim[F_T * NP + pc], Tv = prim[F_TV * NP + pc], pp = prim[F_P * NP + pc];
  Prim<NS, NT> P;
  prim_from_q<NS, NT>(m, q, P, T, Tv);
  const double Vp = g.V[p];
  // this lane's species row
  const int t = MODE == 0 ? (k >= NF ? k - NF : (k == 0 ? NS - 1 : -1)) : (k < NS ? k : -1);
  double A[G];
  double w_t = 0.0, row[NS], dwT = 0.0, dwTv = 0.0;
#pragma unroll
  for (int u = 0; u < NS; ++u) row[u] = 0.0;
  // vibrational-energy source terms (two temperatures): d omega_ve / d rho_u, dT, dTv
  double dwv_dr[NS], dwv_dT = 0.0, dwv_dTv = 0.0;
  auto ve_terms = [&]() {
    double wv_lt, dr[NS], dT_, dTv_;
    lt_relax<NS>(m, q, T, Tv, pp, wv_lt, dr, dT_, dTv_);
    const double ev = t >= 0 ? eve_s(m, t, Tv) : 0.0, cv = t >= 0 ? cvve_s(m, t, Tv) : 0.0;
    double wr[NS];
#pragma unroll
    for (int u = 0; u < NS; ++u) wr[u] = row[u] * ev;
    double cs[NS];
    group_colsum<NS, G>(buf, k, wr, cs);
#pragma unroll
    for (int u = 0; u < NS; ++u) dwv_dr[u] = dr[u] + cs[u];
    double sv[4] = {dwT * ev, dwTv * ev + w_t * cv, 0.0, 0.0}, ss[4];
    group_sum4<NS, G>(buf, k, sv, ss);
    dwv_dT = dT_ + ss[0];
    dwv_dTv = dTv_ + ss[1];
  };
  bool ok;
  int pos;
  double Inv[G];
  if (MODE == 0) {
    chem_row<NS, NT>(m, q, T, Tv, pp, t, w_t, row, dwT, dwTv);
    if (NT == 2) ve_terms();
    // the total-density row sums every species row
    double S1[NS], s4[4] = {dwT, dwTv, 0.0, 0.0}, S4[4];
    group_colsum<NS, G>(buf, k, row, S1);
    group_sum4<NS, G>(buf, k, s4, S4);
    // row k of dS/dq (storage columns), then of dS/dz
    double Jq[NV];
#pragma unroll
    for (int c = 0; c < NV; ++c) {
      double dT, dTv;
      temp_derivs<NS, NT>(P, c, dT, dTv);
      double v = 0.0;
      if (k >= NF) v = (c < NS ? row[c < NS ? c : 0] : 0.0) + dwT * dT + dwTv * dTv;
      else if (k == 0) v = (c < NS ? S1[c < NS ? c : 0] : 0.0) + S4[0] * dT + S4[1] * dTv;
      else if (NT == 2 && k == 4) v = (c < NS ? dwv_dr[c < NS ? c : 0] : 0.0) + dwv_dT * dT + dwv_dTv * dTv;
      Jq[c] = v;
    }
    const double dK = out.diag[p];
#pragma unroll
    for (int c = 0; c < NB; ++c) {
      const double jz = c == 0 ? Jq[NS - 1] : c < NF ? Jq[NS + c - 1] : Jq[c - NF] - Jq[NS - 1];
      A[c] = (c == k ? dK : 0.0) - Vp * jz;
    }
    ok = group_invert<G>(k, grp * G, A, Inv, pos);
    // row pos of the inverse
    if (real) {
      if (out.group_c > 0) {
        constexpr RecShape S = rec_shape(PART_COUPLED, NS, NT, sizeof(RT));
        RT *St = reinterpret_cast<RT *>(out.gS[0]);
#pragma unroll
        for (int c = 0; c < NB; ++c) St[st_idx(S, g.N, 0, rw_d(S, pos, c), p)] = RT(Inv[c]);
      } else {
        RT *Dcm = reinterpret_cast<RT *>(out.Dinv);
#pragma unroll
        for (int c = 0; c < NB; ++c) Dcm[long(pos * NB + c) * g.N + p] = RT(Inv[c]);
      }
    }
  } else {
    const double dF = out.diag[p], dC = out.diag[g.N + p];
    // surrogate species block, accepted when the group's block is strictly row
    // diagonally dominant with a positive diagonal in molar units
    const bool try_sur = (flags & 4) && out.Jsur && *out.surr_off < 0;
    bool use_sur = false;
    if (try_sur) {
      double off = 0.0;
#pragma unroll
      for (int c = 0; c < NS; ++c) {
        A[c] = (c == k ? dC : 0.0) - Vp * double(out.Jsur[size_t(k * NS + c) * g.N + p]);
        if (c != k) off += fabs(A[c]) * m.M[c];
      }
      const bool dd = A[k < NS ? k : 0] > 0.0 && A[k < NS ? k : 0] * m.M[k] > off;
      const unsigned long long bal = __ballot(dd);
      constexpr unsigned long long gm = G >= 64 ? ~0ull : (1ull << G) - 1;
      use_sur = ((bal >> (grp * G)) & gm) == gm;
      if (!use_sur && k == 0 && real) atomicAdd(out.ddfail, 1ull);
    }
    if (!use_sur || NT == 2) chem_row<NS, NT>(m, q, T, Tv, pp, t, w_t, row, dwT, dwTv);
    if (!use_sur) {
#pragma unroll
      for (int c = 0; c < NS; ++c) A[c] = (c == k ? dC : 0.0) - Vp * row[c];
    }
    // flow block: diagonal 1/dF, and in two temperatures the rho e_ve row
    // -V d omega_ve / d Q_F (frozen Y) eliminated in closed form
    double df6[6] = {1.0 / dF, 0.0, 0.0, 0.0, 0.0, 0.0};
    if (NT == 2) {
      ve_terms();
      double a0 = 0.0;
#pragma unroll
      for (int s = 0; s < NS; ++s) a0 += P.Y[s] * (dwv_dr[s] + dwv_dT * P.dT_dr[s] + dwv_dTv * P.dTv_dr[s]);
      double dwv[5];
      dwv[0] = a0;
#pragma unroll
      for (int c = 1; c < 5; ++c) {
        double dT, dTv;
        temp_derivs<NS, NT>(P, NS - 1 + c, dT, dTv);
        dwv[c] = dwv_dT * dT + dwv_dTv * dTv;
      }
#pragma unroll
      for (int c = 0; c < 4; ++c) df6[1 + c] = Vp * dwv[c];
      const double piv = dF - Vp * dwv[4];
      if (piv == 0.0 && real && out.bad && k == 0) atomicMin(out.bad, p);
      df6[5] = 1.0 / piv;
    }
    ok = group_invert<G>(k, grp * G, A, Inv, pos);
    if (real) {
      if (out.group_c > 0) {
        constexpr RecShape S = rec_shape(PART_SPECIES, NS, NT, sizeof(RT));
        constexpr RecShape SF = rec_shape(PART_FLOW, NS, NT, sizeof(RT));
        RT *St = reinterpret_cast<RT *>(out.gS[1]);
#pragma unroll
        for (int c = 0; c < NS; ++c) St[st_idx(S, g.N, 0, rw_d(S, pos, c), p)] = RT(Inv[c]);
        if (k < NF) {
          RT *Sf = reinterpret_cast<RT *>(out.gS[0]);
#pragma unroll
          for (int c = 0; c < NF; ++c) {
            double v = c == k && k < 4 ? df6[0] : 0.0;
            if (NT == 2 && k == 4) v = c < 4 ? df6[1 + c] * df6[0] * df6[5] : df6[5];
            Sf[st_idx(SF, g.N, 0, rw_d(SF, k, c), p)] = RT(v);
          }
        }
      } else {
        RT *Dcm = reinterpret_cast<RT *>(out.Dinv);
#pragma unroll
        for (int c = 0; c < NS; ++c) Dcm[long(6 + pos * NS + c) * g.N + p] = RT(Inv[c]);
        if (k == 0)
#pragma unroll
          for (int c = 0; c < 6; ++c) Dcm[long(c) * g.N + p] = RT(df6[c]);
      }
    }
  }
  if (!ok && real && k == 0 && out.bad) atomicMin(out.bad, p);
}

}  // namespace csi
