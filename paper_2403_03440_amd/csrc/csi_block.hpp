// Diagonal blocks with many species: one group of G lanes per cell.
//
// The diagonal block of the implicit operator (paper Section 2.2: V/dtau plus
// the spectral radii, minus V times the chemical source Jacobian; Section 2.3
// for the split parts) is ns x ns (split species part) or nb x nb (coupled).
// Held by one thread, its FP64 source Jacobian, the block and the inverse do
// not fit in registers once ns is large.  Here each cell is owned by a group
// of G lanes, lane k owns row k of the block, and the work of the kinetics is
// spread over the group instead of repeated by every lane:
//   * per-cell inputs (X_s, the temperature derivatives, Y_s) come from the
//     cell kernel and are staged in the group's LDS; lane s evaluates the
//     Gibbs energy and enthalpy of species s;
//   * the reactions are taken G at a time, one per lane: the lane evaluates
//     the rates of its reaction and writes its record (dq_r/d rho_u for every
//     u, q_r, dq_r/dT, dq_r/dTv) to LDS;
//   * the lane of species t then adds M_t nu_tr times each record of the
//     chunk to its row (d omega_t / d rho_u, d omega_t / dT, dTv);
//   * sums over species (the total-density row of the coupled block, the
//     vibrational-energy source and its Landau-Teller part, one species per
//     lane) are group sums through LDS;
//   * the block row, then an in-place Gauss-Jordan inversion with partial
//     pivoting across the group (pivot candidates and rows through LDS);
//   * the lane whose row became pivot r writes row r of the inverse, each
//     entry to the column of the lane that was pivot at its step.
// Used for ns >= BLOCK_NS_MIN; the cell kernel writes the right-hand sides, push
// data and the per-cell hand-off that this kernel reads.
#pragma once
#include "csi_kernels.hpp"

namespace csi {

struct BlockOut {
  void *gS[2];                 // group schedule: record staging of part 0 (coupled / flow), 1 (species)
  void *Dinv;                  // hyperplane schedule: cell-major inverses (layout as the cell kernel's)
  int group_c;                 // 0: hyperplane schedule; > 0: group schedule
  const double *hb;            // [hb_fields][N] from the cell kernel
  const float *Jsur;           // surrogate J_C, cell-major [N][ns][ns]
  unsigned long long *ddfail;  // cells whose surrogate block failed the dominance check
  const int *surr_off;         // >= 0: surrogate switched off
  int *bad;                    // first singular cell
  float *jc_out;               // non-null: write the species block's J_C [n_lim][ns][ns] (FP32) and stop
  long n_lim;                  // cells written with jc_out
  SampleMap smap;              // with jc_out: row r of jc_out is cell smap(r)
  // one temperature, flags bit 0 (the cell kernel formed the residual in
  // this pass without the chemical source): R [nv][N] receives the source
  // -V omega_s of the species rows and the right-hand side's species rows
  // -R_s are rewritten (hyperplane schedule: b [nsol][N])
  double *R;
  void *b;
};

template <int NS, int NT, int MODE> struct BlockDims {
  static constexpr int NF = NT == 2 ? 5 : 4, NB = NF + NS - 1, NV = NS + 3 + (NT == 2 ? 1 : 0);
  static constexpr int G = MODE == 0 ? NB : NS, C = 64 / G;
  static constexpr int RW = NS + 3;   // reaction record: dq/d rho_u (u < NS), q, dq/dT, dq/dTv
  static constexpr int NSUM = 9;      // scalars summed over the group
  static constexpr bool SUMS = MODE == 0 || NT == 2;
  // per-group LDS (doubles): hand-off X | dT/dq | dTv/dq | Y, then g/RT | h/RT^2,
  // then a scratch area
  static constexpr int O_X = 0, O_TQ = NS, O_Y = NS + 2 * NV, O_GH = 2 * NS + 2 * NV, O_EV = 4 * NS + 2 * NV;
  static constexpr int O_S = O_EV + (NT == 2 ? NS : 0);
  static constexpr int NHB = 2 * NS + 2 * NV;
  // the scratch area holds, one after the other (wave syncs between them):
  // the chunk's reaction records [G][RW], the scalar sums [NSUM][G] + NSUM,
  // the column sums [G][NS] + NS, the inversion's rows [G][G] + keys/pivots
  static constexpr int O_SUM = 0;
  static constexpr int SCR_SUM = SUMS ? NSUM * G + NSUM : 0;
  static constexpr int SCR_CS = SUMS ? G * NS + NS : 0;
  static constexpr int SCR_INV = G * G + G;
  static constexpr int SCR0 = G * RW > SCR_SUM ? G * RW : SCR_SUM;
  static constexpr int SCR1 = SCR_CS > SCR_INV ? SCR_CS : SCR_INV;
  static constexpr int SCR = SCR0 > SCR1 ? SCR0 : SCR1;
  static constexpr int BUF = O_S + SCR;
};

// Workgroups are handed to the eight XCDs in turn (b mod 8), and each XCD has
// its own L2.  Cells of adjacent blocks share cache lines of the per-cell
// fields (three to five cells per block, sixteen doubles per line), so block b
// takes the logical position that gives every XCD one contiguous run of
// blocks: the lines a block fetches are then mostly in its own XCD's L2.
// A bijection of [0, n).
__device__ __forceinline__ unsigned xcd_block(unsigned b, unsigned n) {
  const unsigned x = b % 8u, k = b / 8u, per = n / 8u, rem = n % 8u;
  return x * per + (x < rem ? x : rem) + k;
}

// Exchange point between the lanes of one wave through LDS: stores made before
// it are seen by loads after it.  The LDS operations of a wave complete in
// order; the fences keep the compiler from moving memory operations across it
// and the (convergent) wave barrier from duplicating or merging the code
// around it.  Every lane of the wave passes it together.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Sum over the group of each lane's vector v[NS]; every lane receives the sums.
// `live`: the lane's group owns the buffer (other lanes only read).
template <int NS, int G>
__device__ __forceinline__ void group_colsum(double *scr, int k, bool live, const double (&v)[NS],
                                             double (&s)[NS]) {
  double *cs = scr, *res = scr + G * NS;
  if (live)
#pragma unroll
    for (int u = 0; u < NS; ++u) cs[k * NS + u] = v[u];
  wave_sync();
  const int kk = k < NS ? k : NS - 1;
  double acc = 0.0;
  for (int j = 0; j < G; ++j) acc += cs[j * NS + kk];
  if (live && k < NS) res[k] = acc;
  wave_sync();
#pragma unroll
  for (int u = 0; u < NS; ++u) s[u] = res[u];
  wave_sync();
}
// sums over the group of N scalars per lane; every lane receives them
// (lane k sums slots k, k + G, ...; sb holds [N][G] then the N sums)
template <int N, int G>
__device__ __forceinline__ void group_sum(double *sb, int k, bool live, const double (&v)[N], double (&s)[N]) {
  if (live)
#pragma unroll
    for (int j = 0; j < N; ++j) sb[j * G + k] = v[j];
  wave_sync();
#pragma unroll
  for (int q0 = 0; q0 < N; q0 += G) {
    const int jj = q0 + k < N ? q0 + k : N - 1;
    double acc = 0.0;
    for (int l = 0; l < G; ++l) acc += sb[jj * G + l];
    if (live && q0 + k < N) sb[N * G + q0 + k] = acc;
  }
  wave_sync();
#pragma unroll
  for (int j = 0; j < N; ++j) s[j] = sb[N * G + j];
  wave_sync();
}

// In-place Gauss-Jordan inversion with partial pivoting of the G x G matrix
// whose row k is A (lane k of the group).  Column kc takes as pivot the unused
// row of largest magnitude; that lane becomes logical row kc (pos = kc).  The
// candidates are ranked by one 32-bit key per lane: the bits of |a| in FP32
// with the low 6 bits replaced by 63 - k (so ties, and magnitudes within
// about 2^-17 of each other, go to the lowest lane; a NaN counts as zero;
// rows already used rank below every unused one).  With the rows so
// permuted, B = P A is inverted in place, one column per step: the pivot row
// is scaled by 1/b_kk (its entry kc becomes 1/b_kk), every other row subtracts
// its multiple of it (its entry kc becomes -b_ik/b_kk).  On return lane k
// holds row pos of B^-1 = A^-1 P^T, i.e. A[r] = (A^-1)[pos][piv(r)], where
// piv(r), the lane chosen at step r, is left in pv[r].  The keys and each
// lane's scaled row go through the group's LDS (every lane writes its own
// slot; the group reads the pivot's), scr: [G][G] rows, then G keys.  False
// on a zero pivot (the group agrees).
template <int G>
__device__ __forceinline__ bool group_invert(double *scr, int *pv, int k, bool live, double (&A)[G], int &pos) {
  static_assert(G <= 64, "lane index in 6 bits");
  double *rows = scr;
  unsigned *keys = reinterpret_cast<unsigned *>(scr + G * G);
  pos = -1;
  bool ok = true;
#pragma unroll
  for (int kc = 0; kc < G; ++kc) {
    const double f = A[kc], ip = 1.0 / f;
    const float a = float(fabs(f));
    const unsigned mag = __float_as_uint(a >= 0.0f ? a : 0.0f) & ~63u;
    const unsigned key = pos >= 0 ? 0u : ((mag > 64u ? mag : 64u) | unsigned(63 - k));
    if (live) {
      keys[k] = key;
#pragma unroll
      for (int c = 0; c < G; ++c) rows[k * G + c] = c == kc ? ip : A[c] * ip;
    }
    wave_sync();
    unsigned best = 0u;
    for (int j = 0; j < G; ++j) best = keys[j] > best ? keys[j] : best;
    if ((best >> 6) <= 1u) ok = false;  // the pivot is zero (or below FP32's range)
    const int piv = 63 - int(best & 63u);
    const bool me = k == piv;
    if (me) pos = kc;
    if (live) pv[kc] = piv;
    // pivot lane: 0 * A + 1 * r; other lanes: A - f r (entry kc: -f r)
    const double fe = me ? -1.0 : f, sc = me ? 0.0 : 1.0;
    const double *pr = rows + piv * G;
#pragma unroll
    for (int c = 0; c < G; ++c) {
      const double r = pr[c];
      A[c] = c == kc ? -fe * r : fma(-fe, r, A[c] * sc);
    }
    wave_sync();
  }
  return ok;
}

// The same inversion as group_invert (pivot order, pivot keys, result layout
// and zero-pivot test alike) with fewer operations per column, used for the
// split species block (at the coupled block's width its larger register
// footprint costs a wave per SIMD).  B = P A is inverted in place, one column
// per step, without
// normalising the pivot row: the pivot lane publishes its row unchanged
// (entry kc then set to 1), every other row subtracts g = b_ik / b_kk times
// it (its entry kc becomes -g); a row that was pivot is p times the
// normalised one for its own pivot value p, and the later steps keep that
// factor, so each lane divides its row by its own pivot value at the end.
// Per column and lane: one multiply-add per entry; only the pivot lanes
// store a row.  On return lane k holds row pos of B^-1 = A^-1 P^T, i.e.
// A[r] = (A^-1)[pos][piv(r)], where piv(r), the lane chosen at step r, is
// left in pv[r].  The keys and the pivot rows go through the group's LDS
// (scr: [G][G] rows, then G keys).  False on a zero pivot (the group agrees).
template <int G>
__device__ __forceinline__ bool group_invert_unnormalised(double *scr, int *pv, int k, bool live, double (&A)[G], int &pos) {
  static_assert(G <= 64, "lane index in 6 bits");
  double *rows = scr;
  unsigned *keys = reinterpret_cast<unsigned *>(scr + G * G);
  pos = -1;
  bool ok = true;
  double myip = 1.0;
#pragma unroll
  for (int kc = 0; kc < G; ++kc) {
    const double f = A[kc];
    const float a = float(fabs(f));
    const unsigned mag = __float_as_uint(a >= 0.0f ? a : 0.0f) & ~63u;
    const unsigned key = pos >= 0 ? 0u : ((mag > 64u ? mag : 64u) | unsigned(63 - k));
    if (live) keys[k] = key;
    wave_sync();
    unsigned best = 0u;
    for (int j = 0; j < G; ++j) best = keys[j] > best ? keys[j] : best;
    if ((best >> 6) <= 1u) ok = false;  // the pivot is zero (or below FP32's range)
    const int piv = 63 - int(best & 63u);
    const bool me = k == piv;
    if (me) pos = kc;
    if (live) pv[kc] = piv;
    // the pivot lane of each group publishes its row (the others store nothing)
    if (me && live) {
#pragma unroll
      for (int c = 0; c < G; ++c) rows[k * G + c] = A[c];
    }
    wave_sync();
    const double *pr = rows + piv * G;
    const double ip = 1.0 / pr[kc];
    const double gk = me ? 0.0 : f * ip;
    if (me) myip = ip;
    // the pivot row in chunks of eight (a scheduling fence between chunks
    // keeps the compiler from holding the whole row in registers at once)
#pragma unroll
    for (int c = 0; c < G; ++c) {
      const double r = pr[c];
      A[c] = c == kc ? (me ? 1.0 : -gk) : fma(-gk, r, A[c]);
      if (c % 8 == 7) __builtin_amdgcn_sched_barrier(0);
    }
  }
#pragma unroll
  for (int c = 0; c < G; ++c) A[c] *= myip;
  wave_sync();
  return ok;
}

// Record of reaction r at (T, Tv) into D[RW] (the same kinetics as
// `chemistry`): D[u] = (dq_r / dX_u) / M_u (third-body efficiencies and the
// law-of-mass-action products), D[NS] = q_r, D[NS+1] = dq_r/dT, D[NS+2] =
// dq_r/dTv, with q_r = M (k_f prod X_reac - k_b prod X_prod).  X, GH: the
// group's concentrations and g/RT, h/RT^2 per species.
template <int NS, int NT>
__device__ __forceinline__ void reaction_record(const Mech &m, int r, double T, double Tv, double lnT, double lnTv,
                                                double lnc0, const double *X, const double *GH, double *D) {
  const Reaction &R = m.rx[r];
  // the reaction's fields and species lists, loaded together (fixed sizes)
  const double lnA = R.lnA, b = R.b, theta = R.theta;
  const int tctl = R.tctl, third = R.third, nreac = R.nreac, nprod = R.nprod, nnet = R.nnet, dnu = R.dnu;
  int rs_[3], ps_[3], es_[6], en_[6];
#pragma unroll
  for (int e = 0; e < 3; ++e) {
    rs_[e] = R.reac[e];
    ps_[e] = R.prod[e];
  }
#pragma unroll
  for (int e = 0; e < 6; ++e) {
    es_[e] = R.net_s[e];
    en_[e] = R.net_nu[e];
  }
  double lnTf = lnT, dTf_dT = 1.0, dTf_dTv = 0.0, Tf = T;
  if (NT == 2 && tctl == 1) {
    lnTf = 0.5 * (lnT + lnTv);
    Tf = exp(lnTf);
    dTf_dT = 0.5 * Tf / T;
    dTf_dTv = 0.5 * Tf / Tv;
  } else if (NT == 2 && tctl == 2) {
    lnTf = lnTv;
    Tf = Tv;
    dTf_dT = 0.0;
    dTf_dTv = 1.0;
  }
  const double kf = exp(lnA + b * lnTf - theta / Tf);
  double lnKc = double(dnu) * lnc0, dlnKc = -double(dnu) / T;
#pragma unroll
  for (int e = 0; e < 6; ++e)
    if (e < nnet) {
      lnKc -= double(en_[e]) * GH[es_[e]];
      dlnKc += double(en_[e]) * GH[NS + es_[e]];
    }
  const double kb = exp(lnA + b * lnT - theta / T - lnKc);
  double Xr[3], Xp[3], Pf = 1.0, Pb = 1.0;
#pragma unroll
  for (int e = 0; e < 3; ++e) {
    Xr[e] = e < nreac ? X[rs_[e]] : 1.0;
    Xp[e] = e < nprod ? X[ps_[e]] : 1.0;
  }
#pragma unroll
  for (int e = 0; e < 3; ++e) {
    if (e < nreac) Pf *= Xr[e];
    if (e < nprod) Pb *= Xp[e];
  }
  double Mc = 1.0;
  if (third) {
    Mc = 0.0;
#pragma unroll
    for (int s = 0; s < NS; ++s) Mc += m.eff[r][s] * X[s];
  }
  const double net = kf * Pf - kb * Pb;
  if (third) {
#pragma unroll
    for (int u = 0; u < NS; ++u) D[u] = m.eff[r][u] * net * m.iM[u];
  } else {
#pragma unroll
    for (int u = 0; u < NS; ++u) D[u] = 0.0;
  }
  // law-of-mass-action products without factor e (in list order, as a plain product)
#pragma unroll
  for (int e = 0; e < 3; ++e)
    if (e < nreac) {
      double lo = 1.0;
#pragma unroll
      for (int f = 0; f < 3; ++f)
        if (f < nreac && f != e) lo *= Xr[f];
      D[rs_[e]] += Mc * kf * lo * m.iM[rs_[e]];
    }
#pragma unroll
  for (int e = 0; e < 3; ++e)
    if (e < nprod) {
      double lo = 1.0;
#pragma unroll
      for (int f = 0; f < 3; ++f)
        if (f < nprod && f != e) lo *= Xp[f];
      D[ps_[e]] -= Mc * kb * lo * m.iM[ps_[e]];
    }
  const double dkf_dTf = kf * (b + theta / Tf) / Tf;
  const double dkb_dT = kb * ((b + theta / T) / T - dlnKc);
  D[NS] = Mc * net;
  D[NS + 1] = Mc * (dkf_dTf * dTf_dT * Pf - dkb_dT * Pb);
  D[NS + 2] = Mc * (dkf_dTf * dTf_dTv * Pf);
}

// One group of G lanes per cell, one wave per block.  MODE 0: coupled block
// (G = nb; lane 0 carries the last species' chemistry row, which only enters
// the total-density row; lanes 1..4 have no species row); MODE 1: split
// species block (G = ns) and the flow block's inverse (lanes k < nf).
template <int NS, int NT, typename RT, int MODE>
__global__ void __launch_bounds__(64) k_block(Geo g, const Mech *__restrict__ mech, const double *__restrict__ Q,
                                              const double *__restrict__ prim, int flags, BlockOut out,
                                              const int *__restrict__ done) {
  using BD = BlockDims<NS, NT, MODE>;
  constexpr int G = BD::G, C = BD::C, NF = BD::NF, NB = BD::NB, NV = BD::NV, RW = BD::RW;
  __shared__ double sh[C][BD::BUF];
  if (done && *done) return;
  const Mech &m = *mech;
  const int lane = threadIdx.x;
  const int grp = lane / G, k = lane - grp * G;
  const bool live = grp < C;  // lanes past the last group read group 0's buffer and write nothing
  double *buf = sh[live ? grp : 0];
  const long cell = long(xcd_block(blockIdx.x, gridDim.x)) * C + grp;
  const bool real = live && cell < (out.jc_out ? out.n_lim : long(g.N));
  // sample mode: output row `cell` holds grid cell smap(cell)
  const int p = int(real ? (out.jc_out ? out.smap(cell, g.N) : cell) : 0);
  const int i = p % g.ni, j = p / g.ni;
  const int pc = padc(g, i, j);
  const size_t NP = g.NP;
  const double T = prim[F_T * NP + pc], Tv = NT == 2 ? prim[F_TV * NP + pc] : T, pp = prim[F_P * NP + pc];
  const double Vp = g.V[p];
  const double *X = buf + BD::O_X, *TQ = buf + BD::O_TQ, *Ysh = buf + BD::O_Y;
  double *GH = buf + BD::O_GH, *scr = buf + BD::O_S;
  // stage the hand-off; lane s evaluates species s's Gibbs energy and enthalpy
  const double lnT = log(T), lnTv = log(Tv);
  if (live) {
    for (int f = k; f < BD::NHB; f += G) {
      // one temperature: the dTv/dq row is not handed over (its derivatives
      // enter with the zero dq/dTv of the reaction records)
      const bool tv_row = f >= NS + NV && f < NS + 2 * NV;
      buf[f] = NT == 1 && tv_row ? 0.0 : out.hb[size_t(HB_X + f) * g.N + p];
    }
    if (k < NS) {
      GH[k] = gRT(m, k, T, lnT);
      GH[NS + k] = hRT2(m, k, T);
      if (NT == 2) buf[BD::O_EV + k] = eve_s(m, k, Tv);
    }
  }
  wave_sync();
  // this lane's species row
  const int t = MODE == 0 ? (k >= NF ? k - NF : (k == 0 ? NS - 1 : -1)) : (k < NS ? k : -1);
  const int tc = t >= 0 ? t : 0;
  double A[G];
  const double d0 = out.hb[p], d1 = MODE == 1 ? out.hb[size_t(g.N) + p] : 0.0;  // dK | dF, dC
  // split form: surrogate species block, accepted when the group's block is
  // strictly row diagonally dominant with a positive diagonal in molar units
  bool use_sur = false;
  if (MODE == 1 && (flags & 4) && out.Jsur && *out.surr_off < 0) {
    double off = 0.0, dkk = 0.0;
#pragma unroll
    for (int c = 0; c < NS; ++c) {
      const double a = (c == k ? d1 : 0.0) - Vp * double(out.Jsur[(size_t(p) * NS + tc) * NS + c]);
      if (c == k) dkk = a;
      else off += fabs(a) * m.M[c];
    }
    const bool dd = dkk > 0.0 && dkk * m.M[tc] > off;
    const unsigned long long bal = __ballot(dd);
    constexpr unsigned long long gm = G >= 64 ? ~0ull : (1ull << G) - 1;
    use_sur = ((bal >> (grp * G)) & gm) == gm;
    if (!use_sur && k == 0 && real) atomicAdd(out.ddfail, 1ull);
  }
  // the exact rows, unless every group of the wave takes the surrogate block
  // (two temperatures: the flow block needs them anyway)
  double w_t = 0.0, row[NS], dwT = 0.0, dwTv = 0.0;
#pragma unroll
  for (int u = 0; u < NS; ++u) row[u] = 0.0;
  const bool exact = MODE == 0 || NT == 2 || __ballot(real && !use_sur) != 0ull;
  // one temperature: the species source of the residual comes from the
  // reaction records here (the cell kernel left it out)
  const bool src = NT == 1 && (flags & 1) && !out.jc_out && out.R;
  if (exact || src) {
    const double lnc0 = log(1.0e5 / (RU * T));
    for (int r0 = 0; r0 < m.nr; r0 += G) {
      if (live && r0 + k < m.nr) reaction_record<NS, NT>(m, r0 + k, T, Tv, lnT, lnTv, lnc0, X, GH, scr + k * RW);
      wave_sync();
      const int nk = m.nr - r0 < G ? m.nr - r0 : G;
      double av[G];  // M_t nu_tr of the chunk's reactions, loaded together
#pragma unroll
      for (int kk = 0; kk < G; ++kk) av[kk] = t >= 0 && kk < nk ? m.nuM[r0 + kk][tc] : 0.0;
#pragma unroll
      for (int kk = 0; kk < G; ++kk) {
        const double a = av[kk];
        if (kk < nk && a != 0.0) {
          const double *D = scr + kk * RW;
          if (exact) {
#pragma unroll
            for (int u = 0; u < NS; ++u) row[u] += a * D[u];
          }
          w_t += a * D[NS];
          dwT += a * D[NS + 1];
          dwTv += a * D[NS + 2];
        }
      }
      wave_sync();
    }
  }
  if (src && real && t >= 0) {
    const double Rt = out.R[size_t(t) * g.N + p] - Vp * w_t;
    out.R[size_t(t) * g.N + p] = Rt;
    // the right-hand side row of species t: split species row t; coupled z
    // row k (the closing species, lane 0, enters only the total density)
    const int row_b = MODE == 1 ? t : (k >= NF ? k : -1);
    if (row_b >= 0) {
      if (out.group_c > 0) {
        constexpr RecShape SB = rec_shape(MODE == 1 ? PART_SPECIES : PART_COUPLED, NS, NT, sizeof(RT));
        RT *Sb = reinterpret_cast<RT *>(out.gS[MODE == 1 ? 1 : 0]);
        Sb[st_idx(SB, g.N, 1, dw_b(row_b), p)] = RT(-Rt);
      } else {
        RT *bb = reinterpret_cast<RT *>(out.b);
        bb[long(MODE == 1 ? NF + row_b : row_b) * g.N + p] = RT(-Rt);
      }
    }
  }
  // group sums: Landau-Teller terms (species k), pressure derivatives, the
  // e_ve-weighted production terms and the total-density row's T columns
  double dwv_dT = 0.0, dwv_dTv = 0.0, Sd0 = 0.0, Sd1 = 0.0, own_dr = 0.0, lt_sum = 0.0;
  const double ev = NT == 2 && t >= 0 ? eve_s(m, tc, Tv) : 0.0;
  if (BD::SUMS) {
    double v[BD::NSUM], S[BD::NSUM];
#pragma unroll
    for (int q = 0; q < BD::NSUM; ++q) v[q] = 0.0;
    if (NT == 2 && k < NS) {
      const double rs = Q[size_t(k) * g.N + p];
      if (m.kind[k] == MOLECULE && m.thv[k] > 0.0) {
        const double Tm13 = exp(-lnT / 3.0);
        const double itau = pp / ATM * exp(18.42 - m.lta[k] * (Tm13 - m.ltb[k]));
        const double evT = evib(m.R[k], m.thv[k], T), evTv = evib(m.R[k], m.thv[k], Tv);
        const double term = rs * (evT - evTv) * itau;
        own_dr = (evT - evTv) * itau;
        v[0] = term;
        v[1] = rs * cvvib(m.R[k], m.thv[k], T) * itau + term * (m.lta[k] / 3.0) * Tm13 / T;
        v[2] = -rs * cvvib(m.R[k], m.thv[k], Tv) * itau;
      }
      const bool el = m.kind[k] == ELECTRON;
      v[3] = el ? 0.0 : rs * m.R[k];
      v[4] = el ? rs * m.R[k] : 0.0;
    }
    if (NT == 2) {
      v[5] = dwT * ev;
      v[6] = dwTv * ev + w_t * (t >= 0 ? cvve_s(m, tc, Tv) : 0.0);
    }
    v[7] = dwT;
    v[8] = dwTv;
    group_sum<BD::NSUM, G>(scr + BD::O_SUM, k, live, v, S);
    lt_sum = S[0];
    dwv_dT = S[1] + lt_sum * S[3] / pp + S[5];
    dwv_dTv = S[2] + lt_sum * S[4] / pp + S[6];
    Sd0 = S[7];
    Sd1 = S[8];
  }
  // d omega_ve / d rho_u: the e_ve-weighted species rows, the Landau-Teller
  // terms of species u and the pressure dependence of the relaxation time
  double dwv_dr[NS];
#pragma unroll
  for (int u = 0; u < NS; ++u) dwv_dr[u] = 0.0;
  if (NT == 2) {
    double wr[NS];
#pragma unroll
    for (int u = 0; u < NS; ++u) wr[u] = row[u] * ev + (u == k ? own_dr : 0.0);
    group_colsum<NS, G>(scr, k, live, wr, dwv_dr);
#pragma unroll
    for (int u = 0; u < NS; ++u) dwv_dr[u] += lt_sum * (m.R[u] * (m.kind[u] == ELECTRON ? Tv : T)) / pp;
  }
  bool ok;
  int pos;
  int *pv = reinterpret_cast<int *>(scr + G * G) + G;  // pivot lane of each step (after the keys)
  if (MODE == 0) {
    // this lane's row of dS/dq (storage columns): a species row, the total
    // density row (the sum of all species rows) or the vibrational-energy row
    double rv[NS], vT = dwT, vTv = dwTv;
    {
      double S1[NS];
      group_colsum<NS, G>(scr, k, live, row, S1);
#pragma unroll
      for (int u = 0; u < NS; ++u) rv[u] = k >= NF ? row[u] : k == 0 ? S1[u] : 0.0;
    }
    if (k == 0) {
      vT = Sd0;
      vTv = Sd1;
    } else if (k < NF) {
      vT = vTv = 0.0;
    }
    if (NT == 2 && k == 4) {
#pragma unroll
      for (int u = 0; u < NS; ++u) rv[u] = dwv_dr[u];
      vT = dwv_dT;
      vTv = dwv_dTv;
    }
    auto jq = [&](int c) { return (c < NS ? rv[c < NS ? c : 0] : 0.0) + vT * TQ[c] + vTv * TQ[NV + c]; };
    const double jl = jq(NS - 1);
#pragma unroll
    for (int c = 0; c < NB; ++c) {
      const double jz = c == 0 ? jl : c < NF ? jq(NS + c - 1) : jq(c - NF) - jl;
      A[c] = (c == k ? d0 : 0.0) - Vp * jz;
    }
    ok = group_invert<G>(scr, pv, k, live, A, pos);
    if (real) {
      if (out.group_c > 0) {
        constexpr RecShape S = rec_shape(PART_COUPLED, NS, NT, sizeof(RT));
        RT *St = reinterpret_cast<RT *>(out.gS[0]);
#pragma unroll
        for (int r = 0; r < NB; ++r) St[st_idx(S, g.N, 0, rw_d(S, pos, pv[r]), p)] = RT(A[r]);
      } else {
        RT *Dcm = reinterpret_cast<RT *>(out.Dinv);
#pragma unroll
        for (int r = 0; r < NB; ++r) Dcm[long(pos * NB + pv[r]) * g.N + p] = RT(A[r]);
      }
    }
  } else {
    const double dF = d0, dC = d1;
    // flags bit 3: the species block with the velocities and the internal
    // (and vibrational) energy densities held, so that the temperatures follow
    // the composition: J_C += d omega_t/dT dT/d rho_c (+ the Tv term), the
    // temperature derivatives taken along the direction that adds mass at the
    // cell's velocity and kinetic energy
    // (flags bit 4, two temperatures: Tv held too, rho e_ve taking the added
    // mass's e_ve,r(Tv) out of the same internal energy)
    const bool te = (flags & 8) != 0 && !use_sur;
    const bool hold_tv = NT == 2 && (flags & 16) != 0;
    const double uu = prim[F_U * NP + pc], vv = prim[F_V * NP + pc], ke = 0.5 * (uu * uu + vv * vv);
    double jr[NS];
#pragma unroll
    for (int c = 0; c < NS; ++c) {
      double jc = use_sur ? double(out.Jsur[(size_t(p) * NS + tc) * NS + c]) : row[c];
      if (te) {
        const double ev = hold_tv ? buf[BD::O_EV + c] : 0.0;
        jc += dwT * (TQ[c] + uu * TQ[NS] + vv * TQ[NS + 1] + ke * TQ[NS + 2] + (NT == 2 ? ev * TQ[NS + 3] : 0.0));
        if (NT == 2)
          jc += dwTv * (TQ[NV + c] + uu * TQ[NV + NS] + vv * TQ[NV + NS + 1] + ke * TQ[NV + NS + 2] +
                        ev * TQ[NV + NS + 3]);
      }
      jr[c] = jc;
      A[c] = (c == k ? dC : 0.0) - Vp * jc;
    }
    // training samples of the species block's source Jacobian (row-major
    // (s, r) per cell); the whole wave leaves here
    if (out.jc_out) {
      if (real && t >= 0)
#pragma unroll
        for (int c = 0; c < NS; ++c) out.jc_out[(size_t(cell) * NS + t) * NS + c] = float(jr[c]);
      return;
    }
    // flow block: diagonal 1/dF, and in two temperatures the rho e_ve row
    // -V d omega_ve / d Q_F (frozen Y) eliminated in closed form
    double df6[6] = {1.0 / dF, 0.0, 0.0, 0.0, 0.0, 0.0};
    if (NT == 2) {
      double a0 = 0.0;
#pragma unroll
      for (int s = 0; s < NS; ++s) a0 += Ysh[s] * (dwv_dr[s] + dwv_dT * TQ[s] + dwv_dTv * TQ[NV + s]);
      double dwv[5];
      dwv[0] = a0;
#pragma unroll
      for (int c = 1; c < 5; ++c) dwv[c] = dwv_dT * TQ[NS - 1 + c] + dwv_dTv * TQ[NV + NS - 1 + c];
#pragma unroll
      for (int c = 0; c < 4; ++c) df6[1 + c] = Vp * dwv[c];
      const double piv = dF - Vp * dwv[4];
      if (piv == 0.0 && real && out.bad && k == 0) atomicMin(out.bad, p);
      df6[5] = 1.0 / piv;
    }
    // the flow block's inverse first (its inputs then end before the inversion)
    if (real) {
      if (out.group_c > 0) {
        if (k < NF) {
          constexpr RecShape SF = rec_shape(PART_FLOW, NS, NT, sizeof(RT));
          RT *Sf = reinterpret_cast<RT *>(out.gS[0]);
#pragma unroll
          for (int c = 0; c < NF; ++c) {
            double v = c == k && k < 4 ? df6[0] : 0.0;
            if (NT == 2 && k == 4) v = c < 4 ? df6[1 + c] * df6[0] * df6[5] : df6[5];
            Sf[st_idx(SF, g.N, 0, rw_d(SF, k, c), p)] = RT(v);
          }
        }
      } else if (k == 0) {
        RT *Dcm = reinterpret_cast<RT *>(out.Dinv);
#pragma unroll
        for (int c = 0; c < 6; ++c) Dcm[long(c) * g.N + p] = RT(df6[c]);
      }
    }
    ok = group_invert_unnormalised<G>(scr, pv, k, live, A, pos);
    if (real) {
      if (out.group_c > 0) {
        constexpr RecShape S = rec_shape(PART_SPECIES, NS, NT, sizeof(RT));
        RT *St = reinterpret_cast<RT *>(out.gS[1]);
#pragma unroll
        for (int r = 0; r < NS; ++r) St[st_idx(S, g.N, 0, rw_d(S, pos, pv[r]), p)] = RT(A[r]);
      } else {
        RT *Dcm = reinterpret_cast<RT *>(out.Dinv);
#pragma unroll
        for (int r = 0; r < NS; ++r) Dcm[long(6 + pos * NS + pv[r]) * g.N + p] = RT(A[r]);
      }
    }
  }
  if (!ok && real && k == 0 && out.bad) atomicMin(out.bad, p);
}

}  // namespace csi
