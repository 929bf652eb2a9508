// Persistent strip-wavefront LU-SGS sweeps.
//
// The i+j hyperplane order of the sweeps (paper Section 2.2, forward
// (D+L) dQ* = RHS and backward (D+U) dQ = D dQ*) is executed by one wavefront
// per strip of W columns.  At step d, lane l of the strip owns cell
// (i0 + l, d - l): its west neighbour was computed by lane l-1 one step
// earlier and its south neighbour by the same lane one step earlier, so the
// off-diagonal products are pushed through a lane shuffle and a register
// instead of memory.  Only the strip boundary goes through HBM: the last
// lane publishes its push for the next strip and a release-ordered progress
// counter; the next strip's first lane waits for it with acquire loads.
// Strips are taken in dependency order from an atomic ticket, so every wait
// targets a strip that is already running (no deadlock); a bounded spin with a
// shared abort flag guarantees that every wave exits.
//
// Per-cell records are stored in "strip layout": position
// ((s * NSTEP + d) * W + l), consecutive lanes of a step adjacent in memory.
#pragma once
#include "csi_sweep.hpp"

namespace csi {

struct StripMap {
  int W, NSTEP, nstrip;
  long LEN;
};

__host__ __device__ inline StripMap strip_map(int ni, int nj, int W) {
  StripMap s;
  s.W = W;
  s.NSTEP = nj + W - 1;
  s.nstrip = (ni + W - 1) / W;
  s.LEN = long(s.nstrip) * s.NSTEP * W;
  return s;
}
__host__ __device__ inline long strip_pos(const StripMap &sm, int i, int j) {
  int s = i / sm.W, l = i - s * sm.W;
  return (long(s) * sm.NSTEP + j + l) * sm.W + l;
}

// record field counts
template <int NS, int NT> struct Rec {
  using D = Dims<NS, NT>;
  static constexpr int NSOL = D::nsplit;                       // b, xs, x rows (max over modes)
  static constexpr int NDINV = (D::nb * D::nb > 6 + NS * NS) ? D::nb * D::nb : 6 + NS * NS;
  static constexpr int NSTATE = 6 + 2 * NS;                    // u v H eve pE pv | Y[NS] pr[NS] (split: prY at 6)
  static constexpr int NFACE = 16;                             // mE mN mW mS (x,y) | cE cN cW cS | cCE cCN cCW cCS
};

struct StripArgs {
  void *b, *Dinv, *state, *face, *xs, *x;  // RT arrays, strip layout, field stride LEN
  void *bnd;                               // RT [nstrip][nj][NSOL] boundary pushes
  int *prog;                               // [nstrip] forward progress (completed steps)
  int *progb;                              // [nstrip] backward progress
  int *ticket;                             // [2] forward / backward tickets
  int *abort_flag;                         // set by a wave whose wait timed out
  int mode;
  int pub_every;  // progress published every pub_every steps (and at the last step)
  long spin_limit;
};

template <typename RT> __device__ __forceinline__ RT shfl_up1(RT v) { return __shfl_up(v, 1, 64); }
template <typename RT> __device__ __forceinline__ RT shfl_down1(RT v) { return __shfl_down(v, 1, 64); }

// Strip-boundary traffic uses device-coherent (agent-scope) atomic loads and
// stores for both the pushed vectors and the progress counters; the producer
// waits for its data stores to complete (s_waitcnt) before it stores the
// counter, so a consumer that reads the counter sees the data.  This avoids
// the L2 write-back a release fence would issue on every step.
__device__ __forceinline__ int load_acquire_relaxed(const int *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void publish(int *p, int v) {
  __builtin_amdgcn_s_waitcnt(0);
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename RT> __device__ __forceinline__ void put_coherent(RT *p, RT v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename RT> __device__ __forceinline__ RT get_coherent(const RT *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// wait until *p >= need; returns false on timeout / abort (then sets the abort flag)
__device__ __forceinline__ bool wait_at_least(const int *p, int need, int *abort_flag, long spin_limit) {
  long n = 0;
  while (load_acquire_relaxed(p) < need) {
    if (__hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return false;
    if (++n > spin_limit) {
      __hip_atomic_store(abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return false;
    }
    __builtin_amdgcn_s_sleep(1);
  }
  return true;
}

// push O_QP x from cell P to neighbour Q: A_P(m) x - c x, m the half-length-
// scaled outward normal of Q across the shared face (coupled / flow parts),
// (u_P . m - cC) x for the species part.
template <int NS, int NT, typename RT>
__device__ __forceinline__ void push_op(int mode, const NbState<NS, RT> &st, RT mx, RT my, RT c, RT cC, const RT *x,
                                        RT *o) {
  using D = Dims<NS, NT>;
  constexpr int NB = D::nb, NF = D::nf;
  if (mode == 0) {
    RT a[NB];
    jvp_coupled<NS, NT, RT>(st, mx, my, x, a);
#pragma unroll
    for (int k = 0; k < NB; ++k) o[k] = a[k] - c * x[k];
  } else {
    RT a[NF];
    jvp_flow<NS, NT, RT>(st, mx, my, x, a);
#pragma unroll
    for (int k = 0; k < NF; ++k) o[k] = a[k] - c * x[k];
    RT coef = st.u * mx + st.v * my - cC;
#pragma unroll
    for (int k = 0; k < NS; ++k) o[NF + k] = coef * x[NF + k];
  }
}

// Per-step record of one cell, loaded in one batch (and, when it fits in
// registers, one step ahead of its use) so that a step costs one memory round
// trip or none.  FWD: the cell's E and N push coefficients; backward: W and S
// pushes plus dQ*.
template <int NS, int NT, typename RT, int MODE, bool FWD> struct StepRec {
  using D = Dims<NS, NT>;
  static constexpr int NSOL = MODE == 0 ? D::nb : D::nsplit;
  static constexpr int ND = MODE == 0 ? D::nb * D::nb : 6 + NS * NS;
  static constexpr int NST = MODE == 0 ? 6 + 2 * NS : 7;
  static constexpr bool PREFETCH = sizeof(RT) * (2 * NSOL + ND + NST + 8) <= 8 * 72;
  RT v[NSOL];  // forward: RHS b; backward: dQ*
  RT Dm[ND];
  RT st[NST];
  RT f[8];     // push 1 (mx, my, c, cC), push 2 (mx, my, c, cC)

  __device__ __forceinline__ void load(const StripArgs &a, long LEN, long pos) {
    const RT *src = reinterpret_cast<const RT *>(FWD ? a.b : a.xs);
    const RT *Di = reinterpret_cast<const RT *>(a.Dinv);
    const RT *stt = reinterpret_cast<const RT *>(a.state);
    const RT *fc = reinterpret_cast<const RT *>(a.face);
#pragma unroll
    for (int k = 0; k < NSOL; ++k) v[k] = src[long(k) * LEN + pos];
#pragma unroll
    for (int k = 0; k < ND; ++k) Dm[k] = Di[long(k) * LEN + pos];
#pragma unroll
    for (int k = 0; k < NST; ++k) st[k] = stt[long(k) * LEN + pos];
    const int m1 = FWD ? 0 : 4, m2 = FWD ? 2 : 6, c1 = FWD ? 8 : 10, c2 = FWD ? 9 : 11;
    f[0] = fc[long(m1) * LEN + pos];
    f[1] = fc[long(m1 + 1) * LEN + pos];
    f[2] = fc[long(c1) * LEN + pos];
    f[3] = fc[long(c1 + 4) * LEN + pos];
    f[4] = fc[long(m2) * LEN + pos];
    f[5] = fc[long(m2 + 1) * LEN + pos];
    f[6] = fc[long(c2) * LEN + pos];
    f[7] = fc[long(c2 + 4) * LEN + pos];
  }

  __device__ __forceinline__ void state(NbState<NS, RT> &s) const {
    s.u = st[0]; s.v = st[1]; s.H = st[2]; s.eve = st[3]; s.pE = st[4]; s.pv = st[5];
    if (MODE == 0) {
#pragma unroll
      for (int k = 0; k < NS; ++k) { s.Y[k] = st[6 + k]; s.pr[k] = st[6 + NS + k]; }
    } else {
#pragma unroll
      for (int k = 0; k < NS; ++k) { s.Y[k] = RT(0); s.pr[k] = RT(0); }
      s.Y[0] = RT(1);
      s.pr[0] = st[6];
    }
  }

  // x = D^-1 r
  __device__ __forceinline__ void dinv(const RT *r, RT *x) const {
    constexpr int NB = D::nb, NF = D::nf;
    if (MODE == 0) {
#pragma unroll
      for (int rr = 0; rr < NB; ++rr) {
        RT acc = RT(0);
#pragma unroll
        for (int c = 0; c < NB; ++c) acc += Dm[rr * NB + c] * r[c];
        x[rr] = acc;
      }
    } else {
#pragma unroll
      for (int k = 0; k < 4; ++k) x[k] = r[k] * Dm[0];
      if (NT == 2) {
        RT acc = r[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) acc += Dm[1 + k] * x[k];
        x[4] = acc * Dm[5];
      }
#pragma unroll
      for (int rr = 0; rr < NS; ++rr) {
        RT acc = RT(0);
#pragma unroll
        for (int c = 0; c < NS; ++c) acc += Dm[6 + rr * NS + c] * r[NF + c];
        x[NF + rr] = acc;
      }
    }
  }
};

// forward sweep: one 64-thread workgroup per strip, lanes [0, W) active
template <int NS, int NT, typename RT, int W, int MODE>
__global__ void __launch_bounds__(64) k_strip_fwd(Geo g, StripArgs a, const int *__restrict__ done) {
  using Rec = StepRec<NS, NT, RT, MODE, true>;
  constexpr int NSOL = Rec::NSOL;
  if (done && *done) return;
  const StripMap sm = strip_map(g.ni, g.nj, W);
  const long LEN = sm.LEN;
  const int lane = threadIdx.x;
  __shared__ int s_strip;
  if (lane == 0) s_strip = atomicAdd(a.ticket, 1);
  __syncthreads();
  const int s = s_strip;
  if (s >= sm.nstrip) return;
  const int i = s * W + lane;
  const bool lane_ok = lane < W && i < g.ni;
  RT *xs = reinterpret_cast<RT *>(a.xs);
  RT *bnd = reinterpret_cast<RT *>(a.bnd);
  RT inW[NSOL], inS[NSOL];
#pragma unroll
  for (int k = 0; k < NSOL; ++k) { inW[k] = RT(0); inS[k] = RT(0); }
  bool ok = true;
  int seen = 0;
  const long base = long(s) * sm.NSTEP * W + lane;
  Rec cur, nxt;
  if (lane < W) cur.load(a, LEN, base);
  for (int d = 0; d < sm.NSTEP; ++d) {
    const int j = d - lane;
    const bool active = lane_ok && j >= 0 && j < g.nj;
    const long pos = base + long(d) * W;
    if (Rec::PREFETCH && lane < W && d + 1 < sm.NSTEP) nxt.load(a, LEN, pos + W);
    if (!Rec::PREFETCH && lane < W && d > 0) cur.load(a, LEN, pos);
    // the first lane takes the west push of the previous strip
    if (s > 0 && lane == 0 && active) {
      if (seen < d + W) {
        if (ok) ok = wait_at_least(a.prog + (s - 1), d + W, a.abort_flag, a.spin_limit);
        seen = load_acquire_relaxed(a.prog + (s - 1));
      }
      const RT *src = bnd + (long(s - 1) * g.nj + j) * NSOL;
#pragma unroll
      for (int k = 0; k < NSOL; ++k) inW[k] = get_coherent(src + k);
    }
    RT pushE[NSOL], pushN[NSOL];
#pragma unroll
    for (int k = 0; k < NSOL; ++k) { pushE[k] = RT(0); pushN[k] = RT(0); }
    if (active) {
      RT r[NSOL], x[NSOL];
#pragma unroll
      for (int k = 0; k < NSOL; ++k) {
        RT v = cur.v[k];
        if (i > 0) v -= inW[k];
        if (j > 0) v -= inS[k];
        r[k] = v;
      }
      cur.dinv(r, x);
#pragma unroll
      for (int k = 0; k < NSOL; ++k) xs[long(k) * LEN + pos] = x[k];
      NbState<NS, RT> st;
      cur.state(st);
      if (i + 1 < g.ni) push_op<NS, NT, RT>(MODE, st, cur.f[0], cur.f[1], cur.f[2], cur.f[3], x, pushE);
      if (j + 1 < g.nj) push_op<NS, NT, RT>(MODE, st, cur.f[4], cur.f[5], cur.f[6], cur.f[7], x, pushN);
      if (lane == W - 1 && i + 1 < g.ni) {
        RT *dst = bnd + (long(s) * g.nj + j) * NSOL;
#pragma unroll
        for (int k = 0; k < NSOL; ++k) put_coherent(dst + k, pushE[k]);
      }
    }
    if (lane == W - 1 && ((d + 1) % a.pub_every == 0 || d + 1 == sm.NSTEP)) publish(a.prog + s, d + 1);
#pragma unroll
    for (int k = 0; k < NSOL; ++k) {
      inW[k] = shfl_up1(pushE[k]);
      inS[k] = pushN[k];
    }
    if (Rec::PREFETCH) cur = nxt;
  }
}

// backward sweep: strips in reverse order, steps descending
template <int NS, int NT, typename RT, int W, int MODE>
__global__ void __launch_bounds__(64) k_strip_bwd(Geo g, StripArgs a, const int *__restrict__ done) {
  using Rec = StepRec<NS, NT, RT, MODE, false>;
  constexpr int NSOL = Rec::NSOL;
  if (done && *done) return;
  const StripMap sm = strip_map(g.ni, g.nj, W);
  const long LEN = sm.LEN;
  const int lane = threadIdx.x;
  __shared__ int s_strip;
  if (lane == 0) s_strip = sm.nstrip - 1 - atomicAdd(a.ticket + 1, 1);
  __syncthreads();
  const int s = s_strip;
  if (s < 0) return;
  const int i = s * W + lane;
  const bool lane_ok = lane < W && i < g.ni;
  RT *xo = reinterpret_cast<RT *>(a.x);
  RT *bnd = reinterpret_cast<RT *>(a.bnd);
  RT inE[NSOL], inN[NSOL];
#pragma unroll
  for (int k = 0; k < NSOL; ++k) { inE[k] = RT(0); inN[k] = RT(0); }
  bool ok = true;
  int seen = 0;
  const long base = long(s) * sm.NSTEP * W + lane;
  Rec cur, nxt;
  if (lane < W) cur.load(a, LEN, base + long(sm.NSTEP - 1) * W);
  for (int d = sm.NSTEP - 1; d >= 0; --d) {
    const int j = d - lane;
    const bool active = lane_ok && j >= 0 && j < g.nj;
    const long pos = base + long(d) * W;
    if (Rec::PREFETCH && lane < W && d > 0) nxt.load(a, LEN, pos - W);
    if (!Rec::PREFETCH && lane < W && d < sm.NSTEP - 1) cur.load(a, LEN, pos);
    if (s < sm.nstrip - 1 && lane == W - 1 && active) {
      // east neighbour (i0 + W, j) is lane 0 of strip s+1, done at its step j
      if (seen < sm.NSTEP - j) {
        if (ok) ok = wait_at_least(a.progb + (s + 1), sm.NSTEP - j, a.abort_flag, a.spin_limit);
        seen = load_acquire_relaxed(a.progb + (s + 1));
      }
      const RT *src = bnd + (long(s) * g.nj + j) * NSOL;
#pragma unroll
      for (int k = 0; k < NSOL; ++k) inE[k] = get_coherent(src + k);
    }
    RT pushW[NSOL], pushS[NSOL];
#pragma unroll
    for (int k = 0; k < NSOL; ++k) { pushW[k] = RT(0); pushS[k] = RT(0); }
    if (active) {
      RT r[NSOL], x[NSOL];
#pragma unroll
      for (int k = 0; k < NSOL; ++k) {
        RT v = RT(0);
        if (i + 1 < g.ni) v += inE[k];
        if (j + 1 < g.nj) v += inN[k];
        r[k] = v;
      }
      cur.dinv(r, x);
#pragma unroll
      for (int k = 0; k < NSOL; ++k) {
        x[k] = cur.v[k] - x[k];
        xo[long(k) * LEN + pos] = x[k];
      }
      NbState<NS, RT> st;
      cur.state(st);
      if (i > 0) push_op<NS, NT, RT>(MODE, st, cur.f[0], cur.f[1], cur.f[2], cur.f[3], x, pushW);
      if (j > 0) push_op<NS, NT, RT>(MODE, st, cur.f[4], cur.f[5], cur.f[6], cur.f[7], x, pushS);
      if (lane == 0 && s > 0) {
        RT *dst = bnd + (long(s - 1) * g.nj + j) * NSOL;
#pragma unroll
        for (int k = 0; k < NSOL; ++k) put_coherent(dst + k, pushW[k]);
      }
    }
    if (lane == 0 && ((sm.NSTEP - d) % a.pub_every == 0 || d == 0)) publish(a.progb + s, sm.NSTEP - d);
#pragma unroll
    for (int k = 0; k < NSOL; ++k) {
      inE[k] = shfl_down1(pushW[k]);
      inN[k] = pushS[k];
    }
    if (Rec::PREFETCH) cur = nxt;
  }
}

template <int NS>
__global__ void __launch_bounds__(64) k_zero_ints(int *p, int n, const int *__restrict__ done) {
  if (done && *done) return;
  for (int k = threadIdx.x; k < n; k += 64) p[k] = 0;
}

}  // namespace csi
