// Persistent strip-wavefront LU-SGS sweeps.
//
// The i+j hyperplane order of the sweeps (paper Section 2.2, forward
// (D+L) dQ* = RHS and backward (D+U) dQ = D dQ*) is executed by one wavefront
// per strip of W columns.  At step d, lane l of the strip owns cell
// (i0 + l, d - l): its west neighbour was computed by lane l-1 one step
// earlier and its south neighbour by the same lane one step earlier, so the
// off-diagonal products are pushed through a cross-lane move and a register
// instead of memory.  Only the strip boundary goes through HBM: the last lane
// publishes its push for the next strip and a progress counter; the next
// strip's first lane waits for it.  Strips are taken in dependency order from
// an atomic ticket, so every wait targets a strip that is already running (no
// deadlock); a bounded spin with a shared abort flag guarantees that every
// wave exits.
//
// In the split form the flow part and the species part of the implicit
// operator are independent (Section 2.3: the cross terms are discarded), so
// they run as two wavefronts per strip with their own tickets and counters.
//
// Per-cell records are stored step-blocked: all cells of one strip step are
// contiguous, field-major inside the step, so that the wave reads a step's
// record from one scalar base address and a lane offset:
//   element (field f of F, strip s, step d, lane l) at ((s NSTEP + d) F + f) W + l.
#pragma once
#include "csi_sweep.hpp"

namespace csi {

// parts of the implicit operator swept by one wavefront
enum { PART_COUPLED = 0, PART_FLOW = 2, PART_SPECIES = 3 };
template <int NS, int NT, int P> struct PartDims {
  using D = Dims<NS, NT>;
  static constexpr int N = P == PART_COUPLED ? D::nb : P == PART_FLOW ? D::nf : NS;  // unknowns
  static constexpr int OFF = P == PART_SPECIES ? D::nf : 0;                          // first row in b / x
  static constexpr int ND = P == PART_COUPLED ? D::nb * D::nb : P == PART_FLOW ? 6 : NS * NS;
  static constexpr int DOFF = P == PART_SPECIES ? 6 : 0;                             // first Dinv field
  static constexpr int NST = P == PART_COUPLED ? 6 + 2 * NS : P == PART_FLOW ? 7 : 2;
};

struct StripArgs {
  void *b, *Dinv, *state, *face, *xs, *x;  // RT arrays, step-blocked
  void *bnd;                               // RT [nstrip][nj][NSOL] boundary pushes
  int *sync;                               // per part: [nstrip] fwd progress, [nstrip] bwd progress, [2] tickets
  int *abort_flag;                         // set by a wave whose wait timed out
  int pub_every;  // progress published every pub_every steps (and at the last step)
  long spin_limit;
};
__host__ __device__ inline int strip_sync_ints(int nstrip) { return 2 * (2 * nstrip + 2); }

// Cross-lane moves by one lane (DPP wavefront shifts; the vacated lane reads 0).
__device__ __forceinline__ int dpp_up1(int v) { return __builtin_amdgcn_update_dpp(0, v, 0x138, 0xF, 0xF, true); }
__device__ __forceinline__ int dpp_down1(int v) { return __builtin_amdgcn_update_dpp(0, v, 0x130, 0xF, 0xF, true); }
template <bool UP> __device__ __forceinline__ float lane_move(float v) {
  int r = UP ? dpp_up1(__builtin_bit_cast(int, v)) : dpp_down1(__builtin_bit_cast(int, v));
  return __builtin_bit_cast(float, r);
}
template <bool UP> __device__ __forceinline__ double lane_move(double v) {
  long long u = __builtin_bit_cast(long long, v);
  int lo = int(u & 0xffffffffll), hi = int(u >> 32);
  lo = UP ? dpp_up1(lo) : dpp_down1(lo);
  hi = UP ? dpp_up1(hi) : dpp_down1(hi);
  return __builtin_bit_cast(double, (long long)(unsigned(lo)) | ((long long)hi << 32));
}

// Strip-boundary traffic uses device-coherent (agent-scope) atomic loads and
// stores for both the pushed vectors and the progress counters; the producer
// waits for its data stores to complete (s_waitcnt) before it stores the
// counter, so a consumer that reads the counter sees the data.  This avoids
// the L2 write-back a release fence would issue on every step.
__device__ __forceinline__ int load_relaxed(const int *p) {
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
  while (load_relaxed(p) < need) {
    if (__hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return false;
    if (++n > spin_limit) {
      __hip_atomic_store(abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return false;
    }
    __builtin_amdgcn_s_sleep(1);
  }
  return true;
}

// Per-step record of one cell for part P, loaded in one batch (and, when it
// fits in registers, one step ahead of its use).  FWD: the cell's E and N
// push coefficients; backward: W and S pushes plus dQ*.
template <int NS, int NT, typename RT, int P, bool FWD> struct StepRec {
  using Pd = PartDims<NS, NT, P>;
  using Rc = Rec<NS, NT>;
  static constexpr int N = Pd::N, ND = Pd::ND, NST = Pd::NST;
  static constexpr bool PREFETCH = sizeof(RT) * (N + ND + NST + 6) <= 8 * 72;
  RT v[N];     // forward: RHS b; backward: dQ*
  RT Dm[ND];
  RT st[NST];
  RT f[6];     // push 1 (mx, my, c), push 2 (mx, my, c)

  // step0 = (s NSTEP + d) W: first cell position of the step (wave-uniform)
  template <int W> __device__ __forceinline__ void load(const StripArgs &a, long step0, unsigned lane) {
    const RT *src = reinterpret_cast<const RT *>(FWD ? a.b : a.xs) + step0 * Rc::NSOL;
    const RT *Di = reinterpret_cast<const RT *>(a.Dinv) + step0 * Rc::NDINV;
    const RT *stt = reinterpret_cast<const RT *>(a.state) + step0 * Rc::NSTATE;
    const RT *fc = reinterpret_cast<const RT *>(a.face) + step0 * Rc::NFACE;
#pragma unroll
    for (int k = 0; k < N; ++k) v[k] = src[unsigned(Pd::OFF + k) * W + lane];
#pragma unroll
    for (int k = 0; k < ND; ++k) Dm[k] = Di[unsigned(Pd::DOFF + k) * W + lane];
#pragma unroll
    for (int k = 0; k < NST; ++k) st[k] = stt[unsigned(k) * W + lane];
    // normals: mE 0-1, mN 2-3, mW 4-5, mS 6-7; radii: c 8-11, species c 12-15 (E N W S)
    constexpr int m1 = FWD ? 0 : 4, m2 = FWD ? 2 : 6;
    constexpr int c1 = (P == PART_SPECIES ? 12 : 8) + (FWD ? 0 : 2), c2 = c1 + 1;
    f[0] = fc[unsigned(m1) * W + lane];
    f[1] = fc[unsigned(m1 + 1) * W + lane];
    f[2] = fc[unsigned(c1) * W + lane];
    f[3] = fc[unsigned(m2) * W + lane];
    f[4] = fc[unsigned(m2 + 1) * W + lane];
    f[5] = fc[unsigned(c2) * W + lane];
  }

  // o = O x for push q (0 or 1): A(m) x - c x (coupled / flow), (u.m - c) x (species)
  __device__ __forceinline__ void push(int q, const RT *x, RT *o) const {
    const RT mx = f[3 * q], my = f[3 * q + 1], c = f[3 * q + 2];
    if (P == PART_SPECIES) {
      const RT coef = st[0] * mx + st[1] * my - c;
#pragma unroll
      for (int k = 0; k < N; ++k) o[k] = coef * x[k];
    } else {
      NbState<NS, RT> s;
      s.u = st[0]; s.v = st[1]; s.H = st[2]; s.eve = st[3]; s.pE = st[4]; s.pv = st[5];
      RT a[N];
      if (P == PART_COUPLED) {
#pragma unroll
        for (int k = 0; k < NS; ++k) { s.Y[k] = st[6 + k]; s.pr[k] = st[6 + NS + k]; }
        jvp_coupled<NS, NT, RT>(s, mx, my, x, a);
      } else {
#pragma unroll
        for (int k = 0; k < NS; ++k) { s.Y[k] = RT(0); s.pr[k] = RT(0); }
        s.Y[0] = RT(1);
        s.pr[0] = st[6];
        jvp_flow<NS, NT, RT>(s, mx, my, x, a);
      }
#pragma unroll
      for (int k = 0; k < N; ++k) o[k] = a[k] - c * x[k];
    }
  }

  // x = D^-1 r
  __device__ __forceinline__ void dinv(const RT *r, RT *x) const {
    if (P == PART_FLOW) {
#pragma unroll
      for (int k = 0; k < 4; ++k) x[k] = r[k] * Dm[0];
      if (NT == 2) {
        RT acc = r[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) acc += Dm[1 + k] * x[k];
        x[4] = acc * Dm[5];
      }
    } else {
#pragma unroll
      for (int rr = 0; rr < N; ++rr) {
        RT acc = RT(0);
#pragma unroll
        for (int c = 0; c < N; ++c) acc += Dm[rr * N + c] * r[c];
        x[rr] = acc;
      }
    }
  }
};

// sync counters of part slot q
struct PartSync {
  int *prog, *progb, *ticket;
};
__device__ __forceinline__ PartSync part_sync(const StripArgs &a, int nstrip, int q) {
  PartSync ps;
  ps.prog = a.sync + q * (2 * nstrip + 2);
  ps.progb = ps.prog + nstrip;
  ps.ticket = ps.prog + 2 * nstrip;
  return ps;
}

template <int NS, int NT, typename RT, int W, int P>
__device__ __forceinline__ void strip_fwd_part(const Geo &g, const StripArgs &a, int q) {
  using R = StepRec<NS, NT, RT, P, true>;
  using Rc = Rec<NS, NT>;
  constexpr int N = R::N, OFF = PartDims<NS, NT, P>::OFF;
  const StripMap sm = strip_map(g.ni, g.nj, W);
  const PartSync ps = part_sync(a, sm.nstrip, q);
  const unsigned lane = threadIdx.x;
  __shared__ int s_strip;
  if (lane == 0) s_strip = atomicAdd(ps.ticket, 1);
  __syncthreads();
  const int s = __builtin_amdgcn_readfirstlane(s_strip);
  if (s >= sm.nstrip) return;
  const int i = s * W + int(lane);
  const bool lane_ok = lane < unsigned(W) && i < g.ni;
  RT *xs = reinterpret_cast<RT *>(a.xs);
  RT *bnd = reinterpret_cast<RT *>(a.bnd);
  RT inW[N], inS[N];
#pragma unroll
  for (int k = 0; k < N; ++k) { inW[k] = RT(0); inS[k] = RT(0); }
  bool ok = true;
  int seen = 0;
  const long sbase = long(s) * sm.NSTEP;
  R cur, nxt;
  if (lane < unsigned(W)) cur.template load<W>(a, sbase * W, lane);
  // one step; `use` holds this step's record, `fill` receives the next one
  auto step = [&](int d, R &use, R &fill) {
    const int j = d - int(lane);
    const bool active = lane_ok && j >= 0 && j < g.nj;
    const long step0 = (sbase + d) * W;
    if (R::PREFETCH && lane < unsigned(W) && d + 1 < sm.NSTEP) fill.template load<W>(a, step0 + W, lane);
    if (!R::PREFETCH && lane < unsigned(W) && d > 0) use.template load<W>(a, step0, lane);
    // the first lane takes the west push of the previous strip
    if (s > 0 && lane == 0 && active) {
      if (seen < d + W) {
        if (ok) ok = wait_at_least(ps.prog + (s - 1), d + W, a.abort_flag, a.spin_limit);
        seen = load_relaxed(ps.prog + (s - 1));
      }
      const RT *src = bnd + (long(s - 1) * g.nj + j) * Rc::NSOL + OFF;
#pragma unroll
      for (int k = 0; k < N; ++k) inW[k] = get_coherent(src + k);
    }
    RT pushE[N], pushN[N];
#pragma unroll
    for (int k = 0; k < N; ++k) { pushE[k] = RT(0); pushN[k] = RT(0); }
    if (active) {
      RT r[N], x[N];
#pragma unroll
      for (int k = 0; k < N; ++k) {
        RT v = use.v[k];
        if (i > 0) v -= inW[k];
        if (j > 0) v -= inS[k];
        r[k] = v;
      }
      use.dinv(r, x);
      RT *dst = xs + step0 * Rc::NSOL;
#pragma unroll
      for (int k = 0; k < N; ++k) dst[unsigned(OFF + k) * W + lane] = x[k];
      if (i + 1 < g.ni) use.push(0, x, pushE);
      if (j + 1 < g.nj) use.push(1, x, pushN);
      if (lane == unsigned(W - 1) && i + 1 < g.ni) {
        RT *bd = bnd + (long(s) * g.nj + j) * Rc::NSOL + OFF;
#pragma unroll
        for (int k = 0; k < N; ++k) put_coherent(bd + k, pushE[k]);
      }
    }
    if (lane == unsigned(W - 1) && ((d + 1) % a.pub_every == 0 || d + 1 == sm.NSTEP)) publish(ps.prog + s, d + 1);
#pragma unroll
    for (int k = 0; k < N; ++k) {
      inW[k] = lane_move<true>(pushE[k]);
      inS[k] = pushN[k];
    }
  };
  // unrolled by two so that the prefetch buffers alternate without copies
  if (R::PREFETCH) {
    for (int d = 0; d < sm.NSTEP; d += 2) {
      step(d, cur, nxt);
      if (d + 1 < sm.NSTEP) step(d + 1, nxt, cur);
    }
  } else {
    for (int d = 0; d < sm.NSTEP; ++d) step(d, cur, cur);
  }
}

template <int NS, int NT, typename RT, int W, int P>
__device__ __forceinline__ void strip_bwd_part(const Geo &g, const StripArgs &a, int q) {
  using R = StepRec<NS, NT, RT, P, false>;
  using Rc = Rec<NS, NT>;
  constexpr int N = R::N, OFF = PartDims<NS, NT, P>::OFF;
  const StripMap sm = strip_map(g.ni, g.nj, W);
  const PartSync ps = part_sync(a, sm.nstrip, q);
  const unsigned lane = threadIdx.x;
  __shared__ int s_strip;
  if (lane == 0) s_strip = sm.nstrip - 1 - atomicAdd(ps.ticket + 1, 1);
  __syncthreads();
  const int s = __builtin_amdgcn_readfirstlane(s_strip);
  if (s < 0) return;
  const int i = s * W + int(lane);
  const bool lane_ok = lane < unsigned(W) && i < g.ni;
  RT *xo = reinterpret_cast<RT *>(a.x);
  RT *bnd = reinterpret_cast<RT *>(a.bnd);
  RT inE[N], inN[N];
#pragma unroll
  for (int k = 0; k < N; ++k) { inE[k] = RT(0); inN[k] = RT(0); }
  bool ok = true;
  int seen = 0;
  const long sbase = long(s) * sm.NSTEP;
  R cur, nxt;
  if (lane < unsigned(W)) cur.template load<W>(a, (sbase + sm.NSTEP - 1) * W, lane);
  auto step = [&](int d, R &use, R &fill) {
    const int j = d - int(lane);
    const bool active = lane_ok && j >= 0 && j < g.nj;
    const long step0 = (sbase + d) * W;
    if (R::PREFETCH && lane < unsigned(W) && d > 0) fill.template load<W>(a, step0 - W, lane);
    if (!R::PREFETCH && lane < unsigned(W) && d < sm.NSTEP - 1) use.template load<W>(a, step0, lane);
    if (s < sm.nstrip - 1 && lane == unsigned(W - 1) && active) {
      // east neighbour (i0 + W, j) is lane 0 of strip s+1, done at its step j
      if (seen < sm.NSTEP - j) {
        if (ok) ok = wait_at_least(ps.progb + (s + 1), sm.NSTEP - j, a.abort_flag, a.spin_limit);
        seen = load_relaxed(ps.progb + (s + 1));
      }
      const RT *src = bnd + (long(s) * g.nj + j) * Rc::NSOL + OFF;
#pragma unroll
      for (int k = 0; k < N; ++k) inE[k] = get_coherent(src + k);
    }
    RT pushW[N], pushS[N];
#pragma unroll
    for (int k = 0; k < N; ++k) { pushW[k] = RT(0); pushS[k] = RT(0); }
    if (active) {
      RT r[N], x[N];
#pragma unroll
      for (int k = 0; k < N; ++k) {
        RT v = RT(0);
        if (i + 1 < g.ni) v += inE[k];
        if (j + 1 < g.nj) v += inN[k];
        r[k] = v;
      }
      use.dinv(r, x);
      RT *dst = xo + step0 * Rc::NSOL;
#pragma unroll
      for (int k = 0; k < N; ++k) {
        x[k] = use.v[k] - x[k];
        dst[unsigned(OFF + k) * W + lane] = x[k];
      }
      if (i > 0) use.push(0, x, pushW);
      if (j > 0) use.push(1, x, pushS);
      if (lane == 0 && s > 0) {
        RT *bd = bnd + (long(s - 1) * g.nj + j) * Rc::NSOL + OFF;
#pragma unroll
        for (int k = 0; k < N; ++k) put_coherent(bd + k, pushW[k]);
      }
    }
    if (lane == 0 && ((sm.NSTEP - d) % a.pub_every == 0 || d == 0)) publish(ps.progb + s, sm.NSTEP - d);
#pragma unroll
    for (int k = 0; k < N; ++k) {
      inE[k] = lane_move<false>(pushW[k]);
      inN[k] = pushS[k];
    }
  };
  if (R::PREFETCH) {
    for (int d = sm.NSTEP - 1; d >= 0; d -= 2) {
      step(d, cur, nxt);
      if (d - 1 >= 0) step(d - 1, nxt, cur);
    }
  } else {
    for (int d = sm.NSTEP - 1; d >= 0; --d) step(d, cur, cur);
  }
}

// One 64-thread workgroup per strip and part, lanes [0, W) active.  Coupled:
// grid (nstrip); split: grid (nstrip, 2), y = 0 flow part, y = 1 species part.
template <int NS, int NT, typename RT, int W, int MODE>
__global__ void __launch_bounds__(64) k_strip_fwd(Geo g, StripArgs a, const int *__restrict__ done) {
  if (done && *done) return;
  if (MODE == 0) strip_fwd_part<NS, NT, RT, W, PART_COUPLED>(g, a, 0);
  else if (blockIdx.y == 0) strip_fwd_part<NS, NT, RT, W, PART_FLOW>(g, a, 0);
  else strip_fwd_part<NS, NT, RT, W, PART_SPECIES>(g, a, 1);
}

template <int NS, int NT, typename RT, int W, int MODE>
__global__ void __launch_bounds__(64) k_strip_bwd(Geo g, StripArgs a, const int *__restrict__ done) {
  if (done && *done) return;
  if (MODE == 0) strip_bwd_part<NS, NT, RT, W, PART_COUPLED>(g, a, 0);
  else if (blockIdx.y == 0) strip_bwd_part<NS, NT, RT, W, PART_FLOW>(g, a, 0);
  else strip_bwd_part<NS, NT, RT, W, PART_SPECIES>(g, a, 1);
}

template <int NS>
__global__ void __launch_bounds__(64) k_zero_ints(int *p, int n, const int *__restrict__ done) {
  if (done && *done) return;
  for (int k = threadIdx.x; k < n; k += 64) p[k] = 0;
}

}  // namespace csi
