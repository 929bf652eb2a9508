// LU-SGS sweeps with one group of lanes per cell.
//
// The i+j hyperplane order of the sweeps (paper Section 2.2, forward
// (D+L) dQ* = RHS and backward (D+U) dQ = D dQ*) is executed strip by strip:
// one workgroup per strip of C columns.  Each cell of the strip is owned by a
// group of G lanes of the compute wavefront, one lane per unknown of the swept
// part (G = nb coupled, nf flow part, ns species part; C <= 64 / G).  At step d
// the group of column c owns cell (i0 + c, d - c); its west neighbour was
// computed by the previous group one step earlier and its south neighbour by
// the same group one step earlier.  A step of lane k is:
//   r_k = b_k - pushW_k - pushS_k,
//   x_k = sum_m (D^-1)_km r_m          (r gathered from the group's lanes),
//   the two pushes O x of this cell towards its east and north neighbours,
//   component k (the flux Jacobian-vector product needs the whole x, gathered
//   again; the species operator is a scalar times x_k).
// The pushes move to the next group through a cross-lane permute.
//
// A step is a short chain of dependent arithmetic, so the sweep is bound by
// latency, not bandwidth.  The workgroup therefore has three wavefronts, so
// that the compute wave never waits for global memory:
//   wave 0  computes; it reads its step records from an LDS ring;
//   wave 1  gathers the records of the step's C cells from the staging
//           array into the ring with 16-byte global-to-LDS copies, up to a
//           ring of DEPTH steps ahead;
//   wave 2  takes the pushes that cross the strip boundary (written by the
//           neighbouring strip's compute wave) and hands them over in LDS.
// A boundary push is its own ready flag: its slot is filled with an all-ones
// pattern (a NaN that arithmetic never produces) before the sweep, and the
// consumer polls the slot until it holds a value, so the producer never waits
// for its stores.  Strips are taken in dependency order from an atomic ticket
// (every strip waits only on strips that already run, so there is no
// deadlock); every wait is bounded and a shared abort flag makes every wave
// exit.  In the split form the flow and species parts are independent
// (Section 2.3 discards the cross terms) and run in separate workgroups.
#pragma once
#include "csi_sweep.hpp"

namespace csi {

// device buffers of one part (inside the workspace)
struct GroupBufs {
  void *S;        // record staging (RT), written by the cell kernel (dQ* by the forward sweep)
  void *x;        // backward results dQ (RT) [blk][G C]
  void *bnd[2];   // boundary pushes of the forward / backward sweep, RT [nstrip][nj][G]
  int *tickets;   // [2] strip tickets of the forward / backward sweep
};
struct GroupPart {
  GroupBufs b;
  int C;          // cells per wave (64 / G)
};
struct GroupArgs {
  GroupPart part[2];  // coupled or flow; species
  int *abort_flag;
  long spin_limit;
  long long *trace;   // optional per-strip trace [part][strip][TR_N] of this sweep
};
// per-strip trace: wall clock (100 MHz) at the compute wave's start and end,
// spins of the compute wave on step records and on boundary pushes, spins of
// the copy wave on free ring slots and of the boundary wave on pushes
enum { TR_T0 = 0, TR_T1, TR_REC, TR_BND, TR_COPY, TR_POLL, TR_N = 8 };

// Ring geometry of a part and sweep direction.  A step's LDS block holds the
// C cells' common and direction sections, cell c at granule c NQ: KB copy
// instructions (1 KiB each) per step, DEPTH slots, at most LAG steps of
// copies in flight (LAG KB <= 60: the vector memory counter has 6 bits).
template <int NS, int NT, typename RT, int P> struct GPipe {
  static constexpr RecShape S = rec_shape(P, NS, NT, sizeof(RT));
  static constexpr int G = S.G, C = 64 / G, GW = S.GW;
  static constexpr int NQ = S.QC + S.QD;               // granules per cell in LDS
  static constexpr int CS = NQ * GW;                   // words per cell in LDS
  static constexpr int KB = (C * NQ + 63) / 64;
  static constexpr int SLOT = KB * 1024 / int(sizeof(RT));  // words per step block
  static constexpr int DEPTH = 128 / KB < 16 ? 128 / KB : 16;
  static constexpr int LAG = 60 / KB < DEPTH - 1 ? 60 / KB : DEPTH - 1;
  static constexpr size_t RING = size_t(DEPTH) * KB * 1024;
  static constexpr size_t LDS = RING + size_t(DEPTH) * G * sizeof(RT);
};
template <int NS, int NT, typename RT, int MODE> constexpr size_t group_lds_bytes() {
  if (MODE == 0) return GPipe<NS, NT, RT, PART_COUPLED>::LDS;
  const size_t a = GPipe<NS, NT, RT, PART_FLOW>::LDS, b = GPipe<NS, NT, RT, PART_SPECIES>::LDS;
  return a > b ? a : b;
}

// ------------------------------------------------------------ synchronisation
__device__ __forceinline__ bool aborted(const int *f) {
  return __hip_atomic_load(f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
}
__device__ __forceinline__ void set_abort(int *f) {
  __hip_atomic_store(f, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// LDS counters shared by the three waves (compute and boundary waves)
__device__ __forceinline__ int lds_get(const int *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void lds_set(int *p, int v) {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
// spin until *p >= need; seen receives the value read, spins the number of
// extra reads; a waiting wave sleeps `sleep` units between reads (0: the
// wave on the critical path, 1: a wave that runs ahead).  False on timeout /
// abort.
__device__ __forceinline__ bool lds_wait(const int *p, int need, int *abort_flag, long spin_limit, long &spins,
                                         int &seen, int sleep) {
  long n = 0;
  while ((seen = lds_get(p)) < need) {
    if (++n > spin_limit) { set_abort(abort_flag); return false; }
    if ((n & 255) == 0 && aborted(abort_flag)) return false;
    if (sleep) __builtin_amdgcn_s_sleep(1);
  }
  spins += n;
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  return true;
}

// The copy wave's own LDS accesses are written in assembly (each waits for
// its result in the same block): the compiler would otherwise make them wait
// for every copy still in flight, since copies and reads share the LDS.
__device__ __forceinline__ unsigned lds_addr(const void *p) {
  // (a C-style cast converts the generic pointer to a 32-bit LDS address)
  return unsigned(reinterpret_cast<uintptr_t>((const __attribute__((address_space(3))) char *)(p)));
}
__device__ __forceinline__ int lds_get_asm(const int *p) {
  int v;
  asm volatile("ds_read_b32 %0, %1\n\ts_waitcnt lgkmcnt(0)" : "=v"(v) : "v"(lds_addr(p)) : "memory");
  return v;
}
__device__ __forceinline__ void lds_set_asm(int *p, int v) {
  asm volatile("ds_write_b32 %0, %1\n\ts_waitcnt lgkmcnt(0)" : : "v"(lds_addr(p)), "v"(v) : "memory");
}
// s_waitcnt immediate that waits for the vector memory counter only
constexpr int vmcnt_imm(int n) { return (n & 0xF) | ((n >> 4) << 14) | (0x7 << 4) | (0xF << 8); }

// boundary pushes: all-ones = empty slot
template <typename RT> struct UBits;
template <> struct UBits<float> { using T = unsigned int; };
template <> struct UBits<double> { using T = unsigned long long; };
template <typename RT> __device__ __forceinline__ void put_push(RT *p, RT v) {
  using U = typename UBits<RT>::T;
  __hip_atomic_store(reinterpret_cast<U *>(p), __builtin_bit_cast(U, v), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename RT>
__device__ __forceinline__ bool take_push(const RT *p, RT &v, int *abort_flag, long spin_limit, long &spins) {
  using U = typename UBits<RT>::T;
  long &n = spins;
  U u;
  while ((u = __hip_atomic_load(reinterpret_cast<const U *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) == ~U(0)) {
    if (++n > spin_limit) { set_abort(abort_flag); return false; }
    if ((n & 63) == 0 && aborted(abort_flag)) return false;
    __builtin_amdgcn_s_sleep(1);
  }
  v = __builtin_bit_cast(RT, u);
  return true;
}

// ------------------------------------------------------------ step arithmetic
// The step arithmetic is written with explicit fused multiply-adds and
// contraction off, so that every cell gets the same rounding whatever its
// position in the unrolled loop (results do not depend on C).
template <typename RT> __device__ __forceinline__ RT fmad(RT a, RT b, RT c) { return fma(a, b, c); }

// per-step record of one lane.  The forward sweep pushes through faces E, N,
// the backward sweep through W, S.
template <int NS, int NT, typename RT, int P, bool FWD> struct GRec {
  using Pp = GPipe<NS, NT, RT, P>;
  static constexpr RecShape S = Pp::S;
  static constexpr int G = S.G, OD = S.QC * S.GW;  // direction section of a cell in LDS
  static constexpr bool JVP = P != PART_SPECIES;
  RT b;          // forward: RHS b_k; backward: dQ*_k
  RT Dr[G];      // row k of D^-1
  // JVP parts: coefficient of a, and per push face: g_k, cp_k, (m_x, m_y, u.m), dp weights
  RT ca, gk[2], cp[2], mx[2], my[2], un[2];
  RT w[JVP ? G : 1];
  RT coef[2];    // species part: u.m - c per push face

  // from one step block in LDS: Q = the cell's record (block + c CS), component k
  __device__ __forceinline__ void load(const RT *Q, int k) {
    const RT *L = Q + k, *DL = Q + k * G;
    b = L[OD + dw_b(0)];
#pragma unroll
    for (int q = 0; q < G; ++q) Dr[q] = DL[q];
    if (JVP) {
      ca = L[rw_ca(S, 0)];
#pragma unroll
      for (int f = 0; f < 2; ++f) {
        gk[f] = L[OD + dw_g(S, f, 0)];
        cp[f] = L[OD + dw_cp(S, f, 0)];
        mx[f] = Q[OD + dw_m(S, f)];
        my[f] = Q[OD + dw_m(S, f) + 1];
        un[f] = Q[OD + dw_m(S, f) + 2];
      }
#pragma unroll
      for (int q = 0; q < G; ++q) w[q] = Q[rw_w(S, q)];
    } else {
#pragma unroll
      for (int f = 0; f < 2; ++f) coef[f] = Q[OD + dw_coef(S, f)];
    }
  }
};

// value of v in the lane whose byte address (4 x lane) is addr
__device__ __forceinline__ float gather(float v, int addr) {
  return __builtin_bit_cast(float, __builtin_amdgcn_ds_bpermute(addr, __builtin_bit_cast(int, v)));
}
__device__ __forceinline__ double gather(double v, int addr) {
  const long long u = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_ds_bpermute(addr, int(u & 0xffffffffll));
  const int hi = __builtin_amdgcn_ds_bpermute(addr, int(u >> 32));
  return __builtin_bit_cast(double, (long long)(unsigned(lo)) | ((long long)hi << 32));
}
// cross-lane moves by one lane (DPP wavefront shifts; the vacated lane reads 0):
// UP: lane l takes lane l - 1, else lane l + 1
template <bool UP> __device__ __forceinline__ int dpp_move(int v) {
  return __builtin_amdgcn_update_dpp(0, v, UP ? 0x138 : 0x130, 0xF, 0xF, true);
}
template <bool UP> __device__ __forceinline__ float lane_move(float v) {
  return __builtin_bit_cast(float, dpp_move<UP>(__builtin_bit_cast(int, v)));
}
template <bool UP> __device__ __forceinline__ double lane_move(double v) {
  const long long u = __builtin_bit_cast(long long, v);
  const int lo = dpp_move<UP>(int(u & 0xffffffffll)), hi = dpp_move<UP>(int(u >> 32));
  return __builtin_bit_cast(double, (long long)(unsigned(lo)) | ((long long)hi << 32));
}

// component k of the push O x through push face f (JVP parts):
//   o_k = ca_k a + [k = 0] dmn + g_k x_k + cp_k dp,
//   dmn = x_1 m_x + x_2 m_y, a = dmn - (u.m) x_0, dp = w.x,
// the spectral-split flux Jacobian-vector product 1/2 S (A(n) x - lam x) minus
// the viscous radius term (m = S/2 n of the receiving cell); species part:
// (u.m - c) x_k.
template <int NS, int NT, typename RT, int P, bool FWD>
__device__ __forceinline__ RT push_comp(const GRec<NS, NT, RT, P, FWD> &R, int f, RT beta, RT xk, const RT *xall,
                                        RT dp) {
#pragma clang fp contract(off)
  if (P == PART_SPECIES) return R.coef[f] * xk;
  const RT dmn = fmad(xall[2], R.my[f], xall[1] * R.mx[f]);
  const RT a = fmad(-R.un[f], xall[0], dmn);
  RT o = fmad(R.gk[f], xk, R.ca * a);
  o = fmad(beta, dmn, o);
  return fmad(R.cp[f], dp, o);
}

// ------------------------------------------------------------ the three waves
struct GroupSync {
  int strip;      // strip of this workgroup
  int rec_ready;  // step records in the ring (copy wave)
  int bnd_ready;  // boundary pushes in LDS (boundary wave)
  int consumed;   // steps whose ring slots the compute wave has read
};

// wave 1: the records of each step's cells, in sweep order, gathered from
// the staging array into the LDS ring.  Copy instruction q of lane l moves
// granule n = 64 q + l of the step block: cell c = n / NQ, granule n % NQ of
// its common then direction section.  Cells outside the grid read a clamped
// (valid) cell; their lanes' results are discarded.
template <int NS, int NT, typename RT, int P, bool FWD>
__device__ __forceinline__ long copy_wave(const Geo &g, const RT *stage, int s, int NSTEP, char *ring, GroupSync &sy,
                                          int *abort_flag, long spin_limit) {
  using Pp = GPipe<NS, NT, RT, P>;
  constexpr RecShape S = Pp::S;
  constexpr int KB = Pp::KB, DEPTH = Pp::DEPTH, LAG = Pp::LAG, NQ = Pp::NQ, C = Pp::C;
  const int lane = threadIdx.x & 63;
  const char *base = reinterpret_cast<const char *>(stage);
  constexpr int QR = S.QC + 2 * S.QD;  // granules per staged record
  int col[KB], gofs[KB];  // the lane's cell column and granule within the record
#pragma unroll
  for (int q = 0; q < KB; ++q) {
    const int n = q * 64 + lane, c = n / NQ, r = n - c * NQ;
    col[q] = c < C ? c : -1;
    gofs[q] = r < S.QC ? r : S.QC + (FWD ? 0 : S.QD) + (r - S.QC);
  }
  int pub = 0, seen = 0, slot = 0;
  long spins = 0;
  for (int e = 0; e < NSTEP; ++e) {
    if (e >= DEPTH && seen < e - DEPTH + 1) {
      // a full ring ahead of the compute wave: publish what has landed and
      // wait for the oldest slot to be read
      __builtin_amdgcn_s_waitcnt(vmcnt_imm(0));
      pub = e;
      lds_set_asm(&sy.rec_ready, pub);
      long n = 0;
      while ((seen = lds_get_asm(&sy.consumed)) < e - DEPTH + 1) {
        if (++n > spin_limit) { set_abort(abort_flag); return spins; }
        if ((n & 255) == 0 && aborted(abort_flag)) return spins;
        __builtin_amdgcn_s_sleep(1);
      }
      spins += n;
    }
    const int d = FWD ? e : NSTEP - 1 - e;
    char *dst = ring + slot * (KB * 1024);
#pragma unroll
    for (int q = 0; q < KB; ++q) {
      const int c = col[q] < 0 ? 0 : col[q];
      const int i = min(s * C + c, g.ni - 1), j = min(max(d - c, 0), g.nj - 1);
      const char *src = base + ((long(j) * g.ni + i) * QR + gofs[q]) * 16;
      __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void *)(dst + q * 1024), 16, 0, 0);
    }
    if (++slot == DEPTH) slot = 0;
    if (e >= LAG) {
      // copies of step e - LAG have landed once at most LAG steps of copies are in flight
      __builtin_amdgcn_s_waitcnt(vmcnt_imm(LAG * KB));
      if (e - LAG + 1 > pub) {
        pub = e - LAG + 1;
        lds_set_asm(&sy.rec_ready, pub);
      }
    }
  }
  __builtin_amdgcn_s_waitcnt(vmcnt_imm(0));
  lds_set_asm(&sy.rec_ready, NSTEP);
  return spins;
}

// spin until *p >= need (rare path of the compute wave); returns the value
// read, or sets the abort flag and clears live on timeout / abort
__device__ __forceinline__ int lds_spin(const int *p, int need, int *abort_flag, long spin_limit, long &spins,
                                        bool &live) {
  int v = lds_get(p);
  long n = 0;
  while (v < need && live) {
    ++n;
    if (n > spin_limit || ((n & 1023) == 0 && aborted(abort_flag))) {
      set_abort(abort_flag);
      live = false;
    }
    v = lds_get(p);
  }
  spins += n;
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  return v;
}

// wave 2: the G pushes that enter the strip at each step, from the
// neighbouring strip.  The steps that take a push form one run [e0, e1); the
// push of step e sits at bnd[at0 + dir (e - e0) G + k].  The wave polls a
// window of up to 64 / G consecutive steps with one load per lane and hands
// over every leading step whose G components have all landed, so that it
// keeps up with the neighbour however far behind it starts.
template <typename RT, int G, int DEPTH>
__device__ __forceinline__ long boundary_wave(const RT *bnd, long at0, int dir, int e0, int e1, int NSTEP, RT *bring,
                                              GroupSync &sy, int *abort_flag, long spin_limit) {
  using U = typename UBits<RT>::T;
  constexpr int W = 64 / G;
  const int lane = threadIdx.x & 63;
  const int w = lane / G, k = lane - w * G;
  if (e0 >= e1) {  // a strip at the edge of the grid takes no pushes
    lds_set(&sy.bnd_ready, NSTEP);
    return 0;
  }
  lds_set(&sy.bnd_ready, e0);
  long spins = 0, n = 0;
  int e = e0, seen = 0;
  while (e < e1) {
    // steps e .. e + nw - 1 fit the ring once the compute wave has read step e + nw - 1 - DEPTH
    int free_slots = seen + DEPTH - e;
    if (free_slots <= 0) {
      long s2 = 0;
      bool live = true;
      seen = lds_spin(&sy.consumed, e - DEPTH + 1, abort_flag, spin_limit, s2, live);
      if (!live) return spins;
      free_slots = seen + DEPTH - e;
    }
    const int nw = min(W, min(free_slots, e1 - e));
    U u = ~U(0);
    if (w < nw)
      u = __hip_atomic_load(reinterpret_cast<const U *>(bnd + at0 + long(dir) * (e - e0 + w) * G + k), __ATOMIC_RELAXED,
                            __HIP_MEMORY_SCOPE_AGENT);
    const unsigned long long got = __ballot(w < nw && u != ~U(0));
    int cnt = 0;
    constexpr unsigned long long gm = (1ull << G) - 1;
    while (cnt < nw && ((got >> (cnt * G)) & gm) == gm) ++cnt;
    if (cnt == 0) {
      if (++n > spin_limit || ((n & 63) == 0 && aborted(abort_flag))) {
        set_abort(abort_flag);
        return spins;
      }
      ++spins;
      __builtin_amdgcn_s_sleep(1);
      continue;
    }
    if (w < cnt) bring[((e + w) % DEPTH) * G + k] = __builtin_bit_cast(RT, u);
    e += cnt;
    lds_set(&sy.bnd_ready, e);
  }
  lds_set(&sy.bnd_ready, NSTEP);
  return spins;
}

// wave 0: the sweep recurrence.  Lane (c, k) = k C + c; the push of column c
// reaches column c + 1 (forward, east) or c - 1 (backward, west) by a one-lane
// move, the north / south push stays in the lane for the next step.  The step
// records are read from the ring one step ahead.  After a timeout the wave
// stops waiting and runs to the end (its results are then discarded).
template <int NS, int NT, typename RT, int P, bool FWD>
__device__ __forceinline__ void compute_wave(const Geo &g, const GroupArgs &a, const GroupPart &gp,
                                             const GroupMap &m, int s, const RT *ring, const RT *bring, GroupSync &sy,
                                             long &rsp, long &bsp) {
#pragma clang fp contract(off)
  using Pp = GPipe<NS, NT, RT, P>;
  using R = GRec<NS, NT, RT, P, FWD>;
  constexpr RecShape S = Pp::S;
  constexpr int G = Pp::G, DEPTH = Pp::DEPTH, SLOT = Pp::SLOT, C = Pp::C;
  constexpr bool JVP = R::JVP;
  const int lane = threadIdx.x & 63;
  const int NSTEP = m.NSTEP;
  const int k = lane / C, c = lane - k * C;
  const bool lane_ok = k < G;
  const int kk = lane_ok ? k : G - 1;  // idle lanes read (and discard) the last component
  const int i = s * C + c;
  const bool col_ok = lane_ok && i < g.ni;
  int gaddr[G];  // byte addresses of the group's lanes (q C + c)
#pragma unroll
  for (int q = 0; q < G; ++q) gaddr[q] = (q * C + c) * 4;
  // forward: dQ* into the staging (backward section); backward: dQ step-blocked
  RT *out = reinterpret_cast<RT *>(FWD ? gp.b.S : gp.b.x);
  RT *bnd = reinterpret_cast<RT *>(gp.b.bnd[FWD ? 0 : 1]);
  const long b0 = long(s) * NSTEP;
  // the column that takes a push from the neighbouring strip
  constexpr int edge = FWD ? 0 : C - 1;
  const bool has_nb = FWD ? s > 0 : s < m.nstrip - 1;
  // lanes that hand their push to the neighbouring strip (only real components)
  const bool send_nb = lane_ok && c == C - 1 - edge && (FWD ? i + 1 < g.ni : s > 0);
  // lanes whose in-strip push source is not a cell: the edge column, and in
  // the backward sweep the last column of the grid (its east neighbour is padding)
  const bool no_src = c == edge || (!FWD && i + 1 >= g.ni);
  const RT beta = k == 0 ? RT(1) : RT(0);
  const int cofs = c * Pp::CS;  // the cell's record in a step block
  bool live = true;
  int rec_seen = lds_spin(&sy.rec_ready, 1, a.abort_flag, a.spin_limit, rsp, live);
  int bnd_seen = 0;
  R A, B;
  A.load(ring + cofs, kk);
  RT in1 = RT(0), in2 = RT(0);  // pushes from the west / south (forward), east / north (backward)
  int slot = 0;
  auto step = [&](int e, R &cur, R &nxt) {
    const int d = FWD ? e : NSTEP - 1 - e;
    const int j = d - c;
    const int jb = d - edge;
    if (has_nb && jb >= 0 && jb < g.nj) {
      if (bnd_seen <= e) bnd_seen = lds_spin(&sy.bnd_ready, e + 1, a.abort_flag, a.spin_limit, bsp, live);
      const RT v = bring[slot * G + kk];
      in1 = c == edge ? v : in1;
    }
    // r = b -/+ pushes, gathered over the group.  in1 is zero at the edge
    // column unless a neighbouring strip pushed; in2 comes from the previous
    // cell of the column, which does not exist at its first cell.
    const bool h2 = FWD ? j > 0 : j + 1 < g.nj;
    RT r = FWD ? cur.b - in1 : in1;
    const RT t2 = h2 ? in2 : RT(0);
    r = FWD ? r - t2 : r + t2;
    RT rg[G];
#pragma unroll
    for (int q = 0; q < G; ++q) rg[q] = gather(r, gaddr[q]);
    // The next step's record.  FP32, and FP64 groups of more than 9 lanes:
    // right behind the gather in the LDS queue.  FP64 groups of up to 9
    // lanes: only once the pushes are formed, since LDS results return in
    // issue order and reads issued between a gather and its use hold up the
    // gather's results (5-species air, 512 x 256, forward sweep: split FP64
    // 0.44 -> 0.41 ms, coupled FP64 0.59 -> 0.57 ms; the FP32 sweeps gain
    // nothing and the coupled FP32 one loses, and so does the 15-lane
    // coupled FP64 block of 11-species air, by 3 %).  The empty statement
    // and the scheduling barriers keep the compiler from hoisting the reads
    // back above the push arithmetic.
    auto next_record = [&]() {
      const int nslot = slot + 1 == DEPTH ? 0 : slot + 1;
      if (e + 1 < NSTEP) {
        if (rec_seen <= e + 1) rec_seen = lds_spin(&sy.rec_ready, e + 2, a.abort_flag, a.spin_limit, rsp, live);
        nxt.load(ring + nslot * SLOT + cofs, kk);
      }
      lds_set(&sy.consumed, e + 1);
      slot = nslot;
    };
    constexpr bool LATE = sizeof(RT) == 8 && G <= 9;
    if (!LATE) next_record();
    RT y = cur.Dr[0] * rg[0];
#pragma unroll
    for (int q = 1; q < G; ++q) y = fmad(cur.Dr[q], rg[q], y);
    const RT x = FWD ? y : cur.b - y;
    RT p1, p2;
    if (JVP) {
      RT xall[G];
      RT dp = RT(0);
#pragma unroll
      for (int q = 0; q < G; ++q) {
        xall[q] = gather(x, gaddr[q]);
        dp = q == 0 ? cur.w[0] * xall[0] : fmad(cur.w[q], xall[q], dp);
      }
      p1 = push_comp<NS, NT, RT, P, FWD>(cur, 0, beta, x, xall, dp);
      p2 = push_comp<NS, NT, RT, P, FWD>(cur, 1, beta, x, xall, dp);
    } else {
      p1 = push_comp<NS, NT, RT, P, FWD>(cur, 0, beta, x, nullptr, RT(0));
      p2 = push_comp<NS, NT, RT, P, FWD>(cur, 1, beta, x, nullptr, RT(0));
    }
    if (LATE) {
      asm volatile("" : : "v"(p1), "v"(p2), "v"(x) : "memory");
      __builtin_amdgcn_sched_barrier(0);
      next_record();
      __builtin_amdgcn_sched_barrier(0);
    }
    // The pushes of a cell outside the grid reach only cells outside the grid
    // (the same j, or i beyond the last column), except the in-column push
    // into the first cell of the column, which h2 excludes, and the backward
    // push from beyond the last column, which no_src excludes.  Backward
    // results outside the grid land in padding slots of the step blocks.
    const bool active = col_ok && j >= 0 && j < g.nj;
    if (FWD) {
      if (active) out[st_idx(S, g.N, 2, dw_b(k), long(j) * g.ni + i)] = x;
    } else if (lane_ok) {
      out[(b0 + d) * m.Lw + k * C + c] = x;
    }
    if (send_nb && j >= 0 && j < g.nj) put_push(bnd + (long(FWD ? s : s - 1) * g.nj + j) * G + k, p1);
    in1 = lane_move<FWD>(p1);
    in1 = no_src ? RT(0) : in1;
    in2 = p2;
  };
#pragma unroll 1
  for (int e = 0; e < NSTEP; e += 2) {
    step(e, A, B);
    if (e + 1 < NSTEP) step(e + 1, B, A);
  }
}

template <int NS, int NT, typename RT, int P, bool FWD>
__device__ __forceinline__ void group_part(const Geo &g, const GroupArgs &a, int q, char *lds, GroupSync &sy) {
  using Pp = GPipe<NS, NT, RT, P>;
  constexpr int G = Pp::G;
  const GroupPart &gp = a.part[q];
  const GroupMap m = group_map(g.ni, g.nj, G);
  if (threadIdx.x == 0) {
    sy.strip = FWD ? atomicAdd(gp.b.tickets, 1) : m.nstrip - 1 - atomicAdd(gp.b.tickets + 1, 1);
    sy.rec_ready = 0;
    sy.bnd_ready = 0;
    sy.consumed = 0;
  }
  __syncthreads();
  const int s = __builtin_amdgcn_readfirstlane(sy.strip);
  if (s < 0 || s >= m.nstrip) return;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const RT *ring = reinterpret_cast<const RT *>(lds);
  RT *bring = reinterpret_cast<RT *>(lds + Pp::RING);
  const long b0 = long(s) * m.NSTEP;
  long long *tr = a.trace ? a.trace + (long(q) * g.ni + s) * TR_N : nullptr;
  const int lane = threadIdx.x & 63;
  if (wave == 1) {
    const long sp = copy_wave<NS, NT, RT, P, FWD>(g, reinterpret_cast<const RT *>(gp.b.S), s, m.NSTEP, lds, sy,
                                                  a.abort_flag, a.spin_limit);
    if (tr && lane == 0) tr[TR_COPY] = sp;
  } else if (wave == 2) {
    const RT *bnd = reinterpret_cast<const RT *>(gp.b.bnd[FWD ? 0 : 1]);
    const int nj = g.nj, C = m.C, NSTEP = m.NSTEP, last = m.nstrip - 1;
    if (FWD) {
      // west pushes of column 0: cell (i0, j = d = e), written by strip s - 1
      const long sp = boundary_wave<RT, G, Pp::DEPTH>(bnd, s > 0 ? long(s - 1) * nj * G : 0L, 1, 0, s > 0 ? nj : 0,
                                                      NSTEP, bring, sy, a.abort_flag, a.spin_limit);
      if (tr && lane == 0) tr[TR_POLL] = sp;
    } else {
      // east pushes of column C - 1: cell (i0 + C - 1, j = d - C + 1), d = NSTEP - 1 - e, written by strip
      // s + 1; j runs from nj - 1 (e = 0) down to 0 (e = nj - 1)
      const long sp = boundary_wave<RT, G, Pp::DEPTH>(bnd, s < last ? (long(s) * nj + nj - 1) * G : 0L, -1, 0,
                                                      s < last ? nj : 0, NSTEP, bring, sy, a.abort_flag,
                                                      a.spin_limit);
      if (tr && lane == 0) tr[TR_POLL] = sp;
    }
  } else {
    const long long t0 = tr ? (long long)wall_clock64() : 0;
    long rsp = 0, bsp = 0;
    compute_wave<NS, NT, RT, P, FWD>(g, a, gp, m, s, ring, bring, sy, rsp, bsp);
    if (tr && lane == 0) {
      tr[TR_T0] = t0;
      tr[TR_T1] = (long long)wall_clock64();
      tr[TR_REC] = rsp;
      tr[TR_BND] = bsp;
    }
  }
}

// One three-wave workgroup per strip and part.  Coupled: grid (nstrip);
// split: grid (max nstrip, 2), y = 0 flow part, y = 1 species part.
template <int NS, int NT, typename RT, int MODE, bool FWD>
__global__ void __launch_bounds__(192) k_group_sweep(Geo g, GroupArgs a, const int *__restrict__ done) {
  extern __shared__ __align__(16) char lds[];
  __shared__ GroupSync sy;
  if (done && *done) return;
  if (MODE == 0) group_part<NS, NT, RT, PART_COUPLED, FWD>(g, a, 0, lds, sy);
  else if (blockIdx.y == 0) group_part<NS, NT, RT, PART_FLOW, FWD>(g, a, 0, lds, sy);
  else group_part<NS, NT, RT, PART_SPECIES, FWD>(g, a, 1, lds, sy);
}

// Before a sweep pair: clears the strip tickets and marks every boundary-push
// slot empty (all-ones); nw: 32-bit words of each boundary array.
struct GroupReset {
  int *tickets[2];
  unsigned *bnd[4];
  long nw[4];
};
template <int NS>
__global__ void __launch_bounds__(256) k_group_reset(GroupReset r, const int *__restrict__ done) {
  if (done && *done) return;
  const long t = long(blockIdx.x) * blockDim.x + threadIdx.x, stride = long(gridDim.x) * blockDim.x;
  if (t < 2) {
    if (r.tickets[0]) r.tickets[0][t] = 0;
    if (r.tickets[1]) r.tickets[1][t] = 0;
  }
  for (int q = 0; q < 4; ++q)
    for (long k = t; k < r.nw[q]; k += stride) r.bnd[q][k] = ~0u;
}

}  // namespace csi
