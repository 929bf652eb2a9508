// Launch sequences of one pseudo-time iteration, templated on the species
// count and the temperature model; instantiated per species count in
// csi_inst.hip and dispatched through the IRunner interface.
#pragma once
#include <string>

#include "../../include/csi.h"
#include "csi_block.hpp"
#include "csi_group.hpp"
#include "csi_surrogate.hpp"

namespace csi {

// device pointers inside the caller-owned workspace
struct WS {
  Mech *mech;
  double *V, *xc, *yc, *xn, *yn, *fi_nx, *fi_ny, *fi_S, *fj_nx, *fj_ny, *fj_S;
  double *qfs, *Q, *prim, *Fi, *Fj, *Ri, *Rj, *R, *dtau, *src, *qw, *part, *norms, *r0, *hist;
  void *b, *dqs, *dq, *Dinv;  // hyperplane schedule: cell-major records and results
  GroupBufs grp[2];           // group schedule: part 0 (coupled / flow), part 1 (species)
  long long *trace;           // optional per-strip sweep trace [fwd, bwd][part][ni][TR_N] (null: off)
  double *diag;               // [hb_fields][N] per-cell hand-off from k_cell to k_block
  double *qbak;               // [nv][N] state at the start of csi_step (surrogate divergence fallback)
  double *qn, *qnm1;          // [nv][N] physical-time levels Q^n, Q^{n-1} (dual time stepping)
  double pt_a, pt_b;          // (1 + theta) / dt and theta / dt (0: steady)
  int fdiff;                  // off-diagonal flux differences (hyperplane schedule, FP64) instead of the JVP
  int *flags;  // [0] bad cell (INT_MAX = none), [1] done, [2] it_done, [3] clipped cells, [4] singular cell
  int nblk_cell, hist_max;
  int group_c;               // 0: one launch per hyperplane; 1: persistent group kernels
  long spin_limit;
  SurArgs sur;               // surrogate network (packed operands, biases, scales) and its J_C buffer
  // species-generic path: species table, and the Gauss-Jordan scratch of the
  // coupled blocks (row interchanges [N][nb], pivot rows [N][64][nb])
  double *wtab;
  int *gj_perm;
  double *gj_xk;
  // the species table as the streaming kernels read it (one temperature)
  WMech mview;
};
// flags[]: ints, with one 64-bit counter at int offset FL_DDFAIL
enum {
  FL_BAD = 0, FL_DONE = 1, FL_ITDONE = 2, FL_CLIP = 3, FL_SING = 4, FL_ABORT = 5, FL_SURR_OFF = 6, FL_DDFAIL = 8,
  FL_N = 16
};
inline unsigned long long *ddfail_counter(int *flags) { return reinterpret_cast<unsigned long long *>(flags + FL_DDFAIL); }

class IRunner {
 public:
  virtual ~IRunner() {}
  virtual int nprim() const = 0;
  // guess: start the temperature solves at the previous iteration's temperatures
  virtual hipError_t prim(const Geo &g, const WS &w, hipStream_t st, bool stoppable, bool guess = false) = 0;
  virtual hipError_t faces(const Geo &g, const WS &w, hipStream_t st, bool stoppable) = 0;
  // sur_ready (optional): event after which the surrogate's blocks are in
  // place; the launch makes the first kernel that reads them wait for it
  // mid (optional): recorded between the cell kernel and the block kernel
  // (right after the cell kernel where there is no block kernel)
  virtual hipError_t cell(const Geo &g, const WS &w, hipStream_t st, double cfl, int mode, int prec, int flags,
                          bool stoppable, hipEvent_t sur_ready = nullptr, hipEvent_t mid = nullptr) = 0;
  virtual hipError_t norms(const WS &w, hipStream_t st, int it, double tol, bool stoppable,
                           StallArgs stall = StallArgs{nullptr, 0, 0, 0.0}) = 0;
  virtual hipError_t surrogate(const Geo &g, const WS &w, hipStream_t st, bool stoppable) = 0;
  // flags bit 3: the species block's reading with the temperatures following the composition
  virtual hipError_t sample(const Geo &g, const WS &w, hipStream_t st, int n, float *xr, float *jc, int flags,
                            SampleMap sm) = 0;
  virtual hipError_t sweeps(const Geo &g, const WS &w, hipStream_t st, int mode, int prec, bool stoppable,
                            hipEvent_t mid = nullptr) = 0;
  virtual hipError_t update(const Geo &g, const WS &w, hipStream_t st, int mode, int prec, int kind,
                            bool stoppable) = 0;
  virtual hipError_t q_from_prim_host(const Mech &m, const double *rs, double u, double v, double T, double Tv,
                                      double *q) = 0;
  // species table the runner reads from the workspace (species-generic
  // runner; null for the compiled ones, which read the Mech record)
  virtual const void *host_table(size_t *bytes) const {
    *bytes = 0;
    return nullptr;
  }
};

IRunner *make_runner(int ns, int nt);
// Streaming primitive and face kernels (one thread per padded cell / face,
// loops over the species instead of per-thread species arrays; one
// temperature).  The compiled runners take them from STREAM_NS_MIN species
// on, where the register-resident versions run at one wave per SIMD.
constexpr int STREAM_NS_MIN = 16;
hipError_t launch_stream_prim(const Geo &g, const WMech &m, const double *Q, const double *qfs, double *prim,
                              int *bad, const int *done, int guess, hipStream_t st);
hipError_t launch_stream_faces(const Geo &g, const WMech &m, const double *prim, double *Fi, double *Ri, double *Fj,
                               double *Rj, double *qw, const int *done, hipStream_t st);
// pivot rows kept per cell by the blocked Gauss-Jordan inversion (its panel width)
constexpr int WGJ_SCRATCH_ROWS = 64;
// species-generic runner (one temperature, no reactions); null with err set
// on a bad species record
IRunner *make_wide_runner(const csi_mechanism *mm, std::string &err);
// in-place blocked Gauss-Jordan inverse of `count` row-major n x n FP64
// matrices at W; perm [count][n] and XK [count][64][n] of scratch; sing
// receives (atomic minimum) the index of a singular matrix
hipError_t wide_invert(double *W, int n, int count, int *perm, double *XK, int *sing, const int *done,
                       hipStream_t st);

inline int nblocks(long n, int b = 256) { return int((n + b - 1) / b); }

// cells per wave of part q (0: coupled / flow, 1: species) under the group
// schedule (group_c > 0): 64 / G, the widest strip of G-lane groups
template <int NS, int NT> inline int group_cells(int group_c, int mode, int q) {
  const int G = rec_shape(q == 1 ? PART_SPECIES : mode == 0 ? PART_COUPLED : PART_FLOW, NS, NT, 8).G;
  return group_c > 0 ? 64 / G : 0;
}

template <int NS, int NT> class Runner : public IRunner {
 public:
  int nprim() const override { return PF<NS>::N; }

  hipError_t prim(const Geo &g, const WS &w, hipStream_t st, bool stoppable, bool guess) override {
    if constexpr (NT == 1 && NS >= STREAM_NS_MIN)
      return launch_stream_prim(g, w.mview, w.Q, w.qfs, w.prim, w.flags + FL_BAD,
                                stoppable ? w.flags + FL_DONE : nullptr, guess ? 1 : 0, st);
    hipLaunchKernelGGL((k_prim<NS, NT>), dim3(nblocks(g.NP)), dim3(256), 0, st, g, w.mech, w.Q, w.qfs, w.prim,
                       w.flags + FL_BAD, stoppable ? w.flags + FL_DONE : nullptr, guess ? 1 : 0);
    return hipGetLastError();
  }

  hipError_t faces(const Geo &g, const WS &w, hipStream_t st, bool stoppable) override {
    const int *done = stoppable ? w.flags + FL_DONE : nullptr;
    // (the streaming face kernels have the first-order HLLE residual only)
    if constexpr (NT == 1 && NS >= STREAM_NS_MIN)
      if (g.scheme == 0) return launch_stream_faces(g, w.mview, w.prim, w.Fi, w.Ri, w.Fj, w.Rj, w.qw, done, st);
    const dim3 bi(nblocks(long(g.ni + 1) * g.nj)), bj(nblocks(long(g.ni) * (g.nj + 1)));
    if (g.scheme == 1) {
      hipLaunchKernelGGL((k_face_i<NS, NT, 1>), bi, dim3(256), 0, st, g, w.mech, w.prim, w.Fi, w.Ri, done,
                         w.flags + FL_BAD);
      hipLaunchKernelGGL((k_face_j<NS, NT, 1>), bj, dim3(256), 0, st, g, w.mech, w.prim, w.Fj, w.Rj, w.qw, done,
                         w.flags + FL_BAD);
    } else {
      hipLaunchKernelGGL((k_face_i<NS, NT, 0>), bi, dim3(256), 0, st, g, w.mech, w.prim, w.Fi, w.Ri, done,
                         w.flags + FL_BAD);
      hipLaunchKernelGGL((k_face_j<NS, NT, 0>), bj, dim3(256), 0, st, g, w.mech, w.prim, w.Fj, w.Rj, w.qw, done,
                         w.flags + FL_BAD);
    }
    return hipGetLastError();
  }

  hipError_t cell(const Geo &g, const WS &w, hipStream_t st, double cfl, int mode, int prec, int flags,
                  bool stoppable, hipEvent_t sur_ready = nullptr, hipEvent_t mid = nullptr) override {
    // with the diagonal blocks built by k_block only that kernel reads the
    // surrogate's blocks, so the cell kernel runs beside the inference
    const bool blk = NS >= BLOCK_NS_MIN && (flags & 2);
    if (sur_ready && !blk) {
      const hipError_t e = hipStreamWaitEvent(st, sur_ready, 0);
      if (e != hipSuccess) return e;
    }
    CellOut o{w.R, w.dtau, w.part, w.Dinv, w.b, {w.grp[0].S, w.grp[1].S}, w.src, w.flags + FL_SING, w.group_c,
              w.diag, w.sur.J, ddfail_counter(w.flags), w.flags + FL_SURR_OFF, w.qn, w.qnm1, w.pt_a, w.pt_b};
    const int *done = stoppable ? w.flags + FL_DONE : nullptr;
    // one temperature with the block kernel: a pass that forms both the
    // residual and the blocks takes the species source from the block
    // kernel's reaction records
    constexpr bool SB = NT == 1 && NS >= BLOCK_NS_MIN;
    const bool src_block = SB && (flags & 3) == 3;
    if (prec == 0) {
      if (src_block)
        launch_cell_sb<double>(g, w, st, cfl, mode, flags, o, done);
      else
        hipLaunchKernelGGL((k_cell<NS, NT, double, false>), dim3(w.nblk_cell), dim3(256), 0, st, g, w.mech, w.Q,
                           w.prim, w.Fi, w.Fj, w.Ri, w.Rj, cfl, mode, flags, o, done);
    } else {
      if (src_block)
        launch_cell_sb<float>(g, w, st, cfl, mode, flags, o, done);
      else
        hipLaunchKernelGGL((k_cell<NS, NT, float, false>), dim3(w.nblk_cell), dim3(256), 0, st, g, w.mech, w.Q,
                           w.prim, w.Fi, w.Fj, w.Ri, w.Rj, cfl, mode, flags, o, done);
    }
    if (mid) {
      const hipError_t e = hipEventRecord(mid, st);
      if (e != hipSuccess) return e;
    }
    if constexpr (NS >= BLOCK_NS_MIN) {
      if (flags & 2) {
        const BlockOut bo{{w.grp[0].S, w.grp[1].S}, w.Dinv, w.group_c, w.diag, w.sur.J, ddfail_counter(w.flags),
                          w.flags + FL_SURR_OFF, w.flags + FL_SING, nullptr, 0, SampleMap{0, 0},
                          src_block ? w.R : nullptr, w.b};
        if (sur_ready) {
          const hipError_t e = hipStreamWaitEvent(st, sur_ready, 0);
          if (e != hipSuccess) return e;
        }
        if (prec == 0) block<double>(g, w, st, mode, flags, bo, done);
        else block<float>(g, w, st, mode, flags, bo, done);
      }
    }
    return hipGetLastError();
  }

  // diagonal blocks with one lane per row (ns >= BLOCK_NS_MIN)
  template <typename RT>
  void block(const Geo &g, const WS &w, hipStream_t st, int mode, int flags, const BlockOut &bo, const int *done) {
    if (mode == 0) {
      constexpr int C = BlockDims<NS, NT, 0>::C;
      hipLaunchKernelGGL((k_block<NS, NT, RT, 0>), dim3(nblocks(g.N, C)), dim3(64), 0, st, g, w.mech, w.Q,
                         w.prim, flags, bo, done);
    } else {
      constexpr int C = BlockDims<NS, NT, 1>::C;
      hipLaunchKernelGGL((k_block<NS, NT, RT, 1>), dim3(nblocks(g.N, C)), dim3(64), 0, st, g, w.mech, w.Q,
                         w.prim, flags, bo, done);
    }
  }

  hipError_t norms(const WS &w, hipStream_t st, int it, double tol, bool stoppable, StallArgs stall) override {
    hipLaunchKernelGGL(k_norms<NS>, dim3(1), dim3(256), 0, st, w.part, w.nblk_cell, w.norms, stoppable ? w.hist : nullptr,
                       it, w.hist_max, stoppable ? w.r0 : nullptr, tol, stoppable ? w.flags + FL_DONE : nullptr,
                       w.flags + FL_ITDONE, stall);
    return hipGetLastError();
  }

  hipError_t surrogate(const Geo &g, const WS &w, hipStream_t st, bool stoppable) override {
    hipLaunchKernelGGL((k_surrogate<NS, NT>), dim3(nblocks(g.N, 64)), dim3(256), 0, st, g, w.prim, w.sur,
                       w.flags + FL_SURR_OFF, stoppable ? w.flags + FL_DONE : nullptr);
    return hipGetLastError();
  }

  hipError_t sample(const Geo &g, const WS &w, hipStream_t st, int n, float *xr, float *jc, int flags,
                    SampleMap sm) override {
    hipError_t e = prim(g, w, st, false, false);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_sample<NS, NT>), dim3(nblocks(n)), dim3(256), 0, st, g, w.mech, w.Q, w.prim, n, xr, jc,
                       flags, sm);
    if constexpr (NS >= BLOCK_NS_MIN) {
      // the species rows from the block kernel (one lane per row)
      hipLaunchKernelGGL((k_handoff<NS, NT>), dim3(nblocks(n)), dim3(256), 0, st, g, w.mech, w.Q, w.prim, n, w.diag,
                         sm);
      BlockOut bo{{nullptr, nullptr}, nullptr, 0, w.diag, nullptr, nullptr, nullptr, nullptr, jc, long(n), sm};
      constexpr int C = BlockDims<NS, NT, 1>::C;
      hipLaunchKernelGGL((k_block<NS, NT, float, 1>), dim3(nblocks(n, C)), dim3(64), 0, st, g, w.mech, w.Q, w.prim,
                         2 | (flags & 24), bo, nullptr);
    }
    return hipGetLastError();
  }

  // one temperature with the block kernel: the cell kernel compiled for the
  // form at hand (each form's instantiation carries only its own branch)
  template <typename RT>
  static void launch_cell_sb(const Geo &g, const WS &w, hipStream_t st, double cfl, int mode, int flags,
                             const CellOut &o, const int *done) {
    constexpr bool SB = NT == 1 && NS >= BLOCK_NS_MIN;
    if (mode == 1)
      hipLaunchKernelGGL((k_cell<NS, NT, RT, SB, 1>), dim3(w.nblk_cell), dim3(256), 0, st, g, w.mech, w.Q, w.prim,
                         w.Fi, w.Fj, w.Ri, w.Rj, cfl, mode, flags, o, done);
    else
      hipLaunchKernelGGL((k_cell<NS, NT, RT, SB, 0>), dim3(w.nblk_cell), dim3(256), 0, st, g, w.mech, w.Q, w.prim,
                         w.Fi, w.Fj, w.Ri, w.Rj, cfl, mode, flags, o, done);
  }

  template <typename RT, int MODE>
  static void launch_pair(const Geo &g, const GroupArgs &a, dim3 gr, dim3 bl, hipStream_t st, const int *done,
                          hipEvent_t mid) {
    constexpr size_t lds = group_lds_bytes<NS, NT, RT, MODE>();
    static_assert(lds + sizeof(GroupSync) <= 160 * 1024, "sweep ring exceeds the LDS");
    static bool attr = false;  // dynamic LDS above 64 KiB must be allowed per kernel
    if (!attr) {
      (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&k_group_sweep<NS, NT, RT, MODE, true>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
      (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&k_group_sweep<NS, NT, RT, MODE, false>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
      attr = true;
    }
    hipLaunchKernelGGL((k_group_sweep<NS, NT, RT, MODE, true>), gr, bl, lds, st, g, a, done);
    if (mid) (void)hipEventRecord(mid, st);
    GroupArgs ab = a;
    if (ab.trace) ab.trace += 2L * g.ni * TR_N;
    hipLaunchKernelGGL((k_group_sweep<NS, NT, RT, MODE, false>), gr, bl, lds, st, g, ab, done);
  }

  // mid (optional) is recorded between the forward and the backward sweep
  template <typename RT>
  hipError_t sweeps_t(const Geo &g, const WS &w, hipStream_t st, int mode, bool stoppable, hipEvent_t mid) {
    const int *done = stoppable ? w.flags + FL_DONE : nullptr;
    if (w.group_c > 0) {
      GroupArgs a{};
      a.abort_flag = w.flags + FL_ABORT;
      a.spin_limit = w.spin_limit;
      a.trace = w.trace;
      const int nparts = mode == 0 ? 1 : 2;
      int nstrip = 0;
      long maxw = 0;
      GroupReset rs{};
      for (int q = 0; q < nparts; ++q) {
        const int C = group_cells<NS, NT>(w.group_c, mode, q);
        a.part[q] = GroupPart{w.grp[q], C};
        const int G = rec_shape(q == 1 ? PART_SPECIES : mode == 0 ? PART_COUPLED : PART_FLOW, NS, NT, 8).G;
        const GroupMap m = group_map(g.ni, g.nj, G);
        nstrip = m.nstrip > nstrip ? m.nstrip : nstrip;
        const long words = long(m.nstrip) * g.nj * G * long(sizeof(RT)) / 4;
        maxw = words > maxw ? words : maxw;
        rs.tickets[q] = w.grp[q].tickets;
        for (int f = 0; f < 2; ++f) {
          rs.bnd[2 * q + f] = reinterpret_cast<unsigned *>(w.grp[q].bnd[f]);
          rs.nw[2 * q + f] = words;
        }
      }
      const int rb = nblocks(maxw) < 1024 ? (nblocks(maxw) > 0 ? nblocks(maxw) : 1) : 1024;
      hipLaunchKernelGGL(k_group_reset<NS>, dim3(rb), dim3(256), 0, st, rs, done);
      // split: one workgroup per strip for each of the two independent parts
      const dim3 gr(nstrip, nparts), bl(192);
      if (mode == 0) launch_pair<RT, 0>(g, a, gr, bl, st, done, mid);
      else launch_pair<RT, 1>(g, a, gr, bl, st, done, mid);
      return hipGetLastError();
    }
    SweepArgs a{w.prim, w.Ri, w.Rj, w.Dinv, w.b, w.dqs, w.dq, mode, w.Q, w.fdiff ? w.mech : nullptr,
                w.flags + FL_BAD};
    const int K = g.ni + g.nj - 1;
    for (int k = 0; k < K; ++k) {
      int j0 = k - g.ni + 1 > 0 ? k - g.ni + 1 : 0, j1 = k < g.nj - 1 ? k : g.nj - 1;
      int len = j1 - j0 + 1;
      hipLaunchKernelGGL((k_sweep_fwd_hp<NS, NT, RT>), dim3(nblocks(len, 64)), dim3(64), 0, st, g, a, k, done);
    }
    if (mid) (void)hipEventRecord(mid, st);
    for (int k = K - 1; k >= 0; --k) {
      int j0 = k - g.ni + 1 > 0 ? k - g.ni + 1 : 0, j1 = k < g.nj - 1 ? k : g.nj - 1;
      int len = j1 - j0 + 1;
      hipLaunchKernelGGL((k_sweep_bwd_hp<NS, NT, RT>), dim3(nblocks(len, 64)), dim3(64), 0, st, g, a, k, done);
    }
    return hipGetLastError();
  }

  hipError_t sweeps(const Geo &g, const WS &w, hipStream_t st, int mode, int prec, bool stoppable,
                    hipEvent_t mid) override {
    return prec == 0 ? sweeps_t<double>(g, w, st, mode, stoppable, mid) : sweeps_t<float>(g, w, st, mode, stoppable, mid);
  }

  hipError_t update(const Geo &g, const WS &w, hipStream_t st, int mode, int prec, int kind, bool stoppable) override {
    const int *done = stoppable ? w.flags + FL_DONE : nullptr;
    IncView iv{{w.grp[0].x, w.grp[1].x}, {0, 0}};
    if (w.group_c > 0) {
      iv.C[0] = group_cells<NS, NT>(w.group_c, mode, 0);
      iv.C[1] = group_cells<NS, NT>(w.group_c, mode, 1);
    }
    if (prec == 0)
      hipLaunchKernelGGL((k_update<NS, NT, double>), dim3(nblocks(g.N)), dim3(256), 0, st, g, w.mech, w.Q, w.dq, mode, kind,
                         w.flags + FL_CLIP, w.flags + FL_BAD, done, iv);
    else
      hipLaunchKernelGGL((k_update<NS, NT, float>), dim3(nblocks(g.N)), dim3(256), 0, st, g, w.mech, w.Q, w.dq, mode, kind,
                         w.flags + FL_CLIP, w.flags + FL_BAD, done, iv);
    return hipGetLastError();
  }

  hipError_t q_from_prim_host(const Mech &m, const double *rs, double u, double v, double T, double Tv,
                              double *q) override {
    q_from_prim<NS, NT>(m, rs, u, v, T, Tv, q);
    return hipSuccess;
  }
};

}  // namespace csi
