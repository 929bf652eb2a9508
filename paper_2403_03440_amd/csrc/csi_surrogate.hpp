// Solver-side kernels of the species-Jacobian surrogate: training samples
// (features and the exact J_C = d omega_s / d rho_r at fixed T, Tv, the block
// the split species diagonal carries, Section 2.3) and network inference per
// cell into an FP32 buffer that the cell kernel assembles D_C from.
#pragma once
#include "csi_kernels.hpp"
#include "csi_mlp_core.hpp"

namespace csi {

struct SurArgs {
  const u16x8 *P;         // packed BF16 operands
  const float *p;         // FP32 master vector (biases)
  const double *scales;   // mu[n_in], sigma[n_in], tau0
  float *J;               // [ns * ns][N], entry (s, r) at row s * ns + r
};

// Cell features (ln T, ln Tv, ln rho, Y_1..Y_ns) of padded cell pc.
template <int NS, int NT>
__device__ inline double sur_feature(const double *__restrict__ prim, size_t NP, long pc, int k) {
  if (k == 0) return log(prim[F_T * NP + pc]);
  if (k == 1) return log(prim[(NT == 2 ? F_TV : F_T) * NP + pc]);
  if (k == 2) return log(prim[F_RHO * NP + pc]);
  return prim[size_t(PF<NS>::Y + k - 3) * NP + pc];
}

template <int NS, int NT>
__global__ void __launch_bounds__(256) k_sample(Geo g, const Mech *__restrict__ mech, const double *__restrict__ Q,
                                                const double *__restrict__ prim, int n, float *__restrict__ xr,
                                                float *__restrict__ jc, int flags, SampleMap sm) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  const int p = int(sm(r, g.N));  // row r of the sample is cell p
  const Mech &m = *mech;
  const size_t NP = g.NP;
  const int i = p % g.ni, j = p / g.ni;
  const long pc = padc(g, i, j);
  constexpr int NIN = NS + 3;
#pragma unroll
  for (int k = 0; k < NIN; ++k) xr[long(r) * NIN + k] = float(sur_feature<NS, NT>(prim, NP, pc, k));
  // the block kernel writes J_C where it builds the species blocks
  if (NS >= BLOCK_NS_MIN) return;
  constexpr int NV = Dims<NS, NT>::nv;
  double q[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) q[k] = Q[size_t(k) * g.N + p];
  const double T = prim[F_T * NP + pc], Tv = prim[F_TV * NP + pc];
  Chem<NS, NT> C;
  chemistry<NS, NT, true>(m, q, T, Tv, prim[F_P * NP + pc], C);
  double dTc[NS], dTvc[NS];
  if (flags & 8) {
    Prim<NS, NT> P;
    prim_from_q<NS, NT>(m, q, P, T, Tv);
#pragma unroll
    for (int c = 0; c < NS; ++c) temp_derivs_fixed_e<NS, NT>(m, P, c, (flags & 16) != 0, dTc[c], dTvc[c]);
  } else {
#pragma unroll
    for (int c = 0; c < NS; ++c) dTc[c] = dTvc[c] = 0.0;
  }
#pragma unroll
  for (int s = 0; s < NS; ++s)
#pragma unroll
    for (int c = 0; c < NS; ++c)
      jc[long(r) * NS * NS + s * NS + c] = float(C.dw_dr[s][c] + C.dw_dT[s] * dTc[c] + C.dw_dTv[s] * dTvc[c]);
}

// sinh in FP32: the Taylor series to y^7 below |y| = 1/2 (truncation below
// 5e-9 relative), (e - 1/e) / 2 with e = exp(|y|) above (where the
// difference loses at most one bit): a few ulp, at a fraction of the cost of
// the library's sinhf; overflows to +-inf where sinhf does
__device__ __forceinline__ float sinh32(float y) {
  const float a = fabsf(y);
  if (a < 0.5f) {
    const float y2 = y * y;
    return y * (1.0f + y2 * (1.0f / 6.0f + y2 * (1.0f / 120.0f + y2 * (1.0f / 5040.0f))));
  }
  const float e = expf(a);
  return copysignf(0.5f * (e - 1.0f / e), y);
}

// One block = 64 cells (4 waves x 16); J = sinh(y) / tau0.
template <int NS, int NT>
__global__ void __launch_bounds__(256) k_surrogate(Geo g, const double *__restrict__ prim, SurArgs a,
                                                   const int *__restrict__ off, const int *__restrict__ done) {
  if ((done && *done) || *off >= 0) return;
  constexpr int NIN = NS + 3, KS1 = (NIN + 31) / 32;
  const MlpDims d = mlp_dims(NIN, NS * NS);
  const int lane = threadIdx.x & 63, gq = lane >> 4, jl = lane & 15;
  const int p = blockIdx.x * 64 + (threadIdx.x >> 6) * 16 + jl;
  const bool valid = p < g.N;
  const long pc = valid ? padc(g, p % g.ni, p / g.ni) : 0;
  u16x8 xin[KS1];
#pragma unroll
  for (int s = 0; s < KS1; ++s)
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int k = mlp_kmap(s, gq, e);
      float v = 0.f;
      if (valid && k < NIN) v = float((sur_feature<NS, NT>(prim, g.NP, pc, k) - a.scales[k]) / a.scales[NIN + k]);
      xin[s][e] = f2bf(v);
    }
  float h1[4][4], h2[4][4];
  u16x8 B2[2];
  mlp_hidden<KS1>(d, a.P, a.p, xin, h1, h2, B2);
  // J is stored in FP32 and y comes from FP32 accumulation: sinh in FP32
  // (a few ulp) keeps the stored value within a few FP32 roundings of the
  // double-precision expression, at a fraction of its cost
  const float itau = float(1.0 / a.scales[2 * NIN]);
  // layout of J: [ns * ns][N] where the cell kernel reads it (one thread per
  // cell, ns < 5); cell-major [N][ns * ns] where the block kernel does (each
  // lane reads one contiguous row of its cell's block)
  constexpr int NN = NS * NS;
  constexpr bool CELL_MAJOR = NS >= BLOCK_NS_MIN;
  for (int t = 0; t < d.nt3; ++t) {
    const f32x4 y = mlp_out_tile(d, a.P, a.p, B2, t);
    const int o0 = 16 * t + 4 * gq;
    f32x4 v;
#pragma unroll
    for (int r = 0; r < 4; ++r) v[r] = sinh32(y[r]) * itau;
    if (!valid) continue;
    if constexpr (CELL_MAJOR && NN % 4 == 0) {
      // a lane's four outputs are consecutive entries of its cell's block and
      // the block starts on a 16-byte boundary: one 16-byte store
      if (o0 < NN) *reinterpret_cast<f32x4 *>(a.J + size_t(p) * NN + o0) = v;
    } else {
#pragma unroll
      for (int r = 0; r < 4; ++r)
        if (o0 + r < NN) a.J[CELL_MAJOR ? size_t(p) * NN + o0 + r : size_t(o0 + r) * g.N + p] = v[r];
    }
  }
}

}  // namespace csi
