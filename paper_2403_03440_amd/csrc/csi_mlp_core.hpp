// Building blocks of the species-Jacobian surrogate network on gfx950 matrix
// cores: x -> tanh(W1 x + b1) -> tanh(W2 h1 + b2) -> W3 h2 + b3, hidden width
// 64, BF16 operands with FP32 accumulation (v_mfma_f32_16x16x32_bf16).
//
// Every product is computed transposed, Z^T = W X^T, so that one wave owns 16
// samples (the MFMA's N dimension) and the activations of one layer are
// already in the lanes the next layer's B operand needs: the accumulator of
// output tile t holds rows 16t + 4g + r (g = lane / 16, r = 0..3) of sample
// lane % 16.  The MFMA pairs A and B elements by (lane group, element), so the
// reduction index k may be assigned to them in any order as long as both
// operands use the same one; here element e of group g in k-step s is
//   k = 32 s + 4 g + e          (e < 4, from accumulator tile 2s)
//   k = 32 s + 16 + 4 g + e - 4 (e >= 4, from accumulator tile 2s + 1)
// and the weights are stored pre-permuted in that order ("packed"), 16 bytes
// per lane per (tile, k-step).
#pragma once
#include <hip/hip_runtime.h>

namespace csi {

constexpr int MLP_H = 64;        // hidden width
constexpr int MLP_MAX_IN = 64;   // n_in <= 64 (two k-steps)
constexpr int MLP_MAX_OUT = 1024;

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(8))) unsigned short u16x8;
typedef __attribute__((ext_vector_type(4))) float f32x4;

// round to nearest even (finite inputs)
__host__ __device__ inline unsigned short f2bf(float f) {
  unsigned u;
  __builtin_memcpy(&u, &f, 4);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return static_cast<unsigned short>(u >> 16);
}
__host__ __device__ inline float bf2f(unsigned short h) {
  unsigned u = unsigned(h) << 16;
  float f;
  __builtin_memcpy(&f, &u, 4);
  return f;
}

__host__ __device__ inline int mlp_kmap(int s, int g, int e) { return 32 * s + (e < 4 ? 4 * g + e : 12 + 4 * g + e); }

__device__ inline f32x4 mfma16(const u16x8 &a, const u16x8 &b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c, 0,
                                                 0, 0);
}

// Geometry of a network with n_in inputs and n_out outputs.
struct MlpDims {
  int n_in, n_out;
  int ks1;   // k-steps of layer 1 (n_in padded to 32 * ks1)
  int nt3;   // output tiles of 16 rows (even: n_out padded to 32 * nt3 / 2)
  int np;    // FP32 master parameters
  // offsets in the master vector
  int oW1, ob1, oW2, ob2, oW3, ob3;
  // offsets (in 16-byte lane slots) of the packed operands
  int pW1, pW2, pW3, pW2T, pW3T, nslots;
};

__host__ __device__ inline MlpDims mlp_dims(int n_in, int n_out) {
  MlpDims d;
  d.n_in = n_in;
  d.n_out = n_out;
  d.ks1 = (n_in + 31) / 32;
  d.nt3 = 2 * ((n_out + 31) / 32);
  d.oW1 = 0;
  d.ob1 = d.oW1 + MLP_H * n_in;
  d.oW2 = d.ob1 + MLP_H;
  d.ob2 = d.oW2 + MLP_H * MLP_H;
  d.oW3 = d.ob2 + MLP_H;
  d.ob3 = d.oW3 + n_out * MLP_H;
  d.np = d.ob3 + n_out;
  d.pW1 = 0;                              // 4 tiles x ks1 steps
  d.pW2 = d.pW1 + 4 * d.ks1 * 64;         // 4 x 2
  d.pW3 = d.pW2 + 8 * 64;                 // nt3 x 2
  d.pW2T = d.pW3 + d.nt3 * 2 * 64;        // 4 x 2
  d.pW3T = d.pW2T + 8 * 64;               // 4 x nt3/2
  d.nslots = d.pW3T + 4 * (d.nt3 / 2) * 64;
  return d;
}

// Packed operand slot q (16 bytes): which matrix, tile, k-step and lane, and
// the eight BF16 values it holds, read from the FP32 master vector.
__device__ inline u16x8 mlp_pack_slot(const MlpDims &d, const float *__restrict__ p, int q) {
  int which, t, s, lane = q & 63, base, ks;
  if (q < d.pW2) { which = 0; base = d.pW1; ks = d.ks1; }
  else if (q < d.pW3) { which = 1; base = d.pW2; ks = 2; }
  else if (q < d.pW2T) { which = 2; base = d.pW3; ks = 2; }
  else if (q < d.pW3T) { which = 3; base = d.pW2T; ks = 2; }
  else { which = 4; base = d.pW3T; ks = d.nt3 / 2; }
  int ts = (q - base) >> 6;
  t = ts / ks;
  s = ts - t * ks;
  int row = 16 * t + (lane & 15), g = lane >> 4;
  u16x8 v;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    int k = mlp_kmap(s, g, e);
    float x = 0.f;
    switch (which) {
      case 0: if (k < d.n_in) x = p[d.oW1 + row * d.n_in + k]; break;           // W1[row][k]
      case 1: x = p[d.oW2 + row * MLP_H + k]; break;                            // W2[row][k]
      case 2: if (row < d.n_out) x = p[d.oW3 + row * MLP_H + k]; break;         // W3[row][k]
      case 3: x = p[d.oW2 + k * MLP_H + row]; break;                            // W2^T
      default: if (k < d.n_out) x = p[d.oW3 + k * MLP_H + row]; break;          // W3^T
    }
    v[e] = f2bf(x);
  }
  return v;
}

// B operand of the next layer from two accumulator tiles (rounded to BF16).
__device__ inline u16x8 mlp_b_from_acc(const float *lo, const float *hi) {
  u16x8 v;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    v[e] = f2bf(lo[e]);
    v[e + 4] = f2bf(hi[e]);
  }
  return v;
}

// Hidden layers for the wave's 16 samples.  xin[s] is the layer-1 B operand
// of k-step s; h1, h2 receive tanh activations (FP32) in accumulator layout and
// B2 the layer-3 B operands.
template <int KS1>
__device__ inline void mlp_hidden(const MlpDims &d, const u16x8 *__restrict__ P, const float *__restrict__ p,
                                  const u16x8 (&xin)[KS1], float (&h1)[4][4], float (&h2)[4][4], u16x8 (&B2)[2]) {
  const int lane = threadIdx.x & 63, g = lane >> 4;
  f32x4 acc[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < KS1; ++s) acc[t] = mfma16(P[d.pW1 + (t * KS1 + s) * 64 + lane], xin[s], acc[t]);
  }
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) h1[t][r] = tanhf(acc[t][r] + p[d.ob1 + 16 * t + 4 * g + r]);
  u16x8 B1[2];
#pragma unroll
  for (int s = 0; s < 2; ++s) B1[s] = mlp_b_from_acc(h1[2 * s], h1[2 * s + 1]);
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < 2; ++s) acc[t] = mfma16(P[d.pW2 + (t * 2 + s) * 64 + lane], B1[s], acc[t]);
  }
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) h2[t][r] = tanhf(acc[t][r] + p[d.ob2 + 16 * t + 4 * g + r]);
#pragma unroll
  for (int s = 0; s < 2; ++s) B2[s] = mlp_b_from_acc(h2[2 * s], h2[2 * s + 1]);
}

// Output tile t (rows 16t + 4g + r) for the wave's samples, bias included.
__device__ inline f32x4 mlp_out_tile(const MlpDims &d, const u16x8 *__restrict__ P, const float *__restrict__ p,
                                     const u16x8 (&B2)[2], int t) {
  const int lane = threadIdx.x & 63, g = lane >> 4;
  f32x4 acc = f32x4{0.f, 0.f, 0.f, 0.f};
  acc = mfma16(P[d.pW3 + (t * 2 + 0) * 64 + lane], B2[0], acc);
  acc = mfma16(P[d.pW3 + (t * 2 + 1) * 64 + lane], B2[1], acc);
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    int o = 16 * t + 4 * g + r;
    acc[r] = o < d.n_out ? acc[r] + p[d.ob3 + o] : 0.f;
  }
  return acc;
}

}  // namespace csi
