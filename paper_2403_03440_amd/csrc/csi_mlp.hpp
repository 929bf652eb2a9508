// Training-side kernels of the species-Jacobian surrogate network: operand
// packing, forward inference over a data set, one fused forward/backward pass
// per block of 64 samples producing per-block gradient partials, the ordered
// reduction of those partials with the Adam update, and the data preparation
// (feature standardisation and the asinh target transform).
//
// Rounding points (BF16 operands, FP32 accumulation) are those stated for the
// reference network: x, h1, h2, W1..W3 and the back-propagated errors g3, g2,
// g1 are rounded to BF16 before each product; biases, tanh, 1 - h^2 and the
// error scaling are FP32; block partials are summed across blocks in FP64 in
// block order, so the result does not depend on the launch schedule.
#pragma once
#include "csi_mlp_core.hpp"

namespace csi {

constexpr int MLP_LDP = 72;          // LDS row pitch (64 samples + 8 pad) in BF16 elements
constexpr int MLP_PREP_BLOCKS = 256; // fixed partition of the data set for the statistics

__global__ void k_mlp_pack(MlpDims d, const float *__restrict__ p, u16x8 *__restrict__ P) {
  int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q < d.nslots) P[q] = mlp_pack_slot(d, p, q);
}

__device__ inline float wave16_sum(float v) {
  v += __shfl_xor(v, 1, 16);
  v += __shfl_xor(v, 2, 16);
  v += __shfl_xor(v, 4, 16);
  v += __shfl_xor(v, 8, 16);
  return v;
}

// y[n][n_out] = network(x[n][n_in]) for standardised FP32 features.
template <int KS1>
__global__ void __launch_bounds__(256) k_mlp_forward(MlpDims d, const u16x8 *__restrict__ P,
                                                     const float *__restrict__ p, const float *__restrict__ x, int n,
                                                     float *__restrict__ y) {
  const int lane = threadIdx.x & 63, g = lane >> 4, j = lane & 15;
  const long smp = long(blockIdx.x) * 64 + (threadIdx.x >> 6) * 16 + j;
  const bool valid = smp < n;
  u16x8 xin[KS1];
#pragma unroll
  for (int s = 0; s < KS1; ++s)
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      int k = mlp_kmap(s, g, e);
      xin[s][e] = f2bf(valid && k < d.n_in ? x[smp * d.n_in + k] : 0.f);
    }
  float h1[4][4], h2[4][4];
  u16x8 B2[2];
  mlp_hidden<KS1>(d, P, p, xin, h1, h2, B2);
  for (int t = 0; t < d.nt3; ++t) {
    f32x4 a = mlp_out_tile(d, P, p, B2, t);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      int o = 16 * t + 4 * g + r;
      if (valid && o < d.n_out) y[smp * d.n_out + o] = a[r];
    }
  }
}

// One block = 64 samples (4 waves x 16).  Writes the block's loss sum and its
// gradient partial [np] (FP32) to row blockIdx.x of the partial arrays.
template <int KS1>
__global__ void __launch_bounds__(256) k_mlp_grad(MlpDims d, const u16x8 *__restrict__ P, const float *__restrict__ p,
                                                  const float *__restrict__ x, const float *__restrict__ tg,
                                                  const int *__restrict__ idx, int batch, int n_data, float scale,
                                                  float *__restrict__ part, double *__restrict__ lpart) {
  __shared__ __attribute__((aligned(16))) unsigned short xT[32 * KS1][MLP_LDP];
  __shared__ __attribute__((aligned(16))) unsigned short h1T[64][MLP_LDP], h2T[64][MLP_LDP];
  __shared__ __attribute__((aligned(16))) unsigned short g2T[64][MLP_LDP], g1T[64][MLP_LDP], g3c[32][MLP_LDP];
  __shared__ float red[4][64];
  __shared__ double lred[4];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, g = lane >> 4, j = lane & 15;
  const int col = wave * 16 + j;
  const long smp = long(blockIdx.x) * 64 + col;
  const int rid = smp < batch ? idx[smp] : -1;
  const bool valid = rid >= 0 && rid < n_data;
  const long row = valid ? long(rid) : 0;
  float *gp = part + long(blockIdx.x) * d.np;

  u16x8 xin[KS1];
#pragma unroll
  for (int s = 0; s < KS1; ++s)
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      int k = mlp_kmap(s, g, e);
      unsigned short b = f2bf(valid && k < d.n_in ? x[row * d.n_in + k] : 0.f);
      xin[s][e] = b;
      xT[k][col] = b;
    }
  float h1[4][4], h2[4][4];
  u16x8 B2[2];
  mlp_hidden<KS1>(d, P, p, xin, h1, h2, B2);
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      h1T[16 * t + 4 * g + r][col] = f2bf(h1[t][r]);
      h2T[16 * t + 4 * g + r][col] = f2bf(h2[t][r]);
    }
  __syncthreads();

  // output layer in pairs of tiles: loss, g3, its contribution to dH2 and the
  // gradients of W3 / b3 for those 32 outputs
  f32x4 aD2[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) aD2[t] = f32x4{0.f, 0.f, 0.f, 0.f};
  double lsum = 0.0;
  const int ks3 = d.nt3 / 2;
  for (int s3 = 0; s3 < ks3; ++s3) {
    float g3[2][4];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int tt = 2 * s3 + h;
      f32x4 yv = mlp_out_tile(d, P, p, B2, tt);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int o = 16 * tt + 4 * g + r;
        double dd = (valid && o < d.n_out) ? double(yv[r]) - double(tg[row * d.n_out + o]) : 0.0;
        lsum += dd * dd;
        g3[h][r] = float(dd * double(scale));
        g3c[16 * h + 4 * g + r][col] = f2bf(g3[h][r]);
        float sr = wave16_sum(g3[h][r]);
        if (j == 0) red[wave][16 * h + 4 * g + r] = sr;
      }
    }
    const u16x8 B3 = mlp_b_from_acc(g3[0], g3[1]);
#pragma unroll
    for (int t = 0; t < 4; ++t) aD2[t] = mfma16(P[d.pW3T + (t * ks3 + s3) * 64 + lane], B3, aD2[t]);
    __syncthreads();
    for (int tile = wave; tile < 8; tile += 4) {
      const int ro = tile >> 2, th = tile & 3;
      f32x4 acc = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        u16x8 a = *reinterpret_cast<const u16x8 *>(&g3c[16 * ro + j][32 * s + 8 * g]);
        u16x8 b = *reinterpret_cast<const u16x8 *>(&h2T[16 * th + j][32 * s + 8 * g]);
        acc = mfma16(a, b, acc);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int o = 32 * s3 + 16 * ro + 4 * g + r;
        if (o < d.n_out) gp[d.oW3 + o * MLP_H + 16 * th + j] = acc[r];
      }
    }
    if (threadIdx.x < 32) {
      const int o = 32 * s3 + threadIdx.x;
      if (o < d.n_out) gp[d.ob3 + o] = ((red[0][threadIdx.x] + red[1][threadIdx.x]) + red[2][threadIdx.x]) + red[3][threadIdx.x];
    }
    __syncthreads();
  }

  // hidden layer 2: g2 = dH2 (1 - h2^2); dH1 = W2^T g2
  float g2[4][4];
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      g2[t][r] = aD2[t][r] * fmaf(-h2[t][r], h2[t][r], 1.f);
      g2T[16 * t + 4 * g + r][col] = f2bf(g2[t][r]);
      float sr = wave16_sum(g2[t][r]);
      if (j == 0) red[wave][16 * t + 4 * g + r] = sr;
    }
  u16x8 Bg[2];
#pragma unroll
  for (int s = 0; s < 2; ++s) Bg[s] = mlp_b_from_acc(g2[2 * s], g2[2 * s + 1]);
  f32x4 aD1[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    aD1[t] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < 2; ++s) aD1[t] = mfma16(P[d.pW2T + (t * 2 + s) * 64 + lane], Bg[s], aD1[t]);
  }
  __syncthreads();
  if (threadIdx.x < 64)
    gp[d.ob2 + threadIdx.x] = ((red[0][threadIdx.x] + red[1][threadIdx.x]) + red[2][threadIdx.x]) + red[3][threadIdx.x];
  __syncthreads();
  float g1[4][4];
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      g1[t][r] = aD1[t][r] * fmaf(-h1[t][r], h1[t][r], 1.f);
      g1T[16 * t + 4 * g + r][col] = f2bf(g1[t][r]);
      float sr = wave16_sum(g1[t][r]);
      if (j == 0) red[wave][16 * t + 4 * g + r] = sr;
    }
  // loss partial
  for (int m = 1; m < 64; m <<= 1) lsum += __shfl_xor(lsum, m, 64);
  if (lane == 0) lred[wave] = lsum;
  __syncthreads();
  if (threadIdx.x < 64)
    gp[d.ob1 + threadIdx.x] = ((red[0][threadIdx.x] + red[1][threadIdx.x]) + red[2][threadIdx.x]) + red[3][threadIdx.x];
  if (threadIdx.x == 0) lpart[blockIdx.x] = ((lred[0] + lred[1]) + lred[2]) + lred[3];
  // dW2 = g2^T h1 (16 tiles) and dW1 = g1^T x (4 x 2 KS1 tiles) over the block's samples
  for (int tile = wave; tile < 16; tile += 4) {
    const int to = tile >> 2, th = tile & 3;
    f32x4 acc = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      u16x8 a = *reinterpret_cast<const u16x8 *>(&g2T[16 * to + j][32 * s + 8 * g]);
      u16x8 b = *reinterpret_cast<const u16x8 *>(&h1T[16 * th + j][32 * s + 8 * g]);
      acc = mfma16(a, b, acc);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) gp[d.oW2 + (16 * to + 4 * g + r) * MLP_H + 16 * th + j] = acc[r];
  }
  for (int tile = wave; tile < 8 * KS1; tile += 4) {
    const int to = tile / (2 * KS1), tk = tile % (2 * KS1);
    f32x4 acc = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      u16x8 a = *reinterpret_cast<const u16x8 *>(&g1T[16 * to + j][32 * s + 8 * g]);
      u16x8 b = *reinterpret_cast<const u16x8 *>(&xT[16 * tk + j][32 * s + 8 * g]);
      acc = mfma16(a, b, acc);
    }
    const int k = 16 * tk + j;
    if (k < d.n_in) {
#pragma unroll
      for (int r = 0; r < 4; ++r) gp[d.oW1 + (16 * to + 4 * g + r) * d.n_in + k] = acc[r];
    }
  }
}

// Ordered sum of the block partials (FP64, block order), optional gradient
// output, optional Adam update of the FP32 master vector and its moments.
__global__ void k_mlp_reduce(int np, int nblk, const float *__restrict__ part, const double *__restrict__ lpart,
                             double loss_scale, double *__restrict__ loss, float *__restrict__ grad,
                             float *__restrict__ prm, float *__restrict__ am, float *__restrict__ av, int step,
                             double lr, double b1, double b2, double eps) {
  int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q == 0 && loss) {
    double s = 0.0;
    for (int b = 0; b < nblk; ++b) s += lpart[b];
    *loss = s * loss_scale;
  }
  if (q >= np) return;
  double s = 0.0;
  for (int b = 0; b < nblk; ++b) s += double(part[long(b) * np + q]);
  const float gq = float(s);
  if (grad) grad[q] = gq;
  if (prm) {
    const double gd = double(gq);
    const double m = b1 * double(am[q]) + (1.0 - b1) * gd;
    const double v = b2 * double(av[q]) + (1.0 - b2) * gd * gd;
    const double mh = m / (1.0 - pow(b1, double(step)));
    const double vh = v / (1.0 - pow(b2, double(step)));
    prm[q] = float(double(prm[q]) - lr * mh / (sqrt(vh) + eps));
    am[q] = float(m);
    av[q] = float(v);
  }
}

// ------------------------------------------------------------ data preparation
// Block partials of per-feature sums (pass 0: x, pass 1: (x - mu)^2) over a
// fixed partition of the samples; feature = blockIdx.y.
__global__ void __launch_bounds__(256) k_prep_moments(int n, int n_in, const float *__restrict__ x,
                                                      const double *__restrict__ mu, double *__restrict__ part) {
  __shared__ double sh[256];
  const int k = blockIdx.y;
  const long per = (long(n) + MLP_PREP_BLOCKS - 1) / MLP_PREP_BLOCKS;
  const long lo = long(blockIdx.x) * per, hi = lo + per < n ? lo + per : n;
  double s = 0.0;
  for (long i = lo + threadIdx.x; i < hi; i += 256) {
    double v = double(x[i * n_in + k]);
    if (mu) v = (v - mu[k]) * (v - mu[k]);
    s += v;
  }
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[long(k) * MLP_PREP_BLOCKS + blockIdx.x] = sh[0];
}

// Block partials of sum ln|J| and of the count of non-zero entries.
__global__ void __launch_bounds__(256) k_prep_logj(long m, const float *__restrict__ J, double *__restrict__ part) {
  __shared__ double sh[256], sc[256];
  const long per = (m + MLP_PREP_BLOCKS - 1) / MLP_PREP_BLOCKS;
  const long lo = long(blockIdx.x) * per, hi = lo + per < m ? lo + per : m;
  double s = 0.0, c = 0.0;
  for (long i = lo + threadIdx.x; i < hi; i += 256) {
    double a = fabs(double(J[i]));
    if (a > 0.0) { s += log(a); c += 1.0; }
  }
  sh[threadIdx.x] = s;
  sc[threadIdx.x] = c;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) { sh[threadIdx.x] += sh[threadIdx.x + w]; sc[threadIdx.x] += sc[threadIdx.x + w]; }
    __syncthreads();
  }
  if (threadIdx.x == 0) { part[blockIdx.x] = sh[0]; part[MLP_PREP_BLOCKS + blockIdx.x] = sc[0]; }
}

// scales = [mu (n_in), sigma (n_in), tau0]; stage 0 finishes mu and tau0,
// stage 1 finishes sigma (sigma := 1 where the standard deviation < 1e-12).
__global__ void k_prep_finish(int stage, int n, int n_in, const double *__restrict__ mpart,
                              const double *__restrict__ jpart, double *__restrict__ scales) {
  int k = threadIdx.x;
  if (k < n_in) {
    double s = 0.0;
    for (int b = 0; b < MLP_PREP_BLOCKS; ++b) s += mpart[long(k) * MLP_PREP_BLOCKS + b];
    if (stage == 0) scales[k] = s / n;
    else {
      double sd = sqrt(s / n);
      scales[n_in + k] = sd < 1e-12 ? 1.0 : sd;
    }
  }
  if (stage == 0 && k == 0) {
    double s = 0.0, c = 0.0;
    for (int b = 0; b < MLP_PREP_BLOCKS; ++b) { s += jpart[b]; c += jpart[MLP_PREP_BLOCKS + b]; }
    scales[2 * n_in] = c > 0.0 ? exp(-s / c) : 1.0;
  }
}

__global__ void k_prep_apply(long n, int n_in, int n_out, const float *__restrict__ xr, const float *__restrict__ J,
                             const double *__restrict__ scales, float *__restrict__ xs, float *__restrict__ t) {
  const long i = long(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n * n_in) {
    int k = int(i % n_in);
    xs[i] = float((double(xr[i]) - scales[k]) / scales[n_in + k]);
  }
  if (i < n * n_out) t[i] = float(asinh(double(J[i]) * scales[2 * n_in]));
}

}  // namespace csi
