// Learned conditional means <phi|V>: the device pieces shared by the step
// kernel and the network kernels -- bfloat16 rounding, the 16x16x16 bfloat16
// MFMA tiles of the network's forward pass, element features and the
// conserving projection with its fallback rule.  Included by the step
// kernel's header after its statistics-record layout.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pdf {
namespace mlp {

constexpr int NFEAT = 32, NHID = 64, NOUT = 8, ROW = 64;
constexpr int OFF_W1 = 0, OFF_B1 = 2048, OFF_W2 = 2112, OFF_B2 = 6208, OFF_W3 = 6272, OFF_B3 = 10368,
              OFF_W4 = 10432, OFF_B4 = 10944, NPARAM = 10952;
constexpr int N_MIN = 8, N_MAX = 64;            // element counts the network serves
constexpr double SIGMA_MIN = 1e-4;              // smaller subsample scalar spread: not a training row
constexpr double T_CLIP = 8.0;                  // standardised targets are clipped to +-T_CLIP
constexpr uint32_t SUB_BLOCK = 0x5EED;          // Philox block word of the subsample draw
constexpr uint32_t TRAIN_BLOCK = 0x7A11;        // Philox block word of the training-row draw
constexpr int TILE = 16;                        // samples per wavefront tile
constexpr int MLP_WAVES = 4;                    // wavefronts per block

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// float -> bfloat16, round to nearest even (finite inputs)
__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// D = A B + C for 16x16 tiles, K = 16.  Lane l holds A[l%16][4(l/16)+i],
// B[4(l/16)+i][l%16] and D[4(l/16)+i][l%16], i = 0..3.
__device__ __forceinline__ f32x4 mfma16(bf16x4 a, bf16x4 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ f32x4 zero4() { return f32x4{0.0f, 0.0f, 0.0f, 0.0f}; }

// A operand: rows 16 mt.. of a row-major (out x in) weight matrix, columns 16 ks..
__device__ __forceinline__ bf16x4 load_w(const uint16_t* W, int in, int mt, int ks, int lane) {
  const int row = 16 * mt + (lane & 15), col = 16 * ks + 4 * (lane >> 4);
  return *(const bf16x4*)(W + row * in + col);
}

// The output layer's A operand, rows 8..15 zero.
__device__ __forceinline__ bf16x4 load_w4(const uint16_t* W4, int ks, int lane) {
  const int row = lane & 15;
  if (row >= NOUT) return bf16x4{0, 0, 0, 0};
  return *(const bf16x4*)(W4 + row * NHID + 16 * ks + 4 * (lane >> 4));
}

// A operand of the transposed product W^T: element (m = in unit, k = out unit)
// is W[k][m]; rows 16 mt.. (in units), columns 16 ks.. (out units).
__device__ __forceinline__ bf16x4 load_wt(const uint16_t* W, int in, int out, int mt, int ks, int lane) {
  const int m = 16 * mt + (lane & 15);
  bf16x4 r;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int k = 16 * ks + 4 * (lane >> 4) + i;
    r[i] = k < out ? (short)W[k * in + m] : (short)0;
  }
  return r;
}

// Bias, ReLU and rounding of one output tile: the B operand of the next layer.
__device__ __forceinline__ bf16x4 bias_relu_bf16(f32x4 acc, const uint16_t* b, int mt, int lane) {
  bf16x4 h;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const float z = acc[i] + bf2f(b[16 * mt + 4 * (lane >> 4) + i]);
    h[i] = (short)f2bf(z > 0.0f ? z : 0.0f);
  }
  return h;
}

// Forward pass of one 16-sample tile.  xb: inputs as B operands (features
// 0..15 and 16..31).  h1..h3: hidden activations, B-operand layout.  Returns
// the output tile: lanes 0..31 hold y[unit 4(l/16)+i] of sample l%16, bias
// included; lanes 32..63 hold zeros.
__device__ __forceinline__ f32x4 forward_tile(const uint16_t* P, const bf16x4 (&xb)[2], bf16x4 (&h1)[4],
                                              bf16x4 (&h2)[4], bf16x4 (&h3)[4], int lane) {
#pragma unroll
  for (int mt = 0; mt < 4; ++mt) {
    f32x4 acc = zero4();
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) acc = mfma16(load_w(P + OFF_W1, NFEAT, mt, ks, lane), xb[ks], acc);
    h1[mt] = bias_relu_bf16(acc, P + OFF_B1, mt, lane);
  }
#pragma unroll
  for (int mt = 0; mt < 4; ++mt) {
    f32x4 acc = zero4();
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) acc = mfma16(load_w(P + OFF_W2, NHID, mt, ks, lane), h1[ks], acc);
    h2[mt] = bias_relu_bf16(acc, P + OFF_B2, mt, lane);
  }
#pragma unroll
  for (int mt = 0; mt < 4; ++mt) {
    f32x4 acc = zero4();
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) acc = mfma16(load_w(P + OFF_W3, NHID, mt, ks, lane), h2[ks], acc);
    h3[mt] = bias_relu_bf16(acc, P + OFF_B3, mt, lane);
  }
  f32x4 y = zero4();
#pragma unroll
  for (int ks = 0; ks < 4; ++ks) y = mfma16(load_w4(P + OFF_W4, ks, lane), h3[ks], y);
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int o = 4 * (lane >> 4) + i;
    y[i] = o < NOUT ? y[i] + bf2f(P[OFF_B4 + o]) : 0.0f;
  }
  return y;
}

// Features of one element (float32) from its statistics as they stand in
// the statistics record: count, means (u, v, w, psi), the ten central second
// moments, bin counts and binned means.
__device__ __forceinline__ void features_from(double n, const double* mean, const double* m2, const double* binn,
                                              const double* binm, float* f) {
  f[0] = (float)(n / 64.0);
#pragma unroll
  for (int q = 0; q < 4; ++q) f[1 + q] = (float)mean[q];
#pragma unroll
  for (int q = 0; q < 10; ++q) f[5 + q] = (float)m2[q];
#pragma unroll
  for (int q = 0; q < 8; ++q) f[15 + q] = n > 0.0 ? (float)(binn[q] / n) : 0.0f;
#pragma unroll
  for (int q = 0; q < 8; ++q) f[23 + q] = (float)binm[q];
  f[31] = (float)sqrt(fmax(m2[9], 0.0));
}

// The learned estimate of one element from its statistics (n, psi mean,
// psi variance, bin counts, binned means) and the network outputs y: the
// projection p_b = y_b - sum_c (n_c / n) y_c, m_b = <psi> + sigma p_b, taken
// only if 8 <= n <= 64, the features were inside the training range, sigma > 0
// and every m_b lies in [0, 1]; otherwise the binned means.  Returns whether
// the network's value was taken.
__device__ __forceinline__ bool learned_estimate(double n, double mean_psi, double var_psi, const double* binn,
                                                 const double* binm, const float* y, bool inbox, double* cm) {
  double wsum = 0.0;
#pragma unroll
  for (int b = 0; b < NOUT; ++b) wsum += (n > 0.0 ? binn[b] / n : 0.0) * (double)y[b];
  const double sig = sqrt(fmax(var_psi, 0.0));
  double m[NOUT];
  bool ok = inbox && n >= (double)N_MIN && n <= (double)N_MAX && sig > 0.0;
#pragma unroll
  for (int b = 0; b < NOUT; ++b) {
    m[b] = mean_psi + sig * ((double)y[b] - wsum);
    ok = ok && m[b] >= 0.0 && m[b] <= 1.0;
  }
#pragma unroll
  for (int b = 0; b < NOUT; ++b) cm[b] = ok ? m[b] : binm[b];
  return ok;
}

}  // namespace mlp
}  // namespace pdf
