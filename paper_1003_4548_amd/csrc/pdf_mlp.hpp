// Learned conditional means <phi|V> for IECM: element features, a small
// multilayer perceptron on the matrix cores, its training and its use inside
// the particle step.
//
// IECM, eq. (7), relaxes a particle's scalar toward the mean scalar of the
// particles of its element whose velocities fall in the same velocity bin.
// With few particles per element that binned mean is noisy; the network maps
// the element's statistics (count, means, second moments, bin fractions and
// binned means) to standardised conditional means, which are projected so
// that IECM still conserves the element's scalar.  The binned means remain
// the fallback wherever the network is not trusted.
//
// Network: 32 -> 64 -> 64 -> 64 -> 8, ReLU, bfloat16 weights and biases,
// float32 accumulation, hidden activations rounded to bfloat16; 10952
// parameters.  Every layer is computed transposed, Z^T = W X^T, with the
// 16x16x16 bfloat16 MFMA: the weights are the A operand, the activations of
// 16 samples the B operand, and the output tile of one layer is, lane for
// lane, the B operand of the next, so the forward pass needs no data
// exchange between lanes.  The backward pass goes through LDS, where the
// activations are kept sample-major.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pdf_kernels.hpp"

namespace pdf {
namespace mlp {

// Features of one element from its statistics record.
__device__ __forceinline__ void features_of(const double* rec, float* f) {
  features_from(rec[ST_N], rec + ST_MEAN, rec + ST_M2, rec + ST_BINN, rec + ST_BINM, f);
}

// ---------------------------------------------------------------------------
// inference: statistics records -> conditional means per cell

struct InferArgs {
  const double* stats;   // ncell x nstat
  int32_t nstat;
  int32_t ncell;
  const uint16_t* w;     // NPARAM bfloat16 codes
  const float* norm;     // 4 x 32: mean, inverse scale, training minimum, training maximum
  double* cm;            // ncell x 8 (out)
  uint32_t* served;      // cells that took the network's value (may be null)
};

__global__ __launch_bounds__(64 * MLP_WAVES) void k_mlp_infer(InferArgs a) {
  __shared__ uint16_t xs[MLP_WAVES][TILE][NFEAT];
  __shared__ float ys[MLP_WAVES][TILE][NOUT];
  __shared__ int inbox[MLP_WAVES][TILE];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int c0 = (blockIdx.x * MLP_WAVES + wv) * TILE;
  const bool live = c0 < a.ncell;
  if (live && lane < TILE) {
    const int cell = c0 + lane;
    float f[NFEAT];
    int ok = 0;
    if (cell < a.ncell) {
      features_of(a.stats + (size_t)cell * a.nstat, f);
      ok = 1;
#pragma unroll
      for (int k = 0; k < NFEAT; ++k) ok &= (f[k] >= a.norm[2 * NFEAT + k] && f[k] <= a.norm[3 * NFEAT + k]) ? 1 : 0;
    } else {
#pragma unroll
      for (int k = 0; k < NFEAT; ++k) f[k] = a.norm[k];
    }
#pragma unroll
    for (int k = 0; k < NFEAT; ++k) xs[wv][lane][k] = f2bf((f[k] - a.norm[k]) * a.norm[NFEAT + k]);
    inbox[wv][lane] = ok;
  }
  __syncthreads();
  if (live) {
    bf16x4 xb[2], h1[4], h2[4], h3[4];
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) xb[ks] = *(const bf16x4*)&xs[wv][lane & 15][16 * ks + 4 * (lane >> 4)];
    const f32x4 y = forward_tile(a.w, xb, h1, h2, h3, lane);
    if (lane < 32) {
#pragma unroll
      for (int i = 0; i < 4; ++i) ys[wv][lane & 15][4 * (lane >> 4) + i] = y[i];
    }
  }
  __syncthreads();
  if (live && lane < TILE && c0 + lane < a.ncell) {
    const int cell = c0 + lane;
    const double* rec = a.stats + (size_t)cell * a.nstat;
    double cmv[NOUT];
    const bool ok = learned_estimate(rec[ST_N], rec[ST_MEAN + 3], rec[ST_M2 + 9], rec + ST_BINN, rec + ST_BINM,
                                     ys[wv][lane], inbox[wv][lane] != 0, cmv);
    double* out = a.cm + (size_t)cell * NOUT;
#pragma unroll
    for (int b = 0; b < NOUT; ++b) out[b] = cmv[b];
    if (ok && a.served) atomicAdd(a.served, 1u);
  }
}

// ---------------------------------------------------------------------------
// plain forward pass over dataset rows (outputs y, no projection)

struct ForwardArgs {
  const float* rows;
  int64_t nrows;
  int32_t stride;        // floats per row; the features are its first 32
  const float* norm;
  const uint16_t* w;
  float* y;              // nrows x 8 (out)
};

__global__ __launch_bounds__(64 * MLP_WAVES) void k_mlp_forward(ForwardArgs a) {
  __shared__ uint16_t xs[MLP_WAVES][TILE][NFEAT];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t r0 = ((int64_t)blockIdx.x * MLP_WAVES + wv) * TILE;
  const bool live = r0 < a.nrows;
  if (live && lane < TILE) {
    const int64_t r = r0 + lane;
#pragma unroll
    for (int k = 0; k < NFEAT; ++k) {
      const float f = r < a.nrows ? a.rows[r * a.stride + k] : a.norm[k];
      xs[wv][lane][k] = f2bf((f - a.norm[k]) * a.norm[NFEAT + k]);
    }
  }
  __syncthreads();
  if (!live) return;
  bf16x4 xb[2], h1[4], h2[4], h3[4];
#pragma unroll
  for (int ks = 0; ks < 2; ++ks) xb[ks] = *(const bf16x4*)&xs[wv][lane & 15][16 * ks + 4 * (lane >> 4)];
  const f32x4 y = forward_tile(a.w, xb, h1, h2, h3, lane);
  const int64_t r = r0 + (lane & 15);
  if (lane < 32 && r < a.nrows) {
#pragma unroll
    for (int i = 0; i < 4; ++i) a.y[r * NOUT + 4 * (lane >> 4) + i] = y[i];
  }
}

// ---------------------------------------------------------------------------
// training: per-tile gradients, then a reduction with the Adam update

struct GradArgs {
  const float* rows;     // nrows x 64: features, targets, loss weights, ...
  int64_t nrows;
  int32_t batch;
  int32_t draw;          // 0: rows 0..batch-1; 1: rows drawn with Philox
  uint32_t k0, k1, iter;
  const float* norm;
  const uint16_t* w;
  float* partial;        // ntiles x NPARAM (out)
  float* loss_partial;   // ntiles (out): sum over the tile of sum_b lw (p - t)^2
};

__device__ __forceinline__ void store_tile_bf16(uint16_t* buf, int ld, int mt, int lane, bf16x4 h) {
  *(bf16x4*)&buf[(lane & 15) * ld + 16 * mt + 4 * (lane >> 4)] = h;
}

// dW[o][k] = sum_s dz[s][o] h[s][k] for the tile at rows 16 mt (o), columns 16 nt (k):
// A[m = o][kk = s] = dz[s][o], B[kk = s][n = k] = h[s][k].
__device__ __forceinline__ f32x4 weight_grad_tile(const uint16_t* dz, int ldz, const uint16_t* h, int ldh, int mt,
                                                  int nt, int lane) {
  bf16x4 A, Bm;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int s = 4 * (lane >> 4) + i;
    A[i] = (short)dz[s * ldz + 16 * mt + (lane & 15)];
    Bm[i] = (short)h[s * ldh + 16 * nt + (lane & 15)];
  }
  return mfma16(A, Bm, zero4());
}

__global__ __launch_bounds__(64 * MLP_WAVES) void k_mlp_grad(GradArgs a) {
  __shared__ uint16_t X[MLP_WAVES][TILE * NFEAT];
  __shared__ uint16_t H1[MLP_WAVES][TILE * NHID];
  __shared__ uint16_t H2[MLP_WAVES][TILE * NHID];
  __shared__ uint16_t H3[MLP_WAVES][TILE * NHID];
  __shared__ uint16_t DA[MLP_WAVES][TILE * NHID];
  __shared__ uint16_t DB[MLP_WAVES][TILE * NHID];
  __shared__ int64_t rowid[MLP_WAVES][TILE];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int tile = blockIdx.x * MLP_WAVES + wv;
  const int ntiles = (a.batch + TILE - 1) / TILE;
  const bool live = tile < ntiles;
  const uint16_t* P = a.w;
  float* G = a.partial + (size_t)(live ? tile : 0) * NPARAM;
  const float inv_b = 1.0f / (float)a.batch;

  // inputs
  if (live && lane < TILE) {
    const int j = tile * TILE + lane;
    int64_t r = -1;
    if (j < a.batch) {
      if (a.draw) {
        uint32_t c0 = (uint32_t)j, c1 = a.iter, c2 = TRAIN_BLOCK, c3 = 0;
        philox4x32_10(c0, c1, c2, c3, a.k0, a.k1);
        r = (int64_t)(c0 % (uint32_t)a.nrows);
      } else {
        r = j;
      }
    }
    rowid[wv][lane] = r;
#pragma unroll
    for (int k = 0; k < NFEAT; ++k) {
      const float f = r >= 0 ? a.rows[r * ROW + k] : a.norm[k];
      X[wv][lane * NFEAT + k] = f2bf((f - a.norm[k]) * a.norm[NFEAT + k]);
    }
  }
  __syncthreads();
  f32x4 y = zero4();
  if (live) {
    bf16x4 xb[2], h1[4], h2[4], h3[4];
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) xb[ks] = *(const bf16x4*)&X[wv][(lane & 15) * NFEAT + 16 * ks + 4 * (lane >> 4)];
    y = forward_tile(P, xb, h1, h2, h3, lane);
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
      store_tile_bf16(H1[wv], NHID, mt, lane, h1[mt]);
      store_tile_bf16(H2[wv], NHID, mt, lane, h2[mt]);
      store_tile_bf16(H3[wv], NHID, mt, lane, h3[mt]);
    }
    // loss and output gradient: projection p = y - sum_c lw_c y_c
    const int64_t r = rowid[wv][lane & 15];
    float t[4], lw[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int o = 4 * (lane >> 4) + i;
      const bool use = lane < 32 && r >= 0;
      t[i] = use ? a.rows[r * ROW + 32 + o] : 0.0f;
      lw[i] = use ? a.rows[r * ROW + 40 + o] : 0.0f;
    }
    float ly = 0.0f;
#pragma unroll
    for (int i = 0; i < 4; ++i) ly += lw[i] * y[i];
    ly += __shfl_xor(ly, 16);
    float g[4], sg = 0.0f, lsum = 0.0f;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const float res = (y[i] - ly) - t[i];
      lsum += lw[i] * res * res;
      g[i] = 2.0f * lw[i] * res * inv_b;
      sg += g[i];
    }
    sg += __shfl_xor(sg, 16);
    bf16x4 dz4;
#pragma unroll
    for (int i = 0; i < 4; ++i) dz4[i] = (short)f2bf(lane < 32 ? g[i] - lw[i] * sg : 0.0f);
    store_tile_bf16(DA[wv], NHID, 0, lane, dz4);     // output units 0..15 (8..15 zero)
    // tile loss: the sum over its lanes
    for (int off = 32; off >= 1; off >>= 1) lsum += __shfl_xor(lsum, off);
    if (lane == 0) a.loss_partial[tile] = lsum;
  }
  __syncthreads();
  // layer 4: dW4, db4, dz3 = (W4^T dz4) * [h3 > 0]
  if (live) {
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      const f32x4 d = weight_grad_tile(DA[wv], NHID, H3[wv], NHID, 0, nt, lane);
      if (lane < 32) {
#pragma unroll
        for (int i = 0; i < 4; ++i) G[OFF_W4 + (4 * (lane >> 4) + i) * NHID + 16 * nt + (lane & 15)] = d[i];
      }
    }
    if (lane < NOUT) {
      float sb = 0.0f;
      for (int s = 0; s < TILE; ++s) sb += bf2f(DA[wv][s * NHID + lane]);
      G[OFF_B4 + lane] = sb;
    }
    const bf16x4 bz = *(const bf16x4*)&DA[wv][(lane & 15) * NHID + 4 * (lane >> 4)];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
      const f32x4 dh = mfma16(load_wt(P + OFF_W4, NHID, NOUT, mt, 0, lane), bz, zero4());
      const bf16x4 hm = *(const bf16x4*)&H3[wv][(lane & 15) * NHID + 16 * mt + 4 * (lane >> 4)];
      bf16x4 dz;
#pragma unroll
      for (int i = 0; i < 4; ++i) dz[i] = (short)f2bf(bf2f((uint16_t)hm[i]) > 0.0f ? dh[i] : 0.0f);
      store_tile_bf16(DB[wv], NHID, mt, lane, dz);
    }
  }
  __syncthreads();
  // layers 3 and 2: dW, db, and the gradient of the layer below
#pragma unroll
  for (int layer = 3; layer >= 2; --layer) {
    const int offw = layer == 3 ? OFF_W3 : OFF_W2, offb = layer == 3 ? OFF_B3 : OFF_B2;
    uint16_t* dzc = layer == 3 ? DB[wv] : DA[wv];      // this layer's pre-activation gradient
    uint16_t* dzn = layer == 3 ? DA[wv] : DB[wv];      // the layer below's
    const uint16_t* hin = layer == 3 ? H2[wv] : H1[wv];
    if (live) {
#pragma unroll
      for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
          const f32x4 d = weight_grad_tile(dzc, NHID, hin, NHID, mt, nt, lane);
#pragma unroll
          for (int i = 0; i < 4; ++i) G[offw + (16 * mt + 4 * (lane >> 4) + i) * NHID + 16 * nt + (lane & 15)] = d[i];
        }
      {
        float sb = 0.0f;
        for (int s = 0; s < TILE; ++s) sb += bf2f(dzc[s * NHID + lane]);
        G[offb + lane] = sb;
      }
      bf16x4 bz[4];
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) bz[ks] = *(const bf16x4*)&dzc[(lane & 15) * NHID + 16 * ks + 4 * (lane >> 4)];
#pragma unroll
      for (int mt = 0; mt < 4; ++mt) {
        f32x4 dh = zero4();
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) dh = mfma16(load_wt(P + offw, NHID, NHID, mt, ks, lane), bz[ks], dh);
        const bf16x4 hm = *(const bf16x4*)&hin[(lane & 15) * NHID + 16 * mt + 4 * (lane >> 4)];
        bf16x4 dz;
#pragma unroll
        for (int i = 0; i < 4; ++i) dz[i] = (short)f2bf(bf2f((uint16_t)hm[i]) > 0.0f ? dh[i] : 0.0f);
        store_tile_bf16(dzn, NHID, mt, lane, dz);
      }
    }
    __syncthreads();
  }
  // layer 1: dW1, db1 (its pre-activation gradient is in DB)
  if (live) {
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
      for (int nt = 0; nt < 2; ++nt) {
        const f32x4 d = weight_grad_tile(DB[wv], NHID, X[wv], NFEAT, mt, nt, lane);
#pragma unroll
        for (int i = 0; i < 4; ++i) G[OFF_W1 + (16 * mt + 4 * (lane >> 4) + i) * NFEAT + 16 * nt + (lane & 15)] = d[i];
      }
    float sb = 0.0f;
    for (int s = 0; s < TILE; ++s) sb += bf2f(DB[wv][s * NHID + lane]);
    G[OFF_B1 + lane] = sb;
  }
}

struct AdamArgs {
  const float* partial;
  const float* loss_partial;
  int32_t ntiles;
  float inv_batch;
  float* loss_out;       // one float (may be null)
  float* grad_out;       // NPARAM (may be null)
  int32_t update;        // 1: Adam step on master and w
  float* master;
  float* m;
  float* v;
  uint16_t* w;
  float lr, b1, b2, eps, bc1, bc2;   // bc1 = 1 - b1^t, bc2 = 1 - b2^t
};

__global__ __launch_bounds__(256) void k_mlp_adam(AdamArgs a) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < NPARAM) {
    float g = 0.0f;
    for (int t = 0; t < a.ntiles; ++t) g += a.partial[(size_t)t * NPARAM + p];
    if (a.grad_out) a.grad_out[p] = g;
    if (a.update) {
      const float m = a.b1 * a.m[p] + (1.0f - a.b1) * g;
      const float v = a.b2 * a.v[p] + (1.0f - a.b2) * (g * g);
      a.m[p] = m;
      a.v[p] = v;
      const float mh = m / a.bc1, vh = v / a.bc2;
      const float th = a.master[p] - a.lr * mh / (sqrtf(vh) + a.eps);
      a.master[p] = th;
      a.w[p] = f2bf(th);
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0 && a.loss_out) {
    float s = 0.0f;
    for (int t = 0; t < a.ntiles; ++t) s += a.loss_partial[t];
    *a.loss_out = s * a.inv_batch;
  }
}

// Feature normalisation from training rows (those with nonzero loss
// weights): per feature (one block each) the mean, the inverse population
// standard deviation (1 if below 1e-12) and the range.
__global__ __launch_bounds__(256) void k_mlp_norm(const float* rows, int64_t nrows, float* norm) {
  __shared__ double red[3][256];
  __shared__ float rmin[256], rmax[256];
  const int k = blockIdx.x, t = threadIdx.x;
  auto used = [&](int64_t r) {
    float s = 0.0f;
#pragma unroll
    for (int q = 0; q < 8; ++q) s += rows[r * ROW + 40 + q];
    return s > 0.0f;
  };
  double cnt = 0.0, sum = 0.0;
  float lo = 3.0e38f, hi = -3.0e38f;
  for (int64_t r = t; r < nrows; r += blockDim.x) {
    if (!used(r)) continue;
    const float f = rows[r * ROW + k];
    cnt += 1.0;
    sum += (double)f;
    lo = fminf(lo, f);
    hi = fmaxf(hi, f);
  }
  red[0][t] = cnt;
  red[1][t] = sum;
  rmin[t] = lo;
  rmax[t] = hi;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (t < h) {
      red[0][t] += red[0][t + h];
      red[1][t] += red[1][t + h];
      rmin[t] = fminf(rmin[t], rmin[t + h]);
      rmax[t] = fmaxf(rmax[t], rmax[t + h]);
    }
    __syncthreads();
  }
  const double n = red[0][0];
  const double mean = n > 0.0 ? red[1][0] / n : 0.0;
  __syncthreads();
  double ss = 0.0;
  for (int64_t r = t; r < nrows; r += blockDim.x) {
    if (!used(r)) continue;
    const double d = (double)rows[r * ROW + k] - mean;
    ss += d * d;
  }
  red[2][t] = ss;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (t < h) red[2][t] += red[2][t + h];
    __syncthreads();
  }
  if (t == 0) {
    const double sd = n > 0.0 ? sqrt(red[2][0] / n) : 0.0;
    norm[k] = (float)mean;
    norm[NFEAT + k] = sd > 1e-12 ? (float)(1.0 / sd) : 1.0f;
    norm[2 * NFEAT + k] = n > 0.0 ? rmin[0] : 0.0f;
    norm[3 * NFEAT + k] = n > 0.0 ? rmax[0] : 0.0f;
  }
}

__global__ void k_mlp_to_bf16(const float* master, uint16_t* w, int n) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < n) w[p] = f2bf(master[p]);
}

// ---------------------------------------------------------------------------
// training rows from a many-particle state: one wavefront per element cell

template <typename T> struct DatasetArgs {
  StateDev<T> buf[2];
  const Ctl* ctl;
  uint32_t parity;        // step parity; with the repack flip it selects the current buffer
  const int32_t* start;
  const int32_t* cap;
  const int32_t* ns;
  const int32_t* nm;
  int32_t ne, ncell;
  int32_t target;
  uint32_t k0, k1, draw;
  float* rows;           // ncell x 64 (out)
};

template <typename T> __global__ __launch_bounds__(256) void k_mlp_dataset(DatasetArgs<T> a) {
  const int lane = lane_id();
  const int cell = blockIdx.x * WAVES_PER_BLOCK + (int)(threadIdx.x / WAVE);
  if (cell >= a.ncell) return;
  const int ens = cell / a.ne;
  const StateDev<T> src = a.buf[a.parity ^ (a.ctl->flip & 1u)];
  const int capc = a.cap[cell], s0 = a.start[cell];
  const int ns = min(a.ns[cell], capc);
  const int nm = min(a.nm[cell], capc - ns);
  const int n = ns + nm;
  float* row = a.rows + (size_t)cell * ROW;
  const double p = n > 0 ? (double)a.target / (double)n : 0.0;
  auto selected = [&](uint32_t id) {
    uint32_t c0 = id, c1 = a.draw, c2 = SUB_BLOCK, c3 = (uint32_t)ens;
    philox4x32_10(c0, c1, c2, c3, a.k0, a.k1);
    return uniform01<double>(c0) < p;
  };
  // subsample means
  double cnt = 0.0, s[4] = {0.0, 0.0, 0.0, 0.0}, sall = 0.0;
  for (int j = lane; j < n; j += WAVE) {
    const int sl = slot_of(j, s0, ns, nm, capc);
    const double psi = (double)src.psi[sl];
    sall += psi;
    if (selected(src.id[sl])) {
      cnt += 1.0;
      s[0] += (double)src.u[sl];
      s[1] += (double)src.v[sl];
      s[2] += (double)src.w[sl];
      s[3] += psi;
    }
  }
  cnt = group_sum<WAVE>(cnt);
  sall = group_sum<WAVE>(sall);
  double mean[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) mean[q] = cnt > 0.0 ? group_sum<WAVE>(s[q]) / cnt : 0.0;
  // central second moments and bins of the subsample; bins of the whole cell
  double m2[10], bs[8], ba[8];
  int nb[8], na[8];
#pragma unroll
  for (int q = 0; q < 10; ++q) m2[q] = 0.0;
#pragma unroll
  for (int q = 0; q < 8; ++q) { bs[q] = 0.0; ba[q] = 0.0; nb[q] = 0; na[q] = 0; }
  for (int base = 0; base < n; base += WAVE) {
    const int j = base + lane;
    int bsel = -1, ball = -1;
    if (j < n) {
      const int sl = slot_of(j, s0, ns, nm, capc);
      const double val[4] = {(double)src.u[sl], (double)src.v[sl], (double)src.w[sl], (double)src.psi[sl]};
      ball = (val[0] > mean[0] ? 1 : 0) + (val[1] > mean[1] ? 2 : 0) + (val[2] > mean[2] ? 4 : 0);
#pragma unroll
      for (int q = 0; q < 8; ++q) ba[q] += ball == q ? val[3] : 0.0;
      if (selected(src.id[sl])) {
        bsel = ball;
        double d[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) d[q] = val[q] - mean[q];
#pragma unroll
        for (int x = 0; x < 4; ++x)
#pragma unroll
          for (int y = x; y < 4; ++y) m2[pair_index(x, y)] += d[x] * d[y];
#pragma unroll
        for (int q = 0; q < 8; ++q) bs[q] += bsel == q ? val[3] : 0.0;
      }
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      nb[q] += (int)__popcll(__ballot(bsel == q));
      na[q] += (int)__popcll(__ballot(ball == q));
    }
  }
#pragma unroll
  for (int q = 0; q < 10; ++q) m2[q] = group_sum<WAVE>(m2[q]);
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    bs[q] = group_sum<WAVE>(bs[q]);
    ba[q] = group_sum<WAVE>(ba[q]);
  }
  if (lane != 0) return;
  if (cnt == 0.0) {
    for (int k = 0; k < ROW; ++k) row[k] = 0.0f;
    return;
  }
  double rec[NSTAT2];
  rec[ST_N] = cnt;
#pragma unroll
  for (int q = 0; q < 4; ++q) rec[ST_MEAN + q] = mean[q];
#pragma unroll
  for (int q = 0; q < 10; ++q) rec[ST_M2 + q] = m2[q] / cnt;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    rec[ST_BINN + q] = (double)nb[q];
    rec[ST_BINM + q] = nb[q] > 0 ? bs[q] / (double)nb[q] : mean[3];
  }
  float f[NFEAT];
  features_of(rec, f);
  for (int k = 0; k < NFEAT; ++k) row[k] = f[k];
  const double mall = sall / (double)n;
  const double sig = sqrt(fmax(rec[ST_M2 + 9], 0.0));
  const bool train = cnt >= 2.0 && sig > SIGMA_MIN;
  for (int q = 0; q < 8; ++q) {
    const double mref = na[q] > 0 ? ba[q] / (double)na[q] : mall;
    const double t = train ? fmin(fmax((mref - mean[3]) / sig, -T_CLIP), T_CLIP) : 0.0;
    row[32 + q] = (float)t;
    row[40 + q] = train ? (float)((double)nb[q] / cnt) : 0.0f;
    row[48 + q] = (float)mref;
    row[56 + q] = (float)na[q];
  }
}

}  // namespace mlp
}  // namespace pdf
