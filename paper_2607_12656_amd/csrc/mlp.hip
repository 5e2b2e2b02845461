// Learned rate estimator: a per-Gaussian MLP 64 -> 128 -> 128 -> 1 on the
// BF16 matrix cores (FP32 accumulation), standing beside the range-based
// rate proxy (paper Sec. 3.3.1) as an estimate of the bits of the paper's
// channel-wise fixed-length coder (Sec. 3.4.1).
//
// Formulation.  Every layer is computed transposed, H_out^T = W^T H_in^T,
// with v_mfma_f32_32x32x16_bf16 (CDNA4): A = 32 rows of W^T (a pre-swizzled
// BF16 fragment per lane, staged in LDS), B = 16 x 32 slice of H_in^T, D =
// 32 x 32 tile of H_out^T.  In the accumulator layout lane l holds batch
// column l%32 and output rows 8(i/4) + 4(l/32) + i%4 (i = 0..15).  A k-step
// of 16 takes, in lane half h = l/32, the rows 16p + 4h + 0..3 and
// 16p + 8 + 4h + 0..3, i.e. accumulator elements 8p .. 8p + 7 of the lane:
// the contraction only needs A and B to agree on which row each of the 16
// k slots holds, and the weight fragments are packed in the same order, so
// activations never leave registers between layers.  The same holds for the
// backward to the inputs (dH1^T = W2 dZ2^T, dX^T = W1 dZ1^T).  Weight
// gradients (training) are split-K GEMMs over the batch on transposed
// activations written by the row kernel.
#include <mutex>

#include "sgs_internal.h"

namespace {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef short bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16v8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int MI = 64, MH = 128;
constexpr int kOffW1 = 0, kOffB1 = MI * MH, kOffW2 = kOffB1 + MH, kOffB2 = kOffW2 + MH * MH,
              kOffW3 = kOffB2 + MH, kOffB3 = kOffW3 + MH, kParams = kOffB3 + 1;
static_assert(kParams == SGS_MLP_PARAMS, "parameter count");
// packed fragment arrays, counted in bf16x4 (two per lane and k-step of 16:
// [t][p][lane][half], half = the two groups of four rows of k-step p)
constexpr int kF1 = 4 * 8 * 64;    // W1^T tiles  [t out 4][p in 4][lane][2]
constexpr int kF2 = 4 * 16 * 64;   // W2^T tiles  [t out 4][p in 8][lane][2]
constexpr int kF2B = 4 * 16 * 64;  // W2 tiles    [t in 4][p out 8][lane][2]
constexpr int kF1B = 2 * 16 * 64;  // W1 tiles    [t in 2][p out 8][lane][2]
constexpr int kPacked = kF1 + kF2 + kF2B + kF1B;
static_assert(kPacked * 8 == SGS_MLP_PACKED_BYTES, "packed size");

// FP32 -> BF16, round to nearest even (the hardware conversion)
__device__ __forceinline__ uint16_t f2bf(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
__device__ __forceinline__ float rbf(float f) { return bf2f(f2bf(f)); }
typedef __bf16 bf16v4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ bf16x4 pack4(float a, float b, float c, float d) {
  const f32x4 v = {a, b, c, d};
  return __builtin_bit_cast(bf16x4, __builtin_convertvector(v, bf16v4));
}
// One k-step of 16: A fragment a, B fragments b0 (rows 16p + 4h + 0..3) and
// b1 (rows 16p + 8 + 4h + 0..3).
__device__ __forceinline__ f32x16 mfma(bf16x8 a, bf16x4 b0, bf16x4 b1, f32x16 c) {
  const bf16x8 b = __builtin_shufflevector(b0, b1, 0, 1, 2, 3, 4, 5, 6, 7);
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16v8, a),
                                                 __builtin_bit_cast(bf16v8, b), c, 0, 0, 0);
}
__device__ __forceinline__ f32x16 mfma(bf16x8 a, bf16x8 b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16v8, a),
                                                 __builtin_bit_cast(bf16v8, b), c, 0, 0, 0);
}
// 32-row tile t of a bias vector in the accumulator layout of lane l
__device__ __forceinline__ f32x16 bias16(const float *b, int t, int lane);
__device__ __forceinline__ f32x16 zero16() {
  f32x16 z;
#pragma unroll
  for (int i = 0; i < 16; ++i) z[i] = 0.0f;
  return z;
}
// output row of accumulator element i for lane l, within a 32-row tile
__device__ __forceinline__ int drow(int i, int lane) { return 8 * (i >> 2) + 4 * (lane >> 5) + (i & 3); }
__device__ __forceinline__ f32x16 bias16(const float *b, int t, int lane) {
  f32x16 z;
#pragma unroll
  for (int i = 0; i < 16; ++i) z[i] = b[32 * t + drow(i, lane)];
  return z;
}

// fp32 master weights -> BF16 fragments
__global__ void k_mlp_pack(const float *__restrict__ th, bf16x4 *__restrict__ out) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= kPacked) return;
  const float *W1 = th + kOffW1, *W2 = th + kOffW2;
  // e = ((t * P + p) * 64 + lane) * 2 + half, k-step of 8 s = 2p + half
  int r = e, lane, s, t;
  float v[4];
  if (r < kF1) {
    lane = (r >> 1) & 63; s = 2 * ((r >> 7) & 3) + (r & 1); t = r >> 9;
    for (int j = 0; j < 4; ++j) v[j] = W1[(8 * s + 4 * (lane >> 5) + j) * MH + 32 * t + (lane & 31)];
  } else if ((r -= kF1) < kF2) {
    lane = (r >> 1) & 63; s = 2 * ((r >> 7) & 7) + (r & 1); t = r >> 10;
    for (int j = 0; j < 4; ++j) v[j] = W2[(8 * s + 4 * (lane >> 5) + j) * MH + 32 * t + (lane & 31)];
  } else if ((r -= kF2) < kF2B) {
    lane = (r >> 1) & 63; s = 2 * ((r >> 7) & 7) + (r & 1); t = r >> 10;
    for (int j = 0; j < 4; ++j) v[j] = W2[(32 * t + (lane & 31)) * MH + 8 * s + 4 * (lane >> 5) + j];
  } else {
    r -= kF2B;
    lane = (r >> 1) & 63; s = 2 * ((r >> 7) & 7) + (r & 1); t = r >> 10;
    for (int j = 0; j < 4; ++j) v[j] = W1[(32 * t + (lane & 31)) * MH + 8 * s + 4 * (lane >> 5) + j];
  }
  out[e] = pack4(v[0], v[1], v[2], v[3]);
}

struct MlpLds {
  bf16x8 F1[4][4][64];
  bf16x8 F2[4][8][64];
  float b1[MH], b2[MH], w3[MH];
  float b3;
};
struct MlpLdsBwd {
  MlpLds f;
  bf16x8 F2B[4][8][64];
  bf16x8 F1B[2][8][64];
};

// Backward-only weights: W2 and W1 fragments and w3 (48.5 KB).
struct MlpLdsB {
  bf16x8 F2B[4][8][64];
  bf16x8 F1B[2][8][64];
  float w3[MH];
};
__device__ void load_lds_b(MlpLdsB &L, const bf16x4 *__restrict__ packed,
                           const float *__restrict__ th) {
  bf16x4 *d = (bf16x4 *)&L.F2B[0][0][0];
  for (int e = threadIdx.x; e < kF2B + kF1B; e += blockDim.x) d[e] = packed[kF1 + kF2 + e];
  for (int k = threadIdx.x; k < MH; k += blockDim.x) L.w3[k] = rbf(th[kOffW3 + k]);
}

__device__ void load_lds(MlpLds &L, const bf16x4 *__restrict__ packed, const float *__restrict__ th) {
  bf16x4 *d1 = (bf16x4 *)&L.F1[0][0][0];
  for (int e = threadIdx.x; e < kF1 + kF2; e += blockDim.x) d1[e] = packed[e];  // F1 then F2
  for (int k = threadIdx.x; k < MH; k += blockDim.x) {
    L.b1[k] = th[kOffB1 + k];
    L.b2[k] = th[kOffB2 + k];
    L.w3[k] = rbf(th[kOffW3 + k]);
  }
  if (threadIdx.x == 0) L.b3 = th[kOffB3];
}
__device__ void load_lds_bwd(MlpLdsBwd &L, const bf16x4 *__restrict__ packed,
                             const float *__restrict__ th) {
  load_lds(L.f, packed, th);
  bf16x4 *d = (bf16x4 *)&L.F2B[0][0][0];
  for (int e = threadIdx.x; e < kF2B + kF1B; e += blockDim.x) d[e] = packed[kF1 + kF2 + e];
}

// Forward of one 32-row tile held by a wave.  xb[s]: B fragments of X^T.
// Leaves pre-activations (with bias) in z1, z2; returns f for row lane%32.
__device__ __forceinline__ float tile_fwd(const MlpLds &L, const bf16x4 xb[8], int lane,
                                          f32x16 z1[4], f32x16 z2[4], bf16x4 hb[16]) {
#pragma unroll
  for (int t = 0; t < 4; ++t) z1[t] = bias16(L.b1, t, lane);  // the sums start at the bias
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int t = 0; t < 4; ++t) z1[t] = mfma(L.F1[t][p][lane], xb[2 * p], xb[2 * p + 1], z1[t]);
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      float h[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        h[j] = fmaxf(z1[t][4 * g + j], 0.0f);
      }
      hb[4 * t + g] = pack4(h[0], h[1], h[2], h[3]);
    }
#pragma unroll
  for (int t = 0; t < 4; ++t) z2[t] = bias16(L.b2, t, lane);
#pragma unroll
  for (int p = 0; p < 8; ++p)
#pragma unroll
    for (int t = 0; t < 4; ++t) z2[t] = mfma(L.F2[t][p][lane], hb[2 * p], hb[2 * p + 1], z2[t]);
  float p = 0.0f;
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int o = 32 * t + drow(i, lane);
      p = fmaf(fmaxf(z2[t][i], 0.0f), L.w3[o], p);
    }
  p += __shfl_xor(p, 32, 64);
  return p + L.b3;
}

// The same forward keeping only the signs of the pre-activations: bit
// 16t + i of m1 / m2 is [z > 0] of accumulator element i of output tile t of
// layer 1 / 2, which is all the backward needs of them.  One set of
// accumulators serves both layers, so the wave holds 64 instead of 128.
__device__ __forceinline__ float tile_fwd_masks(const MlpLds &L, const bf16x4 xb[8], int lane,
                                                uint64_t &m1, uint64_t &m2) {
  f32x16 z[4];
  bf16x4 hb[16];
#pragma unroll
  for (int t = 0; t < 4; ++t) z[t] = bias16(L.b1, t, lane);  // the sums start at the bias
#pragma unroll
  for (int p = 0; p < 4; ++p) {
#pragma unroll
    for (int t = 0; t < 4; ++t) z[t] = mfma(L.F1[t][p][lane], xb[2 * p], xb[2 * p + 1], z[t]);
    // bound the fragments the compiler reads ahead (registers)
    if ((p & 1) == 1) __asm__ volatile("" ::: "memory");
  }
  uint32_t mw[2] = {0u, 0u};  // the two 32-bit halves of m1
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      float h[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int i = 4 * g + j;
        const float zz = z[t][i];
        mw[t >> 1] |= zz > 0.0f ? 1u << (16 * (t & 1) + i) : 0u;
        h[j] = fmaxf(zz, 0.0f);
      }
      hb[4 * t + g] = pack4(h[0], h[1], h[2], h[3]);
    }
  m1 = (uint64_t)mw[0] | ((uint64_t)mw[1] << 32);
#pragma unroll
  for (int t = 0; t < 4; ++t) z[t] = bias16(L.b2, t, lane);
#pragma unroll
  for (int p = 0; p < 8; ++p) {
#pragma unroll
    for (int t = 0; t < 4; ++t) z[t] = mfma(L.F2[t][p][lane], hb[2 * p], hb[2 * p + 1], z[t]);
    // bound the fragments the compiler reads ahead (registers)
    if ((p & 1) == 1) __asm__ volatile("" ::: "memory");
  }
  float p = 0.0f;
  uint32_t nw[2] = {0u, 0u};  // the two 32-bit halves of m2
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int o = 32 * t + drow(i, lane);
      const float zz = z[t][i];
      nw[t >> 1] |= zz > 0.0f ? 1u << (16 * (t & 1) + i) : 0u;
      p = fmaf(fmaxf(zz, 0.0f), L.w3[o], p);
    }
  m2 = (uint64_t)nw[0] | ((uint64_t)nw[1] << 32);
  p += __shfl_xor(p, 32, 64);
  return p + L.b3;
}

// Features of the lane's row for all eight k-steps: x = log2(1 + u),
// u = (y - m) / q for channel 8s + 4(l/32) + jj.  The reciprocal steps rq
// and the minima come from LDS; rows past n and the padding channels are
// zero.
__device__ __forceinline__ void features(const float *__restrict__ y, int64_t npad, int64_t r,
                                         bool valid, const float *s_rq, const float *s_min,
                                         int lane, bf16x4 xb[8]) {
  // all 32 loads first, branch-free (rows past n and padding channels read
  // entry 0 of channel 0 and are dropped), then the arithmetic
  const int64_t rr = valid ? r : 0;
  float yv[8][4];
#pragma unroll
  for (int s = 0; s < 8; ++s)
#pragma unroll
    for (int jj = 0; jj < 4; ++jj) {
      const int j = 8 * s + 4 * (lane >> 5) + jj;
      yv[s][jj] = y[(j < SGS_NCH ? j : 0) * npad + rr];
    }
#pragma unroll
  for (int s = 0; s < 8; ++s) {
    float v[4];
#pragma unroll
    for (int jj = 0; jj < 4; ++jj) {
      const int j = 8 * s + 4 * (lane >> 5) + jj;
      const int jc = j < SGS_NCH ? j : 0;
      const float uu = (valid && j < SGS_NCH) ? (yv[s][jj] - s_min[jc]) * s_rq[jc] : 0.0f;
      v[jj] = __log2f(1.0f + uu);
    }
    xb[s] = pack4(v[0], v[1], v[2], v[3]);
  }
}

__device__ __forceinline__ void load_mins(float *s_min, const uint64_t *__restrict__ stats) {
  for (int j = threadIdx.x; j < SGS_NCH; j += blockDim.x)
    s_min[j] = sgs_unord((uint32_t)(stats[j] >> 32));
}

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;

__device__ __forceinline__ void load_steps(float *s_rq, const float *__restrict__ q) {
  for (int j = threadIdx.x; j < SGS_NCH; j += blockDim.x) s_rq[j] = 1.0f / q[j];
}

// In-loop forward: R partials = sum_r M_r f(x_r) per block (FP64), f optional.
// Keeps f and the activation signs for the backward.
__global__ void __launch_bounds__(kThreads, 2)
k_mlp_rate_fwd(int64_t n, int64_t npad, const bf16x4 *__restrict__ packed,
               const float *__restrict__ th, const float *__restrict__ y,
               const float *__restrict__ q, const uint64_t *__restrict__ stats,
               const uint8_t *__restrict__ hard, float *__restrict__ fout,
               float *__restrict__ fsave, uint4 *__restrict__ signs,
               double *__restrict__ partial) {
  __shared__ MlpLds L;
  __shared__ float s_min[SGS_NCH], s_rq[SGS_NCH];
  __shared__ double s_red[kWaves];
  load_lds(L, packed, th);
  load_mins(s_min, stats);
  load_steps(s_rq, q);
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t ntiles = (n + 31) / 32;
  double acc = 0.0;
  for (int64_t tile = (int64_t)blockIdx.x * kWaves + wave; tile < ntiles;
       tile += (int64_t)gridDim.x * kWaves) {
    // keep the weight fragments in LDS: without this the loop-invariant
    // fragment reads are hoisted into ~200 registers and the kernel spills
    __asm__ volatile("" ::: "memory");
    const int64_t r = tile * 32 + (lane & 31);
    const bool valid = r < n;
    bf16x4 xb[8];
    features(y, npad, r, valid, s_rq, s_min, lane, xb);
    uint64_t m1, m2;
    const float f = tile_fwd_masks(L, xb, lane, m1, m2);
    if (valid) {
      // what the backward needs of this forward: f and the activation signs
      signs[2 * r + (lane >> 5)] =
          make_uint4((uint32_t)m1, (uint32_t)(m1 >> 32), (uint32_t)m2, (uint32_t)(m2 >> 32));
      if (lane < 32) {
        fsave[r] = f;
        if (fout) fout[r] = f;
        if (hard[r]) acc += (double)f;
      }
    }
  }
  acc = sgs_wave_sum_d(acc);
  if (lane == 0) s_red[wave] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < kWaves; ++w) t += s_red[w];
    partial[blockIdx.x] = t;
  }
}

__global__ void k_mlp_rate_finish(int nb, const double *__restrict__ partial, int64_t n_hat,
                                  float *__restrict__ outR) {
  __shared__ double s_w[kWaves];
  double t = 0.0;
  for (int b = threadIdx.x; b < nb; b += blockDim.x) t += partial[b];
  t = sgs_wave_sum_d(t);
  if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = t;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < (int)(blockDim.x / 64); ++w) s += s_w[w];
    outR[0] = (float)(s / (double)n_hat);
  }
}

// In-loop backward of weight * R, R = (1/N_hat) sum_r M_r f(x_r), through the
// MLP to the features, then to the raw parameters and the steps (channel
// minima held fixed); dR/dM_r = f_r / N_hat.  Uses f and the activation
// signs the forward kept (no forward recompute, so only the backward
// weights sit in LDS).  Adds into grad_params, per-block step partials,
// grad_score (mask mode 1) / grad_hard_mask.
// One wave per SIMD: its 344 registers (VGPRs and AGPRs) fit without
// spilling; at two waves it spilled 160 bytes per lane and took 1.3x longer.
__global__ void __launch_bounds__(kThreads, 1)
k_mlp_rate_bwd(int64_t n, int64_t npad, int64_t n_hat, float weight, float tau, int mode,
               const bf16x4 *__restrict__ packed, const float *__restrict__ th,
               const float *__restrict__ y, const float *__restrict__ q,
               const uint64_t *__restrict__ stats, const uint8_t *__restrict__ hard,
               const float *__restrict__ soft, const float *__restrict__ fsave,
               const uint4 *__restrict__ signs, float *__restrict__ gparams,
               float *__restrict__ gscore, float *__restrict__ gmask,
               double *__restrict__ qpartial, int sh_rows) {
  __shared__ MlpLdsB L;
  __shared__ float s_min[SGS_NCH];
  __shared__ float s_rq[SGS_NCH];
  __shared__ double s_gq[kWaves][64];
  load_lds_b(L, packed, th);
  load_mins(s_min, stats);
  load_steps(s_rq, q);
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const float inv_ln2 = 1.4426950408889634f;
  const float cscale = weight / (float)n_hat;
  float gq[32];
#pragma unroll
  for (int k = 0; k < 32; ++k) gq[k] = 0.0f;
  const int64_t ntiles = (n + 31) / 32;
  const int64_t stride = (int64_t)gridDim.x * kWaves;
  // a tile's per-row inputs, loaded one tile ahead (software pipelining: the
  // wave is alone on its SIMD, so nothing else hides their latency)
  struct RowIn {
    uint4 sg;
    float fs, gm, sm, gs;
    bool m;
  };
  auto row_in = [&](int64_t t) {
    RowIn o;
    const int64_t rr = t * 32 + (lane & 31);
    const bool ok = t < ntiles && rr < n;
    o.m = ok && hard[rr];
    o.sg = ok ? signs[2 * rr + (lane >> 5)] : make_uint4(0u, 0u, 0u, 0u);
    const bool own = ok && lane < 32;  // one lane per row writes its mask gradient
    o.fs = own ? fsave[rr] : 0.0f;
    o.gm = own && gmask ? gmask[rr] : 0.0f;
    o.sm = own && mode == 1 && gscore ? soft[rr] : 0.0f;
    o.gs = own && mode == 1 && gscore ? gscore[rr] : 0.0f;
    return o;
  };
  RowIn nxt = row_in((int64_t)blockIdx.x * kWaves + wave);
  for (int64_t tile = (int64_t)blockIdx.x * kWaves + wave; tile < ntiles; tile += stride) {
    // keep the weight fragments in LDS: without this the loop-invariant
    // fragment reads are hoisted into registers and the kernel spills
    __asm__ volatile("" ::: "memory");
    const int64_t r = tile * 32 + (lane & 31);
    const bool valid = r < n;
    const RowIn in = nxt;
    const bool m = in.m;
    const uint4 sg = in.sg;
    // mask gradient
    if (valid && lane < 32) {
      const float gmv = cscale * in.fs;
      if (gmask) gmask[r] = in.gm + gmv;
      if (mode == 1 && gscore) gscore[r] = in.gs + gmv * in.sm * (1.0f - in.sm) / tau;
    }
    const uint64_t m1 = (uint64_t)sg.x | ((uint64_t)sg.y << 32);
    const uint64_t m2 = (uint64_t)sg.z | ((uint64_t)sg.w << 32);
    // this tile's parameter rows and gradient rows for the chain to y and q
    // below, loaded ahead of the MFMA section so that their latency overlaps
    // it (accumulator element (t, i) is channel 32t + drow(i, lane))
    float yv[2][16], old[2][16];
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const int j = 32 * t + drow(i, lane);
        const bool ok = valid && j < SGS_NCH;
        const bool row = ok && (sh_rows || j < SGS_CH_REST || j >= SGS_CH_REST_END);
        yv[t][i] = ok ? y[j * npad + r] : 0.0f;
        old[t][i] = row ? gparams[j * npad + r] : 0.0f;
      }
    nxt = row_in(tile + stride);
    if (__ballot(m) == 0ull) continue;
    const float c = m ? cscale : 0.0f;
    // dz2 = c w3 [z2 > 0]  (BF16, B operand layout)
    bf16x4 dzb[16];
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        float v[4];
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) {
          const int i = 4 * g + jj;
          v[jj] = (m2 >> (16 * t + i)) & 1ull ? c * L.w3[32 * t + drow(i, lane)] : 0.0f;
        }
        dzb[4 * t + g] = pack4(v[0], v[1], v[2], v[3]);
      }
    // dh1^T = W2 dZ2^T, dz1 = dh1 [z1 > 0], dX^T = W1 dZ1^T, by halves of the
    // 128 hidden units (fewer live accumulators)
    f32x16 dx[2];
    dx[0] = zero16();
    dx[1] = zero16();
#pragma unroll
    for (int half = 0; half < 2; ++half) {
      f32x16 dh[2];
      dh[0] = zero16();
      dh[1] = zero16();
#pragma unroll
      for (int p = 0; p < 8; ++p) {
#pragma unroll
        for (int tt = 0; tt < 2; ++tt)
          dh[tt] = mfma(L.F2B[2 * half + tt][p][lane], dzb[2 * p], dzb[2 * p + 1], dh[tt]);
        if ((p & 1) == 1) __asm__ volatile("" ::: "memory");
      }
      bf16x4 d1b[8];
#pragma unroll
      for (int tt = 0; tt < 2; ++tt)
#pragma unroll
        for (int g = 0; g < 4; ++g) {
          const int t = 2 * half + tt;
          float v[4];
#pragma unroll
          for (int jj = 0; jj < 4; ++jj) {
            const int i = 4 * g + jj;
            v[jj] = (m1 >> (16 * t + i)) & 1ull ? dh[tt][i] : 0.0f;
          }
          d1b[4 * tt + g] = pack4(v[0], v[1], v[2], v[3]);
        }
#pragma unroll
      for (int p = 0; p < 4; ++p) {
        dx[0] = mfma(L.F1B[0][4 * half + p][lane], d1b[2 * p], d1b[2 * p + 1], dx[0]);
        dx[1] = mfma(L.F1B[1][4 * half + p][lane], d1b[2 * p], d1b[2 * p + 1], dx[1]);
      }
    }
    // chain to y and q: x = log2(1 + u), u = (y - m) / q
    if (valid) {
#pragma unroll
      for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int i = 0; i < 16; ++i) {
          const int j = 32 * t + drow(i, lane);
          if (t == 0 || j < SGS_NCH) {
            const float uu = (yv[t][i] - s_min[j]) * s_rq[j];
            const float gp = dx[t][i] * __builtin_amdgcn_rcpf(1.0f + uu) * inv_ln2 * s_rq[j];
            if (sh_rows || j < SGS_CH_REST || j >= SGS_CH_REST_END)
              gparams[j * npad + r] = old[t][i] + gp;
            gq[16 * t + i] -= gp * uu;
          }
        }
    }
  }
  // reduce the step gradient: lanes sharing lane>>5 hold the same channels
#pragma unroll
  for (int k = 0; k < 32; ++k) {
    float v = gq[k];
#pragma unroll
    for (int o = 16; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    gq[k] = v;
  }
  if ((lane & 31) == 0) {
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int i = 0; i < 16; ++i) s_gq[wave][32 * t + drow(i, lane)] = (double)gq[16 * t + i];
  }
  __syncthreads();
  if (threadIdx.x < 64) {
    double s = 0.0;
    for (int w = 0; w < kWaves; ++w) s += s_gq[w][threadIdx.x];
    qpartial[(int64_t)blockIdx.x * 64 + threadIdx.x] = s;
  }
}

// Block j: channel j's step gradient, the per-block partials summed by
// strided threads, then wave and block sums (fixed order).
__global__ void __launch_bounds__(256)
k_mlp_q_finish(int nb, const double *__restrict__ qpartial, float *__restrict__ gqstep) {
  __shared__ double s_w[4];
  const int j = blockIdx.x;
  double s = 0.0;
  for (int b = threadIdx.x; b < nb; b += 256) s += qpartial[(int64_t)b * 64 + j];
  s = sgs_wave_sum_d(s);
  if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) gqstep[j] += (float)(((s_w[0] + s_w[1]) + s_w[2]) + s_w[3]);
}

// Inference over given feature rows X [B][64] (BF16) -> f [B].  Three
// workgroups per compute unit (50 KB of LDS and at most 168 registers each).
__global__ void __launch_bounds__(kThreads, 3)
k_mlp_infer(int64_t B, const bf16x4 *__restrict__ packed, const float *__restrict__ th,
            const uint16_t *__restrict__ X, float *__restrict__ fout) {
  __shared__ MlpLds L;
  load_lds(L, packed, th);
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t ntiles = (B + 31) / 32;
  for (int64_t tile = (int64_t)blockIdx.x * kWaves + wave; tile < ntiles;
       tile += (int64_t)gridDim.x * kWaves) {
    // keep the weight fragments in LDS: without this the loop-invariant
    // fragment reads are hoisted into ~200 registers and the kernel spills
    __asm__ volatile("" ::: "memory");
    const int64_t r = tile * 32 + (lane & 31);
    const bool valid = r < B;
    bf16x4 xb[8];
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      if (valid) {
        xb[s] = *(const bf16x4 *)(X + r * MI + 8 * s + 4 * (lane >> 5));
      } else {
        xb[s] = pack4(0.f, 0.f, 0.f, 0.f);
      }
    }
    uint64_t m1, m2;
    const float f = tile_fwd_masks(L, xb, lane, m1, m2);
    if (valid && lane < 32) fout[r] = f;
  }
}

// Training, pass 1 (per row): forward, loss, df = scale (f - t), dz2, dz1;
// writes the transposed operands of the weight-gradient GEMMs.
__global__ void __launch_bounds__(kThreads)
k_mlp_train_rows(int64_t B, float scale, const bf16x4 *__restrict__ packed,
                 const float *__restrict__ th, const uint16_t *__restrict__ X,
                 const float *__restrict__ target, uint16_t *__restrict__ XT,
                 uint16_t *__restrict__ H1T, uint16_t *__restrict__ DZ2T,
                 uint16_t *__restrict__ DZ1T, float *__restrict__ H2T, float *__restrict__ df,
                 double *__restrict__ loss_partial) {
  __shared__ MlpLdsBwd L;
  __shared__ double s_red[kWaves];
  load_lds_bwd(L, packed, th);
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t ntiles = (B + 31) / 32;
  double lacc = 0.0;
  for (int64_t tile = (int64_t)blockIdx.x * kWaves + wave; tile < ntiles;
       tile += (int64_t)gridDim.x * kWaves) {
    // keep the weight fragments in LDS: without this the loop-invariant
    // fragment reads are hoisted into ~200 registers and the kernel spills
    __asm__ volatile("" ::: "memory");
    const int64_t r = tile * 32 + (lane & 31);
    const bool valid = r < B;
    bf16x4 xb[8];
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      if (valid) {
        xb[s] = *(const bf16x4 *)(X + r * MI + 8 * s + 4 * (lane >> 5));
#pragma unroll
        for (int j = 0; j < 4; ++j) XT[(int64_t)(8 * s + 4 * (lane >> 5) + j) * B + r] = (uint16_t)xb[s][j];
      } else {
        xb[s] = pack4(0.f, 0.f, 0.f, 0.f);
      }
    }
    f32x16 z1[4], z2[4];
    bf16x4 hb[16];
    const float f = tile_fwd(L.f, xb, lane, z1, z2, hb);
    float c = 0.0f;
    if (valid) {
      const float d = f - target[r];
      c = scale * d;
      if (lane < 32) {
        lacc += (double)d * (double)d;
        df[r] = c;
      }
    }
    bf16x4 dzb[16];
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        float v[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int i = 4 * g + j;
          const int o = 32 * t + drow(i, lane);
          v[j] = z2[t][i] > 0.0f ? c * L.f.w3[o] : 0.0f;
          if (valid) {
            H2T[(int64_t)o * B + r] = fmaxf(z2[t][i], 0.0f);
            H1T[(int64_t)o * B + r] = (uint16_t)hb[4 * t + g][j];
          }
        }
        dzb[4 * t + g] = pack4(v[0], v[1], v[2], v[3]);
        if (valid) {
#pragma unroll
          for (int j = 0; j < 4; ++j)
            DZ2T[(int64_t)(32 * t + drow(4 * g + j, lane)) * B + r] = (uint16_t)dzb[4 * t + g][j];
        }
      }
    f32x16 dh[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) dh[t] = zero16();
#pragma unroll
    for (int p = 0; p < 8; ++p)
#pragma unroll
      for (int t = 0; t < 4; ++t) dh[t] = mfma(L.F2B[t][p][lane], dzb[2 * p], dzb[2 * p + 1], dh[t]);
    if (valid) {
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int i = 0; i < 16; ++i) {
          const float v = z1[t][i] > 0.0f ? dh[t][i] : 0.0f;
          DZ1T[(int64_t)(32 * t + drow(i, lane)) * B + r] = f2bf(v);
        }
    }
  }
  lacc = sgs_wave_sum_d(lacc);
  if (lane == 0) s_red[wave] = lacc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < kWaves; ++w) t += s_red[w];
    loss_partial[blockIdx.x] = t;
  }
}

// Training, pass 2: split-K GEMMs over the batch.
//   dW2^T [128 out][128 in] = DZ2T [128][B] . H1 [B][128]
//   dW1^T [128 out][ 64 in] = DZ1T [128][B] . X  [B][64]
// Wave w owns output rows 32w..32w+31 of both (4 + 2 tiles of 32 x 32).
// Block b covers batch rows [b*chunk, (b+1)*chunk).  Partials [blocks][24][32][32].
__global__ void __launch_bounds__(kThreads)
k_mlp_wgrad(int64_t B, int64_t chunk, const uint16_t *__restrict__ XT,
            const uint16_t *__restrict__ H1T, const uint16_t *__restrict__ DZ2T,
            const uint16_t *__restrict__ DZ1T, float *__restrict__ partial) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  f32x16 acc[6];
#pragma unroll
  for (int k = 0; k < 6; ++k) acc[k] = zero16();
  const int64_t k0 = (int64_t)blockIdx.x * chunk;
  const int64_t k1 = min(B, k0 + chunk);
  const int row = 32 * wave + (lane & 31);
  for (int64_t kb = k0; kb < k1; kb += 16) {
    // lane half h takes batch rows kb + 8h .. kb + 8h + 7 of both operands
    const int64_t k = kb + 8 * (lane >> 5);
    bf16x8 a2, a1, bh[4], bx[2];
    if (k + 7 < k1) {
      a2 = *(const bf16x8 *)(DZ2T + (int64_t)row * B + k);
      a1 = *(const bf16x8 *)(DZ1T + (int64_t)row * B + k);
#pragma unroll
      for (int u = 0; u < 4; ++u) bh[u] = *(const bf16x8 *)(H1T + (int64_t)(32 * u + (lane & 31)) * B + k);
#pragma unroll
      for (int u = 0; u < 2; ++u) bx[u] = *(const bf16x8 *)(XT + (int64_t)(32 * u + (lane & 31)) * B + k);
    } else {
      // ragged tail: element-wise with zero fill
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const bool ok = k + j < k1;
        a2[j] = ok ? (short)DZ2T[(int64_t)row * B + k + j] : (short)0;
        a1[j] = ok ? (short)DZ1T[(int64_t)row * B + k + j] : (short)0;
#pragma unroll
        for (int u = 0; u < 4; ++u) bh[u][j] = ok ? (short)H1T[(int64_t)(32 * u + (lane & 31)) * B + k + j] : (short)0;
#pragma unroll
        for (int u = 0; u < 2; ++u) bx[u][j] = ok ? (short)XT[(int64_t)(32 * u + (lane & 31)) * B + k + j] : (short)0;
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) acc[u] = mfma(a2, bh[u], acc[u]);
#pragma unroll
    for (int u = 0; u < 2; ++u) acc[4 + u] = mfma(a1, bx[u], acc[4 + u]);
  }
  float *dst = partial + (int64_t)blockIdx.x * 24 * 1024;
#pragma unroll
  for (int u = 0; u < 6; ++u) {
    const int tileid = (u < 4) ? (wave * 4 + u) : (16 + wave * 2 + (u - 4));
#pragma unroll
    for (int i = 0; i < 16; ++i) dst[(int64_t)tileid * 1024 + drow(i, lane) * 32 + (lane & 31)] = acc[u][i];
  }
}

// Training, pass 3: fixed-order sums -> gradient of the flat parameter vector.
//   blocks [0, 768): one row of 32 entries of one of the 24 weight tiles;
//     thread (g, j) sums column j over the chunks of group g (eight groups
//     of consecutive chunks), then the eight group sums are added in order;
//   blocks [768, 768 + 385 kSeg): bias / w3 entries as sums over kSeg
//     segments of the batch (per-segment sums, added by k_mlp_bias_finish).
constexpr int kWRows = 24 * 32;
constexpr int kSeg = 8;
constexpr int64_t kLossParts = 1024;       // loss partials (one per row-kernel block)
constexpr int64_t kSegParts = 385 * kSeg;  // bias / w3 segment sums
__global__ void __launch_bounds__(kThreads)
k_mlp_grad_finish(int64_t B, int nchunks, const float *__restrict__ partial,
                  const uint16_t *__restrict__ DZ2T, const uint16_t *__restrict__ DZ1T,
                  const float *__restrict__ H2T, const float *__restrict__ df,
                  float *__restrict__ g, double *__restrict__ seg_part) {
  const int b = blockIdx.x;
  if (b < kWRows) {
    __shared__ double s_g[8][32];
    const int tile = b >> 5, i = b & 31;  // tile row i (out)
    const int j = threadIdx.x & 31, grp = threadIdx.x >> 5;
    const int per = (nchunks + 7) / 8;
    const int c0 = min(nchunks, grp * per), c1 = min(nchunks, c0 + per);
    const float *src = partial + (int64_t)tile * 1024 + i * 32 + j;
    double s = 0.0;
    // eight loads in flight per round, added in chunk order
    for (int c = c0; c < c1; c += 8) {
      float v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = c + u < c1 ? src[(int64_t)(c + u) * 24 * 1024] : 0.0f;
#pragma unroll
      for (int u = 0; u < 8; ++u) s += (double)v[u];
    }
    s_g[grp][j] = s;
    __syncthreads();
    if (grp == 0) {
      double t = 0.0;
#pragma unroll
      for (int k = 0; k < 8; ++k) t += s_g[k][j];
      if (tile < 16) {
        const int out = 32 * (tile >> 2) + i, in = 32 * (tile & 3) + j;
        g[kOffW2 + in * MH + out] = (float)t;
      } else {
        const int t2 = tile - 16;
        const int out = 32 * (t2 >> 1) + i, in = 32 * (t2 & 1) + j;
        g[kOffW1 + in * MH + out] = (float)t;
      }
    }
    return;
  }
  __shared__ double s_w[kThreads / 64];
  // bias / w3 entry k, segment seg of the batch rows
  const int k = (b - kWRows) / kSeg, seg = (b - kWRows) % kSeg;
  const int64_t per = (B + kSeg - 1) / kSeg;
  const int64_t ra = min(B, seg * per), rb = min(B, ra + per);
  // each thread adds rows ra + threadIdx.x + 256 m in ascending m, eight
  // loads in flight per round
  constexpr int U = 8;
  double s = 0.0;
  for (int64_t r0 = ra + threadIdx.x; r0 < rb; r0 += (int64_t)U * kThreads) {
    double v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t r = r0 + (int64_t)u * kThreads;
      const bool ok = r < rb;
      if (k < 128) v[u] = ok ? (double)bf2f(DZ1T[(int64_t)k * B + r]) : 0.0;
      else if (k < 256) v[u] = ok ? (double)bf2f(DZ2T[(int64_t)(k - 128) * B + r]) : 0.0;
      else if (k < 384) v[u] = ok ? (double)df[r] * (double)H2T[(int64_t)(k - 256) * B + r] : 0.0;
      else v[u] = ok ? (double)df[r] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) s += v[u];
  }
  s = sgs_wave_sum_d(s);
  if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < kThreads / 64; ++w) t += s_w[w];
    seg_part[k * kSeg + seg] = t;
  }
}

// Bias / w3 entries: the kSeg segment sums in order.
__global__ void k_mlp_bias_finish(const double *__restrict__ seg_part, float *__restrict__ g) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= 385) return;
  double t = 0.0;
#pragma unroll
  for (int q = 0; q < kSeg; ++q) t += seg_part[k * kSeg + q];
  if (k < 128) g[kOffB1 + k] = (float)t;
  else if (k < 256) g[kOffB2 + (k - 128)] = (float)t;
  else if (k < 384) g[kOffW3 + (k - 256)] = (float)t;
  else g[kOffB3] = (float)t;
}

// Mean squared error from the per-block partials: a strided sum per thread,
// then wave and block sums, all in a fixed order.
__global__ void __launch_bounds__(kThreads)
k_mlp_loss_finish(int nb, const double *__restrict__ partial, int64_t B, float *__restrict__ loss) {
  __shared__ double s_w[kThreads / 64];
  double s = 0.0;
  for (int b = threadIdx.x; b < nb; b += kThreads) s += partial[b];
  s = sgs_wave_sum_d(s);
  if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < kThreads / 64; ++w) t += s_w[w];
    loss[0] = (float)(t / (double)B);
  }
}

// Adam on the FP32 master parameters.
__global__ void k_adam(int count, float *__restrict__ w, float *__restrict__ m,
                       float *__restrict__ v, const float *__restrict__ g, float lr, float b1,
                       float b2, float eps, float c1, float c2) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= count) return;
  const float gk = g[k];
  const float mk = b1 * m[k] + (1.0f - b1) * gk;
  const float vk = b2 * v[k] + (1.0f - b2) * gk * gk;
  m[k] = mk;
  v[k] = vk;
  w[k] -= lr * (mk / c1) / (sqrtf(vk / c2) + eps);
}

// Feature rows of chosen Gaussians: X[r][j] = the in-loop forward's feature
// of Gaussian idx[r], channel j (0 for j >= 59, and a zero row for an index
// outside [0, n)): one thread per entry.
__global__ void __launch_bounds__(256)
k_mlp_features(int64_t rows, int64_t n, int64_t npad, const float *__restrict__ y,
               const float *__restrict__ q, const uint64_t *__restrict__ stats,
               const int32_t *__restrict__ idx, uint16_t *__restrict__ X) {
  __shared__ float s_min[SGS_NCH], s_rq[SGS_NCH];
  load_mins(s_min, stats);
  load_steps(s_rq, q);
  __syncthreads();
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= rows * 64) return;
  const int64_t r = e >> 6;
  const int j = (int)(e & 63);
  const int64_t i = idx[r];
  float v = 0.0f;
  if (j < SGS_NCH && i >= 0 && i < n) {
    const float uu = (y[j * npad + i] - s_min[j]) * s_rq[j];
    v = __log2f(1.0f + uu);
  }
  X[e] = f2bf(v);
}

}  // namespace

hipError_t launch_mlp_features(sgs_ctx *c, const float *params, const float *q,
                               const uint64_t *stats, const int32_t *idx, int64_t rows,
                               uint16_t *X) {
  SgsProfScope ps(c, SGS_PROF_MLP_FWD);
  if (rows > 0)
    k_mlp_features<<<sgs_blocks(rows * 64, 256), 256, 0, c->stream>>>(rows, c->n, c->npad,
                                                                      params, q, stats, idx, X);
  return hipGetLastError();
}

hipError_t launch_mlp_pack(sgs_ctx *c, const float *theta, void *packed) {
  k_mlp_pack<<<sgs_blocks(kPacked, 256), 256, 0, c->stream>>>(theta, (bf16x4 *)packed);
  return hipGetLastError();
}

// Grid of a grid-stride kernel sized to the workgroups the device holds at
// once, so no second partial round of workgroups runs at low occupancy.
template <typename K>
int resident_grid(K kernel, int64_t rows) {
  static int cap = 0;
  if (cap == 0) {
    int dev = 0, occ = 0, cus = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kernel, kThreads, 0) == hipSuccess &&
        occ > 0 && cus > 0)
      cap = occ * cus;
    else
      cap = 1024;
  }
  const int64_t tiles = (rows + 31) / 32;
  const int64_t want = (tiles + kWaves - 1) / kWaves;
  return (int)(want < cap ? (want < 1 ? 1 : want) : cap);
}

int mlp_grid(int64_t rows) {
  const int64_t tiles = (rows + 31) / 32;
  const int64_t want = (tiles + kWaves - 1) / kWaves;
  return (int)(want < 1024 ? (want < 1 ? 1 : want) : 1024);
}

hipError_t launch_mlp_rate_fwd(sgs_ctx *c, const void *packed, const float *theta,
                               const float *params, const float *q, const uint64_t *stats,
                               const uint8_t *hard, float *outR, float *fout) {
  SgsProfScope ps(c, SGS_PROF_MLP_FWD);
  const int nb = resident_grid(k_mlp_rate_fwd, c->n);
  if (nb > c->red_tmp_words) return hipErrorInvalidValue;
  k_mlp_rate_fwd<<<nb, kThreads, 0, c->stream>>>(c->n, c->npad, (const bf16x4 *)packed, theta,
                                                 params, q, stats, hard, fout, c->mlp_f,
                                                 c->mlp_signs, c->red_tmp);
  k_mlp_rate_finish<<<1, kThreads, 0, c->stream>>>(nb, c->red_tmp, c->n_hat, outR);
  return hipGetLastError();
}

hipError_t launch_mlp_rate_bwd(sgs_ctx *c, const void *packed, const float *theta,
                               const float *params, const float *q, const uint64_t *stats,
                               const uint8_t *hard, const float *soft, int mode, float weight,
                               float *gparams, float *gqstep, float *gscore, float *gmask) {
  SgsProfScope ps(c, SGS_PROF_MLP_BWD);
  const int nb = resident_grid(k_mlp_rate_bwd, c->n);
  if ((int64_t)nb * 64 > c->red_tmp_words) return hipErrorInvalidValue;
  k_mlp_rate_bwd<<<nb, kThreads, 0, c->stream>>>(c->n, c->npad, c->n_hat, weight, c->tau, mode,
                                                 (const bf16x4 *)packed, theta, params, q, stats,
                                                 hard, soft, c->mlp_f, c->mlp_signs, gparams,
                                                 gscore, gmask, c->red_tmp,
                                                 c->grad_sh_rest ? 1 : 0);
  k_mlp_q_finish<<<SGS_NCH, 256, 0, c->stream>>>(nb, c->red_tmp, gqstep);
  return hipGetLastError();
}

hipError_t launch_mlp_infer(sgs_ctx *c, const void *packed, const float *theta,
                            const uint16_t *X, int64_t B, float *fout) {
  SgsProfScope ps(c, SGS_PROF_MLP_FWD);
  k_mlp_infer<<<resident_grid(k_mlp_infer, B), kThreads, 0, c->stream>>>(B, (const bf16x4 *)packed,
                                                                         theta, X, fout);
  return hipGetLastError();
}

// Batch rows per workgroup of the weight-gradient GEMMs: 256 gives a 65,536-row
// batch 256 workgroups (with 2048, 32 of them left most compute units idle).
constexpr int64_t kWgradChunk = 256;

constexpr int64_t train_scratch_bytes(int64_t B) {
  // the takes of launch_mlp_train_step, each rounded up to 256 bytes (only
  // the B * 4 one can be ragged for B a multiple of 8)
  return B * (64 + 3 * 128) * 2 + B * 128 * 4 + B * 4 +
         (B + kWgradChunk - 1) / kWgradChunk * 24 * 1024 * 4 + (kLossParts + kSegParts) * 8 + 256;
}

int64_t mlp_train_scratch_bytes(int64_t B) { return train_scratch_bytes(B); }

// Workspace of sgs_rate_mlp_train_step_static: one copy per GPU, held until
// the process ends, shared by every call on that GPU.  Host code never uses
// this name as an address (it is a host-side stand-in there); it uses the
// device address resolved per device below.
constexpr int64_t kStaticScratchBytes = train_scratch_bytes(SGS_MLP_STATIC_ROWS);
static __device__ __align__(256) unsigned char g_train_scratch[kStaticScratchBytes];

int64_t mlp_static_scratch_bytes() { return kStaticScratchBytes; }

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_static_mu;
void *g_static_ptr[kMaxDevices] = {};
}  // namespace

void *mlp_static_scratch(int device, hipError_t *err) {
  *err = hipSuccess;
  if (device < 0 || device >= kMaxDevices) {
    *err = hipErrorInvalidDevice;
    return nullptr;
  }
  std::lock_guard<std::mutex> lock(g_static_mu);
  if (g_static_ptr[device]) return g_static_ptr[device];
  int cur = 0;
  hipError_t e = hipGetDevice(&cur);
  if (e == hipSuccess && cur != device) e = hipSetDevice(device);
  void *ptr = nullptr;
  if (e == hipSuccess) e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(g_train_scratch));
  if (cur != device) (void)hipSetDevice(cur);
  if (e != hipSuccess || !ptr) {
    *err = e != hipSuccess ? e : hipErrorInvalidSymbol;
    return nullptr;
  }
  g_static_ptr[device] = ptr;
  return ptr;
}

hipError_t launch_mlp_train_step(sgs_ctx *c, float *theta, float *m, float *v, void *packed,
                                 const uint16_t *X, const float *target, int64_t B, float lr,
                                 int64_t step, float *loss, float *gtheta, void *scratch,
                                 bool profile) {
  SgsProfScope ps(c, SGS_PROF_MLP_TRAIN, profile);
  char *p = (char *)scratch;
  auto take = [&](int64_t bytes) {
    char *r = p;
    p += (bytes + 255) / 256 * 256;
    return (void *)r;
  };
  uint16_t *XT = (uint16_t *)take(B * 64 * 2);
  uint16_t *H1T = (uint16_t *)take(B * 128 * 2);
  uint16_t *DZ2T = (uint16_t *)take(B * 128 * 2);
  uint16_t *DZ1T = (uint16_t *)take(B * 128 * 2);
  float *H2T = (float *)take(B * 128 * 4);
  float *df = (float *)take(B * 4);
  const int64_t chunk = kWgradChunk;
  const int nchunks = (int)((B + chunk - 1) / chunk);
  float *part = (float *)take((int64_t)nchunks * 24 * 1024 * 4);
  const int nb = mlp_grid(B);
  double *lpart = (double *)take((kLossParts + kSegParts) * 8);
  if (nb > kLossParts) return hipErrorInvalidValue;
  k_mlp_train_rows<<<nb, kThreads, 0, c->stream>>>(B, 2.0f / (float)B, (const bf16x4 *)packed,
                                                   theta, X, target, XT, H1T, DZ2T, DZ1T, H2T,
                                                   df, lpart);
  k_mlp_loss_finish<<<1, kThreads, 0, c->stream>>>(nb, lpart, B, loss);
  k_mlp_wgrad<<<nchunks, kThreads, 0, c->stream>>>(B, chunk, XT, H1T, DZ2T, DZ1T, part);
  k_mlp_grad_finish<<<kWRows + 385 * kSeg, kThreads, 0, c->stream>>>(
      B, nchunks, part, DZ2T, DZ1T, H2T, df, gtheta, lpart + kLossParts);
  k_mlp_bias_finish<<<2, 256, 0, c->stream>>>(lpart + kLossParts, gtheta);
  if (lr != 0.0f) {
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float c1 = (float)(1.0 - pow(0.9, (double)step));
    const float c2 = (float)(1.0 - pow(0.999, (double)step));
    k_adam<<<sgs_blocks(kParams, 256), 256, 0, c->stream>>>(kParams, theta, m, v, gtheta, lr, b1,
                                                           b2, eps, c1, c2);
    k_mlp_pack<<<sgs_blocks(kPacked, 256), 256, 0, c->stream>>>(theta, (bf16x4 *)packed);
  }
  return hipGetLastError();
}
