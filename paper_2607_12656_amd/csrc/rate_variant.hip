// Rate-proxy variants the paper compares with its range-based multiplicative
// proxy (Sec. 3.3.1 and the supplement's "Comparison with an Alternative
// Rate Proxy"; the ablation's additive masking).
//
// Scale-based Laplace proxy: per channel the mean over the N current
// Gaussians, then b_j = mean |y - mean| (the maximum-likelihood Laplace
// scale) and the mean sign of y - mean; L_j = log2(max(1, 2 e b_j / q_j)).
// Two passes over the parameters (a block per 4096-Gaussian chunk and
// channel, FP64 sums, fixed-order finishes).  Its y gradient is dense:
//     dL_j/dy_ij = (sign(y_ij - mean_j) - mean sign_j) / (N b_j ln 2),
// added by the backward entry after the quantizer backward; the q and mask
// terms go through the compact rate-gradient buffer like the range proxy's.
// Additive masking: the loss carries lambda L_quant + alpha L_mask.
#include <cmath>

#include "sgs_internal.h"

namespace {

constexpr int kVThreads = 256;
constexpr int kVItems = 16;
constexpr int kVChunk = kVThreads * kVItems;

__device__ __forceinline__ double block_sum_d(double v, double *s_w) {
  v = sgs_wave_sum_d(v);
  if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < kVThreads / 64; ++w) t += s_w[w];
  return t;  // valid in thread 0
}

__global__ void __launch_bounds__(kVThreads)
k_lap_sum(int64_t n, int64_t npad, const float *__restrict__ y, int nc,
          double *__restrict__ part) {
  __shared__ double s_w[kVThreads / 64];
  const int j = blockIdx.y;
  const int64_t chunk = blockIdx.x;
  const float *row = y + j * npad;
  // all loads first (entries past n read entry 0 and are dropped)
  float v[kVItems];
#pragma unroll
  for (int e = 0; e < kVItems; ++e) {
    const int64_t i = chunk * kVChunk + (int64_t)e * kVThreads + threadIdx.x;
    v[e] = row[i < n ? i : 0];
  }
  double acc = 0.0;
#pragma unroll
  for (int e = 0; e < kVItems; ++e) {
    const int64_t i = chunk * kVChunk + (int64_t)e * kVThreads + threadIdx.x;
    if (i < n) acc += (double)v[e];
  }
  const double t = block_sum_d(acc, s_w);
  if (threadIdx.x == 0) part[(int64_t)j * nc + chunk] = t;
}

// coef layout (doubles): [0, 64) mean, [64, 128) mean sign, [128, 192) the
// backward's coefficient per channel
__global__ void k_lap_mean(int nc, const double *__restrict__ part, int64_t n,
                           double *__restrict__ coef) {
  __shared__ double s_w[kVThreads / 64];
  const int j = blockIdx.x;
  double acc = 0.0;
  for (int c = threadIdx.x; c < nc; c += kVThreads) acc += part[(int64_t)j * nc + c];
  const double t = block_sum_d(acc, s_w);
  if (threadIdx.x == 0) coef[j] = t / (double)n;
}

__global__ void __launch_bounds__(kVThreads)
k_lap_abs(int64_t n, int64_t npad, const float *__restrict__ y, int nc,
          const double *__restrict__ coef, double *__restrict__ part) {
  __shared__ double s_w[kVThreads / 64];
  const int j = blockIdx.y;
  const int64_t chunk = blockIdx.x;
  const float *row = y + j * npad;
  const double mu = coef[j];
  float v[kVItems];
#pragma unroll
  for (int e = 0; e < kVItems; ++e) {
    const int64_t i = chunk * kVChunk + (int64_t)e * kVThreads + threadIdx.x;
    v[e] = row[i < n ? i : 0];
  }
  double sa = 0.0, ss = 0.0;
#pragma unroll
  for (int e = 0; e < kVItems; ++e) {
    const int64_t i = chunk * kVChunk + (int64_t)e * kVThreads + threadIdx.x;
    if (i < n) {
      const double d = (double)v[e] - mu;
      sa += fabs(d);
      ss += d > 0.0 ? 1.0 : (d < 0.0 ? -1.0 : 0.0);
    }
  }
  const double ta = block_sum_d(sa, s_w);
  __syncthreads();
  const double ts = block_sum_d(ss, s_w);
  if (threadIdx.x == 0) {
    part[(int64_t)j * nc + chunk] = ta;
    part[(int64_t)(SGS_NCH + j) * nc + chunk] = ts;
  }
}

// One wave, lane j = channel j: b_j, mean sign, L_j, L_quant, the loss term,
// the compact rate gradient and the backward's coefficients.
__global__ void k_lap_finish(int nc, const double *__restrict__ part, int64_t n, int64_t n_hat,
                             const float *__restrict__ q, const uint64_t *__restrict__ stats,
                             float weight, int additive, float alpha, double *__restrict__ coef,
                             float *__restrict__ out3, float *__restrict__ rate_grad) {
  const int j = threadIdx.x;
  double L = 0.0, b = 0.0, sbar = 0.0, qj = 1.0;
  bool active = false;
  if (j < SGS_NCH) {
    double sa = 0.0, ss = 0.0;
    for (int c = 0; c < nc; ++c) {
      sa += part[(int64_t)j * nc + c];
      ss += part[(int64_t)(SGS_NCH + j) * nc + c];
    }
    b = sa / (double)n;
    sbar = ss / (double)n;
    qj = (double)q[j];
    const double ratio = 2.0 * 2.718281828459045 * b / qj;
    active = ratio > 1.0;
    L = active ? log2(ratio) : 0.0;
  }
  const double Lq = sgs_wave_sum_d(L);
  const double Lm = (double)stats[118] / (double)n_hat;
  const double f = additive ? 1.0 : Lm;  // factor on the L_quant gradients
  if (j == 0) {
    out3[0] = (float)(additive ? (double)weight * Lq + (double)alpha * Lm : (double)weight * Lm * Lq);
    out3[1] = (float)Lq;
    out3[2] = (float)Lm;
  }
  const double ln2 = 0.6931471805599453;
  if (j < SGS_NCH) {
    coef[64 + j] = sbar;
    coef[128 + j] = active ? (double)weight * f / (b * ln2 * (double)n) : 0.0;
    if (rate_grad) {
      rate_grad[j] = 0.0f;         // no argmax / argmin terms: the y gradient is dense
      rate_grad[64 + j] = 0.0f;
      rate_grad[128 + j] = active ? (float)(-(double)weight * f / (qj * ln2)) : 0.0f;
    }
  }
  if (j == 0 && rate_grad)
    rate_grad[192] = (float)(additive ? (double)alpha / (double)n_hat
                                      : (double)weight * Lq / (double)n_hat);
}

__global__ void __launch_bounds__(kVThreads)
k_lap_bwd(int64_t n, int64_t npad, const float *__restrict__ y, const double *__restrict__ coef,
          float *__restrict__ grad) {
  const int j = blockIdx.y;
  const double mu = coef[j], sbar = coef[64 + j], cj = coef[128 + j];
  if (cj == 0.0) return;
  const int64_t base = (int64_t)blockIdx.x * kVChunk;
  // all loads first (entries past n read entry 0 and are dropped)
  float yv[kVItems], gv[kVItems];
#pragma unroll
  for (int e = 0; e < kVItems; ++e) {
    const int64_t i = base + (int64_t)e * kVThreads + threadIdx.x;
    const int64_t ic = i < n ? i : 0;
    yv[e] = y[j * npad + ic];
    gv[e] = grad[j * npad + ic];
  }
#pragma unroll
  for (int e = 0; e < kVItems; ++e) {
    const int64_t i = base + (int64_t)e * kVThreads + threadIdx.x;
    if (i < n) {
      const double d = (double)yv[e] - mu;
      const double s = d > 0.0 ? 1.0 : (d < 0.0 ? -1.0 : 0.0);
      grad[j * npad + i] = (float)((double)gv[e] + cj * (s - sbar));
    }
  }
}

}  // namespace

int64_t lap_partial_doubles(int64_t n) { return 2 * SGS_NCH * ((n + kVChunk - 1) / kVChunk); }

hipError_t launch_rate_variant(sgs_ctx *c, const float *params, const float *q,
                               const uint64_t *stats, const sgs_rate_options *o, float weight,
                               float *out3, float *rate_grad) {
  SgsProfScope ps(c, SGS_PROF_RATE);
  const int additive = o->masking == 1;
  if (o->proxy == 0)
    return launch_rate_proxy_mode(c, stats, q, weight, additive, o->alpha, out3, rate_grad);
  const int nc = (int)((c->n + kVChunk - 1) / kVChunk);
  if (lap_partial_doubles(c->n) > c->red_tmp_words) return hipErrorInvalidValue;
  double *part = c->red_tmp;
  k_lap_sum<<<dim3(nc, SGS_NCH), kVThreads, 0, c->stream>>>(c->n, c->npad, params, nc, part);
  k_lap_mean<<<SGS_NCH, kVThreads, 0, c->stream>>>(nc, part, c->n, c->lap_coef);
  k_lap_abs<<<dim3(nc, SGS_NCH), kVThreads, 0, c->stream>>>(c->n, c->npad, params, nc,
                                                            c->lap_coef, part);
  k_lap_finish<<<1, 64, 0, c->stream>>>(nc, part, c->n, c->n_hat, q, stats, weight, additive,
                                        o->alpha, c->lap_coef, out3, rate_grad);
  return hipGetLastError();
}

hipError_t launch_rate_variant_bwd(sgs_ctx *c, const float *params, float *grad) {
  SgsProfScope ps(c, SGS_PROF_RATE);
  const int nc = (int)((c->n + kVChunk - 1) / kVChunk);
  k_lap_bwd<<<dim3(nc, SGS_NCH), kVThreads, 0, c->stream>>>(c->n, c->npad, params, c->lap_coef,
                                                            grad);
  return hipGetLastError();
}
