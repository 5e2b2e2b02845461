// L1 distortion and its gradient (the L1 part of the paper's rendering
// distortion, Supplementary "Training Objective").  Two passes: per-block
// FP64 partial sums while writing dL/dC, then a fixed-order sum.
#include "sgs_internal.h"

namespace {

constexpr int kThreads = 256;
constexpr int kItems = 8;

__global__ void __launch_bounds__(kThreads)
k_l1(const float *__restrict__ img, const float *__restrict__ tgt, int64_t count, float inv,
     float *__restrict__ dimg, double *__restrict__ partial) {
  __shared__ double s_w[kThreads / 64];
  const int64_t base = (int64_t)blockIdx.x * kThreads * kItems;
  // all loads first (entries past count read entry 0 and are dropped), then
  // the arithmetic and the stores
  float a[kItems], t[kItems];
#pragma unroll
  for (int k = 0; k < kItems; ++k) {
    const int64_t i = base + (int64_t)k * kThreads + threadIdx.x;
    const int64_t ic = i < count ? i : 0;
    a[k] = img[ic];
    t[k] = tgt[ic];
  }
  double acc = 0.0;
#pragma unroll
  for (int k = 0; k < kItems; ++k) {
    const int64_t i = base + (int64_t)k * kThreads + threadIdx.x;
    if (i < count) {
      const float d = a[k] - t[k];
      acc += (double)fabsf(d);
      dimg[i] = d > 0.0f ? inv : (d < 0.0f ? -inv : 0.0f);
    }
  }
  acc = sgs_wave_sum_d(acc);
  if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < kThreads / 64; ++w) t += s_w[w];
    partial[blockIdx.x] = t;
  }
}

__global__ void k_l1_finish(const double *__restrict__ partial, int nb, int64_t count,
                            float *__restrict__ loss) {
  __shared__ double s_w[kThreads / 64];
  // eight loads in flight per thread (a loop-carried sum would wait on each)
  double a8[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  int b = threadIdx.x;
  for (; b + 7 * kThreads < nb; b += 8 * kThreads) {
#pragma unroll
    for (int u = 0; u < 8; ++u) a8[u] += partial[b + u * kThreads];
  }
  for (; b < nb; b += kThreads) a8[0] += partial[b];
  double acc = ((a8[0] + a8[1]) + (a8[2] + a8[3])) + ((a8[4] + a8[5]) + (a8[6] + a8[7]));
  acc = sgs_wave_sum_d(acc);
  if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < kThreads / 64; ++w) t += s_w[w];
    loss[0] = (float)(t / (double)count);
  }
}

}  // namespace

hipError_t launch_l1(sgs_ctx *c, const float *image, const float *target, float scale,
                     float *loss, float *dimg) {
  const int64_t count = (int64_t)c->V * 3 * c->W * c->H;
  const int64_t per = (int64_t)kThreads * kItems;
  const int nb = (int)((count + per - 1) / per);
  if (nb > c->red_tmp_words) return hipErrorInvalidValue;
  SgsProfScope ps(c, SGS_PROF_L1);
  k_l1<<<nb, kThreads, 0, c->stream>>>(image, target, count, (float)((double)scale / (double)count), dimg,
                                       c->red_tmp);
  k_l1_finish<<<1, kThreads, 0, c->stream>>>(c->red_tmp, nb, count, loss);
  return hipGetLastError();
}
