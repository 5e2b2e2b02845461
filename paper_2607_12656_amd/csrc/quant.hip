// Fake quantization, retention mask, channel statistics, rate proxy and the
// quantizer/mask backward (paper Sec. 3.3.1).  All three kernels stream the
// SoA parameters once: HBM-bound, so each thread owns whole Gaussians and
// walks the 59 channel rows (coalesced across the wave).
#include "sgs_internal.h"

namespace {

constexpr int kQThreads = 256;
constexpr int kQWaves = kQThreads / 64;

__global__ void k_stats_init(uint64_t *stats) {
  const int t = threadIdx.x;
  if (t < SGS_NCH) {
    stats[t] = ~0ull;      // min keys
    stats[SGS_NCH + t] = 0; // max keys
  }
  if (t >= 2 * SGS_NCH && t < SGS_STATS_WORDS) stats[t] = 0;
}

// One pass over params: qparams, hard/soft mask, per-channel min/max keys,
// kept count.  Grid-stride over Gaussians so the number of atomics per
// channel is the number of blocks, not the number of Gaussians.
__global__ void __launch_bounds__(kQThreads)
k_fakequant_prune(int64_t n, int64_t npad, const float *__restrict__ params,
                  const float *__restrict__ q, const float *__restrict__ score, int mode,
                  const uint8_t *__restrict__ given, uint64_t seed, uint64_t step, float tau,
                  float *__restrict__ qparams, uint8_t *__restrict__ hard,
                  float *__restrict__ soft, uint64_t *__restrict__ stats) {
  __shared__ uint64_t s_min[kQWaves][SGS_NCH];
  __shared__ uint64_t s_max[kQWaves][SGS_NCH];
  __shared__ uint32_t s_kept[kQWaves];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t kept = 0;
  // per-thread running extremes would need 2*59 registers; instead each
  // channel is reduced per wave on the fly and merged in LDS.
  for (int j = threadIdx.x; j < kQWaves * SGS_NCH; j += kQThreads) {
    (&s_min[0][0])[j] = ~0ull;
    (&s_max[0][0])[j] = 0ull;
  }
  __syncthreads();
  if (blockIdx.x == 0 && threadIdx.x < SGS_NCH) {
    const float qj = q[threadIdx.x];
    if (!(qj > 0.0f) || !(qj < INFINITY)) atomicOr((unsigned long long *)&stats[119], 1ull);
  }
  const int64_t stride = (int64_t)gridDim.x * kQThreads;
  for (int64_t base = (int64_t)blockIdx.x * kQThreads; base < n; base += stride) {
    const int64_t i = base + threadIdx.x;
    const bool act = i < n;
    for (int j = 0; j < SGS_NCH; ++j) {
      const float qj = q[j];
      float yv = 0.0f;
      uint64_t kmin = ~0ull, kmax = 0ull;
      if (act) {
        yv = params[j * npad + i];
        const float k = rintf(__fdiv_rn(yv, qj));
        qparams[j * npad + i] = k * qj;
        const uint64_t o = (uint64_t)sgs_ord(yv) << 32;
        kmin = o | (uint64_t)(uint32_t)i;
        kmax = o | (uint64_t)(0xFFFFFFFFu - (uint32_t)i);
      }
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) {
        const uint64_t a = __shfl_xor(kmin, off, 64);
        const uint64_t b = __shfl_xor(kmax, off, 64);
        kmin = a < kmin ? a : kmin;
        kmax = b > kmax ? b : kmax;
      }
      if (lane == 0) {
        if (kmin < s_min[wave][j]) s_min[wave][j] = kmin;
        if (kmax > s_max[wave][j]) s_max[wave][j] = kmax;
      }
    }
    if (act) {
      uint8_t m;
      float sm;
      if (mode == 0) {
        m = given[i] ? 1 : 0;
        sm = (float)m;
      } else if (mode == 2) {
        m = 1;
        sm = 1.0f;
      } else {
        const float u = sgs_uniform(seed, step, (uint64_t)i);
        const float s = score[i];
        const float e = sgs_exp_repro(s);
        m = (u * (1.0f + e)) > 1.0f ? 1 : 0;
        const float l = logf(u) - logf(1.0f - u);
        sm = 1.0f / (1.0f + __expf(-(s + l) / tau));
      }
      hard[i] = m;
      if (soft) soft[i] = sm;
      kept += m;
    }
  }
  // kept count
  uint32_t kw = kept;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) kw += __shfl_xor(kw, off, 64);
  if (lane == 0) s_kept[wave] = kw;
  __syncthreads();
  if (threadIdx.x < SGS_NCH) {
    const int j = threadIdx.x;
    uint64_t a = s_min[0][j], b = s_max[0][j];
    for (int w = 1; w < kQWaves; ++w) {
      a = s_min[w][j] < a ? s_min[w][j] : a;
      b = s_max[w][j] > b ? s_max[w][j] : b;
    }
    atomicMin((unsigned long long *)&stats[j], (unsigned long long)a);
    atomicMax((unsigned long long *)&stats[SGS_NCH + j], (unsigned long long)b);
  }
  if (threadIdx.x == 64) {
    uint32_t t = 0;
    for (int w = 0; w < kQWaves; ++w) t += s_kept[w];
    atomicAdd((unsigned long long *)&stats[118], (unsigned long long)t);
  }
}

// Rate proxy from the statistics: one wave, lane j = channel j.
__global__ void k_rate_proxy(const uint64_t *__restrict__ stats, const float *__restrict__ q,
                             int64_t n_hat, float weight, float *__restrict__ out3,
                             float *__restrict__ rate_grad) {
  const int j = threadIdx.x;
  float L = 0.0f, c = 1.0f, R = 0.0f, qj = 1.0f;
  if (j < SGS_NCH) {
    const float vmin = sgs_unord((uint32_t)(stats[j] >> 32));
    const float vmax = sgs_unord((uint32_t)(stats[SGS_NCH + j] >> 32));
    qj = q[j];
    R = vmax - vmin;
    if (R > 0.0f) c = fmaxf(1.0f, ceilf(__fdiv_rn(R, qj)));
    L = log2f(c);
  }
  const float Lq = sgs_wave_sum(L);
  const double kept = (double)stats[118];
  const float Lm = (float)(kept / (double)n_hat);
  if (j == 0) {
    out3[0] = Lm * Lq;
    out3[1] = Lq;
    out3[2] = Lm;
  }
  if (rate_grad) {
    const float ln2 = 0.69314718055994531f;
    if (j < SGS_NCH) {
      float gR = 0.0f, gq = 0.0f;
      if (R > 0.0f) {
        gR = weight * Lm / (c * qj * ln2);
        gq = -weight * Lm * R / (c * qj * qj * ln2);
      }
      rate_grad[j] = gR;
      rate_grad[64 + j] = -gR;
      rate_grad[128 + j] = gq;
    }
    if (j == 0) rate_grad[192] = (float)((double)weight * (double)Lq / (double)n_hat);
  }
}

// Backward, pass 1: straight-through copy, per-block FP64 partial sums of the
// learned-step-size gradient sum_i g_ij (k_ij - y_ij / q_j), score gradient.
constexpr int kBItems = 8;  // Gaussians per thread per block
__global__ void __launch_bounds__(kQThreads)
k_fakequant_bwd(int64_t n, int64_t npad, const float *__restrict__ params,
                const float *__restrict__ q, const float *__restrict__ gq_in,
                float *__restrict__ gparams, double *__restrict__ partial) {
  __shared__ double s_red[kQWaves];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t base = (int64_t)blockIdx.x * kQThreads * kBItems;
  const bool copy = gparams != gq_in;
  for (int j = 0; j < SGS_NCH; ++j) {
    const float qj = q[j];
    double acc = 0.0;
#pragma unroll
    for (int it = 0; it < kBItems; ++it) {
      const int64_t i = base + (int64_t)it * kQThreads + threadIdx.x;
      if (i < n) {
        const float g = gq_in[j * npad + i];
        const float yv = params[j * npad + i];
        const float r = __fdiv_rn(yv, qj);
        acc += (double)g * ((double)rintf(r) - (double)yv / (double)qj);
        if (copy) gparams[j * npad + i] = g;
      }
    }
    acc = sgs_wave_sum_d(acc);
    if (lane == 0) s_red[wave] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = 0.0;
      for (int w = 0; w < kQWaves; ++w) t += s_red[w];
      partial[(int64_t)blockIdx.x * SGS_NCH + j] = t;
    }
    __syncthreads();
  }
}

// Backward, pass 2 (one block): fixed-order sum of the partials + the rate
// proxy's step gradient; scatter of the rate gradient at argmax/argmin.
__global__ void k_fakequant_bwd_finish(int nblocks, const double *__restrict__ partial,
                                       const float *__restrict__ rate_grad,
                                       const uint64_t *__restrict__ stats, int64_t npad,
                                       float *__restrict__ gparams, float *__restrict__ gqstep) {
  const int j = threadIdx.x;
  if (j >= SGS_NCH) return;
  double t = 0.0;
  for (int b = 0; b < nblocks; ++b) t += partial[(int64_t)b * SGS_NCH + j];
  if (rate_grad) {
    t += (double)rate_grad[128 + j];
    const uint32_t imin = (uint32_t)(stats[j] & 0xFFFFFFFFull);
    const uint32_t imax = 0xFFFFFFFFu - (uint32_t)(stats[SGS_NCH + j] & 0xFFFFFFFFull);
    gparams[j * npad + imax] += rate_grad[j];
    gparams[j * npad + imin] += rate_grad[64 + j];
  }
  gqstep[j] = (float)t;
}

__global__ void k_score_bwd(int64_t n, int mode, float tau, const float *__restrict__ soft,
                            const float *__restrict__ gmask, const float *__restrict__ rate_grad,
                            float *__restrict__ gscore) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (mode != 1) {
    gscore[i] = 0.0f;
    return;
  }
  const float g = gmask[i] + (rate_grad ? rate_grad[192] : 0.0f);
  const float s = soft[i];
  gscore[i] = g * s * (1.0f - s) / tau;
}

}  // namespace

hipError_t launch_fakequant_prune(sgs_ctx *c, const float *params, const float *q,
                                  const float *score, int mode, const uint8_t *given,
                                  uint64_t seed, uint64_t step, float *qparams,
                                  uint8_t *hard, float *soft, uint64_t *stats) {
  k_stats_init<<<1, SGS_STATS_WORDS, 0, c->stream>>>(stats);
  const int64_t want = (c->n + kQThreads - 1) / kQThreads;
  const unsigned blocks = (unsigned)(want < 2048 ? want : 2048);
  k_fakequant_prune<<<blocks, kQThreads, 0, c->stream>>>(c->n, c->npad, params, q, score, mode,
                                                         given, seed, step, c->tau, qparams,
                                                         hard, soft, stats);
  return hipGetLastError();
}

hipError_t launch_rate_proxy(sgs_ctx *c, const uint64_t *stats, const float *q, float weight,
                             float *out3, float *rate_grad) {
  k_rate_proxy<<<1, 64, 0, c->stream>>>(stats, q, c->n_hat, weight, out3, rate_grad);
  return hipGetLastError();
}

hipError_t launch_fakequant_bwd(sgs_ctx *c, const float *params, const float *q,
                                const float *soft, int mode, const float *rate_grad,
                                const uint64_t *stats, const float *gq_in,
                                const float *gmask_in, float *gparams, float *gqstep,
                                float *gscore) {
  const int64_t per = (int64_t)kQThreads * kBItems;
  const int nb = (int)((c->n + per - 1) / per);
  if ((int64_t)nb * SGS_NCH > c->red_tmp_words) return hipErrorInvalidValue;
  k_fakequant_bwd<<<nb, kQThreads, 0, c->stream>>>(c->n, c->npad, params, q, gq_in, gparams,
                                                   c->red_tmp);
  k_fakequant_bwd_finish<<<1, 64, 0, c->stream>>>(nb, c->red_tmp, rate_grad, stats, c->npad,
                                                  gparams, gqstep);
  k_score_bwd<<<sgs_blocks(c->n, 256), 256, 0, c->stream>>>(c->n, mode, c->tau, soft, gmask_in,
                                                            rate_grad, gscore);
  return hipGetLastError();
}
