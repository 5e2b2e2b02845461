// Fake quantization, retention mask, channel statistics, rate proxy and the
// quantizer/mask backward (paper Sec. 3.3.1).
//
// The parameter passes are HBM-bound streams over the SoA rows.  A block owns
// one channel row of a chunk of kRPer consecutive Gaussians (16 per thread,
// as four 16-byte loads, coalesced across the wave), so the per-channel
// reductions (range keys, step-size gradient) cost one wave reduction per
// 16 elements of a thread; they are written as per-chunk partials and
// finished by one block per channel.  No contended atomics.
#include "sgs_internal.h"

namespace {

constexpr int kQThreads = 256;
constexpr int kQWaves = kQThreads / 64;
constexpr int kRVec = 4;                        // float4 loads per thread and row
constexpr int kRPer = kQThreads * kRVec * 4;    // Gaussians per chunk
// partial record per block: [0,59) min keys, [59,118) max keys, [118] kept
constexpr int kPartWords = 120;

__device__ __forceinline__ uint64_t wave_min_u64(uint64_t v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const uint64_t o = __shfl_xor(v, off, 64);
    v = o < v ? o : v;
  }
  return v;
}
__device__ __forceinline__ uint64_t wave_max_u64(uint64_t v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const uint64_t o = __shfl_xor(v, off, 64);
    v = o > v ? o : v;
  }
  return v;
}

// Pass 1, block (chunk, j) for j < 59: qparams of row j (WRITE) and the row's
// range keys over the chunk; block (chunk, 59): hard/soft mask and kept count.
// Without WRITE the pass reads the rows for their statistics only (the fused
// path quantizes inside the projection).
template <bool WRITE>
__global__ void __launch_bounds__(kQThreads)
k_fakequant_prune(int64_t n, int64_t npad, const float *__restrict__ params,
                  const float *__restrict__ q, const float *__restrict__ score, int mode,
                  const uint8_t *__restrict__ given, uint64_t seed, uint64_t step, float tau,
                  float *__restrict__ qparams, uint8_t *__restrict__ hard,
                  float *__restrict__ soft, uint64_t *__restrict__ part) {
  __shared__ uint64_t s_a[kQWaves], s_b[kQWaves];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int j = blockIdx.y;
  const int64_t chunk = blockIdx.x;
  const int64_t c0 = chunk * kRPer;
  uint64_t *dst = part + chunk * kPartWords;
  if (j < SGS_NCH) {
    const float qj = q[j];
    const float rq = __fdiv_rn(1.0f, qj);
    const bool fast_ok = sgs_rq_ok(rq);
    const float *row = params + j * npad;
    float *orow = WRITE ? qparams + j * npad : nullptr;
    uint64_t kmin = ~0ull, kmax = 0ull;
    // all loads first (i + 3 < npad for i < n, npad % 64 == 0: a 16-byte load
    // stays in the row; lanes past n load the row's first entries and drop them)
    float4 y4[kRVec];
#pragma unroll
    for (int r = 0; r < kRVec; ++r) {
      const int64_t i = c0 + ((int64_t)r * kQThreads + threadIdx.x) * 4;
      y4[r] = *reinterpret_cast<const float4 *>(row + (i < n ? i : 0));
    }
#pragma unroll
    for (int r = 0; r < kRVec; ++r) {
      const int64_t i = c0 + ((int64_t)r * kQThreads + threadIdx.x) * 4;
      if (i < n) {
        const float4 y = y4[r];
        const float yv[4] = {y.x, y.y, y.z, y.w};
        float o[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          if (WRITE) o[e] = sgs_rint_div(yv[e], qj, rq, fast_ok) * qj;  // rint(fl32(y / q)) q
          if (i + e < n) {
            const uint64_t ok = (uint64_t)sgs_ord(yv[e]) << 32;
            const uint64_t a = ok | (uint64_t)(uint32_t)(i + e);
            const uint64_t b = ok | (uint64_t)(0xFFFFFFFFu - (uint32_t)(i + e));
            kmin = a < kmin ? a : kmin;
            kmax = b > kmax ? b : kmax;
          }
        }
        if (WRITE) {
          if (i + 3 < n) {
            *reinterpret_cast<float4 *>(orow + i) = make_float4(o[0], o[1], o[2], o[3]);
          } else {
#pragma unroll
            for (int e = 0; e < 4; ++e)
              if (i + e < n) orow[i + e] = o[e];
          }
        }
      }
    }
    kmin = wave_min_u64(kmin);
    kmax = wave_max_u64(kmax);
    if (lane == 0) {
      s_a[wave] = kmin;
      s_b[wave] = kmax;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      uint64_t a = s_a[0], b = s_b[0];
#pragma unroll
      for (int w = 1; w < kQWaves; ++w) {
        a = s_a[w] < a ? s_a[w] : a;
        b = s_b[w] > b ? s_b[w] : b;
      }
      dst[j] = a;
      dst[SGS_NCH + j] = b;
    }
    return;
  }
  // the mode is uniform: one branch, then all loads of the given mask or the
  // scores issued together (lanes past n load entry n - 1 and store nothing)
  constexpr int kM = kRVec * 4;
  uint8_t mv[kM];
  float sv[kM];
  if (mode == 0) {
#pragma unroll
    for (int r = 0; r < kM; ++r) {
      const int64_t i = c0 + (int64_t)r * kQThreads + threadIdx.x;
      mv[r] = given[i < n ? i : n - 1] ? 1 : 0;
    }
#pragma unroll
    for (int r = 0; r < kM; ++r) sv[r] = (float)mv[r];
  } else if (mode == 2) {
#pragma unroll
    for (int r = 0; r < kM; ++r) {
      mv[r] = 1;
      sv[r] = 1.0f;
    }
  } else {
    float sc[kM];
#pragma unroll
    for (int r = 0; r < kM; ++r) {
      const int64_t i = c0 + (int64_t)r * kQThreads + threadIdx.x;
      sc[r] = score[i < n ? i : n - 1];
    }
#pragma unroll
    for (int r = 0; r < kM; ++r) {
      const int64_t i = c0 + (int64_t)r * kQThreads + threadIdx.x;
      mv[r] = sgs_gumbel_decide(sc[r], sgs_uniform(seed, step, (uint64_t)i), tau, sv[r]);
    }
  }
  uint32_t kept = 0;
#pragma unroll
  for (int r = 0; r < kM; ++r) {
    const int64_t i = c0 + (int64_t)r * kQThreads + threadIdx.x;
    if (i < n) {
      hard[i] = mv[r];
      if (soft) soft[i] = sv[r];
      kept += mv[r];
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) kept += __shfl_xor(kept, off, 64);
  if (lane == 0) s_a[wave] = kept;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t t = 0;
#pragma unroll
    for (int w = 0; w < kQWaves; ++w) t += s_a[w];
    dst[118] = t;
  }
}

// Pass 2: block j reduces channel j over the block partials; block 0 also
// the kept count and the step-size validity flag.
__global__ void __launch_bounds__(kQThreads)
k_stats_finish(int nblocks, const uint64_t *__restrict__ part, const float *__restrict__ q,
               uint64_t *__restrict__ stats) {
  __shared__ uint64_t s_a[kQWaves], s_b[kQWaves], s_c[kQWaves];
  const int j = blockIdx.x;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint64_t a = ~0ull, b = 0ull, cnt = 0;
  for (int k = threadIdx.x; k < nblocks; k += kQThreads) {
    const uint64_t *p = part + (int64_t)k * kPartWords;
    a = p[j] < a ? p[j] : a;
    b = p[SGS_NCH + j] > b ? p[SGS_NCH + j] : b;
    cnt += p[118];
  }
  a = wave_min_u64(a);
  b = wave_max_u64(b);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) cnt += __shfl_xor(cnt, off, 64);
  if (lane == 0) {
    s_a[wave] = a;
    s_b[wave] = b;
    s_c[wave] = cnt;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  uint64_t ra = s_a[0], rb = s_b[0], rc = 0;
  for (int w = 0; w < kQWaves; ++w) {
    ra = s_a[w] < ra ? s_a[w] : ra;
    rb = s_b[w] > rb ? s_b[w] : rb;
    rc += s_c[w];
  }
  stats[j] = ra;
  stats[SGS_NCH + j] = rb;
  if (j == 0) {
    stats[118] = rc;
    uint64_t flags = 0;
    for (int c = 0; c < SGS_NCH; ++c) {
      const float qc = q[c];
      if (!(qc > 0.0f) || !(qc < INFINITY)) flags |= 1ull;
    }
    stats[119] = flags;
    for (int w = 120; w < SGS_STATS_WORDS; ++w) stats[w] = 0;
  }
}

// Rate proxy from the statistics: one wave, lane j = channel j.  additive:
// the loss carries weight L_quant + alpha L_mask instead of weight L_mask
// L_quant; loss_form: out3[0] is that loss term instead of R = L_mask L_quant.
__global__ void k_rate_proxy(const uint64_t *__restrict__ stats, const float *__restrict__ q,
                             int64_t n_hat, float weight, int additive, float alpha,
                             int loss_form, float *__restrict__ out3,
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
    out3[0] = !loss_form ? Lm * Lq : (additive ? weight * Lq + alpha * Lm : weight * Lm * Lq);
    out3[1] = Lq;
    out3[2] = Lm;
  }
  if (rate_grad) {
    const float ln2 = 0.69314718055994531f;
    const float f = additive ? 1.0f : Lm;  // factor on the L_quant gradients
    if (j < SGS_NCH) {
      float gR = 0.0f, gq = 0.0f;
      if (R > 0.0f) {
        gR = weight * f / (c * qj * ln2);
        gq = -weight * f * R / (c * qj * qj * ln2);
      }
      rate_grad[j] = gR;
      rate_grad[64 + j] = -gR;
      rate_grad[128 + j] = gq;
    }
    if (j == 0)
      rate_grad[192] = additive ? (float)((double)alpha / (double)n_hat)
                                : (float)((double)weight * (double)Lq / (double)n_hat);
  }
}

// Backward pass 1, block (chunk, j): straight-through copy of row j
// (skipped when aliased) and sum_i g_ij (k_ij q_j - y_ij) over the chunk in
// FP64 (the learned-step gradient before the division by q_j).  k q - y is
// formed with one fused multiply-add, so the small residual is exact, and its
// product with g is exact in FP64.
__global__ void __launch_bounds__(kQThreads)
k_fakequant_bwd(int64_t n, int64_t npad, const float *__restrict__ params,
                const float *__restrict__ q, const float *__restrict__ gq_in,
                float *__restrict__ gparams, double *__restrict__ partial) {
  __shared__ double s_red[kQWaves];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int j = blockIdx.y;
  const int64_t chunk = blockIdx.x;
  const int64_t c0 = chunk * kRPer;
  const bool copy = gparams != gq_in;
  const float qj = q[j];
  const float rq = __fdiv_rn(1.0f, qj);
  const bool fast_ok = sgs_rq_ok(rq);
  const float *yrow = params + j * npad;
  const float *grow = gq_in + j * npad;
  float *orow = gparams + j * npad;
  double acc = 0.0;
  // all loads first (i + 3 < npad for i < n; lanes past n read the row's first
  // entries and drop them)
  float4 y4[kRVec], g4[kRVec];
#pragma unroll
  for (int r = 0; r < kRVec; ++r) {
    const int64_t i = c0 + ((int64_t)r * kQThreads + threadIdx.x) * 4;
    const int64_t ic = i < n ? i : 0;
    y4[r] = *reinterpret_cast<const float4 *>(yrow + ic);
    g4[r] = *reinterpret_cast<const float4 *>(grow + ic);
  }
#pragma unroll
  for (int r = 0; r < kRVec; ++r) {
    const int64_t i = c0 + ((int64_t)r * kQThreads + threadIdx.x) * 4;
    if (i < n) {
      const float4 y = y4[r];
      const float4 g = g4[r];
      const float yv[4] = {y.x, y.y, y.z, y.w}, gv[4] = {g.x, g.y, g.z, g.w};
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        if (i + e < n) {
          const float k = sgs_rint_div(yv[e], qj, rq, fast_ok);  // = rint(fl32(y / q))
          acc = fma((double)gv[e], (double)fmaf(k, qj, -yv[e]), acc);
        }
      }
      if (copy) {
        if (i + 3 < n) {
          *reinterpret_cast<float4 *>(orow + i) = g;
        } else {
#pragma unroll
          for (int e = 0; e < 4; ++e)
            if (i + e < n) orow[i + e] = gv[e];
        }
      }
    }
  }
  const double s = sgs_wave_sum_d(acc);
  if (lane == 0) s_red[wave] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < kQWaves; ++w) t += s_red[w];
    partial[chunk * SGS_NCH + j] = t;
  }
}

// Backward pass 2: block j sums channel j's partials (partial[j * jstride +
// b * bstride], fixed order per thread, then a tree), divides by q_j, adds the
// rate proxy's step gradient and scatters its parameter gradient at
// argmax_j / argmin_j.
__global__ void __launch_bounds__(kQThreads)
k_fakequant_bwd_finish(int64_t nblocks, const double *__restrict__ partial, int64_t jstride,
                       int64_t bstride, const float *__restrict__ q,
                       const float *__restrict__ rate_grad, const uint64_t *__restrict__ stats,
                       int64_t npad, float *__restrict__ gparams, float *__restrict__ gqstep,
                       int sh_rows) {
  __shared__ double s_w[kQWaves];
  const int j = blockIdx.x;
  // eight loads in flight per thread (a loop-carried sum would wait on each)
  double t8[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  int64_t b = threadIdx.x;
  for (; b + 7 * kQThreads < nblocks; b += 8 * kQThreads) {
#pragma unroll
    for (int u = 0; u < 8; ++u) t8[u] += partial[j * jstride + (b + u * kQThreads) * bstride];
  }
  for (; b < nblocks; b += kQThreads) t8[0] += partial[j * jstride + b * bstride];
  double t = ((t8[0] + t8[1]) + (t8[2] + t8[3])) + ((t8[4] + t8[5]) + (t8[6] + t8[7]));
  t = sgs_wave_sum_d(t);
  if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = t;
  __syncthreads();
  if (threadIdx.x != 0) return;
  double tot = 0.0;
  for (int w = 0; w < kQWaves; ++w) tot += s_w[w];
  tot /= (double)q[j];
  if (rate_grad) {
    tot += (double)rate_grad[128 + j];
    const uint32_t imin = (uint32_t)(stats[j] & 0xFFFFFFFFull);
    const uint32_t imax = 0xFFFFFFFFu - (uint32_t)(stats[SGS_NCH + j] & 0xFFFFFFFFull);
    if (sh_rows || j < SGS_CH_REST || j >= SGS_CH_REST_END) {
      gparams[j * npad + imax] += rate_grad[j];
      gparams[j * npad + imin] += rate_grad[64 + j];
    }
  }
  gqstep[j] = (float)tot;
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

int64_t quant_partial_words(int64_t n) {
  const int64_t nb = (n + kRPer - 1) / kRPer;
  return nb * (kPartWords > SGS_NCH ? kPartWords : SGS_NCH);
}

hipError_t launch_fakequant_prune(sgs_ctx *c, const float *params, const float *q,
                                  const float *score, int mode, const uint8_t *given,
                                  uint64_t seed, uint64_t step, float *qparams,
                                  uint8_t *hard, float *soft, uint64_t *stats) {
  SgsProfScope ps(c, SGS_PROF_FAKEQUANT);
  const int nb = (int)((c->n + kRPer - 1) / kRPer);
  if ((int64_t)nb * kPartWords > c->red_tmp_words) return hipErrorInvalidValue;
  uint64_t *part = (uint64_t *)c->red_tmp;
  if (qparams)
    k_fakequant_prune<true><<<dim3(nb, SGS_NCH + 1), kQThreads, 0, c->stream>>>(
        c->n, c->npad, params, q, score, mode, given, seed, step, c->tau, qparams, hard, soft,
        part);
  else
    k_fakequant_prune<false><<<dim3(nb, SGS_NCH + 1), kQThreads, 0, c->stream>>>(
        c->n, c->npad, params, q, score, mode, given, seed, step, c->tau, nullptr, hard, soft,
        part);
  k_stats_finish<<<SGS_NCH, kQThreads, 0, c->stream>>>(nb, part, q, stats);
  return hipGetLastError();
}

hipError_t launch_rate_proxy(sgs_ctx *c, const uint64_t *stats, const float *q, float weight,
                             float *out3, float *rate_grad) {
  SgsProfScope ps(c, SGS_PROF_RATE);
  k_rate_proxy<<<1, 64, 0, c->stream>>>(stats, q, c->n_hat, weight, 0, 0.0f, 0, out3, rate_grad);
  return hipGetLastError();
}

hipError_t launch_rate_proxy_mode(sgs_ctx *c, const uint64_t *stats, const float *q,
                                  float weight, int additive, float alpha, float *out3,
                                  float *rate_grad) {
  k_rate_proxy<<<1, 64, 0, c->stream>>>(stats, q, c->n_hat, weight, additive, alpha, 1, out3,
                                        rate_grad);
  return hipGetLastError();
}

hipError_t launch_fakequant_bwd(sgs_ctx *c, const float *params, const float *q,
                                const float *soft, int mode, const float *rate_grad,
                                const uint64_t *stats, const float *gq_in,
                                const float *gmask_in, float *gparams, float *gqstep,
                                float *gscore) {
  const int nb = (int)((c->n + kRPer - 1) / kRPer);
  if ((int64_t)nb * SGS_NCH > c->red_tmp_words) return hipErrorInvalidValue;
  SgsProfScope ps(c, SGS_PROF_FAKEQUANT_BWD);
  k_fakequant_bwd<<<dim3(nb, SGS_NCH), kQThreads, 0, c->stream>>>(c->n, c->npad, params, q,
                                                                  gq_in, gparams, c->red_tmp);
  k_fakequant_bwd_finish<<<SGS_NCH, kQThreads, 0, c->stream>>>(
      nb, c->red_tmp, 1, SGS_NCH, q, rate_grad, stats, c->npad, gparams, gqstep, 1);
  k_score_bwd<<<sgs_blocks(c->n, 256), 256, 0, c->stream>>>(c->n, mode, c->tau, soft, gmask_in,
                                                            rate_grad, gscore);
  return hipGetLastError();
}

hipError_t launch_quant_bwd_finish(sgs_ctx *c, int64_t nblocks, const double *partial,
                                   int64_t jstride, int64_t bstride, const float *q,
                                   const float *rate_grad, const uint64_t *stats,
                                   float *gparams, float *gqstep) {
  SgsProfScope ps(c, SGS_PROF_FAKEQUANT_BWD);
  k_fakequant_bwd_finish<<<SGS_NCH, kQThreads, 0, c->stream>>>(
      nblocks, partial, jstride, bstride, q, rate_grad, stats, c->npad, gparams, gqstep,
      c->grad_sh_rest ? 1 : 0);
  return hipGetLastError();
}
