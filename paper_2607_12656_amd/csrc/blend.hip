// Front-to-back alpha compositing over the per-tile depth-ordered lists
// (paper Sec. 3.1, compositing equation) and its reverse-order backward.
//
// One workgroup per tile.  Each wave64 owns an 8x8 pixel sub-tile (a
// 16x16 tile is four of them), one pixel per lane.  The workgroup stages a
// batch of 48-byte splat records in LDS (one gather per thread, one cache
// line per record); a wave skips every staged splat whose pixel span misses
// its sub-tile (a wave-uniform branch) and stops walking once all its pixels
// have terminated.  All lanes read the same LDS record at the same time
// (broadcast, no bank conflicts).  A pixel stops when T (1 - alpha~) would
// fall below 1e-4; the workgroup stops when every pixel has stopped.
//
// The backward walks the same list from each pixel's stop position towards
// the front, recovers T by division with the same (1 - alpha~) the forward
// multiplied by, and reduces the ten per-splat gradients of a wave with a
// transposing butterfly (17 shuffles for all ten values); ten lanes then
// issue one atomic each.
#include "sgs_internal.h"

namespace {

struct SplatLds {
  float4 a;  // px, py, A, B
  float4 b;  // C, opacity, spanx (x0 | x1 << 16), spany
  float4 c;  // r, g, b, mask
};

__device__ __forceinline__ bool span_meets(const SplatLds &s, int sx0, int sy0) {
  const uint32_t sx = __float_as_uint(s.b.z), sy = __float_as_uint(s.b.w);
  return (int)(sx & 0xFFFF) <= sx0 + 7 && (int)(sx >> 16) >= sx0 &&
         (int)(sy & 0xFFFF) <= sy0 + 7 && (int)(sy >> 16) >= sy0;
}

// alpha of splat `s` at pixel (px, py); the forward and the backward call the
// same code so both see bit-identical values.  Returns false when the pixel is
// outside the splat's pixel span, the exponent is positive or alpha < 1/255.
__device__ __forceinline__ bool splat_alpha(const SplatLds &s, int px, int py, float fx,
                                            float fy, bool &in_span, float &alpha, float &G,
                                            bool &clamped, float &dx, float &dy) {
  const uint32_t sx = __float_as_uint(s.b.z), sy = __float_as_uint(s.b.w);
  in_span = (px >= (int)(sx & 0xFFFF)) && (px <= (int)(sx >> 16)) &&
            (py >= (int)(sy & 0xFFFF)) && (py <= (int)(sy >> 16));
  if (!in_span) return false;
  dx = fx - s.a.x;
  dy = fy - s.a.y;
  const float q1 = s.a.z * dx * dx;
  const float q2 = s.b.x * dy * dy;
  const float q3 = s.a.w * dx * dy;
  const float power = -0.5f * (q1 + q2) - q3;
  if (power > 0.0f) return false;
  G = __expf(power);
  const float raw = s.b.y * G;
  clamped = raw > SGS_ALPHA_MAX;
  alpha = clamped ? SGS_ALPHA_MAX : raw;
  return alpha >= SGS_ALPHA_MIN;
}

template <int TW, int TH>
__global__ void __launch_bounds__(TW * TH)
k_blend_fwd(int64_t n, int W, int H, int GW, int64_t tiles_per_view,
            const uint2 *__restrict__ ranges, const uint32_t *__restrict__ vals,
            const float4 *__restrict__ rec, float *__restrict__ image,
            float *__restrict__ final_T, uint32_t *__restrict__ last,
            unsigned long long *__restrict__ eval_count) {
  constexpr int BS = TW * TH;
  constexpr int SUBW = TW / 8;
  __shared__ SplatLds sh[BS];
  __shared__ unsigned long long s_ev[BS / 64];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t tile = blockIdx.x;
  const int v = (int)(tile / tiles_per_view);
  const int t = (int)(tile - (int64_t)v * tiles_per_view);
  const int tx = t % GW, ty = t / GW;
  const int sx0 = tx * TW + (wave % SUBW) * 8;
  const int sy0 = ty * TH + (wave / SUBW) * 8;
  const int px = sx0 + (lane & 7);
  const int py = sy0 + (lane >> 3);
  const bool inside = px < W && py < H;
  const float fx = (float)px, fy = (float)py;
  const uint2 rg = ranges[tile];
  const int64_t base = (int64_t)v * n;
  float T = 1.0f, C0 = 0.0f, C1 = 0.0f, C2 = 0.0f;
  bool done = !inside;
  uint32_t stop = rg.y - rg.x;
  uint32_t evals = 0;
  for (uint32_t b = rg.x; b < rg.y; b += BS) {
    if (__syncthreads_count(done ? 1 : 0) == BS) break;
    const uint32_t e = b + threadIdx.x;
    if (e < rg.y) {
      const float4 *r = rec + 3 * (base + vals[e]);
      sh[threadIdx.x].a = r[0];
      sh[threadIdx.x].b = r[1];
      sh[threadIdx.x].c = r[2];
    }
    __syncthreads();
    if (__ballot(!done) == 0ull) continue;
    const int cnt = (int)min((uint32_t)BS, rg.y - b);
    for (int k = 0; k < cnt; ++k) {
      const SplatLds &s = sh[k];
      if (!span_meets(s, sx0, sy0)) continue;
      if (!done) {
        bool in_span, clamped;
        float alpha, G, dx, dy;
        const bool ok = splat_alpha(s, px, py, fx, fy, in_span, alpha, G, clamped, dx, dy);
        evals += in_span ? 1u : 0u;
        if (ok) {
          const float at = s.c.w * alpha;
          const float Tn = T * (1.0f - at);
          if (Tn < SGS_T_MIN) {
            done = true;
            stop = b - rg.x + (uint32_t)k;
          } else {
            const float w = at * T;
            C0 = fmaf(s.c.x, w, C0);
            C1 = fmaf(s.c.y, w, C1);
            C2 = fmaf(s.c.z, w, C2);
            T = Tn;
          }
        }
      }
      if (__ballot(!done) == 0ull) break;
    }
  }
  if (inside) {
    const int64_t pix = (int64_t)py * W + px;
    const int64_t plane = (int64_t)W * H;
    image[((int64_t)v * 3 + 0) * plane + pix] = C0;
    image[((int64_t)v * 3 + 1) * plane + pix] = C1;
    image[((int64_t)v * 3 + 2) * plane + pix] = C2;
    final_T[(int64_t)v * plane + pix] = T;
    last[(int64_t)v * plane + pix] = stop;
  }
  if (eval_count) {
    unsigned long long ev = evals;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) ev += __shfl_xor(ev, o, 64);
    if (lane == 0) s_ev[wave] = ev;
    __syncthreads();
    if (threadIdx.x == 0) {
      unsigned long long tot = 0;
      for (int w = 0; w < BS / 64; ++w) tot += s_ev[w];
      if (tot) atomicAdd(eval_count, tot);
    }
  }
}

// Sum each of v[0..15] over the 64 lanes of the wave.  After the call lane L
// holds the total of value ((L>>5)&1)*8 + ((L>>4)&1)*4 + ((L>>3)&1)*2 +
// ((L>>2)&1) (lanes sharing L>>2 hold the same total).
__device__ __forceinline__ float wave_transpose_sum16(float v[16], int lane) {
  float r8[8], r4[4], r2[2];
  {
    const bool hi = lane & 32;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const float mine = hi ? v[8 + i] : v[i];
      const float send = hi ? v[i] : v[8 + i];
      r8[i] = mine + __shfl_xor(send, 32, 64);
    }
  }
  {
    const bool hi = lane & 16;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const float mine = hi ? r8[4 + i] : r8[i];
      const float send = hi ? r8[i] : r8[4 + i];
      r4[i] = mine + __shfl_xor(send, 16, 64);
    }
  }
  {
    const bool hi = lane & 8;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const float mine = hi ? r4[2 + i] : r4[i];
      const float send = hi ? r4[i] : r4[2 + i];
      r2[i] = mine + __shfl_xor(send, 8, 64);
    }
  }
  float x;
  {
    const bool hi = lane & 4;
    const float mine = hi ? r2[1] : r2[0];
    const float send = hi ? r2[0] : r2[1];
    x = mine + __shfl_xor(send, 4, 64);
  }
  x += __shfl_xor(x, 2, 64);
  x += __shfl_xor(x, 1, 64);
  return x;
}

template <int TW, int TH>
__global__ void __launch_bounds__(TW * TH)
k_blend_bwd(int64_t n, int W, int H, int GW, int64_t tiles_per_view,
            const uint2 *__restrict__ ranges, const uint32_t *__restrict__ vals,
            const float4 *__restrict__ rec, const float *__restrict__ final_T,
            const uint32_t *__restrict__ last, const float *__restrict__ dimg,
            float *__restrict__ sgrad) {
  constexpr int BS = TW * TH;
  constexpr int SUBW = TW / 8;
  __shared__ SplatLds sh[BS];
  __shared__ uint32_t s_gid[BS];
  __shared__ uint32_t s_max[BS / 64];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t tile = blockIdx.x;
  const int v = (int)(tile / tiles_per_view);
  const int t = (int)(tile - (int64_t)v * tiles_per_view);
  const int tx = t % GW, ty = t / GW;
  const int sx0 = tx * TW + (wave % SUBW) * 8;
  const int sy0 = ty * TH + (wave / SUBW) * 8;
  const int px = sx0 + (lane & 7);
  const int py = sy0 + (lane >> 3);
  const bool inside = px < W && py < H;
  const float fx = (float)px, fy = (float)py;
  const uint2 rg = ranges[tile];
  const int64_t base = (int64_t)v * n;
  const int64_t plane = (int64_t)W * H;
  const int64_t pix = (int64_t)py * W + px;
  uint32_t my_last = 0;
  float T = 1.0f, g0 = 0.f, g1 = 0.f, g2 = 0.f;
  if (inside) {
    my_last = last[(int64_t)v * plane + pix];
    T = final_T[(int64_t)v * plane + pix];
    g0 = dimg[((int64_t)v * 3 + 0) * plane + pix];
    g1 = dimg[((int64_t)v * 3 + 1) * plane + pix];
    g2 = dimg[((int64_t)v * 3 + 2) * plane + pix];
  }
  // furthest list position reached by any pixel of the wave / workgroup
  uint32_t wave_reach = my_last;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) wave_reach = max(wave_reach, (uint32_t)__shfl_xor(wave_reach, o, 64));
  if (lane == 0) s_max[wave] = wave_reach;
  __syncthreads();
  uint32_t reach = 0;
  for (int w = 0; w < BS / 64; ++w) reach = max(reach, s_max[w]);
  if (reach == 0) return;
  float B0 = 0.f, B1 = 0.f, B2 = 0.f;  // colour seen behind the current splat
  const uint32_t nbatch = (reach + BS - 1) / BS;
  const int vidx = ((lane >> 5) & 1) * 8 + ((lane >> 4) & 1) * 4 + ((lane >> 3) & 1) * 2 +
                   ((lane >> 2) & 1);
  for (int bi = (int)nbatch - 1; bi >= 0; --bi) {
    const uint32_t p0 = (uint32_t)bi * BS;
    const int cnt = (int)min((uint32_t)BS, rg.y - rg.x - p0);
    __syncthreads();
    if ((int)threadIdx.x < cnt) {
      const uint32_t gi = vals[rg.x + p0 + threadIdx.x];
      const float4 *r = rec + 3 * (base + gi);
      s_gid[threadIdx.x] = gi;
      sh[threadIdx.x].a = r[0];
      sh[threadIdx.x].b = r[1];
      sh[threadIdx.x].c = r[2];
    }
    __syncthreads();
    if (p0 >= wave_reach) continue;
    const int kstart = (int)min((uint32_t)cnt, wave_reach - p0) - 1;
    for (int k = kstart; k >= 0; --k) {
      const SplatLds &s = sh[k];
      if (!span_meets(s, sx0, sy0)) continue;
      const uint32_t pos = p0 + (uint32_t)k;
      bool in_span = false, clamped = false, ok = false;
      float alpha = 0.f, G = 0.f, dx = 0.f, dy = 0.f;
      if (inside && pos < my_last)
        ok = splat_alpha(s, px, py, fx, fy, in_span, alpha, G, clamped, dx, dy);
      if (__ballot(ok) == 0ull) continue;
      float d[16];
#pragma unroll
      for (int q = 0; q < 16; ++q) d[q] = 0.0f;
      if (ok) {
        const float m = s.c.w;
        const float at = m * alpha;
        const float Tb = (at == 0.0f) ? T : T / (1.0f - at);
        const float dat = Tb * (g0 * (s.c.x - B0) + g1 * (s.c.y - B1) + g2 * (s.c.z - B2));
        const float wcol = at * Tb;
        d[6] = g0 * wcol;
        d[7] = g1 * wcol;
        d[8] = g2 * wcol;
        d[9] = dat * alpha;
        if (!clamped) {
          const float dal = m * dat;
          d[5] = dal * G;
          const float dp = dal * alpha;
          d[0] = dp * (s.a.z * dx + s.a.w * dy);
          d[1] = dp * (s.a.w * dx + s.b.x * dy);
          d[2] = -0.5f * dp * dx * dx;
          d[3] = -dp * dx * dy;
          d[4] = -0.5f * dp * dy * dy;
        }
        B0 = s.c.x * at + (1.0f - at) * B0;
        B1 = s.c.y * at + (1.0f - at) * B1;
        B2 = s.c.z * at + (1.0f - at) * B2;
        T = Tb;
      }
      const float tot = wave_transpose_sum16(d, lane);
      if ((lane & 3) == 0 && vidx < 10 && tot != 0.0f)
        unsafeAtomicAdd(sgrad + (base + s_gid[k]) * SGS_SGRAD + vidx, tot);
    }
  }
}

template <int TW, int TH>
hipError_t fwd_t(sgs_ctx *c, float *image, float *final_T, uint32_t *last, uint64_t *ec) {
  SgsProfScope ps(c, SGS_PROF_BLEND_FWD);
  const uint32_t *vals = c->pair_val[c->pair_sorted_buf];
  k_blend_fwd<TW, TH><<<(unsigned)c->total_tiles, TW * TH, 0, c->stream>>>(
      c->n, c->W, c->H, c->GW, c->tiles_per_view, c->ranges, vals, c->rec, image, final_T, last,
      (unsigned long long *)ec);
  return hipGetLastError();
}

template <int TW, int TH>
hipError_t bwd_t(sgs_ctx *c, const float *final_T, const uint32_t *last, const float *dimg) {
  SgsProfScope ps(c, SGS_PROF_BLEND_BWD);
  const uint32_t *vals = c->pair_val[c->pair_sorted_buf];
  k_blend_bwd<TW, TH><<<(unsigned)c->total_tiles, TW * TH, 0, c->stream>>>(
      c->n, c->W, c->H, c->GW, c->tiles_per_view, c->ranges, vals, c->rec, final_T, last, dimg,
      c->splat_grad);
  return hipGetLastError();
}

__global__ void k_zero_f32(float *__restrict__ p, int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = 0.0f;
}

}  // namespace

hipError_t launch_blend_fwd(sgs_ctx *c, float *image, float *final_T, uint32_t *last,
                            uint64_t *eval_count) {
  if (c->TW == 16 && c->TH == 16) return fwd_t<16, 16>(c, image, final_T, last, eval_count);
  if (c->TW == 8 && c->TH == 8) return fwd_t<8, 8>(c, image, final_T, last, eval_count);
  if (c->TW == 32 && c->TH == 8) return fwd_t<32, 8>(c, image, final_T, last, eval_count);
  return hipErrorInvalidValue;
}

hipError_t launch_blend_bwd(sgs_ctx *c, const float *final_T, const uint32_t *last,
                            const float *dimg) {
  const int64_t words = c->vn * SGS_SGRAD;
  {
    SgsProfScope ps(c, SGS_PROF_GRAD_CLEAR);
    k_zero_f32<<<sgs_blocks(words, 256), 256, 0, c->stream>>>(c->splat_grad, words);
  }
  if (c->TW == 16 && c->TH == 16) return bwd_t<16, 16>(c, final_T, last, dimg);
  if (c->TW == 8 && c->TH == 8) return bwd_t<8, 8>(c, final_T, last, dimg);
  if (c->TW == 32 && c->TH == 8) return bwd_t<32, 8>(c, final_T, last, dimg);
  return hipErrorInvalidValue;
}
