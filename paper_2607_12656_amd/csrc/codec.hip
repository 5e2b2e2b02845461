// Channel-wise fixed-length coding of the quantized parameters (paper
// Sec. 3.4.1: every channel is stored with the fixed bit width its
// quantization precision implies, plus per-channel metadata).  The codes are
// the quantizer's decisions k_ij = rint(y_ij / q_j) of the kept Gaussians.
//
// Stream: header per channel {q_j, kmin_j, w_j}; payload channel-major, kept
// Gaussians in index order, each (k_ij - kmin_j) in w_j bits LSB first, bit b
// of the stream being bit (b & 7) of byte b >> 3 (so bit b & 31 of 32-bit
// word b >> 5 on a little-endian device); w_j = ceil(log2(kmax_j - kmin_j
// + 1)) over the kept Gaussians (0 for a constant channel).
//
// Encoding: (1) per chunk of 4096 Gaussians and channel, the code range of
// the kept ones, and per chunk the kept count; (2) one block finishes the
// ranges, widths, the chunk ranks of the kept Gaussians and each channel's
// bit offset; (3) the payload words needed are cleared; (4) per chunk and
// channel a block ranks its kept Gaussians, ORs their bit fields into LDS
// words and writes them out (plain stores inside its bit span, atomic OR on
// the first and last word, which neighbouring spans share).  Decoding reads
// each value's one or two words.
#include "sgs_internal.h"

namespace {

constexpr int kCThreads = 256;
constexpr int kCItems = 16;                     // Gaussians per thread
constexpr int kCChunk = kCThreads * kCItems;    // Gaussians per chunk
constexpr int kCWords = kCChunk + 2;            // LDS words of one chunk's span (w <= 32)

// scratch layout (uint32 words): [0, 2*59*nc) chunk ranges (min, max) as
// [chunk][channel][2]; [2*59*nc, 2*59*nc + nc) chunk kept counts, then
// chunk ranks (nc), then per channel bit offsets as uint64 (2*59 words).
__device__ __forceinline__ int32_t code_of(float y, float q, bool &ok) {
  const float k = rintf(__fdiv_rn(y, q));
  ok = k >= -2147483648.0f && k < 2147483648.0f;
  return ok ? (int32_t)k : 0;
}

__global__ void __launch_bounds__(kCThreads)
k_fl_stats(int64_t n, int64_t npad, const float *__restrict__ y, const float *__restrict__ q,
           const uint8_t *__restrict__ hard, int nc, uint32_t *__restrict__ scr,
           uint32_t *__restrict__ flags) {
  __shared__ int32_t s_lo[kCThreads / 64], s_hi[kCThreads / 64];
  __shared__ uint32_t s_cnt[kCThreads / 64];
  const int j = blockIdx.y;
  const int64_t chunk = blockIdx.x;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t base = chunk * kCChunk;
  if (j == SGS_NCH) {
    uint32_t cnt = 0;
    for (int e = 0; e < kCItems; ++e) {
      const int64_t i = base + (int64_t)e * kCThreads + threadIdx.x;
      if (i < n && hard[i]) ++cnt;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o, 64);
    if (lane == 0) s_cnt[wave] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) {
      uint32_t t = 0;
      for (int w = 0; w < kCThreads / 64; ++w) t += s_cnt[w];
      scr[2 * SGS_NCH * nc + chunk] = t;
    }
    return;
  }
  const float qj = q[j];
  int32_t lo = INT32_MAX, hi = INT32_MIN;
  bool bad = false;
  for (int e = 0; e < kCItems; ++e) {
    const int64_t i = base + (int64_t)e * kCThreads + threadIdx.x;
    if (i < n && hard[i]) {
      bool ok;
      const int32_t k = code_of(y[j * npad + i], qj, ok);
      bad |= !ok;
      lo = min(lo, k);
      hi = max(hi, k);
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    lo = min(lo, __shfl_xor(lo, o, 64));
    hi = max(hi, __shfl_xor(hi, o, 64));
  }
  if (bad) atomicOr(flags, 1u);
  if (lane == 0) {
    s_lo[wave] = lo;
    s_hi[wave] = hi;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kCThreads / 64; ++w) {
      lo = min(lo, s_lo[w]);
      hi = max(hi, s_hi[w]);
    }
    uint32_t *d = scr + 2 * (chunk * SGS_NCH + j);
    d[0] = (uint32_t)lo;
    d[1] = (uint32_t)hi;
  }
}

// One block: code ranges -> widths and header; exclusive scan of the chunk
// kept counts; channel bit offsets; totals out[0] = payload bits,
// out[1] = kept Gaussians.
__global__ void __launch_bounds__(kCThreads)
k_fl_plan(int nc, const float *__restrict__ q, uint32_t *__restrict__ scr,
          sgs_fl_channel *__restrict__ hdr, int64_t *__restrict__ out,
          uint32_t *__restrict__ flags, int64_t cap_words) {
  __shared__ int32_t s_w[SGS_NCH];
  __shared__ uint32_t s_part[kCThreads];
  __shared__ uint64_t s_kept;
  const int t = threadIdx.x;
  uint32_t *cnt = scr + 2 * SGS_NCH * nc;
  uint32_t *rank = cnt + nc;
  uint64_t *off = (uint64_t *)(rank + nc);  // 120 nc words in: 8-byte aligned
  // chunk ranks: thread t scans chunks [t*per, (t+1)*per) serially
  const int per = (nc + kCThreads - 1) / kCThreads;
  const int a = min(nc, t * per), b = min(nc, a + per);
  uint32_t s = 0;
  for (int c = a; c < b; ++c) s += cnt[c];
  s_part[t] = s;
  __syncthreads();
  if (t == 0) {
    uint64_t run = 0;
    for (int k = 0; k < kCThreads; ++k) {
      const uint32_t v = s_part[k];
      s_part[k] = (uint32_t)run;
      run += v;
    }
    s_kept = run;
  }
  __syncthreads();
  uint32_t r = s_part[t];
  for (int c = a; c < b; ++c) {
    rank[c] = r;
    r += cnt[c];
  }
  if (t < SGS_NCH) {
    int32_t lo = INT32_MAX, hi = INT32_MIN;
    for (int c = 0; c < nc; ++c) {
      lo = min(lo, (int32_t)scr[2 * (c * SGS_NCH + t)]);
      hi = max(hi, (int32_t)scr[2 * (c * SGS_NCH + t) + 1]);
    }
    int w = 0;
    int32_t kmin = 0;
    if (lo <= hi) {  // some Gaussian is kept
      const uint64_t K = (uint64_t)((int64_t)hi - (int64_t)lo) + 1;
      while (((uint64_t)1 << w) < K) ++w;
      kmin = lo;
    }
    s_w[t] = w;
    hdr[t].q = q[t];
    hdr[t].kmin = kmin;
    hdr[t].width = w;
  }
  __syncthreads();
  if (t == 0) {
    const uint64_t kept = s_kept;
    uint64_t o = 0;
    for (int j = 0; j < SGS_NCH; ++j) {
      off[j] = o;
      o += kept * (uint64_t)s_w[j];
    }
    out[0] = (int64_t)o;
    out[1] = (int64_t)kept;
    if ((int64_t)((o + 31) / 32) > cap_words) atomicOr(flags, 2u);
  }
}

__global__ void k_fl_flags_reset(uint32_t *__restrict__ flags) {
  if (threadIdx.x == 0) *flags = 0u;
}

__global__ void k_fl_zero(uint32_t *__restrict__ payload, int64_t cap_words,
                          const int64_t *__restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t need = min(cap_words, (out[0] + 31) / 32);
  if (i < need) payload[i] = 0u;
}

__global__ void __launch_bounds__(kCThreads)
k_fl_pack(int64_t n, int64_t npad, const float *__restrict__ y, const float *__restrict__ q,
          const uint8_t *__restrict__ hard, int nc, const uint32_t *__restrict__ scr,
          const sgs_fl_channel *__restrict__ hdr, uint32_t *__restrict__ payload,
          int64_t cap_words) {
  __shared__ uint32_t s_words[kCWords];
  __shared__ uint32_t s_wave[kCThreads / 64];
  const int j = blockIdx.y;
  const int64_t chunk = blockIdx.x;
  const int w = hdr[j].width;
  if (w == 0) return;
  const uint32_t *cnt = scr + 2 * SGS_NCH * nc;
  const uint32_t *rank = cnt + nc;
  const uint64_t *off = (const uint64_t *)(rank + nc);
  const uint32_t nkept = cnt[chunk];
  if (nkept == 0) return;
  const uint64_t p0 = off[j] + (uint64_t)rank[chunk] * (uint64_t)w;  // first bit of the span
  const uint64_t wbase = p0 >> 5;
  const uint64_t wlast = (p0 + (uint64_t)nkept * w - 1) >> 5;
  const int nw = (int)(wlast - wbase + 1);
  for (int k = threadIdx.x; k < nw; k += kCThreads) s_words[k] = 0u;
  // thread t owns Gaussians base + 16t .. base + 16t + 15 (index order)
  const int64_t i0 = chunk * kCChunk + (int64_t)threadIdx.x * kCItems;
  uint32_t mine = 0;
#pragma unroll
  for (int e = 0; e < kCItems; ++e) mine += (i0 + e < n && hard[i0 + e]) ? 1u : 0u;
  // block exclusive scan of the per-thread counts
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t x = mine;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t v = __shfl_up(x, o, 64);
    if (lane >= o) x += v;
  }
  if (lane == 63) s_wave[wave] = x;
  __syncthreads();
  uint32_t before = x - mine;
  for (int k = 0; k < wave; ++k) before += s_wave[k];
  const float qj = q[j];
  const int32_t kmin = hdr[j].kmin;
  const uint64_t mask = w == 32 ? 0xFFFFFFFFull : ((1ull << w) - 1ull);
  float yv[kCItems];
  const float *row = y + j * npad + i0;
  if (i0 + kCItems <= n) {  // 64-byte aligned: npad % 64 == 0, 16-byte aligned rows
#pragma unroll
    for (int e = 0; e < kCItems; e += 4) {
      const float4 v4 = *reinterpret_cast<const float4 *>(row + e);
      yv[e] = v4.x;
      yv[e + 1] = v4.y;
      yv[e + 2] = v4.z;
      yv[e + 3] = v4.w;
    }
  } else {
#pragma unroll
    for (int e = 0; e < kCItems; ++e) yv[e] = i0 + e < n ? row[e] : 0.0f;
  }
#pragma unroll
  for (int e = 0; e < kCItems; ++e) {
    const int64_t i = i0 + e;
    if (i < n && hard[i]) {
      bool ok;
      const int32_t k = code_of(yv[e], qj, ok);
      const uint64_t v = (uint64_t)((int64_t)k - (int64_t)kmin) & mask;
      const uint64_t p = p0 + (uint64_t)before * w;   // bit position in the stream
      const int widx = (int)((p >> 5) - wbase);
      const int sh = (int)(p & 31);
      atomicOr(&s_words[widx], (uint32_t)(v << sh));
      if (sh + w > 32) atomicOr(&s_words[widx + 1], (uint32_t)(v >> (32 - sh)));
      ++before;
    }
  }
  __syncthreads();
  for (int k = threadIdx.x; k < nw; k += kCThreads) {
    const uint64_t gw = wbase + k;
    if ((int64_t)gw >= cap_words) break;
    const uint32_t val = s_words[k];
    if (k == 0 || k == nw - 1) {
      if (val) atomicOr(&payload[gw], val);  // shared with the neighbouring span
    } else {
      payload[gw] = val;
    }
  }
}

// Decode: rank r of channel j -> out[j][r] = fl32((kmin + v) q).
__global__ void __launch_bounds__(kCThreads)
k_fl_unpack(int64_t kept, int64_t out_pad, const sgs_fl_channel *__restrict__ hdr,
            const uint32_t *__restrict__ payload, int64_t words, float *__restrict__ out) {
  __shared__ uint64_t s_off;
  const int j = blockIdx.y;
  if (threadIdx.x == 0) {
    uint64_t o = 0;
    for (int c = 0; c < j; ++c) o += (uint64_t)kept * (uint64_t)hdr[c].width;
    s_off = o;
  }
  __syncthreads();
  const int w = hdr[j].width;
  const float qj = hdr[j].q;
  const int32_t kmin = hdr[j].kmin;
  const uint64_t mask = w == 32 ? 0xFFFFFFFFull : ((1ull << w) - 1ull);
  for (int e = 0; e < kCItems; ++e) {
    const int64_t r = (int64_t)blockIdx.x * kCChunk + (int64_t)e * kCThreads + threadIdx.x;
    if (r >= kept) break;
    uint64_t v = 0;
    if (w > 0) {
      const uint64_t p = s_off + (uint64_t)r * w;
      const int64_t wi = (int64_t)(p >> 5);
      const uint64_t lo = wi < words ? payload[wi] : 0u;
      const uint64_t hi = wi + 1 < words ? payload[wi + 1] : 0u;
      v = (((hi << 32) | lo) >> (p & 31)) & mask;
    }
    const int64_t k = (int64_t)kmin + (int64_t)v;
    out[j * out_pad + r] = (float)k * qj;
  }
}

}  // namespace

int64_t fl_scratch_words(int64_t n) {
  const int64_t nc = (n + kCChunk - 1) / kCChunk;
  return 2 * SGS_NCH * nc + 2 * nc + 2 * SGS_NCH + 2;
}

hipError_t launch_fl_encode(sgs_ctx *c, const float *params, const float *q,
                            const uint8_t *hard, sgs_fl_channel *hdr, uint32_t *payload,
                            int64_t cap_words, int64_t *out) {
  SgsProfScope ps(c, SGS_PROF_CODEC);
  const int nc = (int)((c->n + kCChunk - 1) / kCChunk);
  if (fl_scratch_words(c->n) > c->fl_tmp_words) return hipErrorInvalidValue;
  uint32_t *scr = c->fl_tmp;
  uint32_t *flags = (uint32_t *)(out + 2);
  k_fl_flags_reset<<<1, 64, 0, c->stream>>>(flags);
  k_fl_stats<<<dim3(nc, SGS_NCH + 1), kCThreads, 0, c->stream>>>(c->n, c->npad, params, q, hard,
                                                                 nc, scr, flags);
  k_fl_plan<<<1, kCThreads, 0, c->stream>>>(nc, q, scr, hdr, out, flags, cap_words);
  if (cap_words > 0)
    k_fl_zero<<<sgs_blocks(cap_words, 256), 256, 0, c->stream>>>(payload, cap_words, out);
  k_fl_pack<<<dim3(nc, SGS_NCH), kCThreads, 0, c->stream>>>(c->n, c->npad, params, q, hard, nc,
                                                            scr, hdr, payload, cap_words);
  return hipGetLastError();
}

hipError_t launch_fl_decode(sgs_ctx *c, const sgs_fl_channel *hdr, const uint32_t *payload,
                            int64_t words, int64_t kept, int64_t out_pad, float *out) {
  SgsProfScope ps(c, SGS_PROF_CODEC);
  const int64_t nb = (kept + kCChunk - 1) / kCChunk;
  if (nb > 0)
    k_fl_unpack<<<dim3((unsigned)nb, SGS_NCH), kCThreads, 0, c->stream>>>(kept, out_pad, hdr,
                                                                          payload, words, out);
  return hipGetLastError();
}
