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
// Encoding: (1) per chunk of 4096 Gaussians and channel, the smallest and
// largest kept value (the code map y -> rint(y / q) is monotone in y, so the
// code range is the range of the codes of these two values), and per chunk
// the kept count; (2) one block folds the chunk ranges into widths and the
// header, ranks the chunks' kept Gaussians and places each channel's bit
// offset; (3) one thread per chunk span clears the span's two end words (the
// only words two spans share); (4) per chunk and channel a block ranks its
// kept Gaussians and stores their values compacted in LDS; each thread then
// builds whole output words from the values overlapping them and writes its
// span (plain stores inside, atomic OR on the two shared end words).  Decoding stages a block's span of
// payload words in LDS and reads each value's one or two words there.
#include "sgs_internal.h"

namespace {

constexpr int kCThreads = 256;
constexpr int kCItems = 16;                     // Gaussians per thread (one 16-byte mask load)
constexpr int kCChunk = kCThreads * kCItems;    // Gaussians per chunk
constexpr int kCWords = kCChunk + 2;            // LDS words of one chunk's span (w <= 32)
constexpr int kPlanThreads = 1024;

// scratch layout (uint32 words): [0, 118) per-channel bit offsets (uint64);
// [118, 177) per-channel widths; [177, 177 + nc) chunk kept counts;
// [177 + nc, 177 + 2 nc) chunk ranks; then per channel and chunk the smallest
// and largest kept value, [59][nc][2] floats (8-byte aligned).
constexpr int kOffW = 0, kWidW = 2 * SGS_NCH, kCntW = 3 * SGS_NCH;
__host__ __device__ constexpr int64_t range_word(int64_t nc) { return (kCntW + 2 * nc + 1) & ~1LL; }


// thread t of a chunk's block: Gaussians i0 .. i0 + 15; mask bytes and the
// channel-j values (0 past n)
__device__ __forceinline__ void load_items(int64_t n, const float *__restrict__ row,
                                           const uint8_t *__restrict__ hard, int64_t i0,
                                           float (&yv)[kCItems], uint32_t &keep) {
  keep = 0;
  if (i0 + kCItems <= n) {  // rows 64-byte aligned here (npad % 64 == 0, 16-byte aligned rows)
    const uint4 m = *reinterpret_cast<const uint4 *>(hard + i0);
    keep = sgs_nonzero_nibble(m.x) | sgs_nonzero_nibble(m.y) << 4 | sgs_nonzero_nibble(m.z) << 8 |
           sgs_nonzero_nibble(m.w) << 12;
#pragma unroll
    for (int e = 0; e < kCItems; e += 4) {
      const float4 v4 = *reinterpret_cast<const float4 *>(row + i0 + e);
      yv[e] = v4.x;
      yv[e + 1] = v4.y;
      yv[e + 2] = v4.z;
      yv[e + 3] = v4.w;
    }
  } else {
#pragma unroll
    for (int e = 0; e < kCItems; ++e) {
      const bool in = i0 + e < n;
      yv[e] = in ? row[i0 + e] : 0.0f;
      keep |= (in && hard[i0 + e]) ? 1u << e : 0u;
    }
  }
}


__global__ void __launch_bounds__(kCThreads)
k_fl_stats(int64_t n, int64_t npad, const float *__restrict__ y,
           const uint8_t *__restrict__ hard, int nc, uint32_t *__restrict__ scr) {
  __shared__ float s_lo[kCThreads / 64], s_hi[kCThreads / 64];
  __shared__ uint32_t s_cnt[kCThreads / 64];
  const int j = blockIdx.y;
  const int64_t chunk = blockIdx.x;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t i0 = chunk * kCChunk + (int64_t)threadIdx.x * kCItems;
  float yv[kCItems];
  uint32_t keep;
  load_items(n, y + j * npad, hard, i0, yv, keep);
  float lo = __builtin_inff(), hi = -__builtin_inff();
#pragma unroll
  for (int e = 0; e < kCItems; ++e) {
    if (keep & (1u << e)) {
      lo = fminf(lo, yv[e]);
      hi = fmaxf(hi, yv[e]);
    }
  }
  uint32_t cnt = __popc(keep);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    lo = fminf(lo, __shfl_xor(lo, o, 64));
    hi = fmaxf(hi, __shfl_xor(hi, o, 64));
    cnt += __shfl_xor(cnt, o, 64);
  }
  if (lane == 0) {
    s_lo[wave] = lo;
    s_hi[wave] = hi;
    s_cnt[wave] = cnt;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kCThreads / 64; ++w) {
      lo = fminf(lo, s_lo[w]);
      hi = fmaxf(hi, s_hi[w]);
      cnt += s_cnt[w];
    }
    // lo > hi: nothing kept here (or only NaN, which the packing pass flags)
    float *rg = reinterpret_cast<float *>(scr + range_word(nc)) + 2 * ((int64_t)j * nc + chunk);
    rg[0] = lo;
    rg[1] = hi;
    if (j == 0) scr[kCntW + chunk] = cnt;
  }
}

// inclusive scan over a block of kPlanThreads threads (wave scans + wave totals)
__device__ __forceinline__ uint32_t block_scan_incl(uint32_t x, uint32_t *s_wave) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t v = __shfl_up(x, o, 64);
    if (lane >= o) x += v;
  }
  if (lane == 63) s_wave[wave] = x;
  __syncthreads();
  if (wave == 0) {
    uint32_t t = lane < kPlanThreads / 64 ? s_wave[lane] : 0u;
#pragma unroll
    for (int o = 1; o < kPlanThreads / 64; o <<= 1) {
      const uint32_t v = __shfl_up(t, o, 64);
      if (lane >= o) t += v;
    }
    if (lane < kPlanThreads / 64) s_wave[lane] = t;
  }
  __syncthreads();
  const uint32_t r = x + (wave > 0 ? s_wave[wave - 1] : 0u);
  __syncthreads();  // s_wave is reused by the next call
  return r;
}

// One block: chunk ranks (exclusive scan of the kept counts), widths and
// header, channel bit offsets, totals info[0] = payload bits, info[1] = kept,
// and the cleared end words of every span.
__global__ void __launch_bounds__(kPlanThreads)
k_fl_plan(int nc, const float *__restrict__ q, uint32_t *__restrict__ scr,
          sgs_fl_channel *__restrict__ hdr, int64_t *__restrict__ info, int64_t cap_words) {
  __shared__ uint32_t s_wave[kPlanThreads / 64];
  __shared__ uint32_t s_carry;
  __shared__ int32_t s_w[SGS_NCH];
  __shared__ float s_lo[SGS_NCH], s_hi[SGS_NCH];
  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  uint32_t *cnt = scr + kCntW;
  uint32_t *rank = cnt + nc;
  uint64_t *off = reinterpret_cast<uint64_t *>(scr + kOffW);
  uint32_t *flags = reinterpret_cast<uint32_t *>(info + 2);
  if (t == 0) {
    s_carry = 0;
    info[2] = 0;
  }
  // channel ranges: wave v folds channels v, v + 16, ..., lanes striding over chunks
  const float *rg = reinterpret_cast<const float *>(scr + range_word(nc));
  for (int j = wave; j < SGS_NCH; j += kPlanThreads / 64) {
    float lo = __builtin_inff(), hi = -__builtin_inff();
    for (int c = lane; c < nc; c += 64) {
      const float2 r = reinterpret_cast<const float2 *>(rg)[(int64_t)j * nc + c];
      lo = fminf(lo, r.x);
      hi = fmaxf(hi, r.y);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      lo = fminf(lo, __shfl_xor(lo, o, 64));
      hi = fmaxf(hi, __shfl_xor(hi, o, 64));
    }
    if (lane == 0) {
      s_lo[j] = lo;
      s_hi[j] = hi;
    }
  }
  __syncthreads();
  for (int b = 0; b < nc; b += kPlanThreads) {
    const int c = b + t;
    const uint32_t v = c < nc ? cnt[c] : 0u;
    const uint32_t inc = block_scan_incl(v, s_wave);
    const uint32_t carry = s_carry;
    if (c < nc) rank[c] = carry + inc - v;
    __syncthreads();
    if (t == kPlanThreads - 1) s_carry = carry + inc;
    __syncthreads();
  }
  const uint64_t kept = s_carry;
  if (t < SGS_NCH) {
    int w = 0;
    int32_t kmin = 0;
    const float lo = s_lo[t], hi = s_hi[t];
    if (kept > 0) {
      bool ok_lo = false, ok_hi = false;
      if (lo <= hi) {
        const float qt = q[t];
        const int32_t a = sgs_code_of(lo, qt, ok_lo);
        const int32_t z = sgs_code_of(hi, qt, ok_hi);
        kmin = min(a, z);  // q < 0 reverses the order
        const uint64_t K = (uint64_t)((int64_t)max(a, z) - (int64_t)kmin) + 1;
        w = K <= 1 ? 0 : 64 - __clzll((long long)(K - 1));
      }
      if (!ok_lo || !ok_hi) atomicOr(flags, 1u);
    }
    s_w[t] = w;
    scr[kWidW + t] = (uint32_t)w;
    hdr[t].q = q[t];
    hdr[t].kmin = kmin;
    hdr[t].width = w;
  }
  __syncthreads();
  if (t < 64) {  // exclusive scan of kept * w over the channels
    uint64_t x = t < SGS_NCH ? kept * (uint64_t)s_w[t] : 0ull;
    const uint64_t mine = x;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint64_t v = __shfl_up(x, o, 64);
      if (t >= o) x += v;
    }
    if (t < SGS_NCH) off[t] = x - mine;
    if (t == 63) {
      info[0] = (int64_t)x;
      info[1] = (int64_t)kept;
      if ((int64_t)((x + 31) / 32) > cap_words) atomicOr(flags, 2u);
    }
  }
}

// One thread per chunk span: clear its first and last payload words.
__global__ void k_fl_edges(int nc, const uint32_t *__restrict__ scr,
                           uint32_t *__restrict__ payload, int64_t cap_words) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= (int64_t)nc * SGS_NCH) return;
  const int j = (int)(s / nc), c = (int)(s - (int64_t)j * nc);
  const uint64_t w = scr[kWidW + j];
  const uint32_t m = scr[kCntW + c];
  if (w == 0 || m == 0) return;
  const uint64_t p0 = reinterpret_cast<const uint64_t *>(scr + kOffW)[j] +
                      (uint64_t)scr[kCntW + nc + c] * w;
  const int64_t w0 = (int64_t)(p0 >> 5), w1 = (int64_t)((p0 + m * w - 1) >> 5);
  if (w0 < cap_words) payload[w0] = 0u;
  if (w1 < cap_words) payload[w1] = 0u;
}

__global__ void __launch_bounds__(kCThreads)
k_fl_pack(int64_t n, int64_t npad, const float *__restrict__ y, const uint8_t *__restrict__ hard,
          int nc, const uint32_t *__restrict__ scr, const sgs_fl_channel *__restrict__ hdr,
          uint32_t *__restrict__ payload, int64_t cap_words, int64_t *__restrict__ info) {
  __shared__ uint32_t s_vals[kCChunk + 64];  // kept values (k - kmin) by rank; then per-lane discards
  __shared__ uint32_t s_wave[kCThreads / 64];
  const int j = blockIdx.y;
  const int64_t chunk = blockIdx.x;
  const int w = (int)scr[kWidW + j];
  if (w == 0) return;
  const uint32_t nkept = scr[kCntW + chunk];
  if (nkept == 0) return;
  const int64_t i0 = chunk * kCChunk + (int64_t)threadIdx.x * kCItems;
  float yv[kCItems];
  uint32_t keep;
  load_items(n, y + j * npad, hard, i0, yv, keep);
  // block exclusive scan of the per-thread kept counts
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint32_t mine = __popc(keep);
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
  const float qj = hdr[j].q;
  const uint32_t kmin = (uint32_t)hdr[j].kmin;
  const float rq = __fdiv_rn(1.0f, qj);
  const bool fast_ok = fabsf(rq) >= 1.17549435e-38f && fabsf(rq) <= 3.40282347e+38f;
  const uint32_t vmask = w == 32 ? 0xFFFFFFFFu : ((1u << w) - 1u);
  bool bad = false;
#pragma unroll
  for (int e = 0; e < kCItems; ++e) {  // every slot is coded; dropped ones land in a discard
    bool ok;
    const int32_t k = sgs_code_fast(yv[e], qj, rq, fast_ok, ok);
    const bool kept = (keep >> e) & 1u;
    bad |= kept && !ok;
    s_vals[kept ? before + __popc(keep & ((1u << e) - 1u)) : kCChunk + lane] =
        ((uint32_t)k - kmin) & vmask;
  }
  if (bad) atomicOr(reinterpret_cast<uint32_t *>(info + 2), 1u);
  __syncthreads();
  // the span: bits [p0, p0 + nkept w) of the stream; word kw of it gathers
  // the values overlapping its 32 bits
  const uint64_t p0 = reinterpret_cast<const uint64_t *>(scr + kOffW)[j] +
                      (uint64_t)scr[kCntW + nc + chunk] * (uint64_t)w;
  const int s0 = (int)(p0 & 31);
  const int64_t wbase = (int64_t)(p0 >> 5);
  const int nbits = (int)nkept * w;
  const int nw = ((s0 + nbits - 1) >> 5) + 1;
  // floor(x / w) for 0 <= x < 2^17 as mulhi(x, ceil(2^32 / w)): the error is
  // below x / 2^32 < 2^-15 < 1 / w
  const uint32_t wmul = w == 1 ? 0u : (uint32_t)((0x100000000ull + (uint64_t)w - 1) / (uint64_t)w);
  for (int kw = threadIdx.x; kw < nw; kw += kCThreads) {
    const int64_t gw = wbase + kw;
    if (gw >= cap_words) break;
    const int b_lo = 32 * kw - s0;                         // span bit at the word's bit 0
    const uint32_t xa = (uint32_t)max(b_lo, 0), xb = (uint32_t)(min(b_lo + 32, nbits) - 1);
    const int a = (int)(w == 1 ? xa : __umulhi(xa, wmul));
    const int b = (int)(w == 1 ? xb : __umulhi(xb, wmul));
    // values a..b at bits 0, w, 2w, ... of acc ((b - a) w < 31 + w <= 63);
    // the word's bit 0 is acc's bit b_lo - a w, in [0, w), or lies s0 bits
    // below acc's bit 0 (b_lo - a w = -s0: word 0 of a span that starts
    // inside a word)
    uint64_t acc = 0;
    int pos = 0;
    for (int r = a; r <= b; ++r, pos += w) acc |= (uint64_t)s_vals[r] << pos;
    const int sh = b_lo - a * w;
    const uint32_t word = (uint32_t)(sh >= 0 ? acc >> sh : acc << -sh);
    if (kw == 0 || kw == nw - 1) {
      if (word) atomicOr(&payload[gw], word);  // shared with the neighbouring span
    } else {
      payload[gw] = word;
    }
  }
}

// Decode: rank r of channel j -> out[j][r] = fl32((kmin + v) q).  A block
// covers ranks [4096 b, 4096 b + 4096) of channel j: it stages the payload
// words of that span in LDS (coalesced), then each thread reads its values'
// words there.
__global__ void __launch_bounds__(kCThreads)
k_fl_unpack(int64_t kept, int64_t out_pad, const sgs_fl_channel *__restrict__ hdr,
            const uint32_t *__restrict__ payload, int64_t words, float *__restrict__ out) {
  __shared__ uint32_t s_words[kCWords];
  __shared__ uint64_t s_off;
  const int j = blockIdx.y;
  if (threadIdx.x < 64) {  // channel offset: sum of kept * w over earlier channels
    const int l = threadIdx.x;
    uint64_t x = l < j ? (uint64_t)kept * (uint64_t)hdr[l].width : 0ull;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    if (l == 0) s_off = x;
  }
  const int w = hdr[j].width;
  const float qj = hdr[j].q;
  const int32_t kmin = hdr[j].kmin;
  const int64_t rb = (int64_t)blockIdx.x * kCChunk;
  const int nr = (int)min((int64_t)kCChunk, kept - rb);
  __syncthreads();
  const uint64_t p0 = s_off + (uint64_t)rb * w;
  const int64_t wbase = (int64_t)(p0 >> 5);
  // words holding bits [p0, p0 + nr w), plus one so every value reads two
  const int nw = w > 0 ? (int)((((p0 & 31) + (uint64_t)nr * w - 1) >> 5) + 2) : 0;
  for (int k = threadIdx.x; k < nw; k += kCThreads) {
    const int64_t g = wbase + k;
    s_words[k] = g < words ? payload[g] : 0u;
  }
  __syncthreads();
  const uint32_t mask = w == 32 ? 0xFFFFFFFFu : ((1u << w) - 1u);
  float *orow = out + j * out_pad + rb;
#pragma unroll
  for (int e = 0; e < kCItems; ++e) {
    const int r = e * kCThreads + threadIdx.x;
    if (r < nr) {
      uint32_t v = 0;
      if (w > 0) {
        const uint32_t p = (uint32_t)(p0 & 31) + (uint32_t)r * (uint32_t)w;
        const uint64_t pair = ((uint64_t)s_words[(p >> 5) + 1] << 32) | s_words[p >> 5];
        v = (uint32_t)(pair >> (p & 31)) & mask;
      }
      orow[r] = (float)((int64_t)kmin + (int64_t)v) * qj;
    }
  }
}

}  // namespace

int64_t fl_scratch_words(int64_t n) {
  const int64_t nc = (n + kCChunk - 1) / kCChunk;
  return range_word(nc) + 2 * SGS_NCH * nc;
}

hipError_t launch_fl_encode(sgs_ctx *c, const float *params, const float *q,
                            const uint8_t *hard, sgs_fl_channel *hdr, uint32_t *payload,
                            int64_t cap_words, int64_t *info) {
  SgsProfScope ps(c, SGS_PROF_CODEC);
  const int nc = (int)((c->n + kCChunk - 1) / kCChunk);
  if (fl_scratch_words(c->n) > c->fl_tmp_words) return hipErrorInvalidValue;
  uint32_t *scr = c->fl_tmp;
  k_fl_stats<<<dim3(nc, SGS_NCH), kCThreads, 0, c->stream>>>(c->n, c->npad, params, hard, nc,
                                                             scr);
  k_fl_plan<<<1, kPlanThreads, 0, c->stream>>>(nc, q, scr, hdr, info, cap_words);
  if (cap_words > 0)
    k_fl_edges<<<sgs_blocks((int64_t)nc * SGS_NCH, 256), 256, 0, c->stream>>>(nc, scr, payload,
                                                                              cap_words);
  k_fl_pack<<<dim3(nc, SGS_NCH), kCThreads, 0, c->stream>>>(c->n, c->npad, params, hard, nc, scr,
                                                            hdr, payload, cap_words, info);
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
