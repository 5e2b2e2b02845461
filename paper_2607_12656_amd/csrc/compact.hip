// Pruning by the learned mask (the supplement's formation schedule applies
// the mask every 1,000 iterations): stable compaction of the kept Gaussians
// of several SoA arrays.  (1) per 4096-Gaussian chunk the kept count; (2) one
// block scans the counts into chunk ranks and the total; (3) per chunk and
// array row a block ranks its kept Gaussians and writes them at the chunk's
// rank (reads coalesced, writes contiguous per chunk).
#include "sgs_internal.h"

namespace {

constexpr int kKThreads = 256;
constexpr int kKItems = 16;
constexpr int kKChunk = kKThreads * kKItems;
constexpr int kKScan = 1024;

// scratch (the coder's, uint32 words): [0, nc) chunk counts, [nc, 2 nc)
// chunk ranks, [2 nc] the kept count
__device__ __forceinline__ uint32_t keep_bits(const uint8_t *__restrict__ hard, int64_t i0,
                                              int64_t n) {
  if (i0 + kKItems <= n) {
    const uint4 m = *reinterpret_cast<const uint4 *>(hard + i0);
    return sgs_nonzero_nibble(m.x) | sgs_nonzero_nibble(m.y) << 4 |
           sgs_nonzero_nibble(m.z) << 8 | sgs_nonzero_nibble(m.w) << 12;
  }
  uint32_t k = 0;
  for (int e = 0; e < kKItems; ++e)
    if (i0 + e < n && hard[i0 + e]) k |= 1u << e;
  return k;
}

__global__ void __launch_bounds__(kKThreads)
k_compact_count(int64_t n, const uint8_t *__restrict__ hard, uint32_t *__restrict__ cnt) {
  __shared__ uint32_t s_w[kKThreads / 64];
  const int64_t i0 = (int64_t)blockIdx.x * kKChunk + (int64_t)threadIdx.x * kKItems;
  uint32_t c = __popc(keep_bits(hard, i0, n));
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
  if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t t = 0;
    for (int w = 0; w < kKThreads / 64; ++w) t += s_w[w];
    cnt[blockIdx.x] = t;
  }
}

__global__ void __launch_bounds__(kKScan)
k_compact_scan(int nc, const uint32_t *__restrict__ cnt, uint32_t *__restrict__ rank,
               uint32_t *__restrict__ total) {
  __shared__ uint32_t s_wave[kKScan / 64];
  __shared__ uint32_t s_carry;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  if (t == 0) s_carry = 0;
  __syncthreads();
  for (int b = 0; b < nc; b += kKScan) {
    const int c = b + t;
    const uint32_t v = c < nc ? cnt[c] : 0u;
    uint32_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t u = __shfl_up(x, o, 64);
      if (lane >= o) x += u;
    }
    if (lane == 63) s_wave[wave] = x;
    __syncthreads();
    uint32_t before = 0;
    for (int w = 0; w < wave; ++w) before += s_wave[w];
    const uint32_t carry = s_carry;
    if (c < nc) rank[c] = carry + before + x - v;
    __syncthreads();
    if (t == kKScan - 1) s_carry = carry + before + x;
    __syncthreads();
  }
  if (t == 0) *total = s_carry;
}

__global__ void __launch_bounds__(kKThreads)
k_compact_scatter(int64_t n, int64_t src_pad, int64_t dst_pad, const uint8_t *__restrict__ hard,
                  const uint32_t *__restrict__ rank, SgsCompactArrays A) {
  __shared__ uint32_t s_wave[kKThreads / 64];
  const int64_t chunk = blockIdx.x;
  const int row = blockIdx.y;
  int a = 0;
  while (a + 1 < A.narrays && row >= A.row0[a + 1]) ++a;
  const int r = row - A.row0[a];
  const float *__restrict__ src = A.src[a] + r * src_pad;
  float *__restrict__ dst = A.dst[a] + r * dst_pad;
  const int64_t i0 = chunk * kKChunk + (int64_t)threadIdx.x * kKItems;
  const uint32_t keep = keep_bits(hard, i0, n);
  float v[kKItems];
  if (i0 + kKItems <= n) {
#pragma unroll
    for (int e = 0; e < kKItems; e += 4) {
      const float4 f = *reinterpret_cast<const float4 *>(src + i0 + e);
      v[e] = f.x;
      v[e + 1] = f.y;
      v[e + 2] = f.z;
      v[e + 3] = f.w;
    }
  } else {
#pragma unroll
    for (int e = 0; e < kKItems; ++e) v[e] = i0 + e < n ? src[i0 + e] : 0.0f;
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint32_t mine = __popc(keep);
  uint32_t x = mine;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t u = __shfl_up(x, o, 64);
    if (lane >= o) x += u;
  }
  if (lane == 63) s_wave[wave] = x;
  __syncthreads();
  uint32_t before = rank[chunk] + x - mine;
  for (int w = 0; w < wave; ++w) before += s_wave[w];
#pragma unroll
  for (int e = 0; e < kKItems; ++e)
    if (keep & (1u << e)) dst[before + __popc(keep & ((1u << e) - 1u))] = v[e];
}

}  // namespace

hipError_t launch_compact_count(sgs_ctx *c, const uint8_t *hard, uint32_t *d_total) {
  const int nc = (int)((c->n + kKChunk - 1) / kKChunk);
  if (2 * (int64_t)nc + 1 > c->fl_tmp_words) return hipErrorInvalidValue;
  k_compact_count<<<nc, kKThreads, 0, c->stream>>>(c->n, hard, c->fl_tmp);
  k_compact_scan<<<1, kKScan, 0, c->stream>>>(nc, c->fl_tmp, c->fl_tmp + nc, d_total);
  return hipGetLastError();
}

hipError_t launch_compact_scatter(sgs_ctx *c, const uint8_t *hard, const SgsCompactArrays &A,
                                  int64_t dst_pad) {
  const int nc = (int)((c->n + kKChunk - 1) / kKChunk);
  const int rows = A.row0[A.narrays];
  k_compact_scatter<<<dim3(nc, rows), kKThreads, 0, c->stream>>>(c->n, c->npad, dst_pad, hard,
                                                                 c->fl_tmp + nc, A);
  return hipGetLastError();
}
