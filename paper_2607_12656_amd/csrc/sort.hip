// Tile binning and the (tile, depth) order (paper Sec. 3.1: tile-based
// rasterization of depth-sorted Gaussians).
//
// The splats are sorted by depth once (V*N keys, 32 bits).  The pairs are
// then ordered in two levels instead of by a radix sort over every pair:
//  1. items: each splat, in depth order, yields one item per super-tile
//     (8x8 tiles) its tile rectangle meets, written at its item offset; the
//     items are stably sorted by super-tile id, so each super-tile's items
//     stay in depth order;
//  2. each super-tile's items are cut into chunks of 1024; a chunk's
//     workgroup turns every item into a 64-bit mask of the super-tile's tiles
//     it covers, counts the pairs per tile (one ballot per tile bit), and,
//     once the per-tile counts are scanned into tile offsets, writes every
//     pair's Gaussian index straight to its final position: its tile's
//     offset, plus the tile's pairs in earlier chunks, earlier waves and
//     earlier lanes (ranks from the same ballots).
// The pairs come out in (tile, depth, index) order, exactly the order of a
// stable sort by tile of the depth-ordered pairs, and the tile ranges come
// from the tile offsets.  At 3M Gaussians x 8 views the items number about a
// fourteenth of the pairs, and each pair crosses HBM once (its final write).
#include "sgs_internal.h"

namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
constexpr int kItems = 16;
constexpr int kTile = kThreads * kItems;  // elements per block
constexpr int kChunk = 16;                 // histogram rows per chunk of the digit scan

// ---------------------------------------------------------------------------
// Exclusive scan of uint32 (reduce -> scan of block sums -> downsweep).
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t *s_wave,
                                                         uint32_t &total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t t = __shfl_up(x, o, 64);
    if (lane >= o) x += t;
  }
  if (lane == 63) s_wave[wave] = x;
  __syncthreads();
  uint32_t off = 0;
  total = 0;
  for (int w = 0; w < kWaves; ++w) {
    const uint32_t t = s_wave[w];
    if (w < wave) off += t;
    total += t;
  }
  __syncthreads();
  return off + x - v;
}

__global__ void __launch_bounds__(kThreads)
k_scan_reduce(const uint32_t *__restrict__ in, int64_t count, uint32_t *__restrict__ sums) {
  __shared__ uint32_t s_wave[kWaves];
  const int64_t base = (int64_t)blockIdx.x * kTile;
  uint32_t acc = 0;
#pragma unroll
  for (int k = 0; k < kItems; ++k) {
    const int64_t i = base + (int64_t)k * kThreads + threadIdx.x;
    if (i < count) acc += in[i];
  }
  uint32_t total;
  block_exclusive_scan(acc, s_wave, total);
  if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

// single block: exclusive scan of the block sums in place; total to *total_out
// (with cap >= 0 also total_out[1] = min(total, cap), 0 for a saturated total,
// and bit 0 of total_out[2] set when the total exceeds cap)
__global__ void __launch_bounds__(kThreads)
k_scan_sums(uint32_t *__restrict__ sums, int64_t nb, uint32_t *__restrict__ total_out,
            uint32_t *__restrict__ tail, int64_t cap) {
  __shared__ uint64_t s_wave[kWaves];
  __shared__ uint64_t s_total;
  // each thread a run of consecutive sums (its loads in flight together),
  // the runs' totals scanned over the workgroup in 64 bits (a block sum fits
  // in 32 bits, the total may not), then the run rewritten
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t per = (nb + kThreads - 1) / kThreads;
  const int64_t b0 = min(nb, (int64_t)threadIdx.x * per), b1 = min(nb, b0 + per);
  uint64_t s = 0;
#pragma unroll 8
  for (int64_t b = b0; b < b1; ++b) s += sums[b];
  uint64_t x = s;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint64_t t = __shfl_up(x, o, 64);
    if (lane >= o) x += t;
  }
  if (lane == 63) s_wave[wave] = x;
  __syncthreads();
  uint64_t run = x - s;
  for (int w = 0; w < wave; ++w) run += s_wave[w];
  if (threadIdx.x == kThreads - 1) s_total = run + s;
#pragma unroll 8
  for (int64_t b = b0; b < b1; ++b) {
    const uint32_t v = sums[b];
    sums[b] = (uint32_t)run;
    run += v;
  }
  __syncthreads();
  const uint64_t carry = s_total;
  if (threadIdx.x == 0) {
    const uint32_t t = carry >= kPairsSaturated ? kPairsSaturated : (uint32_t)carry;
    if (total_out) *total_out = t;
    if (tail) *tail = t;
    if (total_out && cap >= 0) {
      // a saturated total leaves the offsets wrapped: emit nothing
      total_out[1] = t == kPairsSaturated ? 0u : (uint32_t)((int64_t)t < cap ? (int64_t)t : cap);
      if ((int64_t)t > cap) total_out[2] |= 1u;
    }
  }
}

// Each wave scans 16 x 64 consecutive elements of the block's 4096 as 64
// consecutive elements at a time (so every load and store is one coalesced
// access), carrying the running sum from group to group; the waves' totals
// are then scanned across the block.
__global__ void __launch_bounds__(kThreads)
k_scan_down(const uint32_t *__restrict__ in, int64_t count, const uint32_t *__restrict__ sums,
            uint32_t *__restrict__ out) {
  __shared__ uint32_t s_wave[kWaves];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t base = (int64_t)blockIdx.x * kTile + (int64_t)wave * (kItems * 64) + lane;
  uint32_t v[kItems];
#pragma unroll
  for (int k = 0; k < kItems; ++k) v[k] = (base + k * 64 < count) ? in[base + k * 64] : 0u;
  // inclusive scans of the 16 groups (independent, interleaved), then carries
  uint32_t x[kItems];
#pragma unroll
  for (int k = 0; k < kItems; ++k) x[k] = v[k];
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
      const uint32_t t = __shfl_up(x[k], o, 64);
      if (lane >= o) x[k] += t;
    }
  }
  uint32_t carry = 0;
#pragma unroll
  for (int k = 0; k < kItems; ++k) {
    const uint32_t tot = (uint32_t)__shfl(x[k], 63, 64);
    x[k] += carry - v[k];  // exclusive within the wave's segment
    carry += tot;
  }
  if (lane == 0) s_wave[wave] = carry;
  __syncthreads();
  uint32_t off = sums[blockIdx.x];
  for (int w = 0; w < wave; ++w) off += s_wave[w];
#pragma unroll
  for (int k = 0; k < kItems; ++k)
    if (base + k * 64 < count) out[base + k * 64] = off + x[k];
}

// ---------------------------------------------------------------------------
// Stable LSD radix sort, 8-bit digits (the last pass of a key narrower than
// a multiple of 8 bits takes only the bits left: nb < 8), reduce-then-scan.
// Elements of a block are taken in rounds of 256 (position base + r*256 +
// tid); within a round each wave finds the lanes sharing its digit with nb
// ballots, so ranks follow (round, wave, lane) = input order.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t match_digit(uint32_t d, bool valid, int nb) {
  const uint64_t v = __ballot(valid);
  uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
#pragma unroll
  for (int b = 0; b < 8; ++b) {
    if (b >= nb) break;  // the pass's digit has nb bits (wave-uniform)
    // s: all ones where the lane's bit b is set; a lane keeps the lanes whose
    // bit b equals its own, i.e. those where the ballot agrees with s (kept
    // as 32-bit halves so that each half is one three-input bitwise op)
    const uint32_t s = (uint32_t)__builtin_amdgcn_sbfe((int)d, b, 1);
    const uint64_t bal = __ballot(s != 0u);
    lo &= ~((uint32_t)bal ^ s);
    hi &= ~((uint32_t)(bal >> 32) ^ s);
  }
  return ((uint64_t)hi << 32) | lo;
}

// Blocks of `tile` elements that hold live elements: the sort kernels of a
// grid sized for a capacity loop over these only (the count is on the
// device), and the digit-offset kernels scan only their histogram rows.
__device__ __forceinline__ int64_t live_blocks(int64_t count_static,
                                               const uint32_t *__restrict__ dcount,
                                               int64_t tile) {
  const int64_t count = dcount ? (int64_t)*dcount : count_static;
  return (count + tile - 1) / tile;
}

// Block histogram of one digit.  Lanes count into 32 sub-histograms (eight
// lanes each, rows padded to 257 words so that equal digits of different
// sub-histograms sit in different banks): the pass over the high digit sees
// long runs of equal digits, and same-address LDS atomics serialize.  A grid
// of resident size loops over the live blocks (rows of other blocks are
// neither written nor read).
template <int IT>
__global__ void __launch_bounds__(kThreads)
k_radix_hist(const uint32_t *__restrict__ keys, int64_t count_static,
             const uint32_t *__restrict__ dcount, int shift, int nb, uint32_t *__restrict__ hist) {
  constexpr int TILE = kThreads * IT;
  __shared__ uint32_t s_sub[kThreads / 8][257];
  const int64_t count = dcount ? (int64_t)*dcount : count_static;
  const int64_t live = (count + TILE - 1) / TILE;
  const uint32_t dmask = (1u << nb) - 1u;
  const SgsXcdWalk wk = sgs_xcd_walk(blockIdx.x, gridDim.x, live);
  for (int64_t blk = wk.first; blk < wk.end; blk += wk.step) {
    const int64_t base = blk * TILE;
#pragma unroll
    for (int w = 0; w < kThreads / 8; ++w) s_sub[w][threadIdx.x] = 0;
    // all loads of the block in flight at once
    uint32_t kr[IT];
#pragma unroll
    for (int r = 0; r < IT; ++r) {
      const int64_t i = base + (int64_t)r * kThreads + threadIdx.x;
      kr[r] = i < count ? keys[i] : 0u;
    }
    __syncthreads();
    if (nb <= 3) {
      // at most 8 digits: the keys share few addresses, which LDS atomics
      // would serialize on; a ballot per digit value and round counts them
      // instead, and lane v of each wave adds the wave's count of digit v once
      const uint32_t lane = threadIdx.x & 63u;
      uint32_t own = 0;
#pragma unroll
      for (int r = 0; r < IT; ++r) {
        const bool ok = base + (int64_t)r * kThreads + threadIdx.x < count;
        const uint32_t d = (kr[r] >> shift) & dmask;
        for (uint32_t v = 0; v <= dmask; ++v) {
          const uint32_t n = (uint32_t)__popcll(__ballot(ok && d == v));
          if (lane == v) own += n;
        }
      }
      if (lane <= dmask) atomicAdd(&s_sub[0][lane], own);
    } else {
      uint32_t *mine = s_sub[threadIdx.x >> 3];
#pragma unroll
      for (int r = 0; r < IT; ++r) {
        const int64_t i = base + (int64_t)r * kThreads + threadIdx.x;
        if (i < count) atomicAdd(&mine[(kr[r] >> shift) & dmask], 1u);
      }
    }
    __syncthreads();
    uint32_t tot = 0;
#pragma unroll
    for (int w = 0; w < kThreads / 8; ++w) tot += s_sub[w][threadIdx.x];
    hist[blk * 256 + threadIdx.x] = tot;
    __syncthreads();  // the sums are read before the next block clears them
  }
}

// Digit offsets from the block-major histogram rows H[b][d]: the position of
// block b's first element with digit d is
//   sum_{d' < d} total[d'] + sum_{b' < b} H[b'][d].
// Rows are grouped in chunks of kChunk; every access below reads or writes
// whole 1 KB rows (coalesced), unlike a scan over a digit-major table, whose
// per-block stores and loads are 4 bytes each, a row apart.
__global__ void __launch_bounds__(kThreads)
k_hist_chunk_sums(const uint32_t *__restrict__ H, int64_t count_static,
                  const uint32_t *__restrict__ dcount, int64_t tile, uint32_t *__restrict__ CS) {
  const int64_t nb = live_blocks(count_static, dcount, tile);
  const int64_t g = blockIdx.x;
  const int64_t b0 = g * kChunk, b1 = min(nb, b0 + kChunk);
  if (b0 >= nb) return;
  uint32_t s = 0;
#pragma unroll 8
  for (int64_t b = b0; b < b1; ++b) s += H[b * 256 + threadIdx.x];
  CS[g * 256 + threadIdx.x] = s;
}

// One block per digit: exclusive scan of the chunk sums over chunks (in
// place) and the digit total.
__global__ void __launch_bounds__(kThreads)
k_hist_chunk_scan(uint32_t *__restrict__ CS, int64_t count_static,
                  const uint32_t *__restrict__ dcount, int64_t tile, uint32_t *__restrict__ total) {
  __shared__ uint32_t s_wave[kWaves];
  const int64_t ng = (live_blocks(count_static, dcount, tile) + kChunk - 1) / kChunk;
  const int d = blockIdx.x;
  const int64_t per = (ng + kThreads - 1) / kThreads;
  const int64_t g0 = min(ng, (int64_t)threadIdx.x * per), g1 = min(ng, g0 + per);
  uint32_t s = 0;
  for (int64_t g = g0; g < g1; ++g) s += CS[g * 256 + d];
  uint32_t tot;
  uint32_t run = block_exclusive_scan(s, s_wave, tot);
  for (int64_t g = g0; g < g1; ++g) {
    const uint32_t v = CS[g * 256 + d];
    CS[g * 256 + d] = run;
    run += v;
  }
  if (threadIdx.x == 0) total[d] = tot;
}

__global__ void __launch_bounds__(kThreads)
k_hist_chunk_down(const uint32_t *__restrict__ H, int64_t count_static,
                  const uint32_t *__restrict__ dcount, int64_t tile,
                  const uint32_t *__restrict__ CB, const uint32_t *__restrict__ total,
                  uint32_t *__restrict__ O) {
  __shared__ uint32_t s_wave[kWaves];
  const int64_t nb = live_blocks(count_static, dcount, tile);
  const int64_t g = blockIdx.x;
  if (g * kChunk >= nb) return;
  uint32_t tot;
  uint32_t run = block_exclusive_scan(total[threadIdx.x], s_wave, tot) + CB[g * 256 + threadIdx.x];
  const int64_t b0 = g * kChunk, b1 = min(nb, b0 + kChunk);
#pragma unroll 8
  for (int64_t b = b0; b < b1; ++b) {
    const uint32_t v = H[b * 256 + threadIdx.x];
    O[b * 256 + threadIdx.x] = run;
    run += v;
  }
}

// Digit offsets for at most kColRows blocks in one launch: block d scans
// column d of H[b][d] over b (each thread a run of consecutive rows), writing
// O[b][d] = sum_{b' < b} H[b'][d] and total[d].  The scatter adds the
// digit's base (the exclusive scan of the totals) itself.  Beyond kColRows
// the column reads (one word per 1 KB row) would not stay in L2, and the
// chunked kernels above take over.
constexpr int64_t kColRows = 2048;
__global__ void __launch_bounds__(kThreads)
k_digit_cols(const uint32_t *__restrict__ H, int64_t count_static,
             const uint32_t *__restrict__ dcount, int64_t tile, uint32_t *__restrict__ O,
             uint32_t *__restrict__ total) {
  __shared__ uint32_t s_wave[kWaves];
  const int64_t nb = live_blocks(count_static, dcount, tile);
  const int d = blockIdx.x;
  const int64_t per = (nb + kThreads - 1) / kThreads;
  const int64_t b0 = min(nb, (int64_t)threadIdx.x * per), b1 = min(nb, b0 + per);
  uint32_t s = 0;
#pragma unroll 8
  for (int64_t b = b0; b < b1; ++b) s += H[b * 256 + d];
  uint32_t tot;
  uint32_t run = block_exclusive_scan(s, s_wave, tot);
#pragma unroll 8
  for (int64_t b = b0; b < b1; ++b) {
    const uint32_t v = H[b * 256 + d];
    O[b * 256 + d] = run;
    run += v;
  }
  if (threadIdx.x == 0) total[d] = tot;
}

// The scanned histogram entry of this thread's digit: with digit_tot (the
// column path) the digit's base, the exclusive scan of the digit totals, is
// added here; the chunked path has it included already.  Every thread of the
// block calls this (it synchronizes).
__device__ __forceinline__ uint32_t scanned_offset(const uint32_t *__restrict__ hist_scanned,
                                                   const uint32_t *__restrict__ digit_tot,
                                                   int64_t blk) {
  __shared__ uint32_t s_wave[kWaves];
  uint32_t h = hist_scanned[blk * 256 + threadIdx.x];
  if (digit_tot) {
    uint32_t tot;
    h += block_exclusive_scan(digit_tot[threadIdx.x], s_wave, tot);
  }
  return h;
}

// The same entry for a sort of equal segments (seg_len elements, seg_blocks
// blocks each) sorted each on its own: the digit's position in the block's
// segment, from the global offsets (the elements of the digit in earlier
// blocks of the segment are the difference of two of them; the segment's
// digit counts, scanned, give the digits' bases).  total: the digit totals;
// with_base: hist_scanned includes the digits' bases (the chunked path).
__device__ __forceinline__ uint32_t segment_offset(const uint32_t *__restrict__ hist_scanned,
                                                   const uint32_t *__restrict__ total,
                                                   bool with_base, int64_t blk, int64_t nb,
                                                   int64_t seg_blocks, int64_t seg_len) {
  __shared__ uint32_t s_wave[kWaves];
  const int t = threadIdx.x;
  const int64_t sg = blk / seg_blocks, fb = sg * seg_blocks, fe = fb + seg_blocks;
  const uint32_t hb = hist_scanned[blk * 256 + t], hf = hist_scanned[fb * 256 + t];
  uint32_t he, tot;
  if (fe < nb) {
    he = hist_scanned[fe * 256 + t];
  } else {  // the last segment ends at the digit's total (past its base)
    const uint32_t tt = total[t];
    const uint32_t ex = block_exclusive_scan(tt, s_wave, tot);
    he = (with_base ? ex : 0u) + tt;
  }
  const uint32_t seg_ex = block_exclusive_scan(he - hf, s_wave, tot);
  return (uint32_t)(sg * seg_len) + seg_ex + (hb - hf);
}

// Scatter of one pass for the block's elements in the wave-segment layout:
// wave w holds elements w * IT * 64 + r * 64 + lane of the block in kr[r],
// vr[r], so the input order is (wave, round, lane).  Each wave ranks its own
// elements digit by digit with ballots and wave-private running counts in
// LDS (no workgroup barrier inside the rounds); one barrier later the
// per-wave counts become prefixes, and every element lands at
//   block offset of its digit + elements of that digit in earlier waves
//   + its rank within its wave,
// i.e. the block's elements in LDS in stable digit order; each digit's run is
// then written to its global position with consecutive threads on
// consecutive addresses (coalesced).
// The block's count of each digit (the offsets inside the block) comes from
// the ranking itself.  h_scan: this thread's digit (= tid) entry of the
// block's scanned histogram row, loaded by the caller ahead of its other work.
// V2: a second value array rides along (vr2 -> vout2 through s_val2).
template <int IT, bool V2>
__device__ __forceinline__ void scatter_block(const uint32_t (&kr)[IT],
                                              const uint32_t (&vr)[IT],
                                              const uint32_t (&vr2)[IT], int64_t base,
                                              int64_t count, int shift, int nb, uint32_t h_scan,
                                              uint32_t *__restrict__ kout,
                                              uint32_t *__restrict__ vout,
                                              uint32_t *__restrict__ vout2, uint32_t *s_key,
                                              uint32_t *s_val, uint32_t *s_val2) {
  __shared__ uint32_t s_base[256];
  __shared__ uint32_t s_loff[256];
  __shared__ uint32_t s_cnt[kWaves][256];
  __shared__ uint32_t s_wave[kWaves];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint32_t dmask = (1u << nb) - 1u;
  s_base[threadIdx.x] = h_scan;
#pragma unroll
  for (int w = 0; w < kWaves; ++w) s_cnt[w][threadIdx.x] = 0;
  __syncthreads();
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const int64_t wbase = base + (int64_t)wave * IT * 64;
  uint32_t rank[IT];
#pragma unroll
  for (int r = 0; r < IT; ++r) {
    const bool valid = wbase + (int64_t)r * 64 + lane < count;
    const uint32_t d = (kr[r] >> shift) & dmask;
    const uint64_t m = match_digit(d, valid, nb);
    const uint32_t before = valid ? s_cnt[wave][d] : 0u;
    const uint32_t below = (uint32_t)__popcll(m & lt);  // same-digit lanes before this one
    rank[r] = before + below;
    wave_lds_sync();  // every lane has read before the leader writes
    // the leader (lowest lane of the digit) has none before it
    if (valid && below == 0u) s_cnt[wave][d] = before + (uint32_t)__popcll(m);
    wave_lds_sync();
  }
  __syncthreads();
  {
    const int t = threadIdx.x;
    uint32_t run = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) {
      const uint32_t c = s_cnt[w][t];
      s_cnt[w][t] = run;
      run += c;
    }
    uint32_t tot;
    s_loff[t] = block_exclusive_scan(run, s_wave, tot);  // run: the block's count of digit t
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < IT; ++r) {
    if (wbase + (int64_t)r * 64 + lane < count) {
      const uint32_t d = (kr[r] >> shift) & dmask;
      const uint32_t lp = s_loff[d] + s_cnt[wave][d] + rank[r];  // < kThreads * IT
      s_key[lp] = kr[r];
      s_val[lp] = vr[r];
      if (V2) s_val2[lp] = vr2[r];
    }
  }
  __syncthreads();
  const int nloc = (int)min((int64_t)(kThreads * IT), count - base);
#pragma unroll 4
  for (int p = threadIdx.x; p < nloc; p += kThreads) {
    const uint32_t k = s_key[p];
    const uint32_t d = (k >> shift) & dmask;
    const uint32_t pos = s_base[d] + ((uint32_t)p - s_loff[d]);
    kout[pos] = k;
    vout[pos] = s_val[p];
    if (V2) vout2[pos] = s_val2[p];
  }
}

// One workgroup per block of the capacity-sized grid (a loop over the live
// blocks would need more registers than four workgroups per compute unit
// leave); blocks past the live count return at once.
template <int IT, bool V2>
__global__ void __launch_bounds__(kThreads)
k_radix_scatter(const uint32_t *__restrict__ kin, const uint32_t *__restrict__ vin,
                const uint32_t *__restrict__ vin2, uint32_t *__restrict__ kout,
                uint32_t *__restrict__ vout, uint32_t *__restrict__ vout2,
                int64_t count_static, const uint32_t *__restrict__ dcount, int shift, int nb,
                const uint32_t *__restrict__ hist_scanned,
                const uint32_t *__restrict__ digit_tot, const uint32_t *__restrict__ total,
                int64_t seg_blocks, int64_t seg_len) {
  constexpr int TILE = kThreads * IT;
  __shared__ uint32_t s_key[TILE];
  __shared__ uint32_t s_val[TILE];
  __shared__ uint32_t s_val2[V2 ? TILE : 1];
  const int64_t count = dcount ? (int64_t)*dcount : count_static;
  const int64_t blk = sgs_xcd_block_live(blockIdx.x, gridDim.x, (count + TILE - 1) / TILE);
  const int64_t base = blk * TILE;
  if (base >= count) return;
  // all loads of the block in flight at once, in the wave-segment layout
  const int64_t wbase = base + (int64_t)(threadIdx.x >> 6) * IT * 64 + (threadIdx.x & 63);
  uint32_t kr[IT], vr[IT], vr2[IT];
#pragma unroll
  for (int r = 0; r < IT; ++r) {
    const int64_t i = wbase + (int64_t)r * 64;
    kr[r] = i < count ? kin[i] : 0u;
    vr[r] = i < count ? vin[i] : 0u;
    vr2[r] = V2 && i < count ? vin2[i] : 0u;
  }
  const uint32_t h_scan =
      seg_blocks ? segment_offset(hist_scanned, total, digit_tot == nullptr, blk,
                                  (count + TILE - 1) / TILE, seg_blocks, seg_len)
                 : scanned_offset(hist_scanned, digit_tot, blk);
  scatter_block<IT, V2>(kr, vr, vr2, base, count, shift, nb, h_scan, kout, vout, vout2, s_key,
                        s_val, s_val2);
}

// ---------------------------------------------------------------------------
// Binning input in depth order
// ---------------------------------------------------------------------------
// The tile rectangle of a binning record (first tile id, width in tiles,
// Gaussian, pairs) as columns [tx0, tx1] and rows [ty0, ty1] of its view.
struct TileRect {
  uint32_t v;
  int tx0, tx1, ty0, ty1;
};
__device__ __forceinline__ TileRect tile_rect(const uint4 &b, uint32_t tiles_per_view, int GW) {
  TileRect r;
  r.v = b.x / tiles_per_view;
  const uint32_t t = b.x - r.v * tiles_per_view;
  r.ty0 = (int)(t / (uint32_t)GW);
  r.tx0 = (int)(t - (uint32_t)r.ty0 * (uint32_t)GW);
  r.tx1 = r.tx0 + (int)b.y - 1;
  r.ty1 = r.ty0 + (int)(b.w / b.y) - 1;
  return r;
}

// Items per splat: the 8x8-tile super-tiles its tile rectangle meets.
__device__ __forceinline__ uint32_t super_tiles_met(const uint4 &b, uint32_t tiles_per_view,
                                                    int GW) {
  const TileRect r = tile_rect(b, tiles_per_view, GW);
  return (uint32_t)(((r.tx1 >> 3) - (r.tx0 >> 3) + 1) * ((r.ty1 >> 3) - (r.ty0 >> 3) + 1));
}

// The binning record (first tile id, width in tiles, Gaussian, pairs) of the
// splat at place i of the depth order, rebuilt from its splat index and the
// tile rectangle the depth sort carried along; only a splat whose rectangle
// did not fit the packed word has its record gathered (depth order is
// random in splat index, and every such read fetches a whole cache line).
// An invalid splat (or a segment's padding) has an empty record.
__device__ __forceinline__ uint4 depth_record(int64_t i, const uint32_t *__restrict__ order,
                                              const uint32_t *__restrict__ dkey,
                                              const uint32_t *__restrict__ rect,
                                              const uint4 *__restrict__ bin_splat, uint32_t n,
                                              int GW, uint32_t tiles_per_view) {
  if (dkey[i] == 0xFFFFFFFFu) return make_uint4(0u, 1u, 0u, 0u);
  const uint32_t sp = order[i], r = rect[i];
  if (r == kNoRect) return bin_splat[sp];
  const uint32_t v = sp / n, tw = ((r >> 20) & 63u) + 1u, th = (r >> 26) + 1u;
  return make_uint4(v * tiles_per_view + ((r >> 10) & 1023u) * (uint32_t)GW + (r & 1023u), tw,
                    sp - v * n, tw * th);
}

// The item count of every splat in depth order (input of the item offsets
// scan), and per block of kTile splats the pair count (their sum is the pair
// total; no per-splat pair offset is needed) and the item count (the block
// sums of the item offsets scan).
__global__ void __launch_bounds__(kThreads)
k_gather_bins(const uint32_t *__restrict__ order, const uint32_t *__restrict__ dkey,
              const uint32_t *__restrict__ rect, const uint4 *__restrict__ bin_splat,
              int64_t count, uint32_t n, int GW, uint32_t tiles_per_view,
              uint32_t *__restrict__ icnt, uint32_t *__restrict__ psums,
              uint32_t *__restrict__ isums) {
  __shared__ uint64_t s_sum[kWaves];
  __shared__ uint32_t s_isum[kWaves];
  const int64_t base = (int64_t)blockIdx.x * kTile;
  uint64_t acc = 0;
  uint32_t iacc = 0;
  // eight records at a time (a gathered one waits on two loads before it)
  constexpr int kHalf = kItems / 2;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    uint4 b[kHalf];
#pragma unroll
    for (int k = 0; k < kHalf; ++k) {
      const int64_t i = base + (int64_t)(h * kHalf + k) * kThreads + threadIdx.x;
      b[k] = i < count ? depth_record(i, order, dkey, rect, bin_splat, n, GW, tiles_per_view)
                       : make_uint4(0u, 1u, 0u, 0u);
    }
#pragma unroll
    for (int k = 0; k < kHalf; ++k) {
      const int64_t i = base + (int64_t)(h * kHalf + k) * kThreads + threadIdx.x;
      if (i < count) {
        acc += b[k].w;
        const uint32_t ic = b[k].w ? super_tiles_met(b[k], tiles_per_view, GW) : 0u;
        icnt[i] = ic;
        iacc += ic;
      }
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    acc += __shfl_xor(acc, o, 64);
    iacc += (uint32_t)__shfl_xor((int)iacc, o, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    s_sum[threadIdx.x >> 6] = acc;
    s_isum[threadIdx.x >> 6] = iacc;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t t = 0;
    uint32_t it = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) {
      t += s_sum[w];
      it += s_isum[w];
    }
    // a saturated block sum saturates the total (k_scan_sums)
    psums[blockIdx.x] = t >= kPairsSaturated ? kPairsSaturated : (uint32_t)t;
    isums[blockIdx.x] = it;  // at most 4096 splats x the super-tiles of a view
  }
}

// ---------------------------------------------------------------------------
// Level 1: super-tile items
// ---------------------------------------------------------------------------
// An item's key: the super-tile id (super-tile in its view) << vbits | view
// in bits [0, 16) (at most 65536 ids; the sort's 8-bit digits stay inside
// these bits) and, riding along above bit 20, the covered tile rectangle
// inside the super-tile: first and last column and row, 3 bits each.  The
// items come in (view, depth) order, so one stable sort on the super-tile
// bits alone leaves each super-tile's items together and in depth order.
constexpr int kStBits = 20;
constexpr uint32_t kStMask = (1u << kStBits) - 1u;

// The items of every splat, in (view, depth) order, at its item offset: key =
// super-tile id | covered tile rectangle inside it (see kStBits), value =
// Gaussian index.  Items at or beyond the live item count (a capacity) are
// not written.
__global__ void k_emit_items(const uint32_t *__restrict__ order, const uint32_t *__restrict__ dkey,
                             const uint32_t *__restrict__ rect,
                             const uint4 *__restrict__ bin_splat, uint32_t n,
                             const uint32_t *__restrict__ ioff, int64_t vn, int64_t count_static,
                             const uint32_t *__restrict__ dcount, int GW,
                             uint32_t tiles_per_view, int SGW, int vbits,
                             uint32_t *__restrict__ kout, uint32_t *__restrict__ vout) {
  const int64_t d = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (d >= vn || dkey[d] == 0xFFFFFFFFu) return;
  const uint4 b = depth_record(d, order, dkey, rect, bin_splat, n, GW, tiles_per_view);
  const int64_t count = dcount ? (int64_t)*dcount : count_static;
  int64_t o = ioff[d];
  const TileRect r = tile_rect(b, tiles_per_view, GW);
  for (int sy = r.ty0 >> 3; sy <= (r.ty1 >> 3); ++sy)
    for (int sx = r.tx0 >> 3; sx <= (r.tx1 >> 3); ++sx, ++o) {
      if (o >= count) return;
      const uint32_t cx0 = (uint32_t)max(r.tx0 - 8 * sx, 0), cx1 = (uint32_t)min(r.tx1 - 8 * sx, 7);
      const uint32_t cy0 = (uint32_t)max(r.ty0 - 8 * sy, 0), cy1 = (uint32_t)min(r.ty1 - 8 * sy, 7);
      kout[o] = ((((uint32_t)sy * (uint32_t)SGW + (uint32_t)sx) << vbits) | r.v) |
                (cx0 << kStBits) | (cx1 << (kStBits + 3)) | (cy0 << (kStBits + 6)) |
                (cy1 << (kStBits + 9));
      vout[o] = b.z;
    }
}

// Item range of every super-tile: binary search of the sorted items on the
// super-tile bits of their keys (lower bounds of g and g + 1 over [0, I)).
__global__ void __launch_bounds__(256)
k_st_ranges(const uint32_t *__restrict__ key, int64_t I_static, const uint32_t *__restrict__ dcount,
            uint32_t nst, uint2 *__restrict__ ranges) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= nst) return;
  const int64_t I = dcount ? (int64_t)*dcount : I_static;
  const uint32_t k0 = (uint32_t)g, k1 = (uint32_t)g + 1u;
  int64_t lo0 = 0, hi0 = I, lo1 = 0, hi1 = I;
  while (lo0 < hi0 || lo1 < hi1) {
    const int64_t m0 = (lo0 + hi0) >> 1, m1 = (lo1 + hi1) >> 1;
    const uint32_t v0 = lo0 < hi0 ? key[m0] & kStMask : 0u;
    const uint32_t v1 = lo1 < hi1 ? key[m1] & kStMask : 0u;
    if (lo0 < hi0) {
      if (v0 < k0) lo0 = m0 + 1; else hi0 = m0;
    }
    if (lo1 < hi1) {
      if (v1 < k1) lo1 = m1 + 1; else hi1 = m1;
    }
  }
  ranges[g] = lo0 < lo1 ? make_uint2((uint32_t)lo0, (uint32_t)lo1) : make_uint2(0u, 0u);
}

// ---------------------------------------------------------------------------
// Level 2: tiles inside a super-tile
// ---------------------------------------------------------------------------
constexpr int kL2Items = 1024;  // items per chunk: 4 waves x 4 rounds x 64 lanes

// chunk_first[g] = sum over super-tiles g' < g of ceil(items / kL2Items);
// chunk_first[nst] = the number of chunks (one workgroup); chunk_first[nst + 1]
// (the level-2 scatter's queue of chunks) is cleared.
__global__ void __launch_bounds__(kThreads)
k_st_chunks(const uint2 *__restrict__ st_ranges, int64_t nst, uint32_t *__restrict__ first) {
  __shared__ uint32_t s_wave[kWaves];
  uint32_t carry = 0;
  for (int64_t b0 = 0; b0 < nst; b0 += kThreads) {
    const int64_t g = b0 + threadIdx.x;
    uint32_t v = 0;
    if (g < nst) {
      const uint2 r = st_ranges[g];
      v = (r.y - r.x + kL2Items - 1) / kL2Items;
    }
    uint32_t total;
    const uint32_t ex = block_exclusive_scan(v, s_wave, total);
    if (g < nst) first[g] = carry + ex;
    carry += total;
  }
  if (threadIdx.x == 0) {
    first[nst] = carry;
    first[nst + 1] = 0;
  }
}

// The super-tile of chunk q: the last g with first[g] <= q (q < first[nst]).
__device__ __forceinline__ uint32_t chunk_super(const uint32_t *__restrict__ first, uint32_t nst,
                                                uint32_t q) {
  uint32_t lo = 0, hi = nst;
  while (hi - lo > 1) {
    const uint32_t m = (lo + hi) >> 1;
    if (first[m] <= q) lo = m; else hi = m;
  }
  return lo;
}

// Bit 8 row + column for every tile of the super-tile that the item with
// this key covers (its rectangle rides in the key's high bits): the row's
// bits repeated in every row, cut to the covered rows.
__device__ __forceinline__ uint64_t item_mask(uint32_t key) {
  const uint32_t cx0 = (key >> kStBits) & 7u, cx1 = (key >> (kStBits + 3)) & 7u;
  const uint32_t cy0 = (key >> (kStBits + 6)) & 7u, cy1 = (key >> (kStBits + 9)) & 7u;
  const uint64_t row = (uint64_t)((0xFFu >> (7u - (cx1 - cx0))) << cx0);
  const uint64_t rows = (~0ull >> (8u * (7u - cy1))) & (~0ull << (8u * cy0));
  return (row * 0x0101010101010101ull) & rows;
}

// The value of lane L ^ S, moved without LDS: the half and row swaps of
// gfx950 (each returns both halves of the pair; lanes in the upper half or
// odd row take the first) and DPP within rows (S = 4: mirror the eight, then
// reverse the quad).
template <int kCtrl>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t x) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, kCtrl, 0xF, 0xF, false);
}
template <int S>
__device__ __forceinline__ uint32_t xor_lane(uint32_t x, int lane) {
  if constexpr (S == 32) {
    const auto sw = __builtin_amdgcn_permlane32_swap(x, x, false, false);
    return (lane & 32) ? sw[0] : sw[1];
  } else if constexpr (S == 16) {
    const auto sw = __builtin_amdgcn_permlane16_swap(x, x, false, false);
    return (lane & 16) ? sw[0] : sw[1];
  } else if constexpr (S == 8) {
    return dpp_u32<0x128>(x);                  // row_ror:8
  } else if constexpr (S == 4) {
    return dpp_u32<0x1B>(dpp_u32<0x141>(x));   // row_half_mirror, quad_perm [3,2,1,0]
  } else if constexpr (S == 2) {
    return dpp_u32<0x4E>(x);                   // quad_perm [2,3,0,1]
  } else {
    return dpp_u32<0xB1>(x);                   // quad_perm [1,0,3,2]
  }
}

// One butterfly stage: lanes L and L ^ S exchange the blocks of S bits that
// belong to the other one (m: the blocks a lane with bit S clear keeps).
template <int S>
__device__ __forceinline__ uint64_t transpose_stage(uint64_t r, int lane, uint64_t m) {
  const uint32_t olo = xor_lane<S>((uint32_t)r, lane);
  const uint32_t ohi = xor_lane<S>((uint32_t)(r >> 32), lane);
  const uint64_t o = ((uint64_t)ohi << 32) | olo;
  const bool up = lane & S;
  const uint64_t keep = up ? ~m : m;
  const uint64_t in = up ? (o >> S) : (o << S);
  return (r & keep) | (in & ~keep);
}

// 64 x 64 bit transpose over the wave: lane L holds row L (bit t set when
// item L covers tile t); afterwards lane t holds column t (bit L set when
// item L covers tile t).  Six butterfly stages.
__device__ __forceinline__ uint64_t wave_transpose64(uint64_t r, int lane) {
  r = transpose_stage<32>(r, lane, 0x00000000FFFFFFFFull);
  r = transpose_stage<16>(r, lane, 0x0000FFFF0000FFFFull);
  r = transpose_stage<8>(r, lane, 0x00FF00FF00FF00FFull);
  r = transpose_stage<4>(r, lane, 0x0F0F0F0F0F0F0F0Full);
  r = transpose_stage<2>(r, lane, 0x3333333333333333ull);
  r = transpose_stage<1>(r, lane, 0x5555555555555555ull);
  return r;
}

// The chunk's items: masks and Gaussian indices, four rounds per wave
// (item first + 256 wave + 64 round + lane, in item order).
struct Chunk {
  uint32_t g, first, end;
  int tx_base, ty_base;
  uint32_t view;
};

__device__ __forceinline__ bool chunk_of(uint32_t q, const uint32_t *__restrict__ cfirst,
                                         uint32_t nst, const uint2 *__restrict__ st_ranges,
                                         int SGW, int vbits, Chunk &ch) {
  if (q >= cfirst[nst]) return false;
  ch.g = chunk_super(cfirst, nst, q);
  const uint2 r = st_ranges[ch.g];
  ch.first = r.x + (q - cfirst[ch.g]) * (uint32_t)kL2Items;
  ch.end = r.y;
  ch.view = ch.g & ((1u << vbits) - 1u);
  const uint32_t gs = ch.g >> vbits;
  const uint32_t sy = gs / (uint32_t)SGW;
  ch.ty_base = 8 * (int)sy;
  ch.tx_base = 8 * (int)(gs - sy * (uint32_t)SGW);
  return true;
}

// Per-chunk pair counts of the 64 tiles: cnt[q][t].  A grid of resident
// size loops over the chunks (their number is on the device).
__global__ void __launch_bounds__(kThreads)
k_l2_count(const uint32_t *__restrict__ cfirst, uint32_t nst, const uint2 *__restrict__ st_ranges,
           const uint32_t *__restrict__ ikey, int SGW, int vbits, uint32_t *__restrict__ cnt) {
  __shared__ uint32_t s_w[kWaves][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const SgsXcdWalk wk = sgs_xcd_walk(blockIdx.x, gridDim.x, cfirst[nst]);
  // a chunk's keys (0xFFFFFFFF: no item), loaded one chunk ahead
  auto keys_of = [&](int64_t q, uint32_t (&k)[4]) {
    Chunk ch;
    const bool live = q < wk.end && chunk_of((uint32_t)q, cfirst, nst, st_ranges, SGW, vbits, ch);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const uint32_t idx = live ? ch.first + (uint32_t)(wave * 256 + r * 64 + lane) : 0u;
      k[r] = live && idx < ch.end ? ikey[idx] : 0xFFFFFFFFu;
    }
  };
  uint32_t kn[4];
  keys_of(wk.first, kn);
  for (int64_t q = wk.first; q < wk.end; q += wk.step) {
    uint32_t kr[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) kr[r] = kn[r];
    keys_of(q + wk.step, kn);
    uint32_t acc = 0;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const uint64_t m = kr[r] == 0xFFFFFFFFu ? 0ull : item_mask(kr[r]);
      // lane t: the round's items covering tile t
      acc += (uint32_t)__popcll(wave_transpose64(m, lane));
    }
    s_w[wave][lane] = acc;
    __syncthreads();
    if (wave == 0)
      cnt[q * 64 + lane] = s_w[0][lane] + s_w[1][lane] + s_w[2][lane] + s_w[3][lane];
    __syncthreads();  // read before the next chunk writes
  }
}

// Per super-tile (four waves, lane t = tile t): the chunk counts become the
// tile's pairs in earlier chunks (in place), and the tile's total goes to
// tile_cnt (tiles past the image edge have no pairs and no entry).  Wave w
// takes the w-th quarter of the super-tile's chunks: it sums them, the four
// sums give each quarter its start, and the wave rewrites its quarter.
constexpr int kL2ScanWaves = 4;
__global__ void __launch_bounds__(64 * kL2ScanWaves)
k_l2_scan(const uint32_t *__restrict__ cfirst, uint32_t *__restrict__ cnt, int GW, int GH,
          int SGW, int vbits, int V, uint32_t tiles_per_view, uint32_t *__restrict__ tile_cnt) {
  __shared__ uint32_t s_part[kL2ScanWaves][64];
  const uint32_t g = blockIdx.x;
  const int t = threadIdx.x & 63, w = threadIdx.x >> 6;
  const uint32_t q0 = cfirst[g], q1 = cfirst[g + 1];
  const uint32_t per = (q1 - q0 + kL2ScanWaves - 1) / kL2ScanWaves;
  const uint32_t a = min(q1, q0 + per * (uint32_t)w), e = min(q1, a + per);
  uint32_t part = 0;
  for (uint32_t qb = a; qb < e; qb += 32) {
    uint32_t c[32];
#pragma unroll
    for (int k = 0; k < 32; ++k) c[k] = qb + k < e ? cnt[(int64_t)(qb + k) * 64 + t] : 0u;
#pragma unroll
    for (int k = 0; k < 32; ++k) part += c[k];
  }
  s_part[w][t] = part;
  __syncthreads();
  uint32_t run = 0, total = 0;
#pragma unroll
  for (int k = 0; k < kL2ScanWaves; ++k) {
    if (k < w) run += s_part[k][t];
    total += s_part[k][t];
  }
  for (uint32_t qb = a; qb < e; qb += 32) {
    uint32_t c[32];
#pragma unroll
    for (int k = 0; k < 32; ++k) c[k] = qb + k < e ? cnt[(int64_t)(qb + k) * 64 + t] : 0u;
#pragma unroll
    for (int k = 0; k < 32; ++k)
      if (qb + k < e) {
        cnt[(int64_t)(qb + k) * 64 + t] = run;
        run += c[k];
      }
  }
  const uint32_t v = g & ((1u << vbits) - 1u), gs = g >> vbits;
  if (w != 0 || v >= (uint32_t)V) return;  // (ids of views >= V hold no items)
  const uint32_t sy = gs / (uint32_t)SGW, sx = gs - sy * (uint32_t)SGW;
  const int tx = 8 * (int)sx + (t & 7), ty = 8 * (int)sy + (t >> 3);
  if (tx < GW && ty < GH) tile_cnt[(int64_t)v * tiles_per_view + (int64_t)ty * GW + tx] = total;
}

// Tile ranges from the tile offsets, clamped to the pairs the buffer holds
// (the pair count, or the capacity it was clamped to); empty tiles (0, 0).
__global__ void k_l2_ranges(const uint32_t *__restrict__ tile_cnt,
                            const uint32_t *__restrict__ tile_start, int64_t tiles,
                            int64_t held_static, const uint32_t *__restrict__ dheld,
                            uint2 *__restrict__ ranges) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= tiles) return;
  const int64_t held = dheld ? (int64_t)*dheld : held_static;
  const int64_t n = tile_cnt[t];
  const int64_t a = min((int64_t)tile_start[t], held), e = min((int64_t)tile_start[t] + n, held);
  ranges[t] = n && a < e ? make_uint2((uint32_t)a, (uint32_t)e) : make_uint2(0u, 0u);
}

// Every pair of the chunk to its final position, tile run by tile run: the
// chunk's pairs of tile t are consecutive in the output (from the tile's
// offset + its pairs in earlier chunks), in item order (wave, round, lane).
// They are laid out in LDS tile after tile, each as the item's slot in the
// chunk (10 bits) and the tile (6 bits), and copied out by the whole
// workgroup with consecutive threads on consecutive entries, which look the
// slot's Gaussian index and the tile's destination up, so that each output
// line is written whole in one burst (writing each wave's and round's few
// dozen bytes on their own left lines half written in the cache, and most
// were written out twice).
// A chunk whose pairs exceed the LDS array takes its tiles in groups that
// fit (one tile's pairs of a chunk are at most kL2Items).
constexpr int kL2Out = 12288;
static_assert(kL2Out >= kL2Items, "one tile's pairs of a chunk must fit");

__global__ void __launch_bounds__(kThreads)
k_l2_scatter(const uint32_t *__restrict__ cfirst, uint32_t *__restrict__ queue, uint32_t nst,
             const uint2 *__restrict__ st_ranges, const uint32_t *__restrict__ ikey,
             const uint32_t *__restrict__ ival, int GW, int GH, uint32_t tiles_per_view, int SGW,
             int vbits, const uint32_t *__restrict__ rel,
             const uint32_t *__restrict__ tile_start, int64_t held_static,
             const uint32_t *__restrict__ dheld, uint32_t *__restrict__ vals) {
  __shared__ uint16_t s_out[kL2Out];
  __shared__ uint32_t s_gid[kL2Items];  // slot wave * 256 + round * 64 + lane
  __shared__ uint16_t s_cnt[kWaves][4][64];  // wave, round: its items covering tile t
  __shared__ uint32_t s_dst[64];  // tile t's entry e of the group goes to s_dst[t] + e
  __shared__ uint32_t s_q[2];
  const uint32_t held = (uint32_t)(dheld ? (int64_t)*dheld : held_static);
  const uint32_t nchunks = cfirst[nst];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // a chunk's inputs: lane t's tile start in the output (dst0) and the
  // wave's keys (0xFFFFFFFF: no item) and Gaussian indices of its four rounds
  auto chunk_in = [&](int64_t q, uint32_t &dst0, uint32_t (&key)[4], uint32_t (&gid)[4]) {
    Chunk ch;
    const bool live = q < nchunks && chunk_of((uint32_t)q, cfirst, nst, st_ranges, SGW, vbits, ch);
    const int tx = ch.tx_base + (lane & 7), ty = ch.ty_base + (lane >> 3);
    dst0 = 0;
    if (live && tx < GW && ty < GH)
      dst0 = tile_start[(int64_t)ch.view * tiles_per_view + (int64_t)ty * GW + tx] +
             rel[q * 64 + lane];
#pragma unroll
    for (int r = 0; r < 4; ++r) {  // all four rounds' loads in flight at once
      const uint32_t idx = live ? ch.first + (uint32_t)(wave * 256 + r * 64 + lane) : 0u;
      const bool ok = live && idx < ch.end;
      key[r] = ok ? ikey[idx] : 0xFFFFFFFFu;
      gid[r] = ok ? ival[idx] : 0u;
    }
  };
  // chunks from the queue, one per workgroup at a time (their work varies
  // with the items' footprints; a fixed share per workgroup left a tail);
  // the next chunk's ticket and inputs are fetched while one is worked on
  if (threadIdx.x == 0) s_q[0] = atomicAdd(queue, 1u);
  __syncthreads();
  int64_t q = s_q[0];
  uint32_t dst0n, keyn[4], gidn[4];
  chunk_in(q, dst0n, keyn, gidn);
  for (uint32_t it = 0; q < nchunks; ++it) {
    // slot (it + 1) & 1 was last read two chunks ago, before this chunk's barriers
    if (threadIdx.x == 0) s_q[(it + 1) & 1] = atomicAdd(queue, 1u);
    const uint32_t dst0 = dst0n;
    uint32_t key[4], gid[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      key[r] = keyn[r];
      gid[r] = gidn[r];
    }
    uint64_t col[4];  // lane t: the round's items covering tile t (bit L: lane L's item)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      col[r] = wave_transpose64(key[r] == 0xFFFFFFFFu ? 0ull : item_mask(key[r]), lane);
      s_gid[wave * 256 + r * 64 + lane] = gid[r];
      s_cnt[wave][r][lane] = (uint16_t)__popcll(col[r]);
    }
    __syncthreads();
    const int64_t qn = s_q[(it + 1) & 1];
    chunk_in(qn, dst0n, keyn, gidn);
    // lane t: the tile's pairs in this chunk, and in its earlier waves
    uint32_t tot = 0, before = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const uint32_t v = s_cnt[w][r][lane];
        tot += v;
        before += w < wave ? v : 0u;
      }
    uint32_t incl = tot;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t v = (uint32_t)__shfl_up((int)incl, o, 64);
      if (lane >= o) incl += v;
    }
    // groups of consecutive tiles whose pairs fit the LDS array (the same in
    // every wave: each computes the same prefix)
    uint32_t base = 0;  // pairs of the tiles in earlier groups
    for (int t0 = 0; t0 < 64;) {
      // incl rises with the lane: the tiles that fit are t0 .. t1 - 1
      const uint64_t fits = __ballot(lane >= t0 && incl - base <= (uint32_t)kL2Out);
      const int t1 = 64 - (int)__builtin_clzll(fits);
      if (lane >= t0 && lane < t1) {
        if (wave == 0) s_dst[lane] = dst0 - (incl - tot - base);
        uint32_t lp = incl - tot - base + before;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          // the two halves of the column on their own (32-bit bit scans)
          const uint32_t slot = (uint32_t)(wave * 256 + r * 64) | (uint32_t)lane << 10;
          uint32_t lo = (uint32_t)col[r], hi = (uint32_t)(col[r] >> 32);
          while (lo) {
            s_out[lp++] = (uint16_t)(slot | __builtin_ctz(lo));
            lo &= lo - 1u;
          }
          while (hi) {
            s_out[lp++] = (uint16_t)(slot | (32u + __builtin_ctz(hi)));
            hi &= hi - 1u;
          }
        }
      }
      __syncthreads();
      // copy-out: the group's entries over the workgroup, four per thread in
      // flight at once
      const uint32_t end = (uint32_t)__builtin_amdgcn_readlane((int)incl, t1 - 1);
      const uint32_t ng = end - base;
      for (uint32_t e0 = 0; e0 < ng; e0 += 4u * kThreads) {
        uint32_t v[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const uint32_t e = e0 + (uint32_t)(k * kThreads) + threadIdx.x;
          v[k] = s_out[min(e, (uint32_t)kL2Out - 1u)];  // past the group: read, dropped
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const uint32_t e = e0 + (uint32_t)(k * kThreads) + threadIdx.x;
          const uint32_t d = s_dst[v[k] >> 10] + e;
          const uint32_t g = s_gid[v[k] & 1023u];
          if (e < ng && d < held) vals[d] = g;
        }
      }
      __syncthreads();  // the next group or chunk refills the arrays
      base = end;
      t0 = t1;
    }
    q = qn;
  }
}

}  // namespace

hipError_t ensure_tmp(sgs_ctx *c, int64_t scan_words, int64_t hist_words) {
  if (scan_words > c->scan_tmp_words) {
    if (c->scan_tmp) (void)hipFree(c->scan_tmp);
    c->scan_tmp = nullptr;
    hipError_t e = hipMalloc(&c->scan_tmp, sizeof(uint32_t) * scan_words);
    if (e != hipSuccess) { c->scan_tmp_words = 0; return e; }
    c->scan_tmp_words = scan_words;
  }
  if (hist_words > c->sort_hist_words) {
    if (c->sort_hist) (void)hipFree(c->sort_hist);
    c->sort_hist = nullptr;
    hipError_t e = hipMalloc(&c->sort_hist, sizeof(uint32_t) * hist_words);
    if (e != hipSuccess) { c->sort_hist_words = 0; return e; }
    c->sort_hist_words = hist_words;
  }
  return hipSuccess;
}

int64_t radix_blocks(int64_t count) { return (count + kTile - 1) / kTile; }

// Chunks of kL2Items items for at most cap items over total_st super-tiles
// (each super-tile's last chunk may be partial).
int64_t l2_chunks_for(int64_t cap, int64_t total_st) { return cap / kL2Items + total_st + 1; }

// A plain radix pass over at most kSmallSort elements takes kSmallItems per
// thread: with 4096 per block a 1M-element sort would launch fewer blocks
// than there are compute units.
constexpr int64_t kSmallSort = (int64_t)1 << 22;
constexpr int kSmallItems = 4;
// With a second value array a large pass takes kV2Items per thread (three
// 4096-word LDS arrays would leave two workgroups per compute unit).
constexpr int kV2Items = 8;
int64_t radix_tile(int64_t count, bool v2 = false) {
  if (count <= kSmallSort) return (int64_t)kThreads * kSmallItems;
  return v2 ? (int64_t)kThreads * kV2Items : (int64_t)kTile;
}

// (sized for the smaller of the tiles a sort of count elements may take)
int64_t radix_hist_words(int64_t count) {
  const int64_t tile = radix_tile(count, true);
  const int64_t nb = (count + tile - 1) / tile;
  const int64_t ng = (nb + kChunk - 1) / kChunk;
  return 2 * nb * 256 + ng * 256 + 256 + 1;
}

// scan_tmp must hold ceil(count / kTile) words
hipError_t launch_exclusive_scan(sgs_ctx *c, const uint32_t *in, uint32_t *out, int64_t count,
                                 uint32_t *total_out, int64_t cap) {
  const int64_t nb = (count + kTile - 1) / kTile;
  if (nb == 0) {
    k_scan_sums<<<1, kThreads, 0, c->stream>>>(c->scan_tmp, 0, total_out, out, cap);
    return hipGetLastError();
  }
  if (nb > c->scan_tmp_words) return hipErrorInvalidValue;
  k_scan_reduce<<<(unsigned)nb, kThreads, 0, c->stream>>>(in, count, c->scan_tmp);
  k_scan_sums<<<1, kThreads, 0, c->stream>>>(c->scan_tmp, nb, total_out, out + count, cap);
  k_scan_down<<<(unsigned)nb, kThreads, 0, c->stream>>>(in, count, c->scan_tmp, out);
  return hipGetLastError();
}

namespace {

struct SortBufs {
  int64_t nb, ng;
  uint32_t *hraw, *hscan, *chunk, *total;
};

bool sort_bufs(sgs_ctx *c, int64_t count, SortBufs &b, int64_t tile = kTile) {
  b.nb = (count + tile - 1) / tile;
  b.ng = (b.nb + kChunk - 1) / kChunk;
  if (radix_hist_words(count) > c->sort_hist_words) return false;
  b.hraw = c->sort_hist;
  b.hscan = b.hraw + b.nb * 256;
  b.chunk = b.hscan + b.nb * 256;
  b.total = b.chunk + b.ng * 256;
  return true;
}

// Digit offsets of every block from the raw block histograms (raw counts kept
// for the block-local placement).  Returns the digit totals the scatter must
// add the digit bases of (column path), or null (chunked path: included).
const uint32_t *launch_digit_offsets(sgs_ctx *c, const SortBufs &b, int64_t count,
                                     const uint32_t *dcount, int64_t tile) {
  if (b.nb <= kColRows) {
    k_digit_cols<<<256, kThreads, 0, c->stream>>>(b.hraw, count, dcount, tile, b.hscan, b.total);
    return b.total;
  }
  k_hist_chunk_sums<<<(unsigned)b.ng, kThreads, 0, c->stream>>>(b.hraw, count, dcount, tile,
                                                                b.chunk);
  k_hist_chunk_scan<<<256, kThreads, 0, c->stream>>>(b.chunk, count, dcount, tile, b.total);
  k_hist_chunk_down<<<(unsigned)b.ng, kThreads, 0, c->stream>>>(b.hraw, count, dcount, tile,
                                                                b.chunk, b.total, b.hscan);
  return nullptr;
}

// Workgroups of a grid that loops over its blocks: all that fit on the device
// at once (occupancy x compute units), at most `blocks`.  One instance (and
// cached count) per kernel.
template <auto Kernel>
unsigned resident_blocks(int64_t blocks) {
  static int cap = 0;
  if (cap == 0) {
    int dev = 0, occ = 0, cus = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, Kernel, kThreads, 0) == hipSuccess &&
        occ > 0 && cus > 0)
      cap = occ * cus;
    else
      cap = 1024;
  }
  return (unsigned)max((int64_t)1, min(blocks, (int64_t)cap));
}

}  // namespace

// Passes shift0, shift0 + 8, ... < bits of the stable LSD sort; the data
// starts in buffer cur0 and *which receives the buffer holding the result.
hipError_t launch_radix_sort(sgs_ctx *c, uint32_t *keys[2], uint32_t *vals[2], int64_t count,
                             int bits, int *which, const uint32_t *dcount, int shift0,
                             int cur0, uint32_t **vals2, int64_t seg_len) {
  int cur = cur0;
  *which = cur0;
  if (count <= 1 || shift0 >= bits) return hipSuccess;
  const bool small = count <= kSmallSort, v2 = vals2 != nullptr;
  const int64_t tile = radix_tile(count, v2);
  // segments: whole blocks, a static count
  if (seg_len && (seg_len % tile != 0 || count % seg_len != 0 || dcount))
    return hipErrorInvalidValue;
  const int64_t seg_blocks = seg_len / tile;
  SortBufs b;
  if (!sort_bufs(c, count, b, tile)) return hipErrorInvalidValue;
  for (int shift = shift0; shift < bits; shift += 8) {
    const int nb = min(8, bits - shift);  // digit bits of this pass
    if (small)
      k_radix_hist<kSmallItems><<<resident_blocks<k_radix_hist<kSmallItems>>(b.nb), kThreads, 0,
                                  c->stream>>>(keys[cur], count, dcount, shift, nb, b.hraw);
    else if (v2)
      k_radix_hist<kV2Items><<<resident_blocks<k_radix_hist<kV2Items>>(b.nb), kThreads, 0,
                               c->stream>>>(keys[cur], count, dcount, shift, nb, b.hraw);
    else
      k_radix_hist<kItems><<<resident_blocks<k_radix_hist<kItems>>(b.nb), kThreads, 0,
                             c->stream>>>(keys[cur], count, dcount, shift, nb, b.hraw);
    const uint32_t *dtot = launch_digit_offsets(c, b, count, dcount, tile);
    uint32_t *in2 = v2 ? vals2[cur] : nullptr, *out2 = v2 ? vals2[cur ^ 1] : nullptr;
    if (small && v2)
      k_radix_scatter<kSmallItems, true><<<(unsigned)b.nb, kThreads, 0, c->stream>>>(
          keys[cur], vals[cur], in2, keys[cur ^ 1], vals[cur ^ 1], out2, count, dcount, shift,
          nb, b.hscan, dtot, b.total,
          seg_blocks, seg_len);
    else if (small)
      k_radix_scatter<kSmallItems, false><<<(unsigned)b.nb, kThreads, 0, c->stream>>>(
          keys[cur], vals[cur], nullptr, keys[cur ^ 1], vals[cur ^ 1], nullptr, count, dcount,
          shift, nb, b.hscan, dtot, b.total,
          seg_blocks, seg_len);
    else if (v2)
      k_radix_scatter<kV2Items, true><<<(unsigned)b.nb, kThreads, 0, c->stream>>>(
          keys[cur], vals[cur], in2, keys[cur ^ 1], vals[cur ^ 1], out2, count, dcount, shift,
          nb, b.hscan, dtot, b.total,
          seg_blocks, seg_len);
    else
      k_radix_scatter<kItems, false><<<(unsigned)b.nb, kThreads, 0, c->stream>>>(
          keys[cur], vals[cur], nullptr, keys[cur ^ 1], vals[cur ^ 1], nullptr, count, dcount,
          shift, nb, b.hscan, dtot, b.total,
          seg_blocks, seg_len);
    cur ^= 1;
  }
  *which = cur;
  return hipGetLastError();
}

// Depth sort of all (view, Gaussian) splats (view-major: each view's segment
// sorted on its own), the item counts in that order and their offsets, and
// the pair total.
hipError_t launch_depth_order(sgs_ctx *c) {
  int which = 0;
  {
    SgsProfScope ps(c, SGS_PROF_DEPTH_SORT);
    // each view's segment on its own (the order is view, then depth); the
    // packed tile rectangles ride along as a second value
    hipError_t e = launch_radix_sort(c, c->depth_key, c->depth_val, c->vn_pad, 32, &which,
                                     nullptr, 0, 0, c->depth_rect, c->vseg);
    if (e != hipSuccess) return e;
  }
  c->depth_sorted_buf = which;
  SgsProfScope ps(c, SGS_PROF_SCAN);
  // item counts in depth order (-> scratch: the other key buffer is free
  // now), pair counts summed per block of kTile splats
  uint32_t *tmp = c->depth_key[which ^ 1];
  const int64_t nb = (c->vn_pad + kTile - 1) / kTile;
  if (nb == 0 || 2 * nb > c->scan_tmp_words) return hipErrorInvalidValue;
  uint32_t *psums = c->scan_tmp, *isums = c->scan_tmp + nb;
  k_gather_bins<<<(unsigned)nb, kThreads, 0, c->stream>>>(
      c->depth_val[which], c->depth_key[which], c->depth_rect[which], c->bin_splat, c->vn_pad,
      (uint32_t)c->n, c->GW, (uint32_t)c->tiles_per_view, tmp, psums, isums);
  // the pair total (with a fixed pair capacity also clamped to it)
  const int64_t cap = c->fixed_cap ? c->cap_limit : -1;
  k_scan_sums<<<1, kThreads, 0, c->stream>>>(psums, nb, c->d_pairs_total, nullptr, cap);
  // the item offsets (an exclusive scan whose block sums the gather wrote)
  k_scan_sums<<<1, kThreads, 0, c->stream>>>(isums, nb, c->d_pairs_total + 4,
                                             c->ioffsets + c->vn_pad, cap);
  k_scan_down<<<(unsigned)nb, kThreads, 0, c->stream>>>(tmp, c->vn_pad, isums, c->ioffsets);
  return hipGetLastError();
}

// Items -> super-tile sort -> per-super-tile tile counts -> tile offsets and
// ranges -> pairs at their final positions.  With a fixed pair capacity the
// counts never leave the device: grids are sized by the capacity (items and
// chunks are bounded by it) and every kernel reads the live counts, clamped
// to the capacity (overflow flagged by the pair scan).
hipError_t launch_bin_pairs(sgs_ctx *c) {
  const bool dev = c->fixed_cap;
  const int64_t cap = dev ? c->cap_limit : c->pair_cap;
  const int64_t P = dev ? cap : c->pairs;   // pairs the buffer holds (bound)
  const int64_t I = dev ? cap : c->items;   // items (bound; an item has at least one pair)
  const uint32_t *dP = dev ? c->d_pairs_total + 1 : nullptr;
  const uint32_t *dI = dev ? c->d_pairs_total + 5 : nullptr;
  const uint32_t tpv = (uint32_t)c->tiles_per_view;
  const uint32_t nst = (uint32_t)c->st_slots;
  const int ds = c->depth_sorted_buf;
  const int vb = c->st_vbits;
  int bits = vb;  // the super-tile bits above the view's
  while (((int64_t)1 << (bits - vb)) < c->st_per_view) ++bits;
  int which = 0;
  const int64_t chunks = min(c->l2_chunks, l2_chunks_for(I, c->total_st));
  {
    SgsProfScope ps(c, SGS_PROF_TILE_SORT);
    // items in (view, depth) order (buffer 0), stably sorted by the super-tile
    // in the view
    if (I > 0)
      k_emit_items<<<sgs_blocks(c->vn_pad, 256), 256, 0, c->stream>>>(
          c->depth_val[ds], c->depth_key[ds], c->depth_rect[ds], c->bin_splat, (uint32_t)c->n,
          c->ioffsets, c->vn_pad, I, dI, c->GW, tpv, c->SGW, vb, c->tile_key[0],
          c->pair_val[0]);
    hipError_t e = launch_radix_sort(c, c->tile_key, c->pair_val, I, bits, &which, dI, vb, 0);
    if (e != hipSuccess) return e;
    k_st_ranges<<<sgs_blocks(nst, 256), 256, 0, c->stream>>>(c->tile_key[which], I, dI, nst,
                                                            c->st_ranges);
    k_st_chunks<<<1, kThreads, 0, c->stream>>>(c->st_ranges, nst, c->chunk_first);
    if (chunks > 0)
      k_l2_count<<<resident_blocks<k_l2_count>(chunks), kThreads, 0, c->stream>>>(
          c->chunk_first, nst, c->st_ranges, c->tile_key[which], c->SGW, vb, c->l2_cnt);
    k_l2_scan<<<nst, 64 * kL2ScanWaves, 0, c->stream>>>(c->chunk_first, c->l2_cnt, c->GW, c->GH,
                                                         c->SGW, vb, c->V, tpv, c->tile_cnt);
  }
  {
    SgsProfScope ps(c, SGS_PROF_RANGES);
    hipError_t e = launch_exclusive_scan(c, c->tile_cnt, c->tile_start, c->total_tiles, nullptr);
    if (e != hipSuccess) return e;
    k_l2_ranges<<<sgs_blocks(c->total_tiles, 256), 256, 0, c->stream>>>(
        c->tile_cnt, c->tile_start, c->total_tiles, P, dP, c->ranges);
  }
  {
    SgsProfScope ps(c, SGS_PROF_DUPLICATE);
    if (chunks > 0)
      k_l2_scatter<<<resident_blocks<k_l2_scatter>(chunks), kThreads, 0, c->stream>>>(
          c->chunk_first, c->chunk_first + nst + 1, nst, c->st_ranges, c->tile_key[which],
          c->pair_val[which], c->GW, c->GH, tpv, c->SGW, vb, c->l2_cnt, c->tile_start, P,
          dP, c->pair_val[which ^ 1]);
  }
  c->pair_sorted_buf = which ^ 1;
  return launch_tile_order(c);
}
