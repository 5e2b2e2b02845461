// Learned-coding stage, lossless parts (paper Sec. 3.4.2): the octree
// occupancy tokens of the quantized geometry, their decoding back to
// positions, and an entropy coder for byte streams.
//
// Octree tokens.  The kept Gaussians' position codes k_c = rint(fl32(y_c /
// q_c)) (the quantizer's decision) become voxel coordinates u_c = k_c -
// kmin_c < 2^D and one Morton code each (bit 3b+2: x bit b, 3b+1: y, 3b: z).
// After a radix sort of the codes, element j starts a node of depth d when
// its code differs from element j-1's in the top 3d bits; the inclusive count
// of such starts up to j, minus one, is the rank of j's depth-d node.  Node
// ranks in Morton order are the token order within a level, so every node of
// depth d >= 1 sets its child bit in its parent's token directly (the parent
// is j's node of depth d-1).  Depth-D starts are the distinct voxels; their
// run lengths give the duplicate counts, kept as a sparse list.
//
// Decoding walks the tokens level by level: one scan of the tokens' child
// counts gives every child's node number, and each level's tokens expand
// their nodes' codes into the next level's.
//
// Entropy coder: range ANS (32-bit state in [2^16, 2^32), 16-bit words,
// frequencies summing to 4096) interleaved over the 64 lanes of a wave.  A
// block of 64 S symbols is one wave: lane l owns the block's l-th run of S
// symbols (its order-1 context is its own previous symbol), all lanes take
// one step per iteration, and the lanes whose state falls below 2^16 read
// the block's next words in lane order (a ballot and a popcount).  The
// encoder runs the same steps backwards, lanes descending, which is what
// puts the words in that order.  Blocks decode independently.
#include <vector>

#include "sgs_internal.h"

namespace {

constexpr int kMaxDepth = 21;
constexpr int kLevels = kMaxDepth + 1;  // node depths 0 .. D
constexpr int kOcThreads = 256;
constexpr uint32_t kAnsPB = 12, kAnsM = 1u << kAnsPB, kAnsL = 1u << 16;
constexpr int kCtx = 257;
constexpr uint32_t kNoSym = 0xFFFFFFFFu;  // decode-table entry of an unused slot

// Device state of one octree encode / decode.
struct OcState {
  int32_t kmin[3], kmax[3];
  uint32_t kept, fill, flags;
  int32_t depth;
  uint32_t ntot[kLevels];  // nodes per depth
  uint32_t toff[kLevels];  // first token of every level
  uint32_t tokens, unique, dups, total;
};

__device__ __forceinline__ uint64_t lanemask_lt() {
  const int lane = threadIdx.x & 63;
  return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

__device__ __forceinline__ uint64_t morton3(uint32_t x, uint32_t y, uint32_t z, int depth) {
  uint64_t c = 0;
  for (int b = 0; b < depth; ++b)
    c |= ((uint64_t)((x >> b) & 1u) << (3 * b + 2)) | ((uint64_t)((y >> b) & 1u) << (3 * b + 1)) |
         ((uint64_t)((z >> b) & 1u) << (3 * b));
  return c;
}

__device__ __forceinline__ int depth_of(const OcState *s) {
  if (s->kept == 0) return 1;
  int D = 1;
  for (int c = 0; c < 3; ++c) {
    const uint64_t r = (uint64_t)((int64_t)s->kmax[c] - (int64_t)s->kmin[c]);
    const int b = r ? 64 - __clzll(r) : 0;  // bit length: r < 2^b
    D = b > D ? b : D;
  }
  return D;
}

// ---------------------------------------------------------------------------
// Octree encode
// ---------------------------------------------------------------------------
__global__ void k_oc_init(OcState *s) {
  if (threadIdx.x != 0) return;
  for (int c = 0; c < 3; ++c) {
    s->kmin[c] = 0x7FFFFFFF;
    s->kmax[c] = (int32_t)0x80000000;
  }
  s->kept = s->fill = s->flags = 0;
  s->depth = 1;
  s->tokens = s->unique = s->dups = s->total = 0;
}

__device__ __forceinline__ void codes_of(const float *__restrict__ params, int64_t npad,
                                         const float *__restrict__ q, int64_t i, int32_t (&v)[3],
                                         bool &ok) {
  ok = true;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    bool o;
    v[c] = sgs_code_of(params[c * npad + i], q[c], o);
    ok = ok && o;
  }
}

// Range of the kept codes per axis and the kept count: per workgroup
// partials {min x3, max x3, count, bad} (no atomics), reduced by k_oc_depth.
constexpr int kOcRangeBlocks = 512;
__global__ void __launch_bounds__(kOcThreads)
k_oc_range(const float *__restrict__ params, int64_t npad, int64_t n, const float *__restrict__ q,
           const uint8_t *__restrict__ hard, int32_t *__restrict__ part) {
  __shared__ int32_t s_p[kOcThreads / 64][8];
  int32_t mn[3] = {0x7FFFFFFF, 0x7FFFFFFF, 0x7FFFFFFF};
  int32_t mx[3] = {(int32_t)0x80000000, (int32_t)0x80000000, (int32_t)0x80000000};
  int32_t cnt = 0;
  bool bad = false;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    if (!hard[i]) continue;
    int32_t v[3];
    bool ok;
    codes_of(params, npad, q, i, v, ok);
    bad = bad || !ok;
    ++cnt;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      mn[c] = min(mn[c], v[c]);
      mx[c] = max(mx[c], v[c]);
    }
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      mn[c] = min(mn[c], __shfl_xor(mn[c], o, 64));
      mx[c] = max(mx[c], __shfl_xor(mx[c], o, 64));
    }
    cnt += __shfl_xor(cnt, o, 64);
  }
  const bool anybad = __ballot(bad) != 0ull;
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    for (int c = 0; c < 3; ++c) {
      s_p[wave][c] = mn[c];
      s_p[wave][3 + c] = mx[c];
    }
    s_p[wave][6] = cnt;
    s_p[wave][7] = anybad ? 1 : 0;
  }
  __syncthreads();
  if (threadIdx.x < 8) {
    const int k = threadIdx.x;
    int32_t r = s_p[0][k];
    for (int w = 1; w < kOcThreads / 64; ++w) {
      const int32_t v = s_p[w][k];
      r = k < 3 ? min(r, v) : k < 6 ? max(r, v) : k == 6 ? r + v : (r | v);
    }
    part[blockIdx.x * 8 + k] = r;
  }
}

// The partials reduced (one workgroup, fixed order); depth and the header's
// geometry fields.
__global__ void __launch_bounds__(256)
k_oc_depth(const int32_t *__restrict__ part, int nparts, OcState *s, sgs_octree_header *h) {
  __shared__ int32_t s_r[256][8];
  int32_t r[8] = {0x7FFFFFFF, 0x7FFFFFFF, 0x7FFFFFFF, (int32_t)0x80000000, (int32_t)0x80000000,
                  (int32_t)0x80000000, 0, 0};
  for (int b = threadIdx.x; b < nparts; b += 256) {
    for (int k = 0; k < 8; ++k) {
      const int32_t v = part[b * 8 + k];
      r[k] = k < 3 ? min(r[k], v) : k < 6 ? max(r[k], v) : k == 6 ? r[k] + v : (r[k] | v);
    }
  }
  for (int k = 0; k < 8; ++k) s_r[threadIdx.x][k] = r[k];
  __syncthreads();
  if (threadIdx.x != 0) return;
  for (int t = 1; t < 256; ++t)
    for (int k = 0; k < 8; ++k) {
      const int32_t v = s_r[t][k];
      r[k] = k < 3 ? min(r[k], v) : k < 6 ? max(r[k], v) : k == 6 ? r[k] + v : (r[k] | v);
    }
  for (int c = 0; c < 3; ++c) {
    s->kmin[c] = r[c];
    s->kmax[c] = r[3 + c];
  }
  s->kept = (uint32_t)r[6];
  if (r[7]) s->flags |= 1u;
  int D = depth_of(s);
  if (D > kMaxDepth) {
    s->flags |= 1u;
    D = kMaxDepth;
  }
  if (s->kept == 0)
    for (int c = 0; c < 3; ++c) s->kmin[c] = s->kmax[c] = 0;
  s->depth = D;
  h->depth = D;
  for (int c = 0; c < 3; ++c) h->kmin[c] = s->kmin[c];
  h->kept = s->kept;
}

// Morton codes of the kept Gaussians at their positions in index order
// (pos: exclusive scan of the kept flags), split into low and high words
// for the radix sort.
__global__ void __launch_bounds__(kOcThreads)
k_oc_codes(const float *__restrict__ params, int64_t npad, int64_t n, const float *__restrict__ q,
           const uint8_t *__restrict__ hard, const uint32_t *__restrict__ pos, const OcState *s,
           uint32_t *__restrict__ lo, uint32_t *__restrict__ hi) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || !hard[i]) return;
  int32_t v[3];
  bool ok;
  codes_of(params, npad, q, i, v, ok);
  const int D = s->depth;
  const uint64_t c =
      morton3((uint32_t)((int64_t)v[0] - s->kmin[0]), (uint32_t)((int64_t)v[1] - s->kmin[1]),
              (uint32_t)((int64_t)v[2] - s->kmin[2]), D);
  const uint32_t p = pos[i];
  lo[p] = (uint32_t)c;
  hi[p] = (uint32_t)(c >> 32);
}

// Node starts of every depth (bit d of heads[j]) and their count per block.
__global__ void __launch_bounds__(kOcThreads)
k_oc_heads(const uint32_t *__restrict__ lo, const uint32_t *__restrict__ hi, const OcState *s,
           uint32_t *__restrict__ heads, uint32_t *__restrict__ blkcnt) {
  __shared__ uint32_t s_cnt[kOcThreads / 64][kLevels];
  const int64_t j = (int64_t)blockIdx.x * kOcThreads + threadIdx.x;
  const int64_t kept = s->kept;
  const int D = s->depth;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  uint32_t mask = 0;
  if (j < kept) {
    const uint64_t c = ((uint64_t)hi[j] << 32) | lo[j];
    const uint64_t p = j > 0 ? ((uint64_t)hi[j - 1] << 32) | lo[j - 1] : 0ull;
    for (int d = 0; d <= D; ++d) {
      const int sh = 3 * (D - d);
      if (j == 0 || (c >> sh) != (p >> sh)) mask |= 1u << d;
    }
    heads[j] = mask;
  }
#pragma unroll
  for (int d = 0; d < kLevels; ++d) {
    const uint64_t b = __ballot((mask >> d) & 1u);
    if (lane == 0) s_cnt[wave][d] = (uint32_t)__popcll(b);
  }
  __syncthreads();
  if (threadIdx.x < kLevels) {
    uint32_t t = 0;
    for (int w = 0; w < kOcThreads / 64; ++w) t += s_cnt[w][threadIdx.x];
    blkcnt[blockIdx.x * kLevels + threadIdx.x] = t;
  }
}

// Block d: exclusive scan of column d of blkcnt over the blocks; total nodes
// of depth d.
__global__ void __launch_bounds__(256)
k_oc_level_scan(const uint32_t *__restrict__ blkcnt, int64_t nb, uint32_t *__restrict__ blkpre,
                OcState *s) {
  __shared__ uint32_t s_part[256];
  const int d = blockIdx.x;
  const int64_t per = (nb + 255) / 256;
  const int64_t b0 = min(nb, (int64_t)threadIdx.x * per), b1 = min(nb, b0 + per);
  uint32_t t = 0;
  for (int64_t b = b0; b < b1; ++b) t += blkcnt[b * kLevels + d];
  s_part[threadIdx.x] = t;
  __syncthreads();
  uint32_t run = 0, tot = 0;
  for (int k = 0; k < 256; ++k) {
    const uint32_t v = s_part[k];
    if (k < (int)threadIdx.x) run += v;
    tot += v;
  }
  for (int64_t b = b0; b < b1; ++b) {
    const uint32_t v = blkcnt[b * kLevels + d];
    blkpre[b * kLevels + d] = run;
    run += v;
  }
  if (threadIdx.x == 0) s->ntot[d] = tot;
}

// Level sizes and token offsets; the header's token fields.
__global__ void k_oc_levels(OcState *s, sgs_octree_header *h, int64_t token_cap) {
  if (threadIdx.x != 0) return;
  const int D = s->depth;
  uint32_t t = 0;
  for (int d = 0; d < kLevels; ++d) {
    s->toff[d] = t;
    if (d < D) t += s->ntot[d];
    if (d < kMaxDepth) h->level_size[d] = d < D ? s->ntot[d] : 0;
  }
  s->tokens = t;
  s->unique = s->ntot[D];
  h->tokens = t;
  h->unique = s->ntot[D];
  if ((int64_t)t > token_cap) s->flags |= 2u;
}

// Zero the token words that the tokens occupy (within the capacity).
__global__ void k_oc_zero(uint32_t *__restrict__ words, int64_t cap_words, const OcState *s) {
  const int64_t need = min(cap_words, ((int64_t)s->tokens + 3) / 4);
  for (int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; w < need;
       w += (int64_t)gridDim.x * blockDim.x)
    words[w] = 0u;
}

// Every node of depth d >= 1 sets its bit in its parent's token; distinct
// voxels are written in order with their first sorted position.
__global__ void __launch_bounds__(kOcThreads)
k_oc_tokens(const uint32_t *__restrict__ lo, const uint32_t *__restrict__ hi,
            const uint32_t *__restrict__ heads, const uint32_t *__restrict__ blkpre,
            const OcState *s, uint32_t *__restrict__ tok_words, int64_t token_cap,
            uint64_t *__restrict__ codes_out, uint32_t *__restrict__ ustart) {
  __shared__ uint32_t s_cnt[kOcThreads / 64][kLevels];
  const int64_t j = (int64_t)blockIdx.x * kOcThreads + threadIdx.x;
  const int64_t kept = s->kept;
  const int D = s->depth;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const bool valid = j < kept;
  const uint32_t mask = valid ? heads[j] : 0u;
  const uint64_t le = lanemask_lt() | (1ull << lane);
#pragma unroll
  for (int d = 0; d < kLevels; ++d) {
    const uint64_t b = __ballot((mask >> d) & 1u);
    if (lane == 0) s_cnt[wave][d] = (uint32_t)__popcll(b);
  }
  __syncthreads();
  if (!valid) return;
  const uint64_t c = ((uint64_t)hi[j] << 32) | lo[j];
  uint32_t prev_rank = 0;
  for (int d = 0; d <= D; ++d) {
    // inclusive count of depth-d node starts up to j (the lanes of this wave
    // that returned have none)
    uint32_t r = blkpre[blockIdx.x * kLevels + d] +
                 (uint32_t)__popcll(__ballot((mask >> d) & 1u) & le);
    for (int w = 0; w < wave; ++w) r += s_cnt[w][d];
    const uint32_t rank = r - 1u;  // j's node of depth d
    if (d >= 1 && ((mask >> d) & 1u)) {
      const int64_t idx = (int64_t)s->toff[d - 1] + prev_rank;
      const uint32_t child = (uint32_t)(c >> (3 * (D - d))) & 7u;
      if (idx < token_cap)
        atomicOr(&tok_words[idx >> 2], (1u << child) << (8 * (int)(idx & 3)));
    }
    prev_rank = rank;
  }
  if ((mask >> D) & 1u) {
    codes_out[prev_rank] = c;
    ustart[prev_rank] = (uint32_t)j;
  }
}

// Duplicate flags of the distinct voxels (zero beyond them, for the scan).
__global__ void k_oc_dup_flags(const uint32_t *__restrict__ ustart, int64_t cap, const OcState *s,
                               uint32_t *__restrict__ flag) {
  const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= cap) return;
  const int64_t m = s->unique;
  uint32_t f = 0;
  if (u < m) {
    const uint32_t next = u + 1 < m ? ustart[u + 1] : s->kept;
    f = next - ustart[u] > 1u ? 1u : 0u;
  }
  flag[u] = f;
}

__global__ void k_oc_dup_write(const uint32_t *__restrict__ ustart, const uint32_t *__restrict__ pos,
                               int64_t cap, OcState *s, uint32_t *__restrict__ dup_index,
                               uint32_t *__restrict__ dup_count, int64_t dup_cap,
                               sgs_octree_header *h) {
  const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t m = s->unique;
  if (u == 0) {
    h->dups = s->total;
    if ((int64_t)s->total > dup_cap) s->flags |= 4u;
    h->flags = s->flags;
  }
  if (u >= m || u >= cap) return;
  const uint32_t next = u + 1 < m ? ustart[u + 1] : s->kept;
  const uint32_t d = next - ustart[u] - 1u;
  if (d == 0u) return;
  const uint32_t e = pos[u];
  if ((int64_t)e < dup_cap) {
    dup_index[e] = (uint32_t)u;
    dup_count[e] = d;
  }
}

// ---------------------------------------------------------------------------
// Octree decode
// ---------------------------------------------------------------------------
__global__ void k_od_popc(const uint8_t *__restrict__ tokens, int64_t T, uint32_t *__restrict__ pc) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g < T) pc[g] = (uint32_t)__popc((uint32_t)tokens[g]);
}

// Root code; the children over all tokens must number T - 1 + unique.
__global__ void k_od_root(uint64_t *__restrict__ nodes, int64_t T, int64_t unique,
                          const uint32_t *__restrict__ total, int64_t *info) {
  if (threadIdx.x != 0) return;
  if (T > 0) nodes[0] = 0ull;
  if ((int64_t)*total != T - 1 + unique) atomicOr((unsigned long long *)info, 1ull);
}

// Level d's tokens [t0, t0 + cnt) expand their nodes into children numbered
// 1 + chs[g] + k, which must fall in [c0, c1) (the next level's nodes, or
// the leaves: then written to codes_out at ci - leaf0).
__global__ void k_od_expand(const uint8_t *__restrict__ tokens, const uint32_t *__restrict__ chs,
                            uint64_t *__restrict__ nodes, int64_t t0, int64_t cnt, int64_t c0,
                            int64_t c1, int leaves, uint64_t *__restrict__ codes_out,
                            int64_t *info) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= cnt) return;
  const int64_t g = t0 + k;
  const uint32_t t = tokens[g];
  const uint64_t code = nodes[g];
  int64_t ci = 1 + (int64_t)chs[g];
  bool bad = t == 0u;
  for (int b = 0; b < 8; ++b) {
    if (!((t >> b) & 1u)) continue;
    if (ci < c0 || ci >= c1) {
      bad = true;
    } else {
      const uint64_t v = (code << 3) | (uint64_t)b;
      if (leaves) codes_out[ci - c0] = v; else nodes[ci] = v;
    }
    ++ci;
  }
  if (bad) atomicOr((unsigned long long *)info, 1ull);
}

// Positions of the decoded Gaussians: voxel u's copies start at u plus the
// duplicates of the voxels before it.
__global__ void k_od_positions(const uint64_t *__restrict__ codes, int64_t m, int depth,
                               int64_t kx, int64_t ky, int64_t kz, const float *__restrict__ q,
                               const uint32_t *__restrict__ dup_index,
                               const uint32_t *__restrict__ dup_count,
                               const uint32_t *__restrict__ dup_pre, int64_t dups, int64_t kept,
                               float *__restrict__ xyz, int64_t out_pad, int64_t *info) {
  const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= m) return;
  int64_t a = 0, b = dups;  // first entry with index >= u
  while (a < b) {
    const int64_t mid = (a + b) >> 1;
    if ((int64_t)dup_index[mid] < u) a = mid + 1; else b = mid;
  }
  bool bad = false;
  if (u == 0) {
    // entries ascending and inside [0, m); copies add up to kept
    bad = (int64_t)dup_pre[dups] + m != kept;
  }
  if (a < dups) {
    bad = bad || (int64_t)dup_index[a] >= m || (a > 0 && dup_index[a - 1] >= dup_index[a]) ||
          dup_count[a] == 0u;
  }
  const uint32_t reps = (a < dups && (int64_t)dup_index[a] == u) ? dup_count[a] : 0u;
  const int64_t base = u + (int64_t)dup_pre[a];
  const uint64_t c = codes[u];
  uint32_t w[3] = {0, 0, 0};
  for (int bb = 0; bb < depth; ++bb) {
    w[0] |= (uint32_t)((c >> (3 * bb + 2)) & 1u) << bb;
    w[1] |= (uint32_t)((c >> (3 * bb + 1)) & 1u) << bb;
    w[2] |= (uint32_t)((c >> (3 * bb)) & 1u) << bb;
  }
  const int64_t km[3] = {kx, ky, kz};
  float p[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) p[k] = (float)((int64_t)w[k] + km[k]) * q[k];
  for (uint32_t r = 0; r <= reps; ++r) {
    const int64_t o = base + r;
    if (o >= kept || o >= out_pad) {
      bad = true;
      break;
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) xyz[k * out_pad + o] = p[k];
  }
  if (bad) atomicOr((unsigned long long *)info, 1ull);
}

// ---------------------------------------------------------------------------
// Entropy coder: model
// ---------------------------------------------------------------------------
__global__ void k_fill_u32(uint32_t *__restrict__ p, int64_t count, uint32_t v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__device__ __forceinline__ int ctx_at(const uint8_t *__restrict__ sym, int64_t i, int64_t S,
                                      int order) {
  if (order == 0) return 0;
  return i % S == 0 ? 256 : (int)sym[i - 1];
}

// (context, symbol) counts.  Block (chunk, g) counts the chunk's symbols
// whose context lies in [64 g, 64 g + 64), in LDS as 16-bit halves of 32-bit
// words (a chunk holds at most 65535 symbols), then adds them to the global
// 32-bit counts.
constexpr int kCntThreads = 1024;
constexpr int64_t kCntPerBlock = 65535;
constexpr int kCntRows = 64;
constexpr int kCntGroups = (kCtx + kCntRows - 1) / kCntRows;
__global__ void __launch_bounds__(kCntThreads)
k_ans_count(const uint8_t *__restrict__ sym, int64_t n, int64_t S, int order,
            uint32_t *__restrict__ cnt) {
  __shared__ uint32_t s_h[kCntRows * 128];
  const int g = blockIdx.y, r0 = g * kCntRows;
  for (int w = threadIdx.x; w < kCntRows * 128; w += kCntThreads) s_h[w] = 0u;
  __syncthreads();
  const int64_t a = (int64_t)blockIdx.x * kCntPerBlock;
  const int64_t e = min(n, a + kCntPerBlock);
  for (int64_t i = a + threadIdx.x; i < e; i += kCntThreads) {
    const int x = ctx_at(sym, i, S, order) - r0;
    if (x < 0 || x >= kCntRows) continue;
    const int k = x * 256 + sym[i];
    atomicAdd(&s_h[k >> 1], 1u << (16 * (k & 1)));
  }
  __syncthreads();
  for (int w = threadIdx.x; w < kCntRows * 128; w += kCntThreads) {
    const int k = r0 * 256 + 2 * w;
    if (k >= kCtx * 256) break;
    const uint32_t v = s_h[w];
    if (v & 0xFFFFu) atomicAdd(&cnt[k], v & 0xFFFFu);
    if (v >> 16) atomicAdd(&cnt[k + 1], v >> 16);
  }
}

// One block per context: frequencies from the counts, and the context's
// share of the ideal code length -sum c_s log2(f_s / M).
__global__ void __launch_bounds__(256)
k_ans_normalize(const uint32_t *__restrict__ cnt, uint16_t *__restrict__ freq,
                double *__restrict__ bits_part) {
  __shared__ uint64_t s_n[4];
  __shared__ uint32_t s_k[4], s_sum[4];
  __shared__ uint64_t s_best[4];
  const int x = blockIdx.x, s = threadIdx.x, wave = s >> 6, lane = s & 63;
  const uint32_t c = cnt[x * 256 + s];
  uint64_t N = c;
  uint32_t K = c ? 1u : 0u;
  // most frequent, lowest symbol on ties: maximize (count << 8) | (255 - s)
  uint64_t best = c ? (((uint64_t)c << 8) | (uint64_t)(255 - s)) : 0ull;
  for (int o = 32; o >= 1; o >>= 1) {
    N += __shfl_xor(N, o, 64);
    K += __shfl_xor(K, o, 64);
    const uint64_t ob = __shfl_xor(best, o, 64);
    best = ob > best ? ob : best;
  }
  if (lane == 0) {
    s_n[wave] = N;
    s_k[wave] = K;
    s_best[wave] = best;
  }
  __syncthreads();
  N = s_n[0] + s_n[1] + s_n[2] + s_n[3];
  K = s_k[0] + s_k[1] + s_k[2] + s_k[3];
  best = s_best[0];
  for (int w = 1; w < 4; ++w) best = s_best[w] > best ? s_best[w] : best;
  uint32_t f = 0;
  if (N && c) f = 1u + (uint32_t)((uint64_t)c * (uint64_t)(kAnsM - K) / N);
  uint32_t sum = f;
  for (int o = 32; o >= 1; o >>= 1) sum += __shfl_xor(sum, o, 64);
  __syncthreads();
  if (lane == 0) s_sum[wave] = sum;
  __syncthreads();
  sum = s_sum[0] + s_sum[1] + s_sum[2] + s_sum[3];
  if (N && s == 255 - (int)(best & 0xFFu)) f += kAnsM - sum;
  freq[x * 256 + s] = (uint16_t)f;
  double b = c ? -(double)c * log2((double)f / (double)kAnsM) : 0.0;
  for (int o = 32; o >= 1; o >>= 1) b += __shfl_xor(b, o, 64);
  __shared__ double s_b[4];
  if (lane == 0) s_b[wave] = b;
  __syncthreads();
  if (s == 0) bits_part[x] = ((s_b[0] + s_b[1]) + s_b[2]) + s_b[3];
}

__global__ void k_ans_bits_sum(const double *__restrict__ part, int rows, double *out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double t = 0.0;
  for (int x = 0; x < rows; ++x) t += part[x];
  *out = t;
}

// ---------------------------------------------------------------------------
// Entropy coder: tables
// ---------------------------------------------------------------------------
// Encoder table: (f << 16) | cum per (context, symbol); flags bit 2 when a
// used row does not sum to M.
__global__ void __launch_bounds__(256)
k_ans_enc_table(const uint16_t *__restrict__ freq, uint32_t *__restrict__ tab, int64_t *info) {
  __shared__ uint32_t s_f[256];
  const int x = blockIdx.x, s = threadIdx.x;
  const uint32_t f = freq[x * 256 + s];
  s_f[s] = f;
  __syncthreads();
  uint32_t cum = 0, tot = 0;
  for (int k = 0; k < 256; ++k) {
    const uint32_t v = s_f[k];
    if (k < s) cum += v;
    tot += v;
  }
  tab[x * 256 + s] = (f << 16) | (cum & 0xFFFFu);
  if (s == 0 && tot != 0u && tot != kAnsM) atomicOr((unsigned long long *)info, 4ull);
}

// Decoder table: slot -> sym | (f - 1) << 8 | cum << 20 per context (kNoSym
// where no symbol owns the slot); flags bit 2 for a row not summing to M.
__device__ __forceinline__ void dec_table_row(const uint16_t *__restrict__ freq,
                                              uint32_t *__restrict__ tab, int x, int64_t *info) {
  __shared__ uint32_t s_cum[257];
  const int s = threadIdx.x;
  const uint32_t f = freq[x * 256 + s];
  s_cum[s + 1] = f;
  if (s == 0) s_cum[0] = 0;
  __syncthreads();
  if (s == 0)
    for (int k = 1; k <= 256; ++k) s_cum[k] += s_cum[k - 1];
  __syncthreads();
  const uint32_t tot = s_cum[256];
  if (s == 0 && tot != 0u && tot != kAnsM) atomicOr((unsigned long long *)info, 4ull);
  const bool ok = tot == kAnsM;
  for (uint32_t slot = s; slot < kAnsM; slot += 256) {
    uint32_t e = kNoSym;
    if (ok) {
      int a = 0, b = 255;  // largest k with cum[k] <= slot
      while (a < b) {
        const int mid = (a + b + 1) >> 1;
        if (s_cum[mid] <= slot) a = mid; else b = mid - 1;
      }
      const uint32_t fk = s_cum[a + 1] - s_cum[a];
      if (fk) e = (uint32_t)a | ((fk - 1u) << 8) | (s_cum[a] << 20);
    }
    tab[(int64_t)x * kAnsM + slot] = e;
  }
}

__global__ void __launch_bounds__(256)
k_ans_dec_table(const uint16_t *__restrict__ freq, uint32_t *__restrict__ tab, int64_t *info) {
  dec_table_row(freq, tab, blockIdx.x, info);
}

// ---------------------------------------------------------------------------
// Entropy coder: encode (WRITE = false: count each block's words)
// ---------------------------------------------------------------------------
template <bool WRITE>
__global__ void __launch_bounds__(64)
k_ans_encode(const uint8_t *__restrict__ sym, int64_t n, int64_t S, int order,
             const uint32_t *__restrict__ tab, uint32_t *__restrict__ blk_words,
             const uint32_t *__restrict__ blk_off, uint16_t *__restrict__ words, int64_t word_cap,
             int64_t *info) {
  const int64_t b = blockIdx.x;
  const int lane = threadIdx.x;
  const int64_t a = b * 64 * S + (int64_t)lane * S;  // this lane's first symbol
  const int64_t len = max((int64_t)0, min(S, n - a));
  const uint64_t above = lane == 63 ? 0ull : (~0ull << (lane + 1));
  uint32_t x = kAnsL;
  uint32_t pushes = 0;          // words pushed by the wave so far (push order)
  const uint32_t total = WRITE ? blk_words[b] - 128u : 0u;
  const int64_t base = WRITE ? (int64_t)blk_off[b] : 0;
  bool bad = false;
  for (int64_t t = S - 1; t >= 0; --t) {
    const bool act = t < len;
    uint32_t f = 0, cum = 0;
    if (act) {
      const int64_t i = a + t;
      const uint32_t e = tab[ctx_at(sym, i, S, order) * 256 + sym[i]];
      f = e >> 16;
      cum = e & 0xFFFFu;
      bad = bad || f == 0u;
    }
    const bool push = act && f != 0u && (uint64_t)x >= ((uint64_t)(kAnsL >> kAnsPB) << 16) * f;
    const uint64_t m = __ballot(push);
    if (push) {
      if (WRITE) {
        // lanes push in descending order: those above come first
        const uint32_t k = pushes + (uint32_t)__popcll(m & above);
        const int64_t pos = base + 128 + (int64_t)(total - 1u - k);
        if (pos < word_cap) words[pos] = (uint16_t)(x & 0xFFFFu);
      }
      x >>= 16;
    }
    pushes += (uint32_t)__popcll(m);
    if (act && f != 0u) x = ((x / f) << kAnsPB) + (x % f) + cum;
  }
  if (WRITE) {
    const int64_t p = base + 2 * lane;
    if (p + 1 < word_cap) {
      words[p] = (uint16_t)(x >> 16);
      words[p + 1] = (uint16_t)(x & 0xFFFFu);
    }
  } else if (lane == 0) {
    blk_words[b] = 128u + pushes;
  }
  if (__ballot(bad) != 0ull && lane == 0) atomicOr((unsigned long long *)info + 1, 1ull);
}

// Block offsets (int64) and the totals; flags bit 1 when the words exceed
// the capacity.
__global__ void k_ans_offsets(const uint32_t *__restrict__ scan, int64_t nb,
                              int64_t *__restrict__ block_off, int64_t word_cap, int64_t *info) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b > nb) return;
  block_off[b] = scan[b];
  if (b == nb) {
    info[0] = scan[nb];
    if ((int64_t)scan[nb] > word_cap) atomicOr((unsigned long long *)info + 1, 2ull);
  }
}

// ---------------------------------------------------------------------------
// Entropy coder: decode
// ---------------------------------------------------------------------------
// Decode of rANS block b by one wave.  tab: the decode table (LDS for an
// order-0 stream, else global).  The block's words are read through a
// window of 256 in four registers per lane (lane i holds word base + 64 r +
// i of register r): a lane's next word is taken from the window with a
// cross-lane read, and the window slides by 64 when the first register is
// used up, its refill loaded two slides before it is read.  Symbols are
// kept in registers and stored 16 at a time where the lane's run is 16-byte
// aligned.
__device__ __forceinline__ void decode_block(const uint16_t *__restrict__ words, int64_t n_words,
                                             const int64_t *__restrict__ block_off, int64_t n,
                                             int64_t S, int order, const uint32_t *tab,
                                             uint8_t *__restrict__ sym, int64_t *info, int64_t b) {
  const int lane = threadIdx.x & 63;
  const int64_t a = b * 64 * S + (int64_t)lane * S;
  const int64_t len = max((int64_t)0, min(S, n - a));
  const int64_t off = block_off[b], end = block_off[b + 1];
  bool bad = off < 0 || end > n_words || end - off < 128;
  if (__ballot(bad) != 0ull) {
    if (lane == 0) atomicOr((unsigned long long *)info, 1ull);
    return;
  }
  uint32_t x = ((uint32_t)words[off + 2 * lane] << 16) | words[off + 2 * lane + 1];
  int64_t p = off + 128, base = p;
  auto wload = [&](int64_t i) -> uint32_t { return i < end ? (uint32_t)words[i] : 0u; };
  uint32_t w0 = wload(base + lane), w1 = wload(base + 64 + lane), w2 = wload(base + 128 + lane),
           w3 = wload(base + 192 + lane);
  const uint64_t lt = lanemask_lt();
  const bool vec = ((uintptr_t)(sym + a) & 15u) == 0u;
  int ctx = order ? 256 : 0;
  bool alive = true;
  for (int64_t t0 = 0; t0 < S; t0 += 16) {
    uint32_t pk[4] = {0u, 0u, 0u, 0u};
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const int64_t t = t0 + j;
      const bool act = t < len && alive;
      bool need = false;
      if (act) {
        const uint32_t slot = x & (kAnsM - 1u);
        const uint32_t e = tab[ctx * (int)kAnsM + (int)slot];
        if (e == kNoSym) {
          alive = false;
          bad = true;
        } else {
          const uint32_t sv = e & 0xFFu, f = ((e >> 8) & 0xFFFu) + 1u, cum = e >> 20;
          x = f * (x >> kAnsPB) + slot - cum;
          pk[j >> 2] |= sv << (8 * (j & 3));
          if (order) ctx = (int)sv;
          need = x < kAnsL;
        }
      }
      const uint64_t m = __ballot(need);
      if (m) {
        // the window: offsets < 64 + 63 always lie in its first two registers
        const int o = (int)(p - base) + __popcll(m & lt);
        const uint32_t r0 = (uint32_t)__shfl((int)w0, o & 63, 64);
        const uint32_t r1 = (uint32_t)__shfl((int)w1, o & 63, 64);
        if (need) {
          if (p + __popcll(m & lt) < end) {
            x = (x << 16) | (o < 64 ? r0 : r1);
          } else {
            alive = false;
            bad = true;
          }
        }
        p += __popcll(m);
        if (p - base >= 64) {
          w0 = w1;
          w1 = w2;
          w2 = w3;
          w3 = wload(base + 256 + lane);
          base += 64;
        }
      }
    }
    // this lane's symbols of the round
    const int64_t cnt = min((int64_t)16, len - t0);
    if (cnt == 16 && vec) {
      *(uint4 *)(sym + a + t0) = make_uint4(pk[0], pk[1], pk[2], pk[3]);
    } else if (cnt > 0) {
      for (int k = 0; k < (int)cnt; ++k) sym[a + t0 + k] = (uint8_t)(pk[k >> 2] >> (8 * (k & 3)));
    }
  }
  // every word read, every lane back at the encoder's initial state
  bad = bad || (lane == 0 && p != end) || x != kAnsL;
  if (__ballot(bad) != 0ull && lane == 0) atomicOr((unsigned long long *)info, 1ull);
}

// Four waves per workgroup, wave w decoding block 4 blockIdx.x + w; an
// order-0 stream's table (16 KB) is staged in LDS once for the four.
constexpr int kDecWaves = 4;
__device__ __forceinline__ void decode_blocks(const uint16_t *__restrict__ words, int64_t n_words,
                                              const int64_t *__restrict__ block_off, int64_t n,
                                              int64_t S, int order, int64_t nb,
                                              const uint32_t *__restrict__ gtab,
                                              uint8_t *__restrict__ sym, int64_t *info,
                                              int64_t group) {
  __shared__ uint32_t s_tab[kAnsM];
  if (order == 0) {
    for (int e = threadIdx.x; e < (int)kAnsM; e += blockDim.x) s_tab[e] = gtab[e];
    __syncthreads();
  }
  const int64_t b = group * kDecWaves + (threadIdx.x >> 6);
  if (b >= nb) return;
  // two call sites so that each sees one address space (LDS reads for the
  // staged table)
  if (order == 0)
    decode_block(words, n_words, block_off, n, S, 0, s_tab, sym, info, b);
  else
    decode_block(words, n_words, block_off, n, S, order, gtab, sym, info, b);
}

__global__ void __launch_bounds__(64 * kDecWaves)
k_ans_decode(const uint16_t *__restrict__ words, int64_t n_words,
             const int64_t *__restrict__ block_off, int64_t n, int64_t S, int order, int64_t nb,
             const uint32_t *__restrict__ tab, uint8_t *__restrict__ sym, int64_t *info) {
  decode_blocks(words, n_words, block_off, n, S, order, nb, tab, sym, info, blockIdx.x);
}

// Several streams in one launch: block (b, s) decodes block b of stream s.
struct AnsDev {
  const uint16_t *words;
  int64_t n_words;
  const int64_t *block_off;
  int64_t n;
  const uint16_t *freq;
  uint8_t *sym;
  uint32_t *tab;
  int64_t S, nb;
  int32_t order, pad;
};

__global__ void __launch_bounds__(256)
k_ans_dec_table_multi(const AnsDev *__restrict__ d, int64_t *info) {
  const AnsDev &a = d[blockIdx.y];
  const int x = blockIdx.x;
  if ((a.order == 0 && x > 0) || a.nb == 0) return;
  dec_table_row(a.freq, a.tab, x, info + blockIdx.y);
}

__global__ void __launch_bounds__(64 * kDecWaves)
k_ans_decode_multi(const AnsDev *__restrict__ d, int64_t *info) {
  const AnsDev &a = d[blockIdx.y];
  if ((int64_t)blockIdx.x * kDecWaves >= a.nb) return;  // whole workgroup: before the barrier
  decode_blocks(a.words, a.n_words, a.block_off, a.n, a.S, a.order, a.nb, a.tab, a.sym,
                info + blockIdx.y, blockIdx.x);
}

// ---------------------------------------------------------------------------
// Attributes: Morton order, DPCM byte planes, reconstruction, Fourier
// positional embedding
// ---------------------------------------------------------------------------
__global__ void k_flags_u8(const uint8_t *__restrict__ m, int64_t n, uint32_t *__restrict__ f) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) f[i] = m[i] ? 1u : 0u;
}

// Key of kept Gaussian i: its voxel's rank among the distinct codes (binary
// search), value: i; at its position in index order.
__global__ void k_mo_keys(const float *__restrict__ params, int64_t npad, int64_t n,
                          const float *__restrict__ q, const uint8_t *__restrict__ hard,
                          const uint32_t *__restrict__ pos, int depth, int64_t kx, int64_t ky,
                          int64_t kz, const uint64_t *__restrict__ codes, int64_t m,
                          uint32_t *__restrict__ key, uint32_t *__restrict__ val) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || !hard[i]) return;
  int32_t v[3];
  bool ok;
  codes_of(params, npad, q, i, v, ok);
  const uint64_t c = morton3((uint32_t)((int64_t)v[0] - kx), (uint32_t)((int64_t)v[1] - ky),
                             (uint32_t)((int64_t)v[2] - kz), depth);
  int64_t a = 0, b = m;  // first code >= c
  while (a < b) {
    const int64_t mid = (a + b) >> 1;
    if (codes[mid] < c) a = mid + 1; else b = mid;
  }
  const uint32_t p = pos[i];
  key[p] = (uint32_t)a;
  val[p] = (uint32_t)i;
}

__global__ void k_copy_u32(const uint32_t *__restrict__ src, int64_t count, int32_t *__restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) dst[i] = (int32_t)src[i];
}

struct AttrChan {
  float q;
  int32_t kmin, planes, row0, pred;
};
struct AttrChans {
  AttrChan ch[SGS_NCH - 3];
};

// Planes of channel 3 + blockIdx.y at serialized position j: the value's
// residual against the previous position of its group, zigzag-mapped, cut
// into bytes (most significant first).
__global__ void k_attr_planes(const float *__restrict__ params, int64_t npad,
                              const int32_t *__restrict__ perm, int64_t kept, int64_t S,
                              AttrChans C, uint8_t *__restrict__ planes) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const AttrChan a = C.ch[blockIdx.y];
  if (j >= kept || a.planes == 0) return;
  const float *y = params + (int64_t)(3 + blockIdx.y) * npad;
  bool ok;
  const int64_t v = (int64_t)sgs_code_of(y[perm[j]], a.q, ok) - a.kmin;
  uint64_t z = (uint64_t)v;  // predictor 0: the value itself
  if (a.pred) {
    const int64_t pv = j % S == 0 ? 0 : (int64_t)sgs_code_of(y[perm[j - 1]], a.q, ok) - a.kmin;
    const int64_t d = v - pv;
    z = d >= 0 ? (uint64_t)(2 * d) : (uint64_t)(-2 * d - 1);
  }
  for (int t = 0; t < a.planes; ++t)
    planes[(int64_t)(a.row0 + t) * kept + j] = (uint8_t)(z >> (8 * (a.planes - 1 - t)));
}

// Group g of channel 3 + blockIdx.y, one wave: the running sum of the
// residuals (a wave scan per round of 256 positions, four per lane, carried
// from round to round), then the dequantized values fl32((kmin + v) q) into
// out [59][out_pad].
__global__ void __launch_bounds__(256)
k_attr_reconstruct(const uint8_t *__restrict__ planes, int64_t kept, int64_t S, AttrChans C,
                   float *__restrict__ out, int64_t out_pad) {
  const AttrChan a = C.ch[blockIdx.y];
  const int lane = threadIdx.x & 63;
  const int64_t g = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int64_t j0 = g * S;
  if (j0 >= kept) return;
  const int64_t j1 = min(kept, j0 + S);
  float *o = out + (int64_t)(3 + blockIdx.y) * out_pad;
  int64_t carry = 0;
  for (int64_t c0 = j0; c0 < j1; c0 += 256) {
    int64_t d[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int64_t j = c0 + 4 * lane + k;
      uint64_t z = 0;
      if (j < j1)
        for (int t = 0; t < a.planes; ++t) z = (z << 8) | planes[(int64_t)(a.row0 + t) * kept + j];
      d[k] = (z & 1u) ? -(int64_t)((z + 1) >> 1) : (int64_t)(z >> 1);
      if (!a.pred) {  // predictor 0: the value itself
        if (j < j1) o[j] = (float)(a.kmin + (int64_t)z) * a.q;
      }
    }
    if (!a.pred) continue;
    const int64_t sum = (d[0] + d[1]) + (d[2] + d[3]);
    int64_t incl = sum;
#pragma unroll
    for (int sh = 1; sh < 64; sh <<= 1) {
      const int64_t u = __shfl_up(incl, sh, 64);
      if (lane >= sh) incl += u;
    }
    int64_t run = carry + incl - sum;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int64_t j = c0 + 4 * lane + k;
      run += d[k];
      if (j < j1) o[j] = (float)(a.kmin + run) * a.q;
    }
    carry += __shfl(incl, 63, 64);
  }
}

// PE(mu) = W phi(mu) + b, phi = [mu; sin(2 pi 2^l mu); cos(2 pi 2^l mu)]
// (band-major, axis-minor): one thread per Gaussian, W and b in LDS, the
// features in registers (L fixed per instance), four outputs per store.
constexpr int kPeMaxD = 64;
template <int L>
__global__ void __launch_bounds__(256)
k_pos_embed(const float *__restrict__ xyz, int64_t pad, int64_t count, int d,
            const float *__restrict__ W, const float *__restrict__ bias, float *__restrict__ out) {
  constexpr int F = 3 + 6 * L;
  __shared__ float s_w[kPeMaxD * F];
  __shared__ float s_b[kPeMaxD];
  for (int e = threadIdx.x; e < d * F; e += blockDim.x) s_w[e] = W[e];
  for (int e = threadIdx.x; e < d; e += blockDim.x) s_b[e] = bias[e];
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  float phi[F];
  const float mu[3] = {xyz[i], xyz[pad + i], xyz[2 * pad + i]};
#pragma unroll
  for (int c = 0; c < 3; ++c) phi[c] = mu[c];
#pragma unroll
  for (int l = 0; l < L; ++l)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      // sin(2 pi 2^l mu) = sinpi(2^(l+1) mu); the product is exact
      const float x = ldexpf(mu[c], l + 1);
      phi[3 + 3 * l + c] = sinpif(x);
      phi[3 + 3 * L + 3 * l + c] = cospif(x);
    }
  float4 *o = (float4 *)(out + i * d);
  for (int k = 0; k < d; k += 4) {
    float acc[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const float *w = s_w + (k + u) * F;
      float a = s_b[k + u];
#pragma unroll
      for (int f = 0; f < F; ++f) a = fmaf(w[f], phi[f], a);
      acc[u] = a;
    }
    o[k >> 2] = make_float4(acc[0], acc[1], acc[2], acc[3]);
  }
}

}  // namespace

// ---------------------------------------------------------------------------
// Scratch
// ---------------------------------------------------------------------------
struct SgsCoding {
  OcState *st = nullptr;
  int32_t *oc_part = nullptr;  // range partials [kOcRangeBlocks][8]
  int64_t cap_n = 0;        // elements the octree buffers hold
  uint32_t *key[4] = {nullptr, nullptr, nullptr, nullptr};  // lo0, lo1, hi0, hi1
  uint32_t *heads = nullptr, *ustart = nullptr, *dflag = nullptr, *dpos = nullptr;
  uint32_t *blkcnt = nullptr, *blkpre = nullptr;
  int64_t cap_tok = 0;      // tokens the decode buffers hold
  uint64_t *nodes = nullptr;
  uint32_t *pc = nullptr, *chs = nullptr;
  int64_t cap_dup = 0;
  uint32_t *dpre = nullptr;
  uint32_t *ans_cnt = nullptr, *ans_enc = nullptr, *ans_dec = nullptr;
  double *ans_bits = nullptr;
  int64_t cap_blocks = 0;
  uint32_t *ans_blk = nullptr, *ans_scan = nullptr;
  uint32_t *multi_tab = nullptr;   // decode tables of a multi-stream decode
  int64_t multi_tab_words = 0;
  unsigned char *multi_desc = nullptr;  // its stream descriptors
  int32_t multi_cap = 0;
};

namespace {

template <typename T>
void cfree(T *&p) {
  if (p) (void)hipFree((void *)p);
  p = nullptr;
}

template <typename T>
hipError_t calloc_(T *&p, int64_t count) {
  cfree(p);
  return hipMalloc((void **)&p, sizeof(T) * (size_t)(count > 0 ? count : 1));
}

hipError_t coding_base(sgs_ctx *c) {
  if (!c->coding) c->coding = new (std::nothrow) SgsCoding();
  if (!c->coding) return hipErrorOutOfMemory;
  SgsCoding *k = c->coding;
  if (!k->st) {
    hipError_t e = calloc_(k->st, 1);
    if (e != hipSuccess) return e;
    if ((e = calloc_(k->oc_part, kOcRangeBlocks * 8)) != hipSuccess) return e;
    if ((e = calloc_(k->ans_cnt, kCtx * 256)) != hipSuccess) return e;
    if ((e = calloc_(k->ans_enc, kCtx * 256)) != hipSuccess) return e;
    if ((e = calloc_(k->ans_dec, (int64_t)kCtx * kAnsM)) != hipSuccess) return e;
    if ((e = calloc_(k->ans_bits, kCtx + 1)) != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t coding_octree(sgs_ctx *c, int64_t n) {
  hipError_t e = coding_base(c);
  if (e != hipSuccess) return e;
  SgsCoding *k = c->coding;
  if (n > k->cap_n) {
    const int64_t nb = (n + kOcThreads - 1) / kOcThreads;
    k->cap_n = 0;
    for (int i = 0; i < 4; ++i)
      if ((e = calloc_(k->key[i], n)) != hipSuccess) return e;
    if ((e = calloc_(k->heads, n)) != hipSuccess) return e;
    if ((e = calloc_(k->ustart, n)) != hipSuccess) return e;
    if ((e = calloc_(k->dflag, n)) != hipSuccess) return e;
    if ((e = calloc_(k->dpos, n + 1)) != hipSuccess) return e;
    if ((e = calloc_(k->blkcnt, nb * kLevels)) != hipSuccess) return e;
    if ((e = calloc_(k->blkpre, nb * kLevels)) != hipSuccess) return e;
    k->cap_n = n;
  }
  return ensure_tmp(c, (n + 4095) / 4096 + 1, radix_hist_words(n));
}

hipError_t coding_decode(sgs_ctx *c, int64_t T, int64_t dups) {
  hipError_t e = coding_base(c);
  if (e != hipSuccess) return e;
  SgsCoding *k = c->coding;
  if (T > k->cap_tok) {
    k->cap_tok = 0;
    if ((e = calloc_(k->nodes, T)) != hipSuccess) return e;
    if ((e = calloc_(k->pc, T)) != hipSuccess) return e;
    if ((e = calloc_(k->chs, T + 1)) != hipSuccess) return e;
    k->cap_tok = T;
  }
  if (dups + 1 > k->cap_dup) {
    k->cap_dup = 0;
    if ((e = calloc_(k->dpre, dups + 1)) != hipSuccess) return e;
    k->cap_dup = dups + 1;
  }
  const int64_t most = T > dups ? T : dups;
  return ensure_tmp(c, (most + 4095) / 4096 + 1, 0);
}

hipError_t coding_blocks(sgs_ctx *c, int64_t nb) {
  hipError_t e = coding_base(c);
  if (e != hipSuccess) return e;
  SgsCoding *k = c->coding;
  if (nb + 1 > k->cap_blocks) {
    k->cap_blocks = 0;
    if ((e = calloc_(k->ans_blk, nb + 1)) != hipSuccess) return e;
    if ((e = calloc_(k->ans_scan, nb + 1)) != hipSuccess) return e;
    k->cap_blocks = nb + 1;
  }
  return ensure_tmp(c, (nb + 4095) / 4096 + 1, 0);
}

unsigned grid_for(int64_t count, int threads, int64_t most = 65536) {
  int64_t g = (count + threads - 1) / threads;
  if (g < 1) g = 1;
  return (unsigned)(g < most ? g : most);
}

}  // namespace

void coding_free(sgs_ctx *c) {
  SgsCoding *k = c->coding;
  if (!k) return;
  cfree(k->st);
  cfree(k->oc_part);
  for (auto &p : k->key) cfree(p);
  cfree(k->heads);
  cfree(k->ustart);
  cfree(k->dflag);
  cfree(k->dpos);
  cfree(k->blkcnt);
  cfree(k->blkpre);
  cfree(k->nodes);
  cfree(k->pc);
  cfree(k->chs);
  cfree(k->dpre);
  cfree(k->ans_cnt);
  cfree(k->ans_enc);
  cfree(k->ans_dec);
  cfree(k->ans_bits);
  cfree(k->ans_blk);
  cfree(k->ans_scan);
  cfree(k->multi_tab);
  cfree(k->multi_desc);
  delete k;
  c->coding = nullptr;
}

int64_t sgs_ans_max_words(int64_t n, int32_t lane_len) {
  if (n < 0 || lane_len < 1) return -1;
  const int64_t B = 64 * (int64_t)lane_len;
  return 128 * ((n + B - 1) / B) + n;
}

hipError_t launch_octree_encode(sgs_ctx *c, const float *params, int64_t npad, int64_t n,
                                const float *q, const uint8_t *hard, uint8_t *tokens,
                                int64_t token_cap, uint64_t *codes, uint32_t *dup_index,
                                uint32_t *dup_count, int64_t dup_cap, sgs_octree_header *h) {
  hipError_t e = coding_octree(c, n);
  if (e != hipSuccess) return e;
  SgsCoding *k = c->coding;
  hipStream_t st = c->stream;
  const int64_t nb = (n + kOcThreads - 1) / kOcThreads;
  k_oc_init<<<1, 64, 0, st>>>(k->st);
  const int nparts = (int)grid_for(n, kOcThreads, kOcRangeBlocks);
  k_oc_range<<<nparts, kOcThreads, 0, st>>>(params, npad, n, q, hard, k->oc_part);
  k_oc_depth<<<1, 256, 0, st>>>(k->oc_part, nparts, k->st, h);
  k_flags_u8<<<grid_for(n, 256, 1 << 30), 256, 0, st>>>(hard, n, k->dflag);
  e = launch_exclusive_scan(c, k->dflag, k->dpos, n, nullptr);
  if (e != hipSuccess) return e;
  k_oc_codes<<<(unsigned)nb, kOcThreads, 0, st>>>(params, npad, n, q, hard, k->dpos, k->st,
                                                   k->key[0], k->key[2]);
  // 64-bit keys: low words (carrying the high ones), then the high words
  // (carrying the low ones); both passes stable
  int w1 = 0, w2 = 0;
  {
    uint32_t *keys[2] = {k->key[0], k->key[1]}, *vals[2] = {k->key[2], k->key[3]};
    e = launch_radix_sort(c, keys, vals, n, 32, &w1, &k->st->kept);
    if (e != hipSuccess) return e;
  }
  {
    uint32_t *keys[2] = {k->key[2], k->key[3]}, *vals[2] = {k->key[0], k->key[1]};
    e = launch_radix_sort(c, keys, vals, n, 32, &w2, &k->st->kept, 0, w1);
    if (e != hipSuccess) return e;
  }
  const uint32_t *lo = k->key[w2], *hi = k->key[2 + w2];
  k_oc_heads<<<(unsigned)nb, kOcThreads, 0, st>>>(lo, hi, k->st, k->heads, k->blkcnt);
  k_oc_level_scan<<<kLevels, 256, 0, st>>>(k->blkcnt, nb, k->blkpre, k->st);
  k_oc_levels<<<1, 64, 0, st>>>(k->st, h, token_cap);
  k_oc_zero<<<grid_for(token_cap / 4, 256, 4096), 256, 0, st>>>((uint32_t *)tokens,
                                                                 token_cap / 4, k->st);
  k_oc_tokens<<<(unsigned)nb, kOcThreads, 0, st>>>(lo, hi, k->heads, k->blkpre, k->st,
                                                    (uint32_t *)tokens, token_cap, codes,
                                                    k->ustart);
  k_oc_dup_flags<<<grid_for(n, 256, 1 << 30), 256, 0, st>>>(k->ustart, n, k->st, k->dflag);
  e = launch_exclusive_scan(c, k->dflag, k->dpos, n, &k->st->total);
  if (e != hipSuccess) return e;
  k_oc_dup_write<<<grid_for(n, 256, 1 << 30), 256, 0, st>>>(k->ustart, k->dpos, n, k->st,
                                                            dup_index, dup_count, dup_cap, h);
  return hipGetLastError();
}

hipError_t launch_octree_decode(sgs_ctx *c, const sgs_octree_header *h, const uint8_t *tokens,
                                const uint32_t *dup_index, const uint32_t *dup_count,
                                const float *q, uint64_t *codes, float *xyz, int64_t out_pad,
                                int64_t *info) {
  const int64_t T = h->tokens, m = h->unique, dups = h->dups;
  hipError_t e = coding_decode(c, T, dups);
  if (e != hipSuccess) return e;
  SgsCoding *k = c->coding;
  hipStream_t st = c->stream;
  k_fill_u32<<<1, 64, 0, st>>>((uint32_t *)info, 2, 0u);
  if (T == 0) return hipGetLastError();
  k_od_popc<<<grid_for(T, 256, 1 << 30), 256, 0, st>>>(tokens, T, k->pc);
  e = launch_exclusive_scan(c, k->pc, k->chs, T, nullptr);
  if (e != hipSuccess) return e;
  k_od_root<<<1, 64, 0, st>>>(k->nodes, T, m, k->chs + T, info);
  int64_t t0 = 0;
  for (int d = 0; d < h->depth; ++d) {
    const int64_t cnt = h->level_size[d];
    const bool leaves = d + 1 == h->depth;
    const int64_t c0 = leaves ? T : t0 + cnt, c1 = leaves ? T + m : c0 + h->level_size[d + 1];
    if (cnt > 0)
      k_od_expand<<<grid_for(cnt, 256, 1 << 30), 256, 0, st>>>(
          tokens, k->chs, k->nodes, t0, cnt, c0, c1, leaves ? 1 : 0, codes, info);
    t0 += cnt;
  }
  e = launch_exclusive_scan(c, dup_count, k->dpre, dups, nullptr);
  if (e != hipSuccess) return e;
  if (m > 0)
    k_od_positions<<<grid_for(m, 256, 1 << 30), 256, 0, st>>>(
        codes, m, h->depth, h->kmin[0], h->kmin[1], h->kmin[2], q, dup_index, dup_count, k->dpre,
        dups, h->kept, xyz, out_pad, info);
  return hipGetLastError();
}

hipError_t launch_ans_model(sgs_ctx *c, const uint8_t *sym, int64_t n, int order, int64_t S,
                            uint16_t *freq, double *bits) {
  hipError_t e = coding_base(c);
  if (e != hipSuccess) return e;
  SgsCoding *k = c->coding;
  hipStream_t st = c->stream;
  k_fill_u32<<<64, 256, 0, st>>>(k->ans_cnt, kCtx * 256, 0u);
  if (n > 0) {
    const dim3 grid((unsigned)((n + kCntPerBlock - 1) / kCntPerBlock), order ? kCntGroups : 1);
    k_ans_count<<<grid, kCntThreads, 0, st>>>(sym, n, S, order, k->ans_cnt);
  }
  k_ans_normalize<<<kCtx, 256, 0, st>>>(k->ans_cnt, freq, k->ans_bits);
  if (bits) k_ans_bits_sum<<<1, 64, 0, st>>>(k->ans_bits, kCtx, bits);
  return hipGetLastError();
}

hipError_t launch_ans_encode(sgs_ctx *c, const uint8_t *sym, int64_t n, int order, int64_t S,
                             const uint16_t *freq, uint16_t *words, int64_t word_cap,
                             int64_t *block_off, int64_t *info) {
  const int64_t nb = (n + 64 * S - 1) / (64 * S);
  hipError_t e = coding_blocks(c, nb);
  if (e != hipSuccess) return e;
  SgsCoding *k = c->coding;
  hipStream_t st = c->stream;
  k_fill_u32<<<1, 64, 0, st>>>((uint32_t *)info, 4, 0u);
  k_ans_enc_table<<<kCtx, 256, 0, st>>>(freq, k->ans_enc, info + 1);
  if (nb > 0)
    k_ans_encode<false><<<(unsigned)nb, 64, 0, st>>>(sym, n, S, order, k->ans_enc, k->ans_blk,
                                                     nullptr, nullptr, 0, info);
  e = launch_exclusive_scan(c, k->ans_blk, k->ans_scan, nb, nullptr);
  if (e != hipSuccess) return e;
  k_ans_offsets<<<grid_for(nb + 1, 256, 1 << 30), 256, 0, st>>>(k->ans_scan, nb, block_off,
                                                                word_cap, info);
  if (nb > 0)
    k_ans_encode<true><<<(unsigned)nb, 64, 0, st>>>(sym, n, S, order, k->ans_enc, k->ans_blk,
                                                    k->ans_scan, words, word_cap, info);
  return hipGetLastError();
}

hipError_t launch_ans_decode(sgs_ctx *c, const uint16_t *words, int64_t n_words,
                             const int64_t *block_off, int64_t n, int order, int64_t S,
                             const uint16_t *freq, uint8_t *sym, int64_t *info) {
  hipError_t e = coding_base(c);
  if (e != hipSuccess) return e;
  SgsCoding *k = c->coding;
  hipStream_t st = c->stream;
  const int64_t nb = (n + 64 * S - 1) / (64 * S);
  k_fill_u32<<<1, 64, 0, st>>>((uint32_t *)info, 2, 0u);
  k_ans_dec_table<<<kCtx, 256, 0, st>>>(freq, k->ans_dec, info);
  if (nb > 0)
    k_ans_decode<<<(unsigned)((nb + kDecWaves - 1) / kDecWaves), 64 * kDecWaves, 0, st>>>(
        words, n_words, block_off, n, S, order, nb, k->ans_dec,
                                               sym, info);
  return hipGetLastError();
}

hipError_t launch_ans_decode_multi(sgs_ctx *c, int32_t count, const sgs_ans_stream *st,
                                   int64_t *info) {
  hipError_t e = coding_base(c);
  if (e != hipSuccess) return e;
  SgsCoding *k = c->coding;
  // decode tables: 4096 entries per order-0 stream, 257 x 4096 per order-1
  std::vector<AnsDev> h((size_t)count);
  int64_t tab_words = 0, most = 0;
  for (int32_t i = 0; i < count; ++i) {
    const int64_t S = st[i].lane_len;
    h[i] = AnsDev{st[i].words, st[i].n_words, st[i].block_off, st[i].n, st[i].freq, st[i].sym,
                  nullptr, S, (st[i].n + 64 * S - 1) / (64 * S), st[i].order, 0};
    tab_words += (st[i].order ? kCtx : 1) * (int64_t)kAnsM;
    most = h[i].nb > most ? h[i].nb : most;
  }
  if (tab_words > k->multi_tab_words) {
    k->multi_tab_words = 0;
    if ((e = calloc_(k->multi_tab, tab_words)) != hipSuccess) return e;
    k->multi_tab_words = tab_words;
  }
  if (count > k->multi_cap) {
    k->multi_cap = 0;
    if ((e = calloc_(k->multi_desc, (int64_t)count * (int64_t)sizeof(AnsDev))) != hipSuccess) return e;
    k->multi_cap = count;
  }
  int64_t o = 0;
  for (int32_t i = 0; i < count; ++i) {
    h[i].tab = k->multi_tab + o;
    o += (h[i].order ? kCtx : 1) * (int64_t)kAnsM;
  }
  hipStream_t s = c->stream;
  e = hipMemcpyAsync(k->multi_desc, h.data(), sizeof(AnsDev) * (size_t)count,
                     hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return e;
  const AnsDev *d = (const AnsDev *)k->multi_desc;
  k_fill_u32<<<grid_for(2 * (int64_t)count, 256, 64), 256, 0, s>>>((uint32_t *)info,
                                                                  2 * (int64_t)count, 0u);
  k_ans_dec_table_multi<<<dim3(kCtx, (unsigned)count), 256, 0, s>>>(d, info);
  if (most > 0)
    k_ans_decode_multi<<<dim3((unsigned)((most + kDecWaves - 1) / kDecWaves), (unsigned)count),
                         64 * kDecWaves, 0, s>>>(d, info);
  // the host copy of the descriptors must outlive the transfer
  e = hipStreamSynchronize(s);
  if (e != hipSuccess) return e;
  return hipGetLastError();
}

hipError_t launch_morton_order(sgs_ctx *c, const float *params, int64_t npad, int64_t n,
                               const float *q, const uint8_t *hard, const sgs_octree_header *h,
                               const uint64_t *codes, int32_t *perm) {
  hipError_t e = coding_octree(c, n);
  if (e != hipSuccess) return e;
  SgsCoding *k = c->coding;
  hipStream_t s = c->stream;
  const int64_t kept = h->kept, m = h->unique;
  k_flags_u8<<<grid_for(n, 256, 1 << 30), 256, 0, s>>>(hard, n, k->dflag);
  e = launch_exclusive_scan(c, k->dflag, k->dpos, n, nullptr);
  if (e != hipSuccess) return e;
  k_mo_keys<<<grid_for(n, 256, 1 << 30), 256, 0, s>>>(params, npad, n, q, hard, k->dpos,
                                                      (int)h->depth, h->kmin[0], h->kmin[1],
                                                      h->kmin[2], codes, m, k->key[0], k->key[2]);
  int bits = 1;
  while (bits < 32 && ((int64_t)1 << bits) <= m) ++bits;
  int w = 0;
  uint32_t *keys[2] = {k->key[0], k->key[1]}, *vals[2] = {k->key[2], k->key[3]};
  e = ensure_tmp(c, (n + 4095) / 4096 + 1, radix_hist_words(kept));
  if (e != hipSuccess) return e;
  e = launch_radix_sort(c, keys, vals, kept, bits, &w, nullptr);
  if (e != hipSuccess) return e;
  if (kept > 0)
    k_copy_u32<<<grid_for(kept, 256, 1 << 30), 256, 0, s>>>(vals[w], kept, perm);
  return hipGetLastError();
}

static AttrChans attr_chans(const sgs_fl_channel *fl, const uint8_t *pred, int64_t *rows) {
  AttrChans C;
  int32_t r = 0;
  for (int j = 3; j < SGS_NCH; ++j) {
    const int w = fl[j].width;
    const int pj = pred ? (pred[j] ? 1 : 0) : 1;
    const int P = w == 0 ? 0 : pj ? (w + 8) / 8 : (w + 7) / 8;
    C.ch[j - 3] = AttrChan{fl[j].q, fl[j].kmin, P, r, pj};
    r += P;
  }
  *rows = r;
  return C;
}

int64_t attr_plane_rows(const sgs_fl_channel *fl, const uint8_t *pred) {
  int64_t r;
  (void)attr_chans(fl, pred, &r);
  return r;
}

hipError_t launch_attr_planes(sgs_ctx *c, const float *params, int64_t npad, const int32_t *perm,
                              int64_t kept, const sgs_fl_channel *fl, const uint8_t *pred,
                              int32_t S, uint8_t *planes) {
  int64_t rows;
  const AttrChans C = attr_chans(fl, pred, &rows);
  if (kept > 0 && rows > 0)
    k_attr_planes<<<dim3(grid_for(kept, 256, 1 << 30), SGS_NCH - 3), 256, 0, c->stream>>>(
        params, npad, perm, kept, S, C, planes);
  return hipGetLastError();
}

hipError_t launch_attr_reconstruct(sgs_ctx *c, const uint8_t *planes, int64_t kept,
                                   const sgs_fl_channel *fl, const uint8_t *pred, int32_t S,
                                   float *out, int64_t out_pad) {
  int64_t rows;
  const AttrChans C = attr_chans(fl, pred, &rows);
  const int64_t groups = (kept + S - 1) / S;
  if (kept > 0)
    k_attr_reconstruct<<<dim3((unsigned)((groups + 3) / 4), SGS_NCH - 3), 256, 0, c->stream>>>(
        planes, kept, S, C, out, out_pad);
  return hipGetLastError();
}

template <int L>
static void pe_launch(sgs_ctx *c, const float *xyz, int64_t pad, int64_t count, int d,
                      const float *W, const float *b, float *out) {
  k_pos_embed<L><<<grid_for(count, 256, 1 << 30), 256, 0, c->stream>>>(xyz, pad, count, d, W, b,
                                                                       out);
}

hipError_t launch_pos_embed(sgs_ctx *c, const float *xyz, int64_t pad, int64_t count, int L,
                            int d, const float *W, const float *b, float *out) {
  if (count == 0) return hipSuccess;
  switch (L) {
#define SGS_PE_CASE(v) \
  case v: pe_launch<v>(c, xyz, pad, count, d, W, b, out); break;
    SGS_PE_CASE(1) SGS_PE_CASE(2) SGS_PE_CASE(3) SGS_PE_CASE(4) SGS_PE_CASE(5) SGS_PE_CASE(6)
    SGS_PE_CASE(7) SGS_PE_CASE(8) SGS_PE_CASE(9) SGS_PE_CASE(10) SGS_PE_CASE(11)
    SGS_PE_CASE(12) SGS_PE_CASE(13) SGS_PE_CASE(14) SGS_PE_CASE(15) SGS_PE_CASE(16)
#undef SGS_PE_CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}
