// Front-to-back alpha compositing over the per-tile depth-ordered lists
// (paper Sec. 3.1, compositing equation) and its reverse-order backward.
//
// The lists are binned per tile (16x16 by default); the work item of a launch
// is one 8x8 sub-tile of a tile, done by one wave64 as its own workgroup, one
// pixel per lane.  The wave stages 64 list entries at a time in its LDS (one
// 48-byte record per lane, one cache line each), marks with one ballot those
// whose pixel span meets its sub-tile and walks only those; all lanes read the
// same LDS record at the same time (broadcast, no bank conflicts).  A pixel
// stops when T (1 - alpha~) would fall below 1e-4; the wave stops when all its
// pixels have stopped.  Sub-tiles of one tile finish independently and a
// finished wave's slot takes the next work item at once.
//
// The backward walks the same list from the wave's furthest stop towards
// the front, recovers T by multiplying with the reciprocal of the same
// (1 - alpha~) the forward multiplied by, and reduces the ten per-splat
// gradients of a wave with a transposing butterfly (eight lane swaps and
// five DPP exchanges for all ten values); ten lanes then issue one atomic each.
#include "blend_reach.h"
#include "sgs_internal.h"

namespace {

struct SplatLds {
  float4 a;  // px, py, A', B' (the conic scaled by SGS_CONIC_KAC / KB)
  float4 b;  // C', opacity, spanx (x0 | x1 << 16), spany
  float4 c;  // r, g, b, mask
};

// Evaluation of splat s at pixel (px, py), branch-free: every lane computes
// every value and `ok` says whether the pair contributes (pixel inside the
// splat's pixel span, exponent not positive, alpha >= 1/255).  The forward and
// the backward call the same code so both see bit-identical values.
struct SplatEval {
  bool in_span, ok, clamped;
  float alpha, G, dx, dy;
};

__device__ __forceinline__ SplatEval eval_splat(const SplatLds &s, int px, int py, float fx,
                                                float fy) {
  SplatEval r;
  const uint32_t sx = __float_as_uint(s.b.z), sy = __float_as_uint(s.b.w);
  r.in_span = (px >= (int)(sx & 0xFFFF)) && (px <= (int)(sx >> 16)) &&
              (py >= (int)(sy & 0xFFFF)) && (py <= (int)(sy >> 16));
  r.dx = fx - s.a.x;
  r.dy = fy - s.a.y;
  // log2(e) power = A' dx^2 + C' dy^2 + B' dx dy (the record's scaled conic)
  const float p2 = fmaf(s.a.z * r.dx, r.dx, fmaf(s.b.x * r.dy, r.dy, s.a.w * r.dx * r.dy));
  r.G = __builtin_amdgcn_exp2f(p2);
  const float raw = s.b.y * r.G;
  r.clamped = raw > SGS_ALPHA_MAX;
  r.alpha = fminf(raw, SGS_ALPHA_MAX);  // raw is finite: the same value as the clamp
  r.ok = r.in_span && !(p2 > 0.0f) && r.alpha >= SGS_ALPHA_MIN;
  return r;
}

// Whether a splat (record a, b) can pass the alpha cut-off at any pixel
// centre of the 8x8 sub-tile at (sx0, sy0); a test per list entry, made once
// per batch (blend_reach.h states the rule and its margin).
__device__ __forceinline__ bool may_reach(const float4 &a, const float4 &b, int sx0, int sy0) {
  return sgs_may_reach(a.x, a.y, a.z, a.w, b.x, -__log2f(255.0f * b.y), sx0, sy0);
}

// Whether a splat is large: its tile rectangle (the projection's: tiles per
// view row / column of the span's corners) covers kBigTiles tiles or more.
template <int TW, int TH>
__device__ __forceinline__ bool big_splat(uint32_t sx, uint32_t sy) {
  const uint32_t tw = (sx >> 16) / TW - (sx & 0xFFFFu) / TW + 1u;
  const uint32_t th = (sy >> 16) / TH - (sy & 0xFFFFu) / TH + 1u;
  return tw * th >= kBigTiles;
}

// Where a backward sum of splat gid from tile `tile` goes: its record, or
// for a large splat with a replica slot (big_idx offset to the view),
// replica tile % kBigReps of that slot.
__device__ __forceinline__ double *grad_dst(double *gbase, uint32_t gid, bool big,
                                            const uint32_t *big_idx, double *big_rep,
                                            int tile) {
  if (big) {
    const uint32_t slot = big_idx[gid];
    if (slot != 0xFFFFFFFFu)
      return big_rep + ((size_t)slot * kBigReps + (uint32_t)tile % kBigReps) * SGS_SGRAD;
  }
  return gbase + (size_t)gid * SGS_SGRAD;
}

// A 64-bit mask read from LDS, made wave-uniform (held in scalar registers).
__device__ __forceinline__ uint64_t uniform_mask(uint64_t m) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)m);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(m >> 32));
  return ((uint64_t)hi << 32) | lo;
}

// Evaluation counting of the forward: none (the timed path), every in-span
// pair before termination (the method's evaluations; the reach test is off
// so that every such pair is visited), or the pairs the timed path visits
// (in-span pairs kept by the reach test, before termination).
enum CountMode { kCountNone = 0, kCountSpan = 1, kCountReach = 2 };

// One 8x8 sub-tile of a tile's forward, by one wave (the workgroup): the
// wave stages 64 list entries at a time in its LDS (one 48-byte record per
// lane), marks with a ballot those whose pixel span meets its sub-tile and
// that can pass the alpha cut-off there (may_reach; the counting pass keeps
// every entry whose span meets the sub-tile), and composites them in list
// order, in pairs whose records are read and evaluated together; the next
// 64 records are fetched from global memory during the walk.  It stops once
// all its pixels have stopped.  evals accumulates the lane's in-span pairs.
template <int TW, int TH, int COUNT, int WPB>
__device__ __forceinline__ void blend_fwd_sub(int tile, int sub, int n, int W, int H, int GW,
                                              int tiles_per_view,
                                              const uint2 *__restrict__ ranges,
                                              const uint32_t *__restrict__ vals,
                                              const float4 *__restrict__ rec,
                                              float *__restrict__ image,
                                              float *__restrict__ final_T,
                                              uint32_t *__restrict__ last, uint32_t &evals) {
  constexpr int SUBW = TW / 8;
  __shared__ SplatLds sh_all[WPB][64];  // one region per wave of the workgroup
  SplatLds *sh = sh_all[WPB > 1 ? (threadIdx.x >> 6) : 0];
  const int lane = threadIdx.x & 63;
  const int v = tile / tiles_per_view;
  const int t = tile - v * tiles_per_view;
  const int tx = t % GW, ty = t / GW;
  const int sx0 = tx * TW + (sub % SUBW) * 8;
  const int sy0 = ty * TH + (sub / SUBW) * 8;
  const int px = sx0 + (lane & 7);
  const int py = sy0 + (lane >> 3);
  const bool inside = px < W && py < H;
  const float fx = (float)px, fy = (float)py;
  const uint2 rg = ranges[tile];
  const int64_t base = (int64_t)v * n;
  float T = 1.0f, C0 = 0.0f, C1 = 0.0f, C2 = 0.0f;
  bool done = !inside;
  uint32_t stop = rg.y - rg.x;
  // the next batch's records, fetched while the current one is walked
  float4 ra = make_float4(0.f, 0.f, 0.f, 0.f), rb = ra, rc = ra;
  auto fetch = [&](uint32_t b) {
    const uint32_t e = b + (uint32_t)lane;
    if (e < rg.y) {
      const float4 *r = rec + 3 * (base + vals[e]);
      ra = r[0];
      rb = r[1];
      rc = r[2];
    }
  };
  if (rg.x < rg.y) fetch(rg.x);
  for (uint32_t b = rg.x; b < rg.y; b += 64) {
    if (__ballot(!done) == 0ull) break;
    const uint32_t cnt = min(64u, rg.y - b);
    wave_lds_sync();  // the previous batch's records have been read
    uint64_t m;
    {
      const bool valid = (uint32_t)lane < cnt;
      if (valid) {
        sh[lane].a = ra;
        sh[lane].b = rb;
        sh[lane].c = rc;
      }
      // entries whose pixel span meets this sub-tile
      const uint32_t sx = __float_as_uint(rb.z), sy = __float_as_uint(rb.w);
      // (the counting pass keeps every entry whose span meets the sub-tile:
      // it counts in-span pairs)
      m = __ballot(valid && (int)(sx & 0xFFFF) <= sx0 + 7 && (int)(sx >> 16) >= sx0 &&
                   (int)(sy & 0xFFFF) <= sy0 + 7 && (int)(sy >> 16) >= sy0 &&
                   (COUNT == kCountSpan || may_reach(ra, rb, sx0, sy0)));
    }
    wave_lds_sync();
    if (b + 64 < rg.y) fetch(b + 64);
    if (m == 0ull) continue;
    // composite entry k, evaluated as e
    auto step = [&](const SplatLds &cur, const SplatEval &e, int k) {
      const bool act = !done;
      if (COUNT) evals += (act && e.in_span) ? 1u : 0u;
      const bool okc = act && e.ok;
      const float at = cur.c.w * e.alpha;
      const float Tn = T * (1.0f - at);
      const bool term = okc && Tn < SGS_T_MIN;
      const bool contrib = okc && !term;
      // a zero weight leaves C unchanged bit for bit (colours are finite)
      const float w = contrib ? at * T : 0.0f;
      C0 = fmaf(cur.c.x, w, C0);
      C1 = fmaf(cur.c.y, w, C1);
      C2 = fmaf(cur.c.z, w, C2);
      T = contrib ? Tn : T;
      stop = term ? b - rg.x + (uint32_t)k : stop;
      done = done || term;
    };
    // entries in pairs: both records are read and evaluated before either is
    // composited, so two evaluation chains are in flight at once
    while (m != 0ull) {
      const int ka = __builtin_ctzll(m);
      m &= m - 1;
      const bool two = m != 0ull;
      const int kb = two ? __builtin_ctzll(m) : ka;
      if (two) m &= m - 1;
      const SplatLds ra_ = sh[ka], rb_ = sh[kb];
      const SplatEval ea = eval_splat(ra_, px, py, fx, fy);
      const SplatEval eb = eval_splat(rb_, px, py, fx, fy);
      step(ra_, ea, ka);
      if (two) step(rb_, eb, kb);
      // whether any pixel of the wave still runs, every second entry (an
      // entry composited after the last pixel stopped changes nothing)
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
}

// Persistent workers: each workgroup takes tiles from the queue (tiles in the
// order of `order`, longest lists first) until it runs dry; every workgroup
// reaches that exit.
__device__ __forceinline__ int next_tile(uint32_t *head, int total) {
  __shared__ int s_q;
  if (threadIdx.x == 0) s_q = (int)atomicAdd(head, 1u);
  __syncthreads();
  const int q = s_q;
  __syncthreads();  // all threads have read s_q before it is written again
  return q < total ? q : -1;
}

// Blend schedules.  kPerTile: one workgroup per tile (grid = tiles).
// kStride: a resident grid, workgroup g taking positions g, g + grid, ... of
// the length-ordered tile list.  kQueue: a resident grid taking positions of
// that list from an atomic queue head.  Every workgroup of a persistent grid
// leaves its loop once the positions run out.
enum BlendSchedule { kPerTile = 0, kStride = 1, kQueue = 2, kTileBlock = 3 };

template <int SCHED>
__device__ __forceinline__ int first_tile(uint32_t *head, int total) {
  if (SCHED == kQueue) return next_tile(head, total);
  return (int)blockIdx.x < total ? (int)blockIdx.x : -1;
}
template <int SCHED>
__device__ __forceinline__ int later_tile(int q, uint32_t *head, int total) {
  if (SCHED == kPerTile) return -1;
  if (SCHED == kQueue) return next_tile(head, total);
  q += (int)gridDim.x;
  return q < total ? q : -1;
}

// Work item q of a launch: sub-tile q % NW of tile q / NW (in the order of
// `order` for the persistent schedules), one wave per workgroup; with
// kTileBlock a workgroup of NW waves takes whole tiles of that order (striding),
// wave w sub-tile w, the waves walking independently.
template <int TW, int TH, int SCHED, int COUNT>
__global__ void __launch_bounds__(SCHED == kTileBlock ? TW * TH : 64)
k_blend_fwd(int total, const uint32_t *__restrict__ order, uint32_t *__restrict__ head,
            int n, int W, int H, int GW, int tiles_per_view, const uint2 *__restrict__ ranges,
            const uint32_t *__restrict__ vals, const float4 *__restrict__ rec,
            float *__restrict__ image, float *__restrict__ final_T, uint32_t *__restrict__ last,
            unsigned long long *__restrict__ eval_count) {
  constexpr int NW = TW * TH / 64;
  uint32_t evals = 0;
  if (SCHED == kTileBlock) {
    for (int q = (int)blockIdx.x; q < total; q += (int)gridDim.x)
      blend_fwd_sub<TW, TH, COUNT, NW>((int)order[q], (int)(threadIdx.x >> 6), n, W, H, GW,
                                       tiles_per_view, ranges, vals, rec, image, final_T, last,
                                       evals);
  } else {
    for (int q = first_tile<SCHED>(head, total); q >= 0; q = later_tile<SCHED>(q, head, total)) {
      const int ti = q / NW;
      blend_fwd_sub<TW, TH, COUNT, 1>(SCHED == kPerTile ? ti : (int)order[ti], q - ti * NW, n,
                                      W, H, GW, tiles_per_view, ranges, vals, rec, image,
                                      final_T, last, evals);
    }
  }
  if (COUNT) {
    unsigned long long ev = evals;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) ev += __shfl_xor(ev, o, 64);
    // one of SGS_EVAL_SLOTS counters per workgroup (a single counter for
    // 2e5 workgroups serializes); k_eval_finish adds them up
    if ((threadIdx.x & 63) == 0 && ev)
      atomicAdd(eval_count + (blockIdx.x & (SGS_EVAL_SLOTS - 1)), ev);
  }
}

// Adds the slot counters of the blend into the caller's count and clears them
// for the next blend (one wave).
__global__ void k_eval_finish(unsigned long long *__restrict__ slots,
                              unsigned long long *__restrict__ eval_count) {
  unsigned long long v = slots[threadIdx.x];
  slots[threadIdx.x] = 0ull;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  if (threadIdx.x == 0 && v) atomicAdd(eval_count, v);
}

// Sum each of v[0..9] over the 64 lanes of the wave with a transposing
// butterfly: every exchange halves the number of values a lane carries, so
// the ten sums cost five cross-half swaps (v_permlane32_swap), three row
// swaps (v_permlane16_swap; the fifth value is summed over the row pair
// without halving), two DPP exchanges across eights, one across fours and
// two quad reductions.  After the call lane L, with h = L >> 5,
// r = (L >> 4) & 1, b3 = (L >> 3) & 1 and b2 = (L >> 2) & 1, holds the total
// of value sum10_index(L) = 5 h + (b2 ? 2 : b3 ? (r ? 4 : 1) : (r ? 3 : 0)).
template <int kCtrl>
__device__ __forceinline__ float dpp(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), kCtrl, 0xF, 0xF, false));
}
constexpr int kDppRowRor8 = 0x128;       // lane i <- lane (i + 8) mod 16 within a row
constexpr int kDppRowHalfMirror = 0x141; // lane i <- lane 7 - i within each eight
constexpr int kDppQuad2301 = 0x4E;       // lane i <- lane i ^ 2 within a quad
constexpr int kDppQuad1032 = 0xB1;       // lane i <- lane i ^ 1 within a quad

__device__ __forceinline__ int sum10_index(int lane) {
  const int b2 = (lane >> 2) & 1, b3 = (lane >> 3) & 1, r = (lane >> 4) & 1;
  return 5 * (lane >> 5) + (b2 ? 2 : (b3 ? (r ? 4 : 1) : (r ? 3 : 0)));
}

__device__ __forceinline__ float wave_transpose_sum10(const float v[10], int lane) {
  float r5[5], t[3];
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    // lanes 0-31 end with value i, lanes 32-63 with value 5 + i
    const auto sw = __builtin_amdgcn_permlane32_swap(__float_as_uint(v[i]),
                                                     __float_as_uint(v[5 + i]), false, false);
    r5[i] = __uint_as_float(sw[0]) + __uint_as_float(sw[1]);
  }
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    // even rows end with slot i, odd rows with slot 3 + i
    const auto sw = __builtin_amdgcn_permlane16_swap(__float_as_uint(r5[i]),
                                                     __float_as_uint(r5[3 + i]), false, false);
    t[i] = __uint_as_float(sw[0]) + __uint_as_float(sw[1]);
  }
  {
    // slot 2 in every row, summed over the row pair
    const auto sw = __builtin_amdgcn_permlane16_swap(__float_as_uint(r5[2]),
                                                     __float_as_uint(r5[2]), false, false);
    t[2] = __uint_as_float(sw[0]) + __uint_as_float(sw[1]);
  }
  const bool b3 = lane & 8;
  const float u0 = (b3 ? t[1] : t[0]) + dpp<kDppRowRor8>(b3 ? t[0] : t[1]);
  const float u1 = t[2] + dpp<kDppRowRor8>(t[2]);
  const bool b2 = lane & 4;
  float x = (b2 ? u1 : u0) + dpp<kDppRowHalfMirror>(b2 ? u0 : u1);
  x += dpp<kDppQuad2301>(x);
  x += dpp<kDppQuad1032>(x);
  return x;
}

// Deterministic mode: a wave's sum v (FP32) is added as the integer
// X = trunc(v 2^64) (a 96-bit two's-complement number: 2^-64 resolution,
// |v| < 2^31) split into three 32-bit limbs, each added to its own 64-bit
// accumulator (the low two as unsigned, the top one signed).  Integer sums
// do not depend on the order of the additions, so the per-splat totals, and
// every gradient computed from them, are the same bits from run to run and
// from schedule to schedule.  Returns false (nothing added) for |v| >= 2^31
// or a value that is not finite.
__device__ __forceinline__ bool det_add(unsigned long long *acc, float v) {
  const uint32_t b = __float_as_uint(v);
  const int e = (int)((b >> 23) & 0xFFu);
  if (e == 0) return true;                 // zero or below 2^-126
  if (e >= 158) return false;              // |v| >= 2^31, infinite or NaN
  const uint64_t m = (b & 0x7FFFFFu) | 0x800000u;
  const int sh = e - 86;                   // X = m 2^sh
  if (sh <= -24) return true;              // below 2^-64
  uint64_t lo, hi;
  if (sh < 0) {
    lo = m >> -sh;
    hi = 0;
  } else if (sh < 40) {
    lo = m << sh;
    hi = 0;
  } else if (sh < 64) {
    lo = m << sh;
    hi = m >> (64 - sh);
  } else {
    lo = 0;
    hi = m << (sh - 64);
  }
  if (b >> 31) {                           // two's complement of hi:lo
    hi = ~hi + (lo == 0 ? 1u : 0u);
    lo = ~lo + 1u;
  }
  const uint32_t l0 = (uint32_t)lo, l1 = (uint32_t)(lo >> 32);
  const int32_t l2 = (int32_t)(uint32_t)hi;
  if (l0) atomicAdd(acc + 0, (unsigned long long)l0);
  if (l1) atomicAdd(acc + 1, (unsigned long long)l1);
  if (l2) atomicAdd(acc + 2, (unsigned long long)(int64_t)l2);
  return true;
}

// One 8x8 sub-tile of a tile's backward, by one wave: the list from the
// wave's furthest stop towards the front, 64 entries at a time staged in LDS
// with their Gaussian ids, walked back to front.
template <int TW, int TH, int WPB, bool DET>
__device__ __forceinline__ void blend_bwd_sub(int tile, int sub, int n, int W, int H, int GW,
                                              int tiles_per_view,
                                              const uint2 *__restrict__ ranges,
                                              const uint32_t *__restrict__ vals,
                                              const float4 *__restrict__ rec,
                                              const float *__restrict__ final_T,
                                              const uint32_t *__restrict__ last,
                                              const float *__restrict__ dimg,
                                              double *__restrict__ sgrad,
                                              unsigned long long *__restrict__ dacc,
                                              uint32_t *__restrict__ dflag,
                                              const uint32_t *__restrict__ big_idx,
                                              double *__restrict__ big_rep) {
  constexpr int SUBW = TW / 8;
  __shared__ SplatLds sh_all[WPB][64];  // one region per wave of the workgroup
  __shared__ uint32_t s_gid_all[WPB][64];
  SplatLds *sh = sh_all[WPB > 1 ? (threadIdx.x >> 6) : 0];
  uint32_t *s_gid = s_gid_all[WPB > 1 ? (threadIdx.x >> 6) : 0];
  const int lane = threadIdx.x & 63;
  const int v = tile / tiles_per_view;
  const int t = tile - v * tiles_per_view;
  const int tx = t % GW, ty = t / GW;
  const int sx0 = tx * TW + (sub % SUBW) * 8;
  const int sy0 = ty * TH + (sub / SUBW) * 8;
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
  // furthest list position reached by any pixel of the wave
  uint32_t reach = my_last;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) reach = max(reach, (uint32_t)__shfl_xor(reach, o, 64));
  if (reach == 0) return;
  float B0 = 0.f, B1 = 0.f, B2 = 0.f;  // colour seen behind the current splat
  const int nbatch = (int)((reach + 63) / 64);
  const int vidx = sum10_index(lane);
  // the lane that adds value vidx to the splat's gradient (one per value: the
  // first of its quad, and for value 5 h + 2, which 16 lanes hold, the one
  // with r = b3 = 0), and the factor on its own wave sum for the values the
  // conic does not enter
  const bool lead = (lane & 3) == 0 && (((lane >> 2) & 1) == 0 || ((lane >> 3) & 3) == 0);
  const float k_self = (vidx == 2 || vidx == 4) ? -0.5f : (vidx == 3 ? -1.0f : 1.0f);
  // per-lane selectors of the conic entries, which also undo the records'
  // scaling (A = A' / SGS_CONIC_KAC, B = B' / SGS_CONIC_KB, C = C' / KAC;
  // multiplying by 0 and adding 0 is exact)
  const float sel_a = vidx == 0 ? SGS_CONIC_INV_KAC : 0.0f;
  const float sel_c = vidx == 1 ? SGS_CONIC_INV_KAC : 0.0f;
  const float sel_b = vidx < 2 ? SGS_CONIC_INV_KB : 0.0f, k_rest = vidx < 2 ? 0.0f : k_self;
  // per-splat sums in FP64: a splat's terms come from many tiles and
  // cancel, and FP32 sums in arbitrary order lose the small result
  double *const gbase = sgrad + base * SGS_SGRAD;
  const uint32_t *const bigv = big_idx ? big_idx + base : nullptr;
  float4 ra = make_float4(0.f, 0.f, 0.f, 0.f), rb = ra, rc = ra;
  uint32_t rgid = 0;
  auto fetch = [&](int bi) {
    const uint32_t p = (uint32_t)bi * 64 + (uint32_t)lane;
    if (p < reach) {
      rgid = vals[rg.x + p];
      const float4 *r = rec + 3 * (base + rgid);
      ra = r[0];
      rb = r[1];
      rc = r[2];
    }
  };
  fetch(nbatch - 1);
  for (int bi = nbatch - 1; bi >= 0; --bi) {
    const uint32_t p0 = (uint32_t)bi * 64;
    wave_lds_sync();  // the previous batch's records have been read
    uint64_t m, bigm;
    {
      const bool valid = p0 + (uint32_t)lane < reach;
      if (valid) {
        s_gid[lane] = rgid;
        sh[lane].a = ra;
        sh[lane].b = rb;
        sh[lane].c = rc;
      }
      // entries before the wave's furthest stop whose span meets the sub-tile
      const uint32_t sx = __float_as_uint(rb.z), sy = __float_as_uint(rb.w);
      m = __ballot(valid && (int)(sx & 0xFFFF) <= sx0 + 7 && (int)(sx >> 16) >= sx0 &&
                   (int)(sy & 0xFFFF) <= sy0 + 7 && (int)(sy >> 16) >= sy0 &&
                   may_reach(ra, rb, sx0, sy0));
      // the batch's large splats (tile rectangle of kBigTiles tiles or more)
      bigm = big_idx ? __ballot(valid && big_splat<TW, TH>(sx, sy)) : 0ull;
    }
    wave_lds_sync();
    if (bi > 0) fetch(bi - 1);
    if (m == 0ull) continue;
    // gradient of entry k (record cur, Gaussian gid)
    auto step = [&](const SplatLds &cur, const SplatEval &e, int k, uint32_t gid) {
      const uint32_t pos = p0 + (uint32_t)k;
      const bool ok = inside && pos < my_last && e.ok;
      if (__ballot(ok) == 0ull) return;
      // branch-free: lanes without the pair take alpha~ = 0 and dL/dalpha~ = 0,
      // so every value below is 0 there and B, T stay as they are (bit for
      // bit: colours and B are finite and non-negative, 1 - 0 = 1 and its
      // reciprocal is exact)
      const float mk = cur.c.w;
      const float at = ok ? mk * e.alpha : 0.0f;
      const float om = 1.0f - at;
      // T in front of this splat (hardware reciprocal, 1 ulp: the
      // recovered T drifts by about one ulp per blended splat)
      const float Tb = (at == 0.0f) ? T : T * __builtin_amdgcn_rcpf(om);
      const float dsum = fmaf(g0, cur.c.x - B0, fmaf(g1, cur.c.y - B1, g2 * (cur.c.z - B2)));
      const float dat = ok ? Tb * dsum : 0.0f;
      const float wcol = at * Tb;
      float d[10];
      d[6] = g0 * wcol;
      d[7] = g1 * wcol;
      d[8] = g2 * wcol;
      d[9] = dat * e.alpha;
      // moments of dL/dpower over the pixels (zero through the alpha clamp);
      // the conic enters after the wave sum: dL/dpx = A Sx + B Sy,
      // dL/dpy = B Sx + C Sy, dL/dA = -Sxx / 2, dL/dB = -Sxy, dL/dC = -Syy / 2
      const float dal = e.clamped ? 0.0f : mk * dat;
      d[5] = dal * e.G;
      const float dp = dal * e.alpha;
      d[0] = dp * e.dx;
      d[1] = dp * e.dy;
      d[2] = d[0] * e.dx;
      d[3] = d[0] * e.dy;
      d[4] = d[1] * e.dy;
      B0 = fmaf(cur.c.x, at, om * B0);
      B1 = fmaf(cur.c.y, at, om * B1);
      B2 = fmaf(cur.c.z, at, om * B2);
      T = Tb;
      const float tot = wave_transpose_sum10(d, lane);
      // lanes 0-3 hold Sx and lanes 8-11 hold Sy: each reads the other
      const float other = dpp<kDppRowRor8>(tot);
      // cs = A (value 0), C (value 1) or k_self; co = B for values 0 and 1
      const float cs = fmaf(sel_a, cur.a.z, fmaf(sel_c, cur.b.x, k_rest));
      const float co = sel_b * cur.a.w;
      const float gv = fmaf(cs, tot, co * other);
      if (lead && gv != 0.0f) {
        if (DET) {
          const size_t slot = ((size_t)(base + gid) * SGS_SGRAD + vidx) * 3;
          if (!det_add(dacc + slot, gv)) atomicOr(dflag, 1u);
        } else {
          unsafeAtomicAdd(grad_dst(gbase, gid, (bigm >> k) & 1ull, bigv, big_rep, tile) + vidx,
                          (double)gv);
        }
      }
    };
    // back to front, entries in pairs: both records are read and evaluated
    // before either gradient is taken
    while (m != 0ull) {
      const int ka = 63 - __builtin_clzll(m);
      m &= ~(1ull << ka);
      const bool two = m != 0ull;
      const int kb = two ? 63 - __builtin_clzll(m) : ka;
      if (two) m &= ~(1ull << kb);
      const SplatLds ra_ = sh[ka], rb_ = sh[kb];
      const uint32_t ga = s_gid[ka], gb = s_gid[kb];
      const SplatEval ea = eval_splat(ra_, px, py, fx, fy);
      const SplatEval eb = eval_splat(rb_, px, py, fx, fy);
      step(ra_, ea, ka, ga);
      if (two) step(rb_, eb, kb, gb);
    }
  }
}

template <int TW, int TH, int SCHED, bool DET>
__global__ void __launch_bounds__(SCHED == kTileBlock ? TW * TH : 64)
k_blend_bwd(int total, const uint32_t *__restrict__ order, uint32_t *__restrict__ head,
            int n, int W, int H, int GW, int tiles_per_view, const uint2 *__restrict__ ranges,
            const uint32_t *__restrict__ vals, const float4 *__restrict__ rec,
            const float *__restrict__ final_T, const uint32_t *__restrict__ last,
            const float *__restrict__ dimg, double *__restrict__ sgrad,
            unsigned long long *__restrict__ dacc, uint32_t *__restrict__ dflag,
            const uint32_t *__restrict__ big_idx, double *__restrict__ big_rep) {
  constexpr int NW = TW * TH / 64;
  if (SCHED == kTileBlock) {
    for (int q = (int)blockIdx.x; q < total; q += (int)gridDim.x)
      blend_bwd_sub<TW, TH, NW, DET>((int)order[q], (int)(threadIdx.x >> 6), n, W, H, GW,
                                     tiles_per_view, ranges, vals, rec, final_T, last, dimg,
                                     sgrad, dacc, dflag, big_idx, big_rep);
  } else {
    for (int q = first_tile<SCHED>(head, total); q >= 0; q = later_tile<SCHED>(q, head, total)) {
      const int ti = q / NW;
      blend_bwd_sub<TW, TH, 1, DET>(SCHED == kPerTile ? ti : (int)order[ti], q - ti * NW, n, W,
                                    H, GW, tiles_per_view, ranges, vals, rec, final_T, last, dimg,
                                    sgrad, dacc, dflag, big_idx, big_rep);
    }
  }
}

// ---------------------------------------------------------------------------
// Tile order for the persistent blend: tiles bucketed by list length (bucket
// 0 = empty, bucket b >= 1 holds lengths in [2^(b-1), 2^b)), longest bucket
// first; the order inside a bucket is whatever the atomics give (each tile's
// result does not depend on it).  bins: [0,33) counts, [33,66) cursors,
// [66] forward queue head, [67] backward queue head.
// ---------------------------------------------------------------------------
constexpr int kBuckets = 33;

__device__ __forceinline__ int len_bucket(uint2 r) {
  const uint32_t len = r.y - r.x;
  return len ? 32 - __clz(len) : 0;
}

__global__ void k_tile_order_reset(uint32_t *__restrict__ bins) {
  if (threadIdx.x < SGS_TILE_BINS) bins[threadIdx.x] = 0;
}

__global__ void __launch_bounds__(256)
k_tile_order_count(const uint2 *__restrict__ ranges, int tiles, uint32_t *__restrict__ bins) {
  __shared__ uint32_t s_h[kBuckets];
  if (threadIdx.x < kBuckets) s_h[threadIdx.x] = 0;
  __syncthreads();
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < tiles) atomicAdd(&s_h[len_bucket(ranges[t])], 1u);
  __syncthreads();
  if (threadIdx.x < kBuckets && s_h[threadIdx.x]) atomicAdd(&bins[threadIdx.x], s_h[threadIdx.x]);
}

__global__ void __launch_bounds__(256)
k_tile_order_scatter(const uint2 *__restrict__ ranges, int tiles, uint32_t *__restrict__ bins,
                     uint32_t *__restrict__ order) {
  __shared__ uint32_t s_h[kBuckets], s_at[kBuckets];
  if (threadIdx.x < kBuckets) s_h[threadIdx.x] = 0;
  __syncthreads();
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int b = t < tiles ? len_bucket(ranges[t]) : 0;
  const uint32_t rank = t < tiles ? atomicAdd(&s_h[b], 1u) : 0u;
  __syncthreads();
  if (threadIdx.x < kBuckets) {
    const int k = threadIdx.x;
    uint32_t start = 0;  // tiles in longer buckets
    for (int o = k + 1; o < kBuckets; ++o) start += bins[o];
    s_at[k] = start + (s_h[k] ? atomicAdd(&bins[kBuckets + k], s_h[k]) : 0u);
  }
  __syncthreads();
  if (t < tiles) order[s_at[b] + rank] = (uint32_t)t;
}

// Workgroups (of `block` threads) resident on the device for a persistent
// blend kernel, measured once per context and kernel variant (slot).
template <typename K>
int persistent_grid(sgs_ctx *c, int slot, K kernel, int items, int block) {
  if (c->blend_occ[slot] == 0) {
    int dev = 0, occ = 0, n = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kernel, block, 0) != hipSuccess ||
        occ < 1 || n < 1)
      return items;  // one workgroup per item still drains the queue
    c->blend_occ[slot] = occ * n;
  }
  const int g = c->blend_occ[slot];
  return g < items ? g : items;
}

template <int TW, int TH, int SCHED, int COUNT>
hipError_t fwd_tc(sgs_ctx *c, float *image, float *final_T, uint32_t *last, uint64_t *ec) {
  const uint32_t *vals = c->pair_val[c->pair_sorted_buf];
  const int block = SCHED == kTileBlock ? TW * TH : 64;
  const int items = (int)c->total_tiles * (SCHED == kTileBlock ? 1 : TW * TH / 64);
  const int grid = SCHED == kPerTile
                       ? items
                       : persistent_grid(c, COUNT, k_blend_fwd<TW, TH, SCHED, COUNT>,
                                         items, block);
  k_blend_fwd<TW, TH, SCHED, COUNT><<<grid, block, 0, c->stream>>>(
      items, c->tile_order, c->tile_bins + 66, (int)c->n, c->W, c->H, c->GW,
      (int)c->tiles_per_view, c->ranges, vals, c->rec, image, final_T, last,
      (unsigned long long *)c->eval_slots);
  if (COUNT)
    k_eval_finish<<<1, SGS_EVAL_SLOTS, 0, c->stream>>>((unsigned long long *)c->eval_slots,
                                                        (unsigned long long *)ec);
  return hipGetLastError();
}

// the evaluation count is compiled in only when it is asked for
template <int TW, int TH, int SCHED>
hipError_t fwd_t(sgs_ctx *c, float *image, float *final_T, uint32_t *last, uint64_t *ec) {
  if (!ec) return fwd_tc<TW, TH, SCHED, kCountNone>(c, image, final_T, last, ec);
  if (c->count_mode == 1) return fwd_tc<TW, TH, SCHED, kCountReach>(c, image, final_T, last, ec);
  return fwd_tc<TW, TH, SCHED, kCountSpan>(c, image, final_T, last, ec);
}

template <int TW, int TH, int SCHED, bool DET>
hipError_t bwd_td(sgs_ctx *c, const float *final_T, const uint32_t *last, const float *dimg) {
  const uint32_t *vals = c->pair_val[c->pair_sorted_buf];
  const int block = SCHED == kTileBlock ? TW * TH : 64;
  const int items = (int)c->total_tiles * (SCHED == kTileBlock ? 1 : TW * TH / 64);
  const int grid = SCHED == kPerTile
                       ? items
                       : persistent_grid(c, DET ? 4 : 3, k_blend_bwd<TW, TH, SCHED, DET>, items,
                                         block);
  k_blend_bwd<TW, TH, SCHED, DET><<<grid, block, 0, c->stream>>>(
      items, c->tile_order, c->tile_bins + 67, (int)c->n, c->W, c->H, c->GW,
      (int)c->tiles_per_view, c->ranges, vals, c->rec, final_T, last, dimg, c->splat_grad,
      (unsigned long long *)c->det_acc, c->d_pairs_total + 3, DET ? nullptr : c->big_idx,
      DET ? nullptr : c->big_rep);
  return hipGetLastError();
}

template <int TW, int TH, int SCHED>
hipError_t bwd_t(sgs_ctx *c, const float *final_T, const uint32_t *last, const float *dimg) {
  return c->deterministic ? bwd_td<TW, TH, SCHED, true>(c, final_T, last, dimg)
                          : bwd_td<TW, TH, SCHED, false>(c, final_T, last, dimg);
}

template <int TW, int TH>
hipError_t fwd_s(sgs_ctx *c, float *image, float *final_T, uint32_t *last, uint64_t *ec) {
  SgsProfScope ps(c, SGS_PROF_BLEND_FWD);
  if (c->schedule == kStride) return fwd_t<TW, TH, kStride>(c, image, final_T, last, ec);
  if (c->schedule == kTileBlock) {
    // one workgroup per tile: at most 1024 pixels
    if constexpr (TW * TH <= 1024) return fwd_t<TW, TH, kTileBlock>(c, image, final_T, last, ec);
    return hipErrorInvalidValue;
  }
  if (c->schedule == kQueue) return fwd_t<TW, TH, kQueue>(c, image, final_T, last, ec);
  return fwd_t<TW, TH, kPerTile>(c, image, final_T, last, ec);
}

template <int TW, int TH>
hipError_t bwd_s(sgs_ctx *c, const float *final_T, const uint32_t *last, const float *dimg) {
  if (c->schedule == kStride) return bwd_t<TW, TH, kStride>(c, final_T, last, dimg);
  if (c->schedule == kTileBlock) {
    if constexpr (TW * TH <= 1024) return bwd_t<TW, TH, kTileBlock>(c, final_T, last, dimg);
    return hipErrorInvalidValue;
  }
  if (c->schedule == kQueue) return bwd_t<TW, TH, kQueue>(c, final_T, last, dimg);
  return bwd_t<TW, TH, kPerTile>(c, final_T, last, dimg);
}

// Clears the per-splat gradients and the backward queue head.
__global__ void k_zero_grad(double *__restrict__ p, int64_t count, uint32_t *__restrict__ head,
                            uint32_t *__restrict__ big_count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = 0.0;
  if (i == 0 && head) *head = 0u;
  if (i < kBigRanges && big_count) big_count[i] = 0u;
}

// Replica slots of the large splat-views of this step (tile rectangle of at
// least kBigTiles tiles), from range blockIdx % kBigRanges: one counter add
// per wave; a splat finding its range full keeps its own record (slot
// 0xFFFFFFFF).
__global__ void k_big_index(const uint32_t *__restrict__ touched, int64_t vn,
                            uint32_t *__restrict__ big_idx, uint32_t *__restrict__ big_list) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool big = s < vn && touched[s] >= kBigTiles;
  const uint64_t m = __ballot(big);
  if (m == 0ull) return;
  const int lane = (int)(threadIdx.x & 63);
  const int lead = __builtin_ctzll(m);
  const uint32_t range = blockIdx.x % kBigRanges;
  uint32_t first = 0;
  if (lane == lead) first = atomicAdd(big_list + kBigMax + range, (uint32_t)__popcll(m));
  first = (uint32_t)__shfl((int)first, lead, 64);
  if (!big) return;
  const uint32_t local = first + (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
  if (local < (uint32_t)kBigPerRange) {
    const uint32_t slot = range * (uint32_t)kBigPerRange + local;
    big_idx[s] = slot;
    big_list[slot] = (uint32_t)s;
  } else {
    big_idx[s] = 0xFFFFFFFFu;
  }
}

// After the blend: each taken slot's replicas summed in replica order into
// the splat's record (one thread per record value, the only writer of it),
// and cleared for the next step.
__global__ void k_big_fold(const uint32_t *__restrict__ big_list, double *__restrict__ big_rep,
                           double *__restrict__ sgrad) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t slot = i / SGS_SGRAD, j = i - slot * SGS_SGRAD;
  if (slot >= kBigMax) return;
  const int64_t range = slot / kBigPerRange, local = slot - range * kBigPerRange;
  if (local >= min((int64_t)big_list[kBigMax + range], kBigPerRange)) return;
  double *r = big_rep + (size_t)slot * kBigReps * SGS_SGRAD + j;
  double v = 0.0;
#pragma unroll
  for (int k = 0; k < kBigReps; ++k) {
    v += r[k * SGS_SGRAD];
    r[k * SGS_SGRAD] = 0.0;
  }
  sgrad[(size_t)big_list[slot] * SGS_SGRAD + j] += v;
}

// Deterministic mode: clears the fixed-point accumulators (three words per
// value) and the backward queue head.
__global__ void k_zero_acc(unsigned long long *__restrict__ p, int64_t count,
                           uint32_t *__restrict__ head) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = 0ull;
  if (i == 0 && head) *head = 0u;
}

// Deterministic mode: per-splat sums from the accumulators,
//   total = a2 2^64 + a1 2^32 + a0 (units of 2^-64) = hi + lo 2^-64,
// rounded once to FP64 in a fixed way.
__global__ void k_acc_to_grad(const unsigned long long *__restrict__ acc, int64_t count,
                              double *__restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const uint64_t a0 = acc[3 * i], a1 = acc[3 * i + 1];
  const int64_t a2 = (int64_t)acc[3 * i + 2];
  const uint64_t lo = a0 + (a1 << 32);
  const uint64_t carry = (a1 >> 32) + (lo < a0 ? 1u : 0u);
  const int64_t hi = a2 + (int64_t)carry;
  out[i] = (double)hi + ldexp((double)lo, -64);
}

}  // namespace

hipError_t launch_tile_order(sgs_ctx *c) {
  if (c->schedule == kPerTile) return hipSuccess;
  const int tiles = (int)c->total_tiles;
  k_tile_order_reset<<<1, 128, 0, c->stream>>>(c->tile_bins);
  k_tile_order_count<<<sgs_blocks(tiles, 256), 256, 0, c->stream>>>(c->ranges, tiles,
                                                                   c->tile_bins);
  k_tile_order_scatter<<<sgs_blocks(tiles, 256), 256, 0, c->stream>>>(c->ranges, tiles,
                                                                     c->tile_bins, c->tile_order);
  return hipGetLastError();
}

hipError_t launch_blend_fwd(sgs_ctx *c, float *image, float *final_T, uint32_t *last,
                            uint64_t *eval_count) {
  if (c->TW == 16 && c->TH == 16) return fwd_s<16, 16>(c, image, final_T, last, eval_count);
  if (c->TW == 8 && c->TH == 8) return fwd_s<8, 8>(c, image, final_T, last, eval_count);
  if (c->TW == 32 && c->TH == 8) return fwd_s<32, 8>(c, image, final_T, last, eval_count);
  if (c->TW == 32 && c->TH == 16) return fwd_s<32, 16>(c, image, final_T, last, eval_count);
  if (c->TW == 32 && c->TH == 32) return fwd_s<32, 32>(c, image, final_T, last, eval_count);
  return hipErrorInvalidValue;
}

hipError_t launch_blend_bwd(sgs_ctx *c, const float *final_T, const uint32_t *last,
                            const float *dimg) {
  const int64_t words = c->vn * SGS_SGRAD;
  {
    SgsProfScope ps(c, SGS_PROF_GRAD_CLEAR);
    if (c->deterministic)
      k_zero_acc<<<sgs_blocks(3 * words, 256), 256, 0, c->stream>>>(
          (unsigned long long *)c->det_acc, 3 * words, c->tile_bins + 67);
    else {
      k_zero_grad<<<sgs_blocks(words, 256), 256, 0, c->stream>>>(c->splat_grad, words,
                                                                  c->tile_bins + 67,
                                                                  c->big_list + kBigMax);
      k_big_index<<<sgs_blocks(c->vn, 256), 256, 0, c->stream>>>(c->touched, c->vn, c->big_idx,
                                                                 c->big_list);
    }
  }
  // one profiling record per call: the blend and the fold of its sums
  SgsProfScope ps(c, SGS_PROF_BLEND_BWD);
  hipError_t e = hipErrorInvalidValue;
  if (c->TW == 16 && c->TH == 16) e = bwd_s<16, 16>(c, final_T, last, dimg);
  if (c->TW == 8 && c->TH == 8) e = bwd_s<8, 8>(c, final_T, last, dimg);
  if (c->TW == 32 && c->TH == 8) e = bwd_s<32, 8>(c, final_T, last, dimg);
  if (c->TW == 32 && c->TH == 16) e = bwd_s<32, 16>(c, final_T, last, dimg);
  if (c->TW == 32 && c->TH == 32) e = bwd_s<32, 32>(c, final_T, last, dimg);
  if (e != hipSuccess) return e;
  if (!c->deterministic) {
    k_big_fold<<<sgs_blocks(kBigMax * SGS_SGRAD, 256), 256, 0, c->stream>>>(
        c->big_list, c->big_rep, c->splat_grad);
    return hipGetLastError();
  }
  k_acc_to_grad<<<sgs_blocks(words, 256), 256, 0, c->stream>>>(
      (const unsigned long long *)c->det_acc, words, c->splat_grad);
  return hipGetLastError();
}
