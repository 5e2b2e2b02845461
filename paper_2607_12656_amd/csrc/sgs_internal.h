// Internal declarations of libspeedygs: the context, launchers and the
// device-side helpers shared by the kernels.  Compiled for gfx950 only, with
// -ffp-contract=off so every floating-point expression is evaluated exactly
// as written (the discrete decisions below must be reproducible bit for bit).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "../../include/speedygs.h"

#define SGS_CH_MU 0
#define SGS_CH_DC 3
#define SGS_CH_REST 6
#define SGS_CH_REST_END 51  // one past the last higher-SH channel
#define SGS_CH_OPA 51
#define SGS_CH_SCALE 52
#define SGS_CH_ROT 55

// Splat-gradient record stride (floats): px, py, A, B, C, opacity, r, g, b,
// mask, pad, pad.
#define SGS_SGRAD 10  // px, py, A, B, C, opacity, r, g, b, mask (five 16-byte pairs)

// A splat's tile rectangle in one word: first column and row (10 bits each),
// width - 1 and height - 1 (6 bits each); kNoRect when it does not fit.
constexpr uint32_t kNoRect = 0xFFFFFFFFu;
__host__ __device__ __forceinline__ uint32_t sgs_pack_rect(int tx0, int ty0, int tw, int th) {
  if (tx0 >= 1024 || ty0 >= 1024 || tw > 64 || th > 64) return kNoRect;
  return (uint32_t)tx0 | ((uint32_t)ty0 << 10) | ((uint32_t)(tw - 1) << 20) |
         ((uint32_t)(th - 1) << 26);
}

// Large splats in the backward: every tile a splat covers adds its sums to
// the splat's record, and FP64 atomics to one address serialize in the L2.
// A splat-view whose tile rectangle covers at least kBigTiles tiles takes a
// slot with kBigReps replica records, tile t adding to replica t %
// kBigReps; the replicas are folded into the record in a fixed order after
// the blend.  The kBigMax slots form kBigRanges ranges, each with its own
// counter (so that taking slots is not itself one contended address); a
// large splat finding its range full keeps its own record.
constexpr uint32_t kBigTiles = 512;
// Segment granularity of the depth-ordered arrays (a multiple of every radix
// tile the depth sort uses, so that no sort block spans two views).
constexpr int64_t kDepthSeg = 2048;
constexpr int kBigReps = 16;
constexpr int64_t kBigMax = 16384;
constexpr int kBigRanges = 64;
constexpr int64_t kBigPerRange = kBigMax / kBigRanges;

// Blend conventions (the paper does not state them).
#define SGS_NEAR 0.2f
#define SGS_DILATION 0.3f
#define SGS_ALPHA_MAX 0.99f
#define SGS_ALPHA_MIN (1.0f / 255.0f)
#define SGS_T_MIN 1e-4f
// The splat records hold the conic scaled into the blend's exponent of 2:
// A' = -log2(e)/2 A, B' = -log2(e) B, C' = -log2(e)/2 C, so that
// log2(e) power = A' dx^2 + C' dy^2 + B' dx dy and e^power = 2^(that).
#define SGS_CONIC_KAC (-0.72134752044448170368f)   // -log2(e) / 2
#define SGS_CONIC_KB (-1.44269504088896340736f)    // -log2(e)
#define SGS_CONIC_INV_KAC (-1.38629436111989061883f)  // -2 ln 2 = 1 / SGS_CONIC_KAC
#define SGS_CONIC_INV_KB (-0.69314718055994530942f)   // -ln 2 = 1 / SGS_CONIC_KB
#define SGS_FOV_CLAMP 1.3f

struct sgs_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  char err[512] = {0};

  // scene
  int64_t n = 0, npad = 0, n_hat = 0;
  int V = 0, W = 0, H = 0;
  int TW = 16, TH = 16, GW = 0, GH = 0;
  int64_t tiles_per_view = 0, total_tiles = 0;
  float tau = 1.0f;
  int schedule = 0;               // blend launch schedule (sgs_options.schedule)
  int blend_occ[5] = {0, 0, 0, 0, 0}; // resident blend workgroups (fwd, fwd counting in-span,
                                   // fwd counting reach-kept, bwd, bwd deterministic); 0 unknown
  bool deterministic = false;     // sgs_options.deterministic: fixed-point gradient sums
  uint64_t *det_acc = nullptr;    // [vn][SGS_SGRAD][3] fixed-point accumulators (that mode)
  int count_mode = 0;             // sgs_set_eval_count_mode
  bool grad_sh_rest = true;       // sgs_set_grad_sh_rest
  bool scene_set = false;
  bool rendered = false;
  sgs_camera *d_cams = nullptr;
  std::vector<sgs_camera> h_cams; // host copy of the scene's cameras (for re-binding)

  // per (view, Gaussian): V*n entries
  int64_t vn = 0;
  float4 *rec = nullptr;          // [vn][3]: (px,py,A,B) (C,opa,spanx,spany) (r,g,b,mask)
  // [vn_pad] each, view v's splat i at v * vseg + i (value v * n + i)
  uint32_t *depth_key[2] = {nullptr, nullptr};
  uint32_t *depth_val[2] = {nullptr, nullptr};
  // [vn_pad] each: the splat's tile rectangle packed for the depth sort to carry
  // (first column and row 10 bits each, width - 1 and height - 1 6 bits
  // each), or kNoRect when it does not fit (then the record is gathered)
  uint32_t *depth_rect[2] = {nullptr, nullptr};
  uint32_t *touched = nullptr;    // [vn] tiles per splat (0 = culled)
  uint4 *bin_splat = nullptr;     // [vn] (first tile id, width in tiles, Gaussian, pairs),
                                  // written only for rectangles depth_rect cannot hold
  double *splat_grad = nullptr;   // [vn][SGS_SGRAD] per-splat gradient sums (FP64 atomics)
  uint32_t *big_idx = nullptr;    // [vn] replica slot of a large splat (see kBigTiles)
  uint32_t *big_list = nullptr;   // [kBigMax + kBigRanges] splat of each slot, then the
                                  // slots taken in each range
  double *big_rep = nullptr;      // [kBigMax][kBigReps][SGS_SGRAD] replica sums (zero between steps)
  int depth_sorted_buf = 0;       // which depth buffer holds the sorted order

  // super-tiles (8x8 tiles): the first level of the tile binning
  int SGW = 0, SGH = 0;           // super-tiles per view row / column
  int64_t st_per_view = 0, total_st = 0;
  // super-tile ids: (super-tile in its view) << st_vbits | view, st_slots of
  // them (ids of views >= V are empty)
  int st_vbits = 0;
  int64_t st_slots = 0;
  // the depth-ordered arrays hold each view's splats in a segment of vseg
  // entries (n rounded up to kDepthSeg; the padding sorts last), vn_pad in all
  int64_t vseg = 0, vn_pad = 0;
  int64_t items = 0;              // (splat, super-tile) items of the last render (host copy)
  uint32_t *ioffsets = nullptr;   // [vn_pad + 1] exclusive scan of the item counts, in
                                  // (view, depth) order
  uint2 *st_ranges = nullptr;     // [st_slots] item range of every super-tile id
  uint32_t *chunk_first = nullptr;  // [st_slots + 1] first item chunk of every super-tile id
  uint32_t *l2_cnt = nullptr;     // [chunks][64] per-chunk tile counts, then offsets
  int64_t l2_chunks = 0;          // chunks l2_cnt holds
  uint32_t *tile_cnt = nullptr;   // [total_tiles] pairs per tile
  uint32_t *tile_start = nullptr; // [total_tiles + 1] exclusive scan of tile_cnt

  // pairs
  int64_t pair_cap = 0;
  int64_t pairs = 0;
  uint32_t *tile_key[2] = {nullptr, nullptr};
  uint32_t *pair_val[2] = {nullptr, nullptr};
  int pair_sorted_buf = 0;
  uint32_t *blk_start = nullptr;  // first splat (depth order) of every block of sorted pairs
  int64_t blk_start_words = 0;
  uint2 *ranges = nullptr;        // [total_tiles]
  uint32_t *tile_order = nullptr; // [total_tiles] blend order, longest lists first
  uint32_t *tile_bins = nullptr;  // [SGS_TILE_BINS] order counters and blend queue heads
  uint64_t *eval_slots = nullptr; // [SGS_EVAL_SLOTS] evaluation counts of one blend, zero between

  // reusable temporaries
  uint32_t *scan_tmp = nullptr;   int64_t scan_tmp_words = 0;
  uint32_t *sort_hist = nullptr;  int64_t sort_hist_words = 0;
  double *red_tmp = nullptr;      int64_t red_tmp_words = 0;
  uint32_t *fl_tmp = nullptr;     // fixed-length encoder scratch
  int64_t fl_tmp_words = 0;
  double *lap_coef = nullptr;     // Laplace proxy: per-channel mean, mean sign, coefficient
  bool lap_ready = false;         // lap_coef holds the last Laplace forward's values
  double *ssim_tmp = nullptr;     // SSIM gradient maps + block sums (allocated on first use)
  int64_t ssim_tmp_doubles = 0;
  float *mlp_f = nullptr;         // [n] f of the last learned-rate forward
  uint4 *mlp_signs = nullptr;     // [2n] its hidden activation signs (two lanes per row)
  bool mlp_saved = false;         // a learned-rate forward ran since set_scene
  uint32_t *d_pairs_total = nullptr;  // [0] pair count, [1] count clamped to capacity, [2]
                                      // overflow, [3] deterministic range flag, [4] item
                                      // count, [5] item count clamped to capacity, [6] unused
  uint32_t *h_pairs_total = nullptr;  // pinned host mirror of words [0, 5)
  uint32_t *h_aux = nullptr;          // pinned host word (kept count of a compaction)
  bool fixed_cap = false;             // pair capacity fixed by the caller: no host sync per step
  int64_t cap_limit = 0;              // the reserved capacity (buffers may be larger)
  bool capturing = false;             // the stream is being captured into a HIP graph
  struct SgsCoding *coding = nullptr; // octree and entropy-coder scratch (first use)

  // kernel-group timing
  struct ProfRec {
    int group;
    hipEvent_t a, b;
  };
  bool prof = false;
  std::vector<hipEvent_t> ev_free;
  std::vector<ProfRec> prof_recs;
};

// Records a pair of HIP events around the launches in its scope when the
// context's profiling is on.
struct SgsProfScope {
  sgs_ctx *c;
  int g;
  hipEvent_t a = nullptr;
  static hipEvent_t get(sgs_ctx *c) {
    hipEvent_t e = nullptr;
    if (!c->ev_free.empty()) {
      e = c->ev_free.back();
      c->ev_free.pop_back();
    } else if (hipEventCreate(&e) != hipSuccess) {
      e = nullptr;
    }
    return e;
  }
  SgsProfScope(sgs_ctx *ctx, int group, bool on = true) : c(ctx), g(group) {
    if (on && c->prof && !c->capturing) {
      a = get(c);
      if (a) (void)hipEventRecord(a, c->stream);
    }
  }
  ~SgsProfScope() {
    if (!a) return;
    hipEvent_t b = get(c);
    if (!b) return;
    (void)hipEventRecord(b, c->stream);
    c->prof_recs.push_back({g, a, b});
  }
};

// ---- launchers (one translation unit each) --------------------------------
// quant.hip
int64_t quant_partial_words(int64_t n);  // FP64/u64 scratch words the quantizer passes need
hipError_t launch_fakequant_prune(sgs_ctx *c, const float *params, const float *q,
                                  const float *score, int mode, const uint8_t *given,
                                  uint64_t seed, uint64_t step, float *qparams,
                                  uint8_t *hard, float *soft, uint64_t *stats);
hipError_t launch_rate_proxy(sgs_ctx *c, const uint64_t *stats, const float *q,
                             float weight, float *out3, float *rate_grad);
hipError_t launch_fakequant_bwd(sgs_ctx *c, const float *params, const float *q,
                                const float *soft, int mode, const float *rate_grad,
                                const uint64_t *stats, const float *gq_in,
                                const float *gmask_in, float *gparams, float *gqstep,
                                float *gscore);
// Finish of the step-size gradient over block partials partial[j * jstride +
// b * bstride], b < nblocks, with the rate proxy's gradients (rate_grad and
// stats both given, or both null).
hipError_t launch_quant_bwd_finish(sgs_ctx *c, int64_t nblocks, const double *partial,
                                   int64_t jstride, int64_t bstride, const float *q,
                                   const float *rate_grad, const uint64_t *stats,
                                   float *gparams, float *gqstep);
// project.hip
// q non-null: qparams holds the raw rows, quantized inside the projection.
hipError_t launch_preprocess(sgs_ctx *c, const float *qparams, const uint8_t *hard,
                             const float *q = nullptr);
hipError_t launch_preprocess_bwd(sgs_ctx *c, const float *qparams, float *grad_qparams,
                                 float *grad_mask);
// Projection backward fused with the quantizer/mask backward over the raw
// rows; the step-size partials go to partial[j * (*nblocks) + b].
hipError_t launch_preprocess_bwd_fused(sgs_ctx *c, const float *params, const float *q,
                                       int mode, const float *soft, const float *rate_grad,
                                       float *grad_params, float *grad_mask, float *grad_score,
                                       double *partial, int64_t *nblocks);
int64_t proj_partial_doubles(int64_t n);  // FP64 scratch words of the fused backward
// sort.hip
hipError_t ensure_tmp(sgs_ctx *c, int64_t scan_words, int64_t hist_words);
// Pair total reported when the true total does not fit in 32 bits (the
// offsets are then meaningless and no pair is emitted).
constexpr uint32_t kPairsSaturated = 0xFFFFFFFFu;
int64_t radix_blocks(int64_t count);       // blocks of a radix pass over count elements
int64_t l2_chunks_for(int64_t cap, int64_t total_st);  // level-2 chunks for a pair capacity
int64_t radix_hist_words(int64_t count);   // sort_hist words a radix sort of count needs
// Exclusive scan of count words into out[0..count] (out[count] = total); the
// total also to *total_out; with cap >= 0 total_out[1] = min(total, cap) and
// total_out[2] |= 1 on overflow (the pair count of the fixed-capacity mode).
hipError_t launch_exclusive_scan(sgs_ctx *c, const uint32_t *in, uint32_t *out,
                                 int64_t count, uint32_t *total_out, int64_t cap = -1);
// Stable LSD radix sort of 32-bit keys with 32-bit values over bits
// [shift0, bits) starting in buffer cur0; ping-pongs between buffer 0 and 1;
// returns the buffer index that holds the result in *which.  seg_len > 0:
// every seg_len elements are sorted on their own (a multiple of the sort's
// block size, static count).
hipError_t launch_radix_sort(sgs_ctx *c, uint32_t *keys[2], uint32_t *vals[2],
                             int64_t count, int bits, int *which, const uint32_t *dcount,
                             int shift0 = 0, int cur0 = 0, uint32_t **vals2 = nullptr,
                             int64_t seg_len = 0);
hipError_t launch_bin_pairs(sgs_ctx *c);   // depth order -> pairs -> tile sort -> ranges
hipError_t launch_depth_order(sgs_ctx *c); // depth sort + scan (writes d_pairs_total)
// blend.hip
#define SGS_TILE_BINS 68
#define SGS_EVAL_SLOTS 64
// codec.hip
int64_t fl_scratch_words(int64_t n);
hipError_t launch_adam(sgs_ctx *c, const sgs_adam_options *o, float *params, float *pm,
                       float *pv, const float *gp, float *q, float *qm, float *qv,
                       const float *gq, float *s, float *sm, float *sv, const float *gs);
struct SgsCompactArrays {
  const float *src[SGS_COMPACT_MAX_ARRAYS];
  float *dst[SGS_COMPACT_MAX_ARRAYS];
  int32_t row0[SGS_COMPACT_MAX_ARRAYS + 1];  // first row of each array in the launch
  int32_t narrays;
};
hipError_t launch_compact_count(sgs_ctx *c, const uint8_t *hard, uint32_t *d_total);
hipError_t launch_compact_scatter(sgs_ctx *c, const uint8_t *hard, const SgsCompactArrays &A,
                                  int64_t dst_pad);
hipError_t launch_rate_proxy_mode(sgs_ctx *c, const uint64_t *stats, const float *q,
                                  float weight, int additive, float alpha, float *out3,
                                  float *rate_grad);
int64_t lap_partial_doubles(int64_t n);
hipError_t launch_rate_variant(sgs_ctx *c, const float *params, const float *q,
                               const uint64_t *stats, const sgs_rate_options *o, float weight,
                               float *out3, float *rate_grad);
hipError_t launch_rate_variant_bwd(sgs_ctx *c, const float *params, float *grad);
int64_t ssim_scratch_doubles(int64_t V, int64_t W, int64_t H);
hipError_t launch_ssim(sgs_ctx *c, const float *image, const float *target, float weight,
                       float *loss, float *dimg);
hipError_t launch_fl_encode(sgs_ctx *c, const float *params, const float *q, const uint8_t *hard,
                            sgs_fl_channel *hdr, uint32_t *payload, int64_t cap_words,
                            int64_t *out);
hipError_t launch_fl_decode(sgs_ctx *c, const sgs_fl_channel *hdr, const uint32_t *payload,
                            int64_t words, int64_t kept, int64_t out_pad, float *out);
hipError_t launch_tile_order(sgs_ctx *c);  // ranges -> blend tile order (longest first)
hipError_t launch_blend_fwd(sgs_ctx *c, float *image, float *final_T, uint32_t *last,
                            uint64_t *eval_count);
hipError_t launch_blend_bwd(sgs_ctx *c, const float *final_T, const uint32_t *last,
                            const float *dL_dimage);
// mlp.hip
int mlp_grid(int64_t rows);  // blocks of the row kernels (partials per block)
int64_t mlp_train_scratch_bytes(int64_t B);
// Device address of the static training workspace (SGS_MLP_STATIC_ROWS rows)
// on `device`, resolved once per device with that device current; nullptr
// with the HIP error in *err when the symbol cannot be resolved.
void *mlp_static_scratch(int device, hipError_t *err);
int64_t mlp_static_scratch_bytes();
hipError_t launch_mlp_pack(sgs_ctx *c, const float *theta, void *packed);
hipError_t launch_mlp_rate_fwd(sgs_ctx *c, const void *packed, const float *theta,
                               const float *params, const float *q, const uint64_t *stats,
                               const uint8_t *hard, float *outR, float *fout);
hipError_t launch_mlp_rate_bwd(sgs_ctx *c, const void *packed, const float *theta,
                               const float *params, const float *q, const uint64_t *stats,
                               const uint8_t *hard, const float *soft, int mode, float weight,
                               float *gparams, float *gqstep, float *gscore, float *gmask);
hipError_t launch_mlp_features(sgs_ctx *c, const float *params, const float *q,
                               const uint64_t *stats, const int32_t *idx, int64_t rows,
                               uint16_t *X);
hipError_t launch_mlp_infer(sgs_ctx *c, const void *packed, const float *theta,
                            const uint16_t *X, int64_t B, float *fout);
hipError_t launch_mlp_train_step(sgs_ctx *c, float *theta, float *m, float *v, void *packed,
                                 const uint16_t *X, const float *target, int64_t B, float lr,
                                 int64_t step, float *loss, float *gtheta, void *scratch,
                                 bool profile = true);
// loss.hip
// Learned-coding stage (octree tokens, entropy coder)
void coding_free(sgs_ctx *c);
hipError_t launch_octree_encode(sgs_ctx *c, const float *params, int64_t npad, int64_t n,
                                const float *q, const uint8_t *hard, uint8_t *tokens,
                                int64_t token_cap, uint64_t *codes, uint32_t *dup_index,
                                uint32_t *dup_count, int64_t dup_cap, sgs_octree_header *h);
hipError_t launch_octree_decode(sgs_ctx *c, const sgs_octree_header *h, const uint8_t *tokens,
                                const uint32_t *dup_index, const uint32_t *dup_count,
                                const float *q, uint64_t *codes, float *xyz, int64_t out_pad,
                                int64_t *info);
hipError_t launch_ans_model(sgs_ctx *c, const uint8_t *sym, int64_t n, int order, int64_t S,
                            uint16_t *freq, double *bits);
hipError_t launch_ans_encode(sgs_ctx *c, const uint8_t *sym, int64_t n, int order, int64_t S,
                             const uint16_t *freq, uint16_t *words, int64_t word_cap,
                             int64_t *block_off, int64_t *info);
hipError_t launch_ans_decode(sgs_ctx *c, const uint16_t *words, int64_t n_words,
                             const int64_t *block_off, int64_t n, int order, int64_t S,
                             const uint16_t *freq, uint8_t *sym, int64_t *info);
hipError_t launch_ans_decode_multi(sgs_ctx *c, int32_t count, const sgs_ans_stream *st,
                                   int64_t *info);
hipError_t launch_morton_order(sgs_ctx *c, const float *params, int64_t npad, int64_t n,
                               const float *q, const uint8_t *hard, const sgs_octree_header *h,
                               const uint64_t *codes, int32_t *perm);
int64_t attr_plane_rows(const sgs_fl_channel *fl, const uint8_t *pred);
hipError_t launch_attr_planes(sgs_ctx *c, const float *params, int64_t npad, const int32_t *perm,
                              int64_t kept, const sgs_fl_channel *fl, const uint8_t *pred,
                              int32_t S, uint8_t *planes);
hipError_t launch_attr_reconstruct(sgs_ctx *c, const uint8_t *planes, int64_t kept,
                                   const sgs_fl_channel *fl, const uint8_t *pred, int32_t S,
                                   float *out, int64_t out_pad);
hipError_t launch_pos_embed(sgs_ctx *c, const float *xyz, int64_t pad, int64_t count, int L,
                            int d, const float *W, const float *b, float *out);

hipError_t launch_l1(sgs_ctx *c, const float *image, const float *target, float scale,
                     float *loss, float *dimg);

// ---- device helpers ---------------------------------------------------------

// SplitMix64 (Steele, Lea, Flood 2014): the counter hash of the mask noise.
__device__ __forceinline__ uint64_t sgs_splitmix64(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}

// Uniform in (0,1) with 23 random bits plus one half: exact in FP32.
__device__ __forceinline__ float sgs_uniform(uint64_t seed, uint64_t step, uint64_t i) {
  const uint64_t h = sgs_splitmix64(seed ^ ((step << 32) + i));
  return ((float)(uint32_t)(h >> 41) + 0.5f) * 0x1p-23f;
}

// FP32 exponential whose result is reproducible on any IEEE machine:
// Cody-Waite split of x = n ln2 + r, degree-7 Taylor polynomial of e^r in
// Horner form, scaling by 2^n.  Input clamped to [-80, 80].
__device__ __forceinline__ float sgs_exp_repro(float x) {
  x = fminf(fmaxf(x, -80.0f), 80.0f);
  const float n = rintf(x * 0x1.715476p+0f);
  const float r = (x - n * 0x1.62e4p-1f) - n * 0x1.7f7d1cp-20f;
  float p = 1.0f / 5040.0f;
  p = p * r + 1.0f / 720.0f;
  p = p * r + 1.0f / 120.0f;
  p = p * r + 1.0f / 24.0f;
  p = p * r + 1.0f / 6.0f;
  p = p * r + 0.5f;
  p = p * r + 1.0f;
  p = p * r + 1.0f;
  return ldexpf(p, (int)n);
}

// Gumbel-sigmoid retention of a Gaussian with score sc and uniform draw u:
// hard = [u (1 + e^sc) > 1] (= [sc + logit u > 0]), sm = sigmoid((sc + logit
// u) / tau).
__device__ __forceinline__ uint8_t sgs_gumbel_decide(float sc, float u, float tau, float &sm) {
  const float e = sgs_exp_repro(sc);
  const uint8_t m = (u * (1.0f + e)) > 1.0f ? 1 : 0;
  const float l = logf(u) - logf(1.0f - u);
  sm = 1.0f / (1.0f + __expf(-(sc + l) / tau));
  return m;
}

// Retention decision of Gaussian i (Sec. 3.3.1): mode 0 the given mask, 1 the
// Gumbel-sigmoid draw (hard = [u (1 + e^s) > 1], soft = sigmoid((s + logit
// u) / tau)), 2 keep every Gaussian.  Returns the hard mask; sm receives the
// relaxed one (the hard one in modes 0 and 2).
__device__ __forceinline__ uint8_t sgs_mask_decide(int mode, const uint8_t *__restrict__ given,
                                                   const float *__restrict__ score, uint64_t seed,
                                                   uint64_t step, float tau, int64_t i,
                                                   float &sm) {
  if (mode == 0) {
    const uint8_t m = given[i] ? 1 : 0;
    sm = (float)m;
    return m;
  }
  if (mode == 2) {
    sm = 1.0f;
    return 1;
  }
  return sgs_gumbel_decide(score[i], sgs_uniform(seed, step, (uint64_t)i), tau, sm);
}

// Workgroups are dispatched to the eight XCDs round-robin (hardware id i runs
// on XCD i % 8, each XCD with its own L2).  A grid of g workgroups that loops
// over nlive logical blocks (a resident grid whose work count is on the
// device) walks them so that every XCD takes one contiguous share:
// neighbouring blocks, which touch neighbouring memory (the two halves of a
// cache line at a write boundary), then share an L2.  Hardware block i takes
// first, first + step, ... < end; with fewer than eight workgroups some XCD
// has none, and the walk is a plain stride.
struct SgsXcdWalk {
  int64_t first, step, end;
};
__device__ __forceinline__ SgsXcdWalk sgs_xcd_walk(int64_t i, int64_t g, int64_t nlive) {
  if (g < 8) return {i, g, nlive};
  const int64_t x = i & 7, k = i >> 3;
  const int64_t gx = (g >> 3) + (x < (g & 7) ? 1 : 0);  // workgroups on XCD x
  const int64_t per = nlive >> 3, rem = nlive & 7;
  const int64_t start = x * per + (x < rem ? x : rem);
  return {start + k, gx, start + per + (x < rem ? 1 : 0)};
}

// One workgroup per logical block in a grid of nb sized for a capacity, of
// which only the first nlive hold work: the live range is split over the
// eight XCDs as above, so each does an equal share whatever the grid size,
// and the other hardware blocks take the logical blocks nlive, nlive + 1,
// ... in dispatch order (their rank among them: for each XCD, its blocks
// dispatched earlier beyond its live share).  A bijection of [0, nb).
__device__ __forceinline__ int64_t sgs_xcd_block_live(int64_t i, int64_t nb, int64_t nlive) {
  nlive = nlive < nb ? nlive : nb;
  const int64_t x = i & 7, k = i >> 3, per = nlive >> 3, rem = nlive & 7;
  if (k < per + (x < rem ? 1 : 0)) return x * per + (x < rem ? x : rem) + k;
  int64_t r = 0;
#pragma unroll
  for (int xp = 0; xp < 8; ++xp) {
    const int64_t before = k + (xp < x ? 1 : 0), share = per + (xp < rem ? 1 : 0);
    r += before > share ? before - share : 0;
  }
  return nlive + r;
}

// The quantizer's code k = rint(y / q) (FP32 division, ties to even), and
// whether it lies in int32.
__device__ __forceinline__ int32_t sgs_code_of(float y, float q, bool &ok) {
  const float k = rintf(__fdiv_rn(y, q));
  ok = k >= -2147483648.0f && k < 2147483648.0f;
  return ok ? (int32_t)k : 0;
}

// The same decision from y * rq, rq = 1 / q correctly rounded and a normal
// float (fast_ok): then |y rq - y/q| <= (2^-23 + 2^-48) |y/q| (plus 2^-150
// where y rq is subnormal) and the rounded quotient lies within 2^-24 |y/q|
// of y/q, so the two are within about 3 * 2^-24 |y rq| of each other and round
// to the same integer whenever y rq lies farther than 2^-21 |y rq| from every
// half-integer: |y rq - k| < 1/2 - 2^-21 |y rq| with k = rint(y rq) (t - k is
// exact; the bound, rounded once, keeps a margin of more than 2 over the
// error; it is negative from |y rq| = 2^20 on, so k stays far inside int32).
// Otherwise (near a tie, large, not finite) the division decides.  This one
// returns rint(fl32(y / q)) as a float; sgs_code_fast below, the int32 code.
// Ordering of the LDS accesses of one wave among themselves (lanes of a wave
// read what other lanes of the same wave wrote; no workgroup barrier).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// sgs_product_decides(t, k): whether k = rint(t), t = y rq, is that integer.
__device__ __forceinline__ bool sgs_product_decides(float t, float k) {
  return fabsf(t - k) < __fmaf_rn(-fabsf(t), 4.76837158203125e-7f, 0.5f);
}
__device__ __forceinline__ float sgs_rint_div(float y, float q, float rq, bool fast_ok) {
  const float t = y * rq;
  const float k = rintf(t);
  if (fast_ok && sgs_product_decides(t, k)) return k;
  return rintf(__fdiv_rn(y, q));
}
// Whether rq = 1 / q (correctly rounded) is a normal float, so that the
// product rule above holds.
__device__ __forceinline__ bool sgs_rq_ok(float rq) {
  return fabsf(rq) >= 1.17549435e-38f && fabsf(rq) <= 3.40282347e+38f;
}

__device__ __forceinline__ int32_t sgs_code_fast(float y, float q, float rq, bool fast_ok, bool &ok) {
  const float t = y * rq;
  const float k = rintf(t);
  if (fast_ok && sgs_product_decides(t, k)) {
    ok = true;
    return (int32_t)k;
  }
  return sgs_code_of(y, q, ok);
}

// Bit i = (byte i of m) != 0: the high bit of each nonzero byte (the carry of
// its low seven bits plus 0x7F, or its own high bit), gathered by one
// multiply into bits 28..31 (the other partial products land below bit 24).
__device__ __forceinline__ uint32_t sgs_nonzero_nibble(uint32_t m) {
  const uint32_t nz = (((m & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | m) & 0x80808080u;
  return ((nz >> 7) * 0x10204080u) >> 28;
}

// Order-preserving map of float bits to uint32 (for min/max keys).
__device__ __forceinline__ uint32_t sgs_ord(float f) {
  const uint32_t u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__host__ __device__ __forceinline__ float sgs_unord(uint32_t o) {
  const uint32_t u = (o & 0x80000000u) ? (o & 0x7FFFFFFFu) : ~o;
#ifdef __HIP_DEVICE_COMPILE__
  return __uint_as_float(u);
#else
  float f;
  __builtin_memcpy(&f, &u, 4);
  return f;
#endif
}

// Projection of one Gaussian into one view.  The fields up to `x1` are the
// discrete structure (decided in FP32 with a fixed operation order); the rest
// are the continuous values the blend and the backward use.
struct SgsCam {
  float R[9], t[3], fx, fy, cx, cy, campos[3];
};

struct SgsProj {
  bool valid;
  float tz, px, py;
  int x0, x1, y0, y1;
  // intermediates (kept for the backward pass)
  float tx, ty, ux, uy;
  bool clx, cly;
  float qh[4], qn;
  float Rq[9], S[3], M[9];
  float Sg[6];                 // 00 01 02 11 12 22
  float J00, J02, J11, J12;
  float T0[3], T1[3];
  float a, b, c, det;
};

// Discrete structure of one splat.  Operation order (all FP32, no
// contraction, correctly rounded: `sqrtf` and `__fdiv_rn`; the `__fsqrt_rn`
// intrinsic is off by one ulp on a sizeable fraction of inputs and would move
// ceil(3 sqrt(lambda)) where 3 sqrt(lambda) lands next to an integer):
//   t = ((R0 mu0 + R1 mu1) + R2 mu2) + t0 (per row); cull unless tz > 0.2;
//   qq = ((w^2 + x^2) + y^2) + z^2, cull unless qq > 0; q /= sqrt(qq);
//   rotation matrix in the usual unit-quaternion form; S = exp_repro(s);
//   M = Rq diag(S); Sigma_ab = (M_a0 M_b0 + M_a1 M_b1) + M_a2 M_b2;
//   lim = 1.3 ((W/2)/fx); clamped u = min(lim, max(-lim, tx/tz));
//   J00 = fx/tz, J02 = -(fx u)/tz (same for y); T = J R (two products);
//   Sigma' = T Sigma T^T + 0.3 I, with u_a = (S_a0 T0 + S_a1 T1) + S_a2 T2;
//   det = a c - b b, cull unless det > 0; lambda = mid + sqrt(max(0, mid^2 - det));
//   r = ceil(3 sqrt(lambda)); px = fx (tx/tz) + cx;
//   span = [ceil(px - r), floor(px + r)] clipped to the image, cull if empty.
__device__ __forceinline__ void sgs_project(const float *y, const SgsCam &cam, int W, int H,
                                            SgsProj &o) {
  o.valid = false;
  const float mx = y[0], my = y[1], mz = y[2];
  o.tx = ((cam.R[0] * mx + cam.R[1] * my) + cam.R[2] * mz) + cam.t[0];
  o.ty = ((cam.R[3] * mx + cam.R[4] * my) + cam.R[5] * mz) + cam.t[1];
  o.tz = ((cam.R[6] * mx + cam.R[7] * my) + cam.R[8] * mz) + cam.t[2];
  if (!(o.tz > SGS_NEAR)) return;
  float w = y[SGS_CH_ROT], x = y[SGS_CH_ROT + 1], yy = y[SGS_CH_ROT + 2], z = y[SGS_CH_ROT + 3];
  const float qq = ((w * w + x * x) + yy * yy) + z * z;
  if (!(qq > 0.0f)) return;
  o.qn = sqrtf(qq);
  w = __fdiv_rn(w, o.qn);
  x = __fdiv_rn(x, o.qn);
  yy = __fdiv_rn(yy, o.qn);
  z = __fdiv_rn(z, o.qn);
  o.qh[0] = w; o.qh[1] = x; o.qh[2] = yy; o.qh[3] = z;
  float *Rq = o.Rq;
  Rq[0] = 1.0f - 2.0f * (yy * yy + z * z);
  Rq[1] = 2.0f * (x * yy - w * z);
  Rq[2] = 2.0f * (x * z + w * yy);
  Rq[3] = 2.0f * (x * yy + w * z);
  Rq[4] = 1.0f - 2.0f * (x * x + z * z);
  Rq[5] = 2.0f * (yy * z - w * x);
  Rq[6] = 2.0f * (x * z - w * yy);
  Rq[7] = 2.0f * (yy * z + w * x);
  Rq[8] = 1.0f - 2.0f * (x * x + yy * yy);
#pragma unroll
  for (int k = 0; k < 3; ++k) o.S[k] = sgs_exp_repro(y[SGS_CH_SCALE + k]);
#pragma unroll
  for (int e = 0; e < 9; ++e) o.M[e] = Rq[e] * o.S[e % 3];
  const float *M = o.M;
  // Sigma: products commute exactly, so the six distinct entries suffice
  o.Sg[0] = (M[0] * M[0] + M[1] * M[1]) + M[2] * M[2];
  o.Sg[1] = (M[0] * M[3] + M[1] * M[4]) + M[2] * M[5];
  o.Sg[2] = (M[0] * M[6] + M[1] * M[7]) + M[2] * M[8];
  o.Sg[3] = (M[3] * M[3] + M[4] * M[4]) + M[5] * M[5];
  o.Sg[4] = (M[3] * M[6] + M[4] * M[7]) + M[5] * M[8];
  o.Sg[5] = (M[6] * M[6] + M[7] * M[7]) + M[8] * M[8];
  const float limx = 1.3f * __fdiv_rn(0.5f * (float)W, cam.fx);
  const float limy = 1.3f * __fdiv_rn(0.5f * (float)H, cam.fy);
  o.ux = __fdiv_rn(o.tx, o.tz);
  o.uy = __fdiv_rn(o.ty, o.tz);
  const float cux = fminf(limx, fmaxf(-limx, o.ux));
  const float cuy = fminf(limy, fmaxf(-limy, o.uy));
  o.clx = (o.ux < -limx) || (o.ux > limx);
  o.cly = (o.uy < -limy) || (o.uy > limy);
  o.J00 = __fdiv_rn(cam.fx, o.tz);
  o.J02 = __fdiv_rn(-(cam.fx * cux), o.tz);
  o.J11 = __fdiv_rn(cam.fy, o.tz);
  o.J12 = __fdiv_rn(-(cam.fy * cuy), o.tz);
#pragma unroll
  for (int b = 0; b < 3; ++b) {
    o.T0[b] = o.J00 * cam.R[b] + o.J02 * cam.R[6 + b];
    o.T1[b] = o.J11 * cam.R[3 + b] + o.J12 * cam.R[6 + b];
  }
  const float S00 = o.Sg[0], S01 = o.Sg[1], S02 = o.Sg[2], S11 = o.Sg[3], S12 = o.Sg[4],
              S22 = o.Sg[5];
  const float u0 = (S00 * o.T0[0] + S01 * o.T0[1]) + S02 * o.T0[2];
  const float u1 = (S01 * o.T0[0] + S11 * o.T0[1]) + S12 * o.T0[2];
  const float u2 = (S02 * o.T0[0] + S12 * o.T0[1]) + S22 * o.T0[2];
  const float w0 = (S00 * o.T1[0] + S01 * o.T1[1]) + S02 * o.T1[2];
  const float w1 = (S01 * o.T1[0] + S11 * o.T1[1]) + S12 * o.T1[2];
  const float w2 = (S02 * o.T1[0] + S12 * o.T1[1]) + S22 * o.T1[2];
  o.a = ((o.T0[0] * u0 + o.T0[1] * u1) + o.T0[2] * u2) + SGS_DILATION;
  o.b = (o.T0[0] * w0 + o.T0[1] * w1) + o.T0[2] * w2;
  o.c = ((o.T1[0] * w0 + o.T1[1] * w1) + o.T1[2] * w2) + SGS_DILATION;
  o.det = o.a * o.c - o.b * o.b;
  if (!(o.det > 0.0f)) return;
  const float mid = 0.5f * (o.a + o.c);
  const float disc = fmaxf(mid * mid - o.det, 0.0f);
  const float lmax = mid + sqrtf(disc);
  const float rf = ceilf(3.0f * sqrtf(lmax));
  o.px = cam.fx * o.ux + cam.cx;
  o.py = cam.fy * o.uy + cam.cy;
  const float xlo = ceilf(o.px - rf), xhi = floorf(o.px + rf);
  const float ylo = ceilf(o.py - rf), yhi = floorf(o.py + rf);
  if (xhi < 0.0f || xlo > (float)(W - 1) || yhi < 0.0f || ylo > (float)(H - 1)) return;
  o.x0 = xlo < 0.0f ? 0 : (int)xlo;
  o.x1 = xhi > (float)(W - 1) ? W - 1 : (int)xhi;
  o.y0 = ylo < 0.0f ? 0 : (int)ylo;
  o.y1 = yhi > (float)(H - 1) ? H - 1 : (int)yhi;
  o.valid = true;
}

// Real spherical harmonics of degree <= 3 (orthonormal, Condon-Shortley
// phase, index l^2 + l + m) at the unit direction (x, y, z).  Constants are
// K_l^m sqrt(2) times the associated-Legendre factor:
//   Y1: sqrt(3/(4 pi));  Y2: (1/2)sqrt(15/pi), (1/4)sqrt(5/pi), (1/4)sqrt(15/pi);
//   Y3: (1/4)sqrt(35/(2 pi)), (1/2)sqrt(105/pi), (1/4)sqrt(21/(2 pi)),
//       (1/4)sqrt(7/pi), (1/4)sqrt(105/pi).
#define SGS_SH_C0 0.28209479177387814f
#define SGS_SH_C1 0.48860251190291992f
#define SGS_SH_C2A 1.0925484305920792f
#define SGS_SH_C2B 0.31539156525252005f
#define SGS_SH_C2C 0.54627421529603959f
#define SGS_SH_C3A 0.59004358992664352f
#define SGS_SH_C3B 2.8906114426405538f
#define SGS_SH_C3C 0.45704579946446572f
#define SGS_SH_C3D 0.37317633259011540f
#define SGS_SH_C3E 1.4453057213202769f

__device__ __forceinline__ void sgs_sh_basis(float x, float y, float z, float Y[16]) {
  const float xx = x * x, yy = y * y, zz = z * z;
  Y[0] = SGS_SH_C0;
  Y[1] = -SGS_SH_C1 * y;
  Y[2] = SGS_SH_C1 * z;
  Y[3] = -SGS_SH_C1 * x;
  Y[4] = SGS_SH_C2A * x * y;
  Y[5] = -SGS_SH_C2A * y * z;
  Y[6] = SGS_SH_C2B * (2.0f * zz - xx - yy);
  Y[7] = -SGS_SH_C2A * x * z;
  Y[8] = SGS_SH_C2C * (xx - yy);
  Y[9] = -SGS_SH_C3A * y * (3.0f * xx - yy);
  Y[10] = SGS_SH_C3B * x * y * z;
  Y[11] = -SGS_SH_C3C * y * (4.0f * zz - xx - yy);
  Y[12] = SGS_SH_C3D * z * (2.0f * zz - 3.0f * xx - 3.0f * yy);
  Y[13] = -SGS_SH_C3C * x * (4.0f * zz - xx - yy);
  Y[14] = SGS_SH_C3E * z * (xx - yy);
  Y[15] = -SGS_SH_C3A * x * (xx - 3.0f * yy);
}

// Gradient of each basis polynomial w.r.t. (x, y, z).
__device__ __forceinline__ void sgs_sh_grad(float x, float y, float z, float G[16][3]) {
  const float xx = x * x, yy = y * y, zz = z * z;
#pragma unroll
  for (int k = 0; k < 16; ++k) G[k][0] = G[k][1] = G[k][2] = 0.0f;
  G[1][1] = -SGS_SH_C1;
  G[2][2] = SGS_SH_C1;
  G[3][0] = -SGS_SH_C1;
  G[4][0] = SGS_SH_C2A * y; G[4][1] = SGS_SH_C2A * x;
  G[5][1] = -SGS_SH_C2A * z; G[5][2] = -SGS_SH_C2A * y;
  G[6][0] = -2.0f * SGS_SH_C2B * x; G[6][1] = -2.0f * SGS_SH_C2B * y; G[6][2] = 4.0f * SGS_SH_C2B * z;
  G[7][0] = -SGS_SH_C2A * z; G[7][2] = -SGS_SH_C2A * x;
  G[8][0] = 2.0f * SGS_SH_C2C * x; G[8][1] = -2.0f * SGS_SH_C2C * y;
  G[9][0] = -SGS_SH_C3A * 6.0f * x * y; G[9][1] = -SGS_SH_C3A * 3.0f * (xx - yy);
  G[10][0] = SGS_SH_C3B * y * z; G[10][1] = SGS_SH_C3B * x * z; G[10][2] = SGS_SH_C3B * x * y;
  G[11][0] = SGS_SH_C3C * 2.0f * x * y;
  G[11][1] = -SGS_SH_C3C * (4.0f * zz - xx - 3.0f * yy);
  G[11][2] = -SGS_SH_C3C * 8.0f * y * z;
  G[12][0] = -SGS_SH_C3D * 6.0f * x * z;
  G[12][1] = -SGS_SH_C3D * 6.0f * y * z;
  G[12][2] = SGS_SH_C3D * (6.0f * zz - 3.0f * xx - 3.0f * yy);
  G[13][0] = -SGS_SH_C3C * (4.0f * zz - 3.0f * xx - yy);
  G[13][1] = SGS_SH_C3C * 2.0f * x * y;
  G[13][2] = -SGS_SH_C3C * 8.0f * x * z;
  G[14][0] = SGS_SH_C3E * 2.0f * x * z; G[14][1] = -SGS_SH_C3E * 2.0f * y * z;
  G[14][2] = SGS_SH_C3E * (xx - yy);
  G[15][0] = -SGS_SH_C3A * 3.0f * (xx - yy); G[15][1] = SGS_SH_C3A * 6.0f * x * y;
}

__device__ __forceinline__ int sgs_sh_channel(int k, int ch) {
  return k == 0 ? SGS_CH_DC + ch : SGS_CH_REST + 3 * (k - 1) + ch;
}

// Wave-level helpers (wave64).
__device__ __forceinline__ float sgs_wave_sum(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ double sgs_wave_sum_d(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

inline unsigned sgs_blocks(int64_t n, int threads) {
  return (unsigned)((n + threads - 1) / threads);
}
