// C ABI of libspeedygs (declared in include/speedygs.h): argument checks,
// scratch ownership and the order of the launches.  No exception crosses the
// ABI; every failure is a status code plus a message in the context.
#include <stdarg.h>
#include <cmath>
#include <stdio.h>
#include <string.h>

#include <new>

#include "sgs_internal.h"

namespace {

sgs_status fail(sgs_ctx *c, sgs_status s, const char *fmt, ...) {
  if (c) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(c->err, sizeof(c->err), fmt, ap);
    va_end(ap);
  }
  return s;
}

sgs_status hip_fail(sgs_ctx *c, hipError_t e, const char *where) {
  return fail(c, e == hipErrorOutOfMemory ? SGS_ENOMEM : SGS_EHIP, "%s: %s", where,
              hipGetErrorString(e));
}

#define SGS_HIP(call, where)                         \
  do {                                               \
    hipError_t e_ = (call);                          \
    if (e_ != hipSuccess) return hip_fail(c, e_, where); \
  } while (0)

template <typename T>
hipError_t dalloc(T **p, int64_t count) {
  *p = nullptr;
  if (count <= 0) count = 1;
  return hipMalloc((void **)p, sizeof(T) * (size_t)count);
}

template <typename T>
void dfree(T *&p) {
  if (p) (void)hipFree((void *)p);
  p = nullptr;
}

void free_scene(sgs_ctx *c) {
  dfree(c->d_cams);
  dfree(c->rec);
  for (int k = 0; k < 2; ++k) {
    dfree(c->depth_key[k]);
    dfree(c->depth_val[k]);
    dfree(c->depth_rect[k]);
    dfree(c->tile_key[k]);
    dfree(c->pair_val[k]);
  }
  dfree(c->touched);
  dfree(c->ioffsets);
  dfree(c->st_ranges);
  dfree(c->chunk_first);
  dfree(c->l2_cnt);
  c->l2_chunks = 0;
  dfree(c->tile_cnt);
  dfree(c->tile_start);
  dfree(c->bin_splat);
  dfree(c->mlp_f);
  dfree(c->fl_tmp);
  c->fl_tmp_words = 0;
  dfree(c->ssim_tmp);
  c->ssim_tmp_doubles = 0;
  dfree(c->lap_coef);
  c->lap_ready = false;
  dfree(c->mlp_signs);
  c->mlp_saved = false;
  dfree(c->blk_start);
  c->blk_start_words = 0;
  dfree(c->splat_grad);
  dfree(c->big_idx);
  dfree(c->big_list);
  dfree(c->big_rep);
  dfree(c->det_acc);
  dfree(c->ranges);
  dfree(c->tile_order);
  dfree(c->tile_bins);
  dfree(c->eval_slots);
  dfree(c->scan_tmp);
  dfree(c->sort_hist);
  dfree(c->red_tmp);
  dfree(c->d_pairs_total);
  c->scan_tmp_words = c->sort_hist_words = c->red_tmp_words = 0;
  c->pair_cap = 0;
  c->scene_set = false;
  c->rendered = false;
}

bool aligned(const void *p, size_t a) { return ((uintptr_t)p % a) == 0; }

hipError_t grow_pairs(sgs_ctx *c, int64_t P) {
  if (P <= c->pair_cap) return hipSuccess;
  const int64_t cap = P + P / 8 + 1024;
  for (int k = 0; k < 2; ++k) {
    dfree(c->tile_key[k]);
    dfree(c->pair_val[k]);
  }
  dfree(c->blk_start);
  c->blk_start_words = 0;
  dfree(c->l2_cnt);
  c->l2_chunks = 0;
  c->pair_cap = 0;
  for (int k = 0; k < 2; ++k) {
    hipError_t e = dalloc(&c->tile_key[k], cap);
    if (e != hipSuccess) return e;
    e = dalloc(&c->pair_val[k], cap);
    if (e != hipSuccess) return e;
  }
  const int64_t nbs = radix_blocks(cap) + 1;
  hipError_t eb = dalloc(&c->blk_start, nbs);
  if (eb != hipSuccess) return eb;
  c->blk_start_words = nbs;
  const int64_t chunks = l2_chunks_for(cap, c->total_st);
  eb = dalloc(&c->l2_cnt, chunks * 64);
  if (eb != hipSuccess) return eb;
  c->l2_chunks = chunks;
  const int64_t hist = radix_hist_words(cap);
  hipError_t e = ensure_tmp(c, c->scan_tmp_words, hist);
  if (e != hipSuccess) return e;
  c->pair_cap = cap;
  return hipSuccess;
}

}  // namespace

extern "C" {

sgs_status sgs_create(sgs_ctx **out, int device, void *hip_stream) {
  if (!out) return SGS_EINVAL;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return SGS_EINVAL;
  sgs_ctx *c = new (std::nothrow) sgs_ctx();
  if (!c) return SGS_ENOMEM;
  c->device = device;
  c->stream = (hipStream_t)hip_stream;
  if (hipSetDevice(device) != hipSuccess ||
      hipHostMalloc((void **)&c->h_pairs_total, 8 * sizeof(uint32_t), hipHostMallocDefault) !=
          hipSuccess) {
    delete c;
    return SGS_EHIP;
  }
  c->h_aux = c->h_pairs_total + 7;
  // the allocation-free training step's workspace: its device address on
  // this device, resolved once per device with the device current
  hipError_t se = hipSuccess;
  if (!mlp_static_scratch(device, &se)) {
    (void)hipHostFree(c->h_pairs_total);
    delete c;
    return SGS_EHIP;
  }
  *out = c;
  return SGS_OK;
}

void sgs_destroy(sgs_ctx *c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  if (c->stream) (void)hipStreamSynchronize(c->stream); else (void)hipDeviceSynchronize();
  free_scene(c);
  coding_free(c);
  for (auto &r : c->prof_recs) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  for (auto e : c->ev_free) (void)hipEventDestroy(e);
  if (c->h_pairs_total) (void)hipHostFree(c->h_pairs_total);
  delete c;
}

const char *sgs_last_error(const sgs_ctx *c) { return c ? c->err : "null context"; }

sgs_status sgs_set_stream(sgs_ctx *c, void *hip_stream) {
  if (!c) return SGS_EINVAL;
  c->stream = (hipStream_t)hip_stream;
  return SGS_OK;
}

sgs_status sgs_set_scene(sgs_ctx *c, int64_t n, int64_t npad, int64_t n_hat,
                         const sgs_camera *cams, int32_t views, int32_t width, int32_t height,
                         const sgs_options *opt) {
  if (!c) return SGS_EINVAL;
  if (n < 1 || npad < n || npad % 64 != 0 || n_hat < 1)
    return fail(c, SGS_EINVAL, "set_scene: need n >= 1, npad >= n, npad %% 64 == 0, n_hat >= 1");
  if (!cams || views < 1 || width < 1 || height < 1 || width > 32768 || height > 32768)
    return fail(c, SGS_EINVAL, "set_scene: bad cameras or image size");
  if ((int64_t)views * n >= (int64_t)1 << 31)
    return fail(c, SGS_ECAPACITY, "set_scene: views * n must stay below 2^31");
  int tw = 16, th = 16, schedule = 0, det = 0;
  float tau = 1.0f;
  if (opt) {
    if (opt->tile_w || opt->tile_h) {
      tw = opt->tile_w;
      th = opt->tile_h;
    }
    if (opt->tau != 0.0f) tau = opt->tau;
    schedule = opt->schedule;
    det = opt->deterministic;
    for (int k = 0; k < 3; ++k)
      if (opt->reserved[k] != 0) return fail(c, SGS_EINVAL, "set_scene: reserved options must be 0");
  }
  if (det != 0 && det != 1) return fail(c, SGS_EINVAL, "set_scene: deterministic must be 0 or 1");
  if (schedule < 0 || schedule > 3) return fail(c, SGS_EINVAL, "set_scene: schedule must be 0 to 3");
  if (!((tw == 16 && th == 16) || (tw == 8 && th == 8) || (tw == 32 && th == 8) ||
        (tw == 32 && th == 16) || (tw == 32 && th == 32)))
    return fail(c, SGS_EINVAL, "set_scene: tile shape must be 8x8, 16x16, 32x8, 32x16 or 32x32");
  if (!(tau > 0.0f)) return fail(c, SGS_EINVAL, "set_scene: tau must be > 0");
  SGS_HIP(hipSetDevice(c->device), "hipSetDevice");
  if (c->stream) SGS_HIP(hipStreamSynchronize(c->stream), "sync"); else SGS_HIP(hipDeviceSynchronize(), "sync");
  free_scene(c);
  c->n = n;
  c->npad = npad;
  c->n_hat = n_hat;
  c->V = views;
  c->W = width;
  c->H = height;
  c->TW = tw;
  c->TH = th;
  c->tau = tau;
  c->schedule = schedule;
  c->deterministic = det != 0;
  for (int &o : c->blend_occ) o = 0;
  c->GW = (width + tw - 1) / tw;
  c->GH = (height + th - 1) / th;
  c->tiles_per_view = (int64_t)c->GW * c->GH;
  c->total_tiles = c->tiles_per_view * views;
  c->SGW = (c->GW + 7) / 8;
  c->SGH = (c->GH + 7) / 8;
  c->st_per_view = (int64_t)c->SGW * c->SGH;
  c->total_st = c->st_per_view * views;
  c->st_vbits = 0;
  while ((1 << c->st_vbits) < views) ++c->st_vbits;
  c->st_slots = c->st_per_view << c->st_vbits;
  if (c->st_slots > 65536)
    return fail(c, SGS_ECAPACITY,
                "set_scene: super-tiles (8x8 tiles) per view x views rounded up to a power "
                "of two must not exceed 65536 (%lld)", (long long)c->st_slots);
  c->vn = (int64_t)views * n;
  const int64_t vn = c->vn;
  c->vseg = (n + kDepthSeg - 1) / kDepthSeg * kDepthSeg;
  c->vn_pad = (int64_t)views * c->vseg;
  const int64_t vnp = c->vn_pad;
  hipError_t e = hipSuccess;
#define SGS_ALLOC(p, cnt)                                   \
  do {                                                      \
    e = dalloc(&(p), (cnt));                                \
    if (e != hipSuccess) { free_scene(c); return hip_fail(c, e, "set_scene alloc"); } \
  } while (0)
  SGS_ALLOC(c->d_cams, views);
  SGS_ALLOC(c->rec, 3 * vn);
  for (int k = 0; k < 2; ++k) {
    SGS_ALLOC(c->depth_key[k], vnp);
    SGS_ALLOC(c->depth_val[k], vnp);
    SGS_ALLOC(c->depth_rect[k], vnp);
  }
  SGS_ALLOC(c->touched, vn);
  SGS_ALLOC(c->ioffsets, vnp + 1);
  SGS_ALLOC(c->st_ranges, c->st_slots);
  SGS_ALLOC(c->chunk_first, c->st_slots + 2);  // + the level-2 scatter's chunk queue
  SGS_ALLOC(c->tile_cnt, c->total_tiles);
  SGS_ALLOC(c->tile_start, c->total_tiles + 1);
  SGS_ALLOC(c->bin_splat, vn);
  SGS_ALLOC(c->mlp_f, n);
  SGS_ALLOC(c->fl_tmp, fl_scratch_words(n));
  c->fl_tmp_words = fl_scratch_words(n);
  SGS_ALLOC(c->mlp_signs, 2 * n);
  SGS_ALLOC(c->splat_grad, vn * SGS_SGRAD);
  if (c->deterministic) {
    SGS_ALLOC(c->det_acc, vn * SGS_SGRAD * 3);
  } else {
    SGS_ALLOC(c->big_idx, vn);
    SGS_ALLOC(c->big_list, kBigMax + kBigRanges);
    SGS_ALLOC(c->big_rep, kBigMax * kBigReps * SGS_SGRAD);
    // the replicas start at zero and the fold after each blend clears them
    e = hipMemset(c->big_rep, 0, sizeof(double) * kBigMax * kBigReps * SGS_SGRAD);
    if (e != hipSuccess) { free_scene(c); return hip_fail(c, e, "set_scene clear"); }
  }
  SGS_ALLOC(c->ranges, c->total_tiles);
  SGS_ALLOC(c->tile_order, c->total_tiles);
  SGS_ALLOC(c->tile_bins, SGS_TILE_BINS);
  SGS_ALLOC(c->eval_slots, SGS_EVAL_SLOTS);
  SGS_ALLOC(c->d_pairs_total, 8);
  e = hipMemset(c->d_pairs_total, 0, 8 * sizeof(uint32_t));
  if (e == hipSuccess) e = hipMemset(c->eval_slots, 0, SGS_EVAL_SLOTS * sizeof(uint64_t));
  if (e != hipSuccess) { free_scene(c); return hip_fail(c, e, "set_scene clear"); }
  c->fixed_cap = false;
  const int64_t red_q = quant_partial_words(n);
  const int64_t red_l1 = (int64_t)views * 3 * width * height / 2048 + 64;
  const int64_t red_mlp = (int64_t)mlp_grid(n) * 64;
  const int64_t red_lap = lap_partial_doubles(n);
  const int64_t red_proj = proj_partial_doubles(n);
  int64_t red = red_q > red_l1 ? red_q : red_l1;
  red = red > red_mlp ? red : red_mlp;
  red = red > red_proj ? red : red_proj;
  red = (red > red_lap ? red : red_lap) + 64;
  SGS_ALLOC(c->red_tmp, red);
  c->red_tmp_words = red;
  SGS_ALLOC(c->lap_coef, 192);
#undef SGS_ALLOC
  const int64_t hist = radix_hist_words(vnp);
  // block sums of the scans over splats and over tiles
  // (twice the splats' blocks: pair and item sums of the depth order)
  const int64_t scan = 2 * (((vnp > c->total_tiles ? vnp : c->total_tiles) + 4095) / 4096 + 1);
  e = ensure_tmp(c, scan, hist);
  if (e != hipSuccess) { free_scene(c); return hip_fail(c, e, "set_scene alloc"); }
  // initial pair capacity: 4 tiles per splat
  e = grow_pairs(c, 4 * vn);
  if (e != hipSuccess) { free_scene(c); return hip_fail(c, e, "set_scene alloc"); }
  SGS_HIP(hipMemcpy(c->d_cams, cams, sizeof(sgs_camera) * views, hipMemcpyHostToDevice),
          "set_scene camera copy");
  c->h_cams.assign(cams, cams + views);
  c->scene_set = true;
  c->rendered = false;
  return SGS_OK;
}

sgs_status sgs_fakequant_prune(sgs_ctx *c, const float *params, const float *qstep,
                               const float *score, int32_t mask_mode, const uint8_t *given_mask,
                               uint64_t seed, uint64_t step, float *qparams, uint8_t *hard_mask,
                               float *soft_mask, uint64_t *stats) {
  if (!c) return SGS_EINVAL;
  if (!c->scene_set) return fail(c, SGS_ESTATE, "fakequant_prune: set_scene first");
  if (!params || !qstep || !qparams || !hard_mask || !stats)
    return fail(c, SGS_EINVAL, "fakequant_prune: null pointer");
  if (!aligned(params, 16) || !aligned(qparams, 16))
    return fail(c, SGS_EINVAL, "fakequant_prune: parameter rows must be 16-byte aligned");
  if (mask_mode < 0 || mask_mode > 2) return fail(c, SGS_EINVAL, "fakequant_prune: mask_mode");
  if (mask_mode == 0 && !given_mask) return fail(c, SGS_EINVAL, "fakequant_prune: given_mask");
  if (mask_mode == 1 && !score) return fail(c, SGS_EINVAL, "fakequant_prune: score");
  SGS_HIP(launch_fakequant_prune(c, params, qstep, score, mask_mode, given_mask, seed, step,
                                 qparams, hard_mask, soft_mask, stats),
          "fakequant_prune");
  return SGS_OK;
}

sgs_status sgs_rate_proxy(sgs_ctx *c, const uint64_t *stats, const float *qstep,
                          float rate_weight, float *out3, float *rate_grad) {
  if (!c) return SGS_EINVAL;
  if (!c->scene_set) return fail(c, SGS_ESTATE, "rate_proxy: set_scene first");
  if (!stats || !qstep || !out3) return fail(c, SGS_EINVAL, "rate_proxy: null pointer");
  SGS_HIP(launch_rate_proxy(c, stats, qstep, rate_weight, out3, rate_grad), "rate_proxy");
  c->lap_ready = false;
  return SGS_OK;
}

// Everything of the forward render after the projection: depth order, pair
// count (a host synchronization unless the pair capacity is fixed), binning
// and the blend.
static sgs_status render_after_projection(sgs_ctx *c, float *image, float *final_T,
                                          uint32_t *last, uint64_t *eval_count) {
  SGS_HIP(launch_depth_order(c), "render_fwd depth order");
  if (!c->fixed_cap) {
    SGS_HIP(hipMemcpyAsync(c->h_pairs_total, c->d_pairs_total, 5 * sizeof(uint32_t),
                           hipMemcpyDeviceToHost, c->stream),
            "render_fwd pair count");
    SGS_HIP(hipStreamSynchronize(c->stream), "render_fwd pair count");
    c->pairs = c->h_pairs_total[0];
    c->items = c->h_pairs_total[4];
    if (c->pairs == (int64_t)kPairsSaturated)
      return fail(c, SGS_ECAPACITY, "render_fwd: 2^32 - 1 or more (tile, Gaussian) pairs");
    hipError_t e = grow_pairs(c, c->pairs);
    if (e != hipSuccess) return hip_fail(c, e, "render_fwd pair buffers");
  }
  SGS_HIP(launch_bin_pairs(c), "render_fwd binning");
  SGS_HIP(launch_blend_fwd(c, image, final_T, last, eval_count), "render_fwd blend");
  c->rendered = true;
  return SGS_OK;
}

sgs_status sgs_render_fwd(sgs_ctx *c, const float *qparams, const uint8_t *hard_mask,
                          float *image, float *final_T, uint32_t *last, uint64_t *eval_count) {
  if (!c) return SGS_EINVAL;
  if (!c->scene_set) return fail(c, SGS_ESTATE, "render_fwd: set_scene first");
  if (!qparams || !hard_mask || !image || !final_T || !last)
    return fail(c, SGS_EINVAL, "render_fwd: null pointer");
  SGS_HIP(launch_preprocess(c, qparams, hard_mask), "render_fwd preprocess");
  return render_after_projection(c, image, final_T, last, eval_count);
}

sgs_status sgs_quant_render_fwd(sgs_ctx *c, const float *params, const float *qstep,
                                const float *score, int32_t mask_mode,
                                const uint8_t *given_mask, uint64_t seed, uint64_t step,
                                uint8_t *hard_mask, float *soft_mask, uint64_t *stats,
                                float *image, float *final_T, uint32_t *last,
                                uint64_t *eval_count) {
  if (!c) return SGS_EINVAL;
  if (!c->scene_set) return fail(c, SGS_ESTATE, "quant_render_fwd: set_scene first");
  if (!params || !qstep || !hard_mask || !stats || !image || !final_T || !last)
    return fail(c, SGS_EINVAL, "quant_render_fwd: null pointer");
  if (!aligned(params, 16))
    return fail(c, SGS_EINVAL, "quant_render_fwd: parameter rows must be 16-byte aligned");
  if (mask_mode < 0 || mask_mode > 2) return fail(c, SGS_EINVAL, "quant_render_fwd: mask_mode");
  if (mask_mode == 0 && !given_mask) return fail(c, SGS_EINVAL, "quant_render_fwd: given_mask");
  if (mask_mode == 1 && !score) return fail(c, SGS_EINVAL, "quant_render_fwd: score");
  SGS_HIP(launch_fakequant_prune(c, params, qstep, score, mask_mode, given_mask, seed, step,
                                 nullptr, hard_mask, soft_mask, stats),
          "quant_render_fwd statistics");
  SGS_HIP(launch_preprocess(c, params, hard_mask, qstep), "quant_render_fwd preprocess");
  return render_after_projection(c, image, final_T, last, eval_count);
}

sgs_status sgs_l1_loss(sgs_ctx *c, const float *image, const float *target, float scale,
                       float *loss, float *dL_dimage) {
  if (!c) return SGS_EINVAL;
  if (!c->scene_set) return fail(c, SGS_ESTATE, "l1_loss: set_scene first");
  if (!image || !target || !loss || !dL_dimage) return fail(c, SGS_EINVAL, "l1_loss: null pointer");
  SGS_HIP(launch_l1(c, image, target, scale, loss, dL_dimage), "l1_loss");
  return SGS_OK;
}

sgs_status sgs_render_bwd(sgs_ctx *c, const float *qparams, const uint8_t *hard_mask,
                          const float *final_T, const uint32_t *last, const float *dL_dimage,
                          float *grad_qparams, float *grad_hard_mask) {
  if (!c) return SGS_EINVAL;
  if (!c->rendered) return fail(c, SGS_ESTATE, "render_bwd: render_fwd first");
  if (!qparams || !hard_mask || !final_T || !last || !dL_dimage || !grad_qparams ||
      !grad_hard_mask)
    return fail(c, SGS_EINVAL, "render_bwd: null pointer");
  (void)hard_mask;  // the mask is held in the splat records of the forward
  SGS_HIP(launch_blend_bwd(c, final_T, last, dL_dimage), "render_bwd blend");
  SGS_HIP(launch_preprocess_bwd(c, qparams, grad_qparams, grad_hard_mask), "render_bwd project");
  return SGS_OK;
}

sgs_status sgs_fakequant_prune_bwd(sgs_ctx *c, const float *params, const float *qstep,
                                   const float *soft_mask, int32_t mask_mode,
                                   const float *rate_grad, const uint64_t *stats,
                                   const float *grad_qparams, const float *grad_hard_mask,
                                   float *grad_params, float *grad_qstep, float *grad_score) {
  if (!c) return SGS_EINVAL;
  if (!c->scene_set) return fail(c, SGS_ESTATE, "fakequant_prune_bwd: set_scene first");
  if (!params || !qstep || !grad_qparams || !grad_hard_mask || !grad_params || !grad_qstep ||
      !grad_score)
    return fail(c, SGS_EINVAL, "fakequant_prune_bwd: null pointer");
  if ((rate_grad == nullptr) != (stats == nullptr))
    return fail(c, SGS_EINVAL, "fakequant_prune_bwd: rate_grad and stats go together");
  if (mask_mode == 1 && !soft_mask)
    return fail(c, SGS_EINVAL, "fakequant_prune_bwd: soft_mask needed in mask mode 1");
  if (mask_mode < 0 || mask_mode > 2) return fail(c, SGS_EINVAL, "fakequant_prune_bwd: mask_mode");
  if (!aligned(params, 16) || !aligned(grad_qparams, 16) || !aligned(grad_params, 16))
    return fail(c, SGS_EINVAL, "fakequant_prune_bwd: parameter rows must be 16-byte aligned");
  SGS_HIP(launch_fakequant_bwd(c, params, qstep, soft_mask, mask_mode, rate_grad, stats,
                               grad_qparams, grad_hard_mask, grad_params, grad_qstep, grad_score),
          "fakequant_prune_bwd");
  return SGS_OK;
}

sgs_status sgs_quant_render_bwd(sgs_ctx *c, const float *params, const float *qstep,
                                const float *soft_mask, int32_t mask_mode,
                                const float *rate_grad, const uint64_t *stats,
                                const float *final_T, const uint32_t *last,
                                const float *dL_dimage, float *grad_params, float *grad_qstep,
                                float *grad_score, float *grad_hard_mask) {
  if (!c) return SGS_EINVAL;
  if (!c->rendered) return fail(c, SGS_ESTATE, "quant_render_bwd: render forward first");
  if (!params || !qstep || !final_T || !last || !dL_dimage || !grad_params || !grad_qstep ||
      !grad_score || !grad_hard_mask)
    return fail(c, SGS_EINVAL, "quant_render_bwd: null pointer");
  if ((rate_grad == nullptr) != (stats == nullptr))
    return fail(c, SGS_EINVAL, "quant_render_bwd: rate_grad and stats go together");
  if (mask_mode < 0 || mask_mode > 2) return fail(c, SGS_EINVAL, "quant_render_bwd: mask_mode");
  if (mask_mode == 1 && !soft_mask)
    return fail(c, SGS_EINVAL, "quant_render_bwd: soft_mask needed in mask mode 1");
  if (params == grad_params)
    return fail(c, SGS_EINVAL, "quant_render_bwd: grad_params must not alias params");
  double *partial = c->red_tmp;
  int64_t nb = 0;
  SGS_HIP(launch_blend_bwd(c, final_T, last, dL_dimage), "quant_render_bwd blend");
  SGS_HIP(launch_preprocess_bwd_fused(c, params, qstep, mask_mode, soft_mask, rate_grad,
                                      grad_params, grad_hard_mask, grad_score, partial, &nb),
          "quant_render_bwd project");
  SGS_HIP(launch_quant_bwd_finish(c, nb, partial, nb, 1, qstep, rate_grad, stats, grad_params,
                                  grad_qstep),
          "quant_render_bwd step sizes");
  return SGS_OK;
}

sgs_status sgs_rate_variant(sgs_ctx *c, const float *params, const float *qstep,
                            const uint64_t *stats, const sgs_rate_options *o, float rate_weight,
                            float *out3, float *rate_grad) {
  if (!c) return SGS_EINVAL;
  if (!c->scene_set) return fail(c, SGS_ESTATE, "rate_variant: set_scene first");
  if (!o || !qstep || !stats || !out3) return fail(c, SGS_EINVAL, "rate_variant: null pointer");
  if ((o->proxy != 0 && o->proxy != 1) || (o->masking != 0 && o->masking != 1) ||
      o->reserved != 0 || !std::isfinite(o->alpha) || !std::isfinite(rate_weight))
    return fail(c, SGS_EINVAL, "rate_variant: proxy and masking 0/1, reserved 0, finite weights");
  if (o->proxy == 1 && !params)
    return fail(c, SGS_EINVAL, "rate_variant: the Laplace proxy reads params");
  SGS_HIP(launch_rate_variant(c, params, qstep, stats, o, rate_weight, out3, rate_grad),
          "rate_variant");
  c->lap_ready = o->proxy == 1;
  return SGS_OK;
}

sgs_status sgs_rate_variant_bwd(sgs_ctx *c, const float *params, float *grad_params) {
  if (!c) return SGS_EINVAL;
  if (!c->scene_set) return fail(c, SGS_ESTATE, "rate_variant_bwd: set_scene first");
  if (!c->lap_ready) return SGS_OK;  // the range proxy's y gradient went through rate_grad
  if (!params || !grad_params) return fail(c, SGS_EINVAL, "rate_variant_bwd: null pointer");
  SGS_HIP(launch_rate_variant_bwd(c, params, grad_params), "rate_variant_bwd");
  return SGS_OK;
}

sgs_status sgs_ssim_loss(sgs_ctx *c, const float *image, const float *target, float weight,
                         float *loss, float *dL_dimage) {
  if (!c) return SGS_EINVAL;
  if (!c->scene_set) return fail(c, SGS_ESTATE, "ssim_loss: set_scene first");
  if (!image || !target || !loss) return fail(c, SGS_EINVAL, "ssim_loss: null pointer");
  if (!(weight >= 0.0f && weight <= 1.0f))
    return fail(c, SGS_EINVAL, "ssim_loss: weight must lie in [0, 1]");
  const int64_t need = ssim_scratch_doubles(c->V, c->W, c->H);
  if (c->ssim_tmp_doubles < need) {
    if (c->capturing)
      return fail(c, SGS_ESTATE, "ssim_loss: first call (it allocates) during graph capture");
    dfree(c->ssim_tmp);
    c->ssim_tmp_doubles = 0;
    hipError_t e = dalloc(&c->ssim_tmp, need);
    if (e != hipSuccess) return hip_fail(c, e, "ssim_loss scratch");
    c->ssim_tmp_doubles = need;
  }
  SGS_HIP(launch_ssim(c, image, target, weight, loss, dL_dimage), "ssim_loss");
  return SGS_OK;
}

sgs_status sgs_compact(sgs_ctx *c, const uint8_t *hard, int32_t narrays, const float *const *src,
                       float *const *dst, const int32_t *rows, int64_t dst_pad, int64_t *kept) {
  if (!c) return SGS_EINVAL;
  if (!c->scene_set) return fail(c, SGS_ESTATE, "compact: set_scene first");
  if (!hard || !src || !dst || !rows || !kept) return fail(c, SGS_EINVAL, "compact: null pointer");
  if (narrays < 1 || narrays > SGS_COMPACT_MAX_ARRAYS || dst_pad < 0)
    return fail(c, SGS_EINVAL, "compact: need 1 <= narrays <= %d and dst_pad >= 0",
                SGS_COMPACT_MAX_ARRAYS);
  if (!aligned(hard, 16)) return fail(c, SGS_EINVAL, "compact: hard_mask must be 16-byte aligned");
  SgsCompactArrays A;
  A.narrays = narrays;
  A.row0[0] = 0;
  for (int a = 0; a < narrays; ++a) {
    if (!src[a] || !dst[a] || rows[a] < 1 || rows[a] > SGS_NCH || !aligned(src[a], 16))
      return fail(c, SGS_EINVAL, "compact: array %d: null or misaligned pointer, or rows "
                                 "outside 1..59", a);
    A.src[a] = src[a];
    A.dst[a] = dst[a];
    A.row0[a + 1] = A.row0[a] + rows[a];
  }
  const int64_t nc = (c->n + 4095) / 4096;
  uint32_t *d_total = c->fl_tmp + 2 * nc;
  SGS_HIP(launch_compact_count(c, hard, d_total), "compact count");
  SGS_HIP(hipMemcpyAsync(c->h_aux, d_total, sizeof(uint32_t), hipMemcpyDeviceToHost, c->stream),
          "compact count");
  SGS_HIP(hipStreamSynchronize(c->stream), "compact count");
  *kept = (int64_t)*c->h_aux;
  if (*kept > dst_pad)
    return fail(c, SGS_ECAPACITY, "compact: dst_pad %lld < kept %lld", (long long)dst_pad,
                (long long)*kept);
  for (int a = 0; a < narrays; ++a) {  // what is written must not overlap what is read
    const char *d0 = (const char *)dst[a];
    const char *d1 = d0 + ((size_t)(rows[a] - 1) * dst_pad + *kept) * 4;
    for (int b = 0; b < narrays; ++b) {
      const char *s0 = (const char *)src[b];
      const char *s1 = s0 + ((size_t)(rows[b] - 1) * c->npad + c->n) * 4;
      if (*kept > 0 && d0 < s1 && s0 < d1)
        return fail(c, SGS_EINVAL, "compact: dst %d overlaps src %d", a, b);
    }
  }
  if (*kept > 0) SGS_HIP(launch_compact_scatter(c, hard, A, dst_pad), "compact scatter");
  return SGS_OK;
}

sgs_status sgs_adam_step(sgs_ctx *c, const sgs_adam_options *o, float *params, float *pm,
                         float *pv, const float *gp, float *q, float *qm, float *qv,
                         const float *gq, float *s, float *sm, float *sv, const float *gs) {
  if (!c) return SGS_EINVAL;
  if (!c->scene_set) return fail(c, SGS_ESTATE, "adam_step: set_scene first");
  if (!o || !params || !pm || !pv || !gp)
    return fail(c, SGS_EINVAL, "adam_step: null options or parameter buffers");
  const bool qa = q || qm || qv || gq, qall = q && qm && qv && gq;
  const bool sa = s || sm || sv || gs, sall = s && sm && sv && gs;
  if ((qa && !qall) || (sa && !sall))
    return fail(c, SGS_EINVAL, "adam_step: give all four buffers of a variable or none");
  if (o->step < 1 || o->reserved != 0 || (o->sh_rest != 0 && o->sh_rest != 1) ||
      (o->sparse != 0 && o->sparse != 1))
    return fail(c, SGS_EINVAL, "adam_step: need step >= 1, sh_rest and sparse 0/1, reserved 0");
  if (!(o->beta1 >= 0.5f && o->beta1 < 1.0f) || !(o->beta2 >= 0.5f && o->beta2 < 1.0f) ||
      !(o->eps >= 0.0f) || !std::isfinite(o->eps))
    return fail(c, SGS_EINVAL, "adam_step: need beta1, beta2 in [0.5, 1), eps >= 0 finite");
  if (!aligned(params, 16) || !aligned(pm, 16) || !aligned(pv, 16) || !aligned(gp, 16))
    return fail(c, SGS_EINVAL, "adam_step: parameter rows must be 16-byte aligned");
  SGS_HIP(launch_adam(c, o, params, pm, pv, gp, q, qm, qv, gq, s, sm, sv, gs), "adam_step");
  return SGS_OK;
}

sgs_status sgs_fl_encode(sgs_ctx *c, const float *params, const float *qstep,
                         const uint8_t *hard_mask, sgs_fl_channel *header, uint32_t *payload,
                         int64_t payload_words, int64_t *info) {
  if (!c) return SGS_EINVAL;
  if (!c->scene_set) return fail(c, SGS_ESTATE, "fl_encode: set_scene first");
  if (!params || !qstep || !hard_mask || !header || !info || (payload_words > 0 && !payload))
    return fail(c, SGS_EINVAL, "fl_encode: null pointer");
  if (payload_words < 0) return fail(c, SGS_EINVAL, "fl_encode: payload_words < 0");
  if (!aligned(params, 16) || !aligned(hard_mask, 16) || !aligned(info, 8))
    return fail(c, SGS_EINVAL,
                "fl_encode: params and hard_mask must be 16-byte and info 8-byte aligned");
  SGS_HIP(launch_fl_encode(c, params, qstep, hard_mask, header, payload, payload_words, info),
          "fl_encode");
  return SGS_OK;
}

sgs_status sgs_fl_decode(sgs_ctx *c, const sgs_fl_channel *header, const uint32_t *payload,
                         int64_t payload_words, int64_t kept, int64_t out_pad, float *out) {
  if (!c) return SGS_EINVAL;
  if (!header || !out || (payload_words > 0 && !payload))
    return fail(c, SGS_EINVAL, "fl_decode: null pointer");
  if (kept < 0 || out_pad < kept || payload_words < 0)
    return fail(c, SGS_EINVAL, "fl_decode: need 0 <= kept <= out_pad, payload_words >= 0");
  if (kept > (int64_t)INT32_MAX * 4096LL)
    return fail(c, SGS_ECAPACITY, "fl_decode: kept too large");
  SGS_HIP(launch_fl_decode(c, header, payload, payload_words, kept, out_pad, out), "fl_decode");
  return SGS_OK;
}

// ---- learned-coding stage --------------------------------------------------
sgs_status sgs_octree_encode(sgs_ctx *c, const float *params, int64_t npad, int64_t n,
                             const float *qstep, const uint8_t *hard_mask, uint8_t *tokens,
                             int64_t token_cap, uint64_t *codes, uint32_t *dup_index,
                             uint32_t *dup_count, int64_t dup_cap, sgs_octree_header *header) {
  if (!c) return SGS_EINVAL;
  if (c->capturing) return fail(c, SGS_ESTATE, "octree_encode: not inside graph capture");
  if (!params || !qstep || !hard_mask || !tokens || !codes || !header ||
      (dup_cap > 0 && (!dup_index || !dup_count)))
    return fail(c, SGS_EINVAL, "octree_encode: null pointer");
  if (n < 1 || npad < n || n > (int64_t)INT32_MAX)
    return fail(c, SGS_EINVAL, "octree_encode: need 1 <= n <= npad, n < 2^31");
  if (token_cap < 0 || token_cap % 4 != 0 || !aligned(tokens, 4) || dup_cap < 0)
    return fail(c, SGS_EINVAL,
                "octree_encode: token_cap must be a multiple of 4, tokens 4-byte aligned, "
                "dup_cap >= 0");
  SgsProfScope ps(c, SGS_PROF_OCTREE);
  SGS_HIP(launch_octree_encode(c, params, npad, n, qstep, hard_mask, tokens, token_cap, codes,
                               dup_index, dup_count, dup_cap, header),
          "octree_encode");
  return SGS_OK;
}

sgs_status sgs_octree_decode(sgs_ctx *c, const sgs_octree_header *h, const uint8_t *tokens,
                             const uint32_t *dup_index, const uint32_t *dup_count,
                             const float *qstep, uint64_t *codes, float *xyz, int64_t out_pad,
                             int64_t *info) {
  if (!c) return SGS_EINVAL;
  if (c->capturing) return fail(c, SGS_ESTATE, "octree_decode: not inside graph capture");
  if (!h || !qstep || !info || (h->tokens > 0 && (!tokens || !codes || !xyz)) ||
      (h->dups > 0 && (!dup_index || !dup_count)))
    return fail(c, SGS_EINVAL, "octree_decode: null pointer");
  if (h->depth < 1 || h->depth > 21 || h->flags != 0 || h->kept < 0 || h->unique < 0 ||
      h->dups < 0 || h->tokens < 0 || h->kept > (int64_t)INT32_MAX ||
      h->tokens > (int64_t)INT32_MAX)
    return fail(c, SGS_EINVAL, "octree_decode: bad header");
  int64_t sum = 0;
  for (int d = 0; d < 21; ++d) {
    const int64_t v = h->level_size[d];
    if (v < 0 || (d >= h->depth && v != 0)) return fail(c, SGS_EINVAL, "octree_decode: bad level sizes");
    if (d > 0 && d < h->depth && v > 8 * h->level_size[d - 1])
      return fail(c, SGS_EINVAL, "octree_decode: bad level sizes");
    sum += v;
  }
  const bool empty = h->kept == 0;
  if (sum != h->tokens || (empty ? (h->tokens != 0 || h->unique != 0 || h->dups != 0)
                                 : (h->level_size[0] != 1 ||
                                    h->unique > 8 * h->level_size[h->depth - 1] ||
                                    h->unique > h->kept || h->dups > h->unique)))
    return fail(c, SGS_EINVAL, "octree_decode: inconsistent header");
  if (out_pad < h->kept) return fail(c, SGS_EINVAL, "octree_decode: out_pad < kept");
  SgsProfScope ps(c, SGS_PROF_OCTREE);
  SGS_HIP(launch_octree_decode(c, h, tokens, dup_index, dup_count, qstep, codes, xyz, out_pad,
                               info),
          "octree_decode");
  return SGS_OK;
}

static sgs_status ans_args(sgs_ctx *c, const char *who, int64_t n, int32_t order,
                           int32_t lane_len) {
  if (c->capturing) return fail(c, SGS_ESTATE, "%s: not inside graph capture", who);
  if (n < 0 || n > (int64_t)INT32_MAX) return fail(c, SGS_EINVAL, "%s: need 0 <= n < 2^31", who);
  if (order != 0 && order != 1) return fail(c, SGS_EINVAL, "%s: order must be 0 or 1", who);
  if (lane_len < 1 || lane_len > 65536)
    return fail(c, SGS_EINVAL, "%s: lane_len must be in [1, 65536]", who);
  return SGS_OK;
}

sgs_status sgs_ans_model(sgs_ctx *c, const uint8_t *sym, int64_t n, int32_t order,
                         int32_t lane_len, uint16_t *freq, double *ideal_bits) {
  if (!c) return SGS_EINVAL;
  sgs_status r = ans_args(c, "ans_model", n, order, lane_len);
  if (r != SGS_OK) return r;
  if (!freq || (n > 0 && !sym)) return fail(c, SGS_EINVAL, "ans_model: null pointer");
  SgsProfScope ps(c, SGS_PROF_ANS);
  SGS_HIP(launch_ans_model(c, sym, n, order, lane_len, freq, ideal_bits), "ans_model");
  return SGS_OK;
}

sgs_status sgs_ans_encode(sgs_ctx *c, const uint8_t *sym, int64_t n, int32_t order,
                          int32_t lane_len, const uint16_t *freq, uint16_t *words,
                          int64_t word_cap, int64_t *block_off, int64_t *info) {
  if (!c) return SGS_EINVAL;
  sgs_status r = ans_args(c, "ans_encode", n, order, lane_len);
  if (r != SGS_OK) return r;
  if (!freq || !block_off || !info || (n > 0 && (!sym || !words)))
    return fail(c, SGS_EINVAL, "ans_encode: null pointer");
  if (word_cap < 0) return fail(c, SGS_EINVAL, "ans_encode: word_cap < 0");
  SgsProfScope ps(c, SGS_PROF_ANS);
  SGS_HIP(launch_ans_encode(c, sym, n, order, lane_len, freq, words, word_cap, block_off, info),
          "ans_encode");
  return SGS_OK;
}

sgs_status sgs_ans_decode(sgs_ctx *c, const uint16_t *words, int64_t n_words,
                          const int64_t *block_off, int64_t n, int32_t order, int32_t lane_len,
                          const uint16_t *freq, uint8_t *sym, int64_t *info) {
  if (!c) return SGS_EINVAL;
  sgs_status r = ans_args(c, "ans_decode", n, order, lane_len);
  if (r != SGS_OK) return r;
  if (!freq || !block_off || !info || (n > 0 && (!sym || !words)))
    return fail(c, SGS_EINVAL, "ans_decode: null pointer");
  if (n_words < 0) return fail(c, SGS_EINVAL, "ans_decode: n_words < 0");
  SgsProfScope ps(c, SGS_PROF_ANS);
  SGS_HIP(launch_ans_decode(c, words, n_words, block_off, n, order, lane_len, freq, sym, info),
          "ans_decode");
  return SGS_OK;
}

sgs_status sgs_ans_decode_multi(sgs_ctx *c, int32_t count, const sgs_ans_stream *st,
                                int64_t *info) {
  if (!c) return SGS_EINVAL;
  if (count < 0 || count > 65535) return fail(c, SGS_EINVAL, "ans_decode_multi: bad count");
  if (count > 0 && (!st || !info)) return fail(c, SGS_EINVAL, "ans_decode_multi: null pointer");
  for (int32_t i = 0; i < count; ++i) {
    sgs_status r = ans_args(c, "ans_decode_multi", st[i].n, st[i].order, st[i].lane_len);
    if (r != SGS_OK) return r;
    if (!st[i].freq || !st[i].block_off || (st[i].n > 0 && (!st[i].sym || !st[i].words)) ||
        st[i].n_words < 0)
      return fail(c, SGS_EINVAL, "ans_decode_multi: stream %d: bad descriptor", (int)i);
  }
  if (count == 0) return SGS_OK;
  SgsProfScope ps(c, SGS_PROF_ANS);
  SGS_HIP(launch_ans_decode_multi(c, count, st, info), "ans_decode_multi");
  return SGS_OK;
}

sgs_status sgs_morton_order(sgs_ctx *c, const float *params, int64_t npad, int64_t n,
                            const float *qstep, const uint8_t *hard_mask,
                            const sgs_octree_header *h, const uint64_t *codes, int32_t *perm) {
  if (!c) return SGS_EINVAL;
  if (c->capturing) return fail(c, SGS_ESTATE, "morton_order: not inside graph capture");
  if (!params || !qstep || !hard_mask || !h || (h->kept > 0 && (!codes || !perm)))
    return fail(c, SGS_EINVAL, "morton_order: null pointer");
  if (n < 1 || npad < n || n > (int64_t)INT32_MAX)
    return fail(c, SGS_EINVAL, "morton_order: need 1 <= n <= npad, n < 2^31");
  if (h->depth < 1 || h->depth > 21 || h->flags != 0 || h->kept < 0 || h->kept > n ||
      h->unique < 0 || h->unique > h->kept)
    return fail(c, SGS_EINVAL, "morton_order: bad header");
  SgsProfScope ps(c, SGS_PROF_OCTREE);
  SGS_HIP(launch_morton_order(c, params, npad, n, qstep, hard_mask, h, codes, perm),
          "morton_order");
  return SGS_OK;
}

static bool fl_header_ok(const sgs_fl_channel *fl) {
  for (int j = 0; j < 59; ++j)
    if (fl[j].width < 0 || fl[j].width > 32) return false;
  return true;
}

int64_t sgs_attr_plane_rows(const sgs_fl_channel *fl, const uint8_t *predictor) {
  if (!fl || !fl_header_ok(fl)) return -1;
  return attr_plane_rows(fl, predictor);
}

sgs_status sgs_attr_planes(sgs_ctx *c, const float *params, int64_t npad, const int32_t *perm,
                           int64_t kept, const sgs_fl_channel *fl, const uint8_t *predictor,
                           int32_t lane_len, uint8_t *planes) {
  if (!c) return SGS_EINVAL;
  if (!params || !fl || (kept > 0 && (!perm || !planes)))
    return fail(c, SGS_EINVAL, "attr_planes: null pointer");
  if (kept < 0 || kept > npad || kept > (int64_t)INT32_MAX || lane_len < 1 || lane_len > 65536 ||
      !fl_header_ok(fl))
    return fail(c, SGS_EINVAL, "attr_planes: bad sizes or header");
  SgsProfScope ps(c, SGS_PROF_ANS);
  SGS_HIP(launch_attr_planes(c, params, npad, perm, kept, fl, predictor, lane_len, planes),
          "attr_planes");
  return SGS_OK;
}

sgs_status sgs_attr_reconstruct(sgs_ctx *c, const uint8_t *planes, int64_t kept,
                                const sgs_fl_channel *fl, const uint8_t *predictor,
                                int32_t lane_len, float *out, int64_t out_pad) {
  if (!c) return SGS_EINVAL;
  if (!fl || (kept > 0 && !out) || (kept > 0 && attr_plane_rows(fl, predictor) > 0 && !planes))
    return fail(c, SGS_EINVAL, "attr_reconstruct: null pointer");
  if (kept < 0 || out_pad < kept || kept > (int64_t)INT32_MAX || lane_len < 1 ||
      lane_len > 65536 || !fl_header_ok(fl))
    return fail(c, SGS_EINVAL, "attr_reconstruct: bad sizes or header");
  SgsProfScope ps(c, SGS_PROF_ANS);
  SGS_HIP(launch_attr_reconstruct(c, planes, kept, fl, predictor, lane_len, out, out_pad),
          "attr_reconstruct");
  return SGS_OK;
}

sgs_status sgs_positional_embedding(sgs_ctx *c, const float *xyz, int64_t pad, int64_t count,
                                    int32_t L, int32_t d, const float *W, const float *b,
                                    float *out) {
  if (!c) return SGS_EINVAL;
  if (count > 0 && (!xyz || !W || !b || !out))
    return fail(c, SGS_EINVAL, "positional_embedding: null pointer");
  if (count < 0 || pad < count || L < 1 || L > 16 || d < 4 || d > 64 || d % 4 != 0 ||
      !aligned(out, 16))
    return fail(c, SGS_EINVAL,
                "positional_embedding: need 0 <= count <= pad, 1 <= L <= 16, d in {4, 8, .., 64}, "
                "out 16-byte aligned");
  SgsProfScope ps(c, SGS_PROF_ANS);
  SGS_HIP(launch_pos_embed(c, xyz, pad, count, L, d, W, b, out), "positional_embedding");
  return SGS_OK;
}

sgs_status sgs_autotune(sgs_ctx *c, const float *params, const float *qstep,
                        const uint8_t *given_mask, const float *target, int32_t reps,
                        sgs_options *chosen, float *ms_out) {
  if (!c) return SGS_EINVAL;
  if (!c->scene_set) return fail(c, SGS_ESTATE, "autotune: set_scene first");
  if (c->capturing) return fail(c, SGS_ESTATE, "autotune: not inside graph capture");
  if (!params || !qstep || !given_mask || !target || !chosen)
    return fail(c, SGS_EINVAL, "autotune: null pointer");
  if (reps < 1 || reps > 1000) return fail(c, SGS_EINVAL, "autotune: reps must be in [1, 1000]");
  if (!aligned(params, 16)) return fail(c, SGS_EINVAL, "autotune: parameter rows must be 16-byte aligned");
  SGS_HIP(hipSetDevice(c->device), "hipSetDevice");
  // the scene to re-bind for every candidate
  const int64_t n = c->n, npad = c->npad, n_hat = c->n_hat;
  const int V = c->V, W = c->W, H = c->H;
  const float tau = c->tau;
  const int det = c->deterministic ? 1 : 0;
  const std::vector<sgs_camera> cams = c->h_cams;
  const int64_t pix = (int64_t)V * W * H;
  // the step's outputs, in one temporary allocation
  const int64_t words[] = {(n + 3) / 4, n, 2 * SGS_STATS_WORDS, 3 * pix, pix, pix, 3 * pix,
                           SGS_NCH * npad, 64, n, n, 4, 4, SGS_RATE_GRAD_FLOATS};
  int64_t off[15] = {0};
  for (int k = 0; k < 14; ++k) off[k + 1] = off[k] + (words[k] + 63) / 64 * 64;
  float *buf = nullptr;
  hipError_t e = dalloc(&buf, off[14]);
  if (e != hipSuccess) return hip_fail(c, e, "autotune buffers");
  auto at = [&](int k) { return buf + off[k]; };
  uint8_t *hard = (uint8_t *)at(0);
  float *soft = at(1);
  uint64_t *stats = (uint64_t *)at(2);
  float *image = at(3), *fT = at(4);
  uint32_t *last = (uint32_t *)at(5);
  float *dimage = at(6), *gp = at(7), *gq = at(8), *gs = at(9), *gm = at(10);
  float *loss = at(11), *rate3 = at(12), *rgrad = at(13);
  struct Cand { int tw, th, sched; };
  constexpr int kShapes = 5;
  const Cand tiles[kShapes] = {{16, 16, 0}, {8, 8, 0}, {32, 8, 0}, {32, 16, 0}, {32, 32, 0}};
  float times[kShapes + 3] = {0};
  int ntimed = 0;
  hipEvent_t ea = nullptr, eb = nullptr;
  sgs_status st = SGS_OK;
  auto run = [&](const Cand &cd, float *ms) -> sgs_status {
    sgs_options o{};
    o.tile_w = cd.tw;
    o.tile_h = cd.th;
    o.tau = tau;
    o.schedule = cd.sched;
    o.deterministic = det;
    sgs_status r = sgs_set_scene(c, n, npad, n_hat, cams.data(), V, W, H, &o);
    if (r != SGS_OK) return r;
    auto step = [&]() -> sgs_status {
      sgs_status q = sgs_quant_render_fwd(c, params, qstep, nullptr, 0, given_mask, 0, 0, hard,
                                          soft, stats, image, fT, last, nullptr);
      if (q == SGS_OK) q = sgs_rate_proxy(c, stats, qstep, 0.0f, rate3, rgrad);
      if (q == SGS_OK) q = sgs_l1_loss(c, image, target, 1.0f, loss, dimage);
      if (q == SGS_OK)
        q = sgs_quant_render_bwd(c, params, qstep, soft, 0, rgrad, stats, fT, last, dimage, gp,
                                 gq, gs, gm);
      return q;
    };
    r = step();  // sizes the pair buffers
    if (r != SGS_OK) return r;
    if (hipEventRecord(ea, c->stream) != hipSuccess) return fail(c, SGS_EHIP, "autotune event");
    for (int k = 0; k < reps && r == SGS_OK; ++k) r = step();
    if (r != SGS_OK) return r;
    if (hipEventRecord(eb, c->stream) != hipSuccess || hipEventSynchronize(eb) != hipSuccess ||
        hipEventElapsedTime(ms, ea, eb) != hipSuccess)
      return fail(c, SGS_EHIP, "autotune timing");
    *ms /= (float)reps;
    return SGS_OK;
  };
  Cand best = tiles[0];
  float best_ms = 0.0f;
  if (hipEventCreate(&ea) != hipSuccess || hipEventCreate(&eb) != hipSuccess) {
    st = fail(c, SGS_EHIP, "autotune events");
  }
  for (int k = 0; k < kShapes && st == SGS_OK; ++k) {
    st = run(tiles[k], &times[ntimed]);
    if (st == SGS_OK && (ntimed == 0 || times[ntimed] < best_ms)) {
      best = tiles[k];
      best_ms = times[ntimed];
    }
    ++ntimed;
  }
  const Cand shape = best;
  for (int sched = 1; sched <= 3 && st == SGS_OK; ++sched) {
    const Cand cd = {shape.tw, shape.th, sched};
    st = run(cd, &times[ntimed]);
    if (st == SGS_OK && times[ntimed] < best_ms) {
      best = cd;
      best_ms = times[ntimed];
    }
    ++ntimed;
  }
  if (ea) (void)hipEventDestroy(ea);
  if (eb) (void)hipEventDestroy(eb);
  (void)hipStreamSynchronize(c->stream);
  dfree(buf);
  // leave the scene bound with the choice (or, after a failure, as it was)
  sgs_options o{};
  o.tile_w = best.tw;
  o.tile_h = best.th;
  o.tau = tau;
  o.schedule = best.sched;
  o.deterministic = det;
  char keep_err[sizeof(c->err)];
  memcpy(keep_err, c->err, sizeof(keep_err));
  const sgs_status rb = sgs_set_scene(c, n, npad, n_hat, cams.data(), V, W, H, &o);
  if (st != SGS_OK) {
    memcpy(c->err, keep_err, sizeof(keep_err));
    return st;
  }
  if (rb != SGS_OK) return rb;
  *chosen = o;
  if (ms_out)
    for (int k = 0; k < kShapes + 3; ++k) ms_out[k] = times[k];
  return SGS_OK;
}

sgs_status sgs_query_items(sgs_ctx *c, int64_t *items) {
  if (!c || !items) return SGS_EINVAL;
  SGS_HIP(hipSetDevice(c->device), "hipSetDevice");
  SGS_HIP(hipStreamSynchronize(c->stream), "query sync");
  if (c->fixed_cap && c->d_pairs_total) {
    uint32_t v = 0;
    SGS_HIP(hipMemcpy(&v, c->d_pairs_total + 4, sizeof(v), hipMemcpyDeviceToHost), "query items");
    *items = v;
  } else {
    *items = c->items;
  }
  return SGS_OK;
}

sgs_status sgs_set_eval_count_mode(sgs_ctx *c, int32_t mode) {
  if (!c) return SGS_EINVAL;
  if (mode != 0 && mode != 1) return fail(c, SGS_EINVAL, "set_eval_count_mode: mode must be 0 or 1");
  c->count_mode = mode;
  return SGS_OK;
}

sgs_status sgs_set_grad_sh_rest(sgs_ctx *c, int32_t on) {
  if (!c) return SGS_EINVAL;
  if (on != 0 && on != 1) return fail(c, SGS_EINVAL, "set_grad_sh_rest: on must be 0 or 1");
  c->grad_sh_rest = on != 0;
  return SGS_OK;
}

sgs_status sgs_query(sgs_ctx *c, const uint64_t *stats, int64_t *pairs_last, uint64_t *flags) {
  if (!c) return SGS_EINVAL;
  SGS_HIP(hipSetDevice(c->device), "hipSetDevice");
  SGS_HIP(hipStreamSynchronize(c->stream), "query sync");
  bool overflow = false;
  if (c->fixed_cap && c->d_pairs_total) {
    uint32_t counts[3];
    SGS_HIP(hipMemcpy(counts, c->d_pairs_total, sizeof(counts), hipMemcpyDeviceToHost),
            "query counts");
    c->pairs = counts[1];
    overflow = counts[2] != 0;
    if (pairs_last) *pairs_last = counts[0];
    if (overflow) {
      const uint32_t zero = 0;
      SGS_HIP(hipMemcpy(c->d_pairs_total + 2, &zero, sizeof(zero), hipMemcpyHostToDevice),
              "query clear");
    }
  } else if (pairs_last) {
    *pairs_last = c->pairs;
  }
  if (flags) {
    *flags = 0;
    if (stats)
      SGS_HIP(hipMemcpy(flags, stats + 119, sizeof(uint64_t), hipMemcpyDeviceToHost), "query flags");
  }
  if (c->deterministic && c->d_pairs_total) {
    uint32_t dflag = 0;
    SGS_HIP(hipMemcpy(&dflag, c->d_pairs_total + 3, sizeof(dflag), hipMemcpyDeviceToHost),
            "query deterministic flag");
    if (dflag) {
      const uint32_t zero = 0;
      SGS_HIP(hipMemcpy(c->d_pairs_total + 3, &zero, sizeof(zero), hipMemcpyHostToDevice),
              "query clear");
      return fail(c, SGS_ECAPACITY,
                  "deterministic gradient sums: a per-wave term of magnitude >= 2^31 or not "
                  "finite was left out (scale the loss down or use the atomic mode)");
    }
  }
  if (flags && (*flags & 1ull)) return fail(c, SGS_EINVAL, "a step size q_j was <= 0 or not finite");
  if (overflow)
    return fail(c, SGS_ECAPACITY, "pair capacity %lld exceeded (%lld pairs): reserve more and rerun",
                (long long)c->cap_limit, (long long)(pairs_last ? *pairs_last : 0));
  return SGS_OK;
}

sgs_status sgs_reserve_pairs(sgs_ctx *c, int64_t capacity) {
  if (!c) return SGS_EINVAL;
  if (!c->scene_set) return fail(c, SGS_ESTATE, "reserve_pairs: set_scene first");
  if (capacity < 0 || capacity >= ((int64_t)1 << 32) - 1)
    return fail(c, SGS_EINVAL, "reserve_pairs: capacity out of range");
  if (c->capturing) return fail(c, SGS_ESTATE, "reserve_pairs: not during graph capture");
  SGS_HIP(hipSetDevice(c->device), "hipSetDevice");
  SGS_HIP(hipStreamSynchronize(c->stream), "reserve sync");
  if (capacity == 0) {
    c->fixed_cap = false;
    return SGS_OK;
  }
  hipError_t e = grow_pairs(c, capacity);
  if (e != hipSuccess) return hip_fail(c, e, "reserve_pairs");
  SGS_HIP(hipMemset(c->d_pairs_total, 0, 4 * sizeof(uint32_t)), "reserve clear");
  c->cap_limit = capacity;
  c->fixed_cap = true;
  return SGS_OK;
}

struct sgs_graph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

sgs_status sgs_graph_begin(sgs_ctx *c) {
  if (!c) return SGS_EINVAL;
  if (!c->fixed_cap) return fail(c, SGS_ESTATE, "graph_begin: reserve a pair capacity first");
  if (!c->stream) return fail(c, SGS_ESTATE, "graph_begin: the null stream cannot be captured");
  if (c->capturing) return fail(c, SGS_ESTATE, "graph_begin: already capturing");
  SGS_HIP(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal), "graph_begin");
  c->capturing = true;
  return SGS_OK;
}

sgs_status sgs_graph_end(sgs_ctx *c, sgs_graph **out) {
  if (!c || !out) return SGS_EINVAL;
  *out = nullptr;
  if (!c->capturing) return fail(c, SGS_ESTATE, "graph_end: not capturing");
  c->capturing = false;
  sgs_graph *g = new (std::nothrow) sgs_graph();
  if (!g) return SGS_ENOMEM;
  hipError_t e = hipStreamEndCapture(c->stream, &g->graph);
  if (e != hipSuccess) {
    delete g;
    return hip_fail(c, e, "graph_end capture");
  }
  e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(g->graph);
    delete g;
    return hip_fail(c, e, "graph_end instantiate");
  }
  *out = g;
  return SGS_OK;
}

sgs_status sgs_graph_launch(sgs_graph *g, void *hip_stream) {
  if (!g || !g->exec) return SGS_EINVAL;
  return hipGraphLaunch(g->exec, (hipStream_t)hip_stream) == hipSuccess ? SGS_OK : SGS_EHIP;
}

void sgs_graph_destroy(sgs_graph *g) {
  if (!g) return;
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  delete g;
}

sgs_status sgs_rate_mlp_pack(sgs_ctx *c, const float *theta, void *packed) {
  if (!c) return SGS_EINVAL;
  if (!theta || !packed || !aligned(packed, 16))
    return fail(c, SGS_EINVAL, "rate_mlp_pack: null or misaligned pointer");
  SGS_HIP(launch_mlp_pack(c, theta, packed), "rate_mlp_pack");
  return SGS_OK;
}

sgs_status sgs_rate_mlp_fwd(sgs_ctx *c, const void *packed, const float *theta,
                            const float *params, const float *qstep, const uint64_t *stats,
                            const uint8_t *hard_mask, float *out_R, float *per_gaussian) {
  if (!c) return SGS_EINVAL;
  if (!c->scene_set) return fail(c, SGS_ESTATE, "rate_mlp_fwd: set_scene first");
  if (!packed || !theta || !params || !qstep || !stats || !hard_mask || !out_R)
    return fail(c, SGS_EINVAL, "rate_mlp_fwd: null pointer");
  if (!aligned(packed, 16)) return fail(c, SGS_EINVAL, "rate_mlp_fwd: packed must be 16-byte aligned");
  SGS_HIP(launch_mlp_rate_fwd(c, packed, theta, params, qstep, stats, hard_mask, out_R,
                              per_gaussian),
          "rate_mlp_fwd");
  c->mlp_saved = true;
  return SGS_OK;
}

sgs_status sgs_rate_mlp_bwd(sgs_ctx *c, const void *packed, const float *theta,
                            const float *params, const float *qstep, const uint64_t *stats,
                            const uint8_t *hard_mask, const float *soft_mask, int32_t mask_mode,
                            float rate_weight, float *grad_params, float *grad_qstep,
                            float *grad_score, float *grad_hard_mask) {
  if (!c) return SGS_EINVAL;
  if (!c->scene_set) return fail(c, SGS_ESTATE, "rate_mlp_bwd: set_scene first");
  if (!packed || !theta || !params || !qstep || !stats || !hard_mask || !grad_params ||
      !grad_qstep)
    return fail(c, SGS_EINVAL, "rate_mlp_bwd: null pointer");
  if (mask_mode < 0 || mask_mode > 2) return fail(c, SGS_EINVAL, "rate_mlp_bwd: mask_mode");
  if (mask_mode == 1 && grad_score && !soft_mask)
    return fail(c, SGS_EINVAL, "rate_mlp_bwd: soft_mask needed for the score gradient");
  if (!aligned(packed, 16)) return fail(c, SGS_EINVAL, "rate_mlp_bwd: packed must be 16-byte aligned");
  if (!c->mlp_saved) return fail(c, SGS_ESTATE, "rate_mlp_bwd: rate_mlp_fwd first");
  SGS_HIP(launch_mlp_rate_bwd(c, packed, theta, params, qstep, stats, hard_mask, soft_mask,
                              mask_mode, rate_weight, grad_params, grad_qstep,
                              mask_mode == 1 ? grad_score : nullptr, grad_hard_mask),
          "rate_mlp_bwd");
  return SGS_OK;
}

sgs_status sgs_rate_mlp_features(sgs_ctx *c, const float *params, const float *qstep,
                                 const uint64_t *stats, const int32_t *idx, int64_t rows,
                                 uint16_t *X) {
  if (!c) return SGS_EINVAL;
  if (!c->scene_set) return fail(c, SGS_ESTATE, "rate_mlp_features: set_scene first");
  if (!params || !qstep || !stats || !idx || !X || rows < 0)
    return fail(c, SGS_EINVAL, "rate_mlp_features: null pointer or rows < 0");
  if (rows > ((int64_t)1 << 40)) return fail(c, SGS_ECAPACITY, "rate_mlp_features: rows");
  if (!aligned(X, 8)) return fail(c, SGS_EINVAL, "rate_mlp_features: X must be 8-byte aligned");
  SGS_HIP(launch_mlp_features(c, params, qstep, stats, idx, rows, X), "rate_mlp_features");
  return SGS_OK;
}

sgs_status sgs_rate_mlp_infer(sgs_ctx *c, const void *packed, const float *theta,
                              const uint16_t *X, int64_t rows, float *out) {
  if (!c) return SGS_EINVAL;
  if (!packed || !theta || !X || !out || rows < 1)
    return fail(c, SGS_EINVAL, "rate_mlp_infer: null pointer or rows < 1");
  if (!aligned(X, 8) || !aligned(packed, 16))
    return fail(c, SGS_EINVAL, "rate_mlp_infer: misaligned pointer");
  SGS_HIP(launch_mlp_infer(c, packed, theta, X, rows, out), "rate_mlp_infer");
  return SGS_OK;
}

int64_t sgs_rate_mlp_train_scratch_bytes(int64_t rows) {
  return rows < 1 ? 0 : mlp_train_scratch_bytes(rows);
}

sgs_status sgs_rate_mlp_train_step(sgs_ctx *c, float *theta, float *adam_m, float *adam_v,
                                   void *packed, const uint16_t *X, const float *target,
                                   int64_t rows, float lr, int64_t step, float *loss,
                                   float *grad_theta, void *scratch) {
  if (!c) return SGS_EINVAL;
  if (!theta || !packed || !X || !target || !loss || !grad_theta || !scratch)
    return fail(c, SGS_EINVAL, "rate_mlp_train_step: null pointer");
  if (rows < 8 || rows % 8 != 0 || rows > ((int64_t)1 << 26))
    return fail(c, SGS_EINVAL, "rate_mlp_train_step: rows must be a multiple of 8 in [8, 2^26]");
  if (lr > 0.0f && (!adam_m || !adam_v || step < 1))
    return fail(c, SGS_EINVAL, "rate_mlp_train_step: Adam needs moments and step >= 1");
  if (!aligned(X, 8) || !aligned(packed, 16) || !aligned(scratch, 256))
    return fail(c, SGS_EINVAL, "rate_mlp_train_step: misaligned pointer");
  SGS_HIP(launch_mlp_train_step(c, theta, adam_m, adam_v, packed, X, target, rows, lr, step, loss,
                                grad_theta, scratch),
          "rate_mlp_train_step");
  return SGS_OK;
}

sgs_status sgs_rate_mlp_train_step_static(sgs_ctx *c, float *theta, float *adam_m,
                                          float *adam_v, void *packed, const uint16_t *X,
                                          const float *target, int64_t rows, float lr,
                                          int64_t step, float *loss, float *grad_theta) {
  if (!c) return SGS_EINVAL;
  if (!theta || !packed || !X || !target || !loss || !grad_theta)
    return fail(c, SGS_EINVAL, "rate_mlp_train_step_static: null pointer");
  if (rows > SGS_MLP_STATIC_ROWS)
    return fail(c, SGS_ECAPACITY,
                "rate_mlp_train_step_static: %lld rows exceed the static workspace's %d",
                (long long)rows, SGS_MLP_STATIC_ROWS);
  if (rows < 8 || rows % 8 != 0)
    return fail(c, SGS_EINVAL, "rate_mlp_train_step_static: rows must be a multiple of 8");
  if (lr > 0.0f && (!adam_m || !adam_v || step < 1))
    return fail(c, SGS_EINVAL, "rate_mlp_train_step_static: Adam needs moments and step >= 1");
  if (!aligned(X, 8) || !aligned(packed, 16))
    return fail(c, SGS_EINVAL, "rate_mlp_train_step_static: misaligned pointer");
  if (mlp_train_scratch_bytes(rows) > mlp_static_scratch_bytes())
    return fail(c, SGS_ECAPACITY, "rate_mlp_train_step_static: workspace too small");
  // the device address resolved at sgs_create for this context's device
  hipError_t se = hipSuccess;
  void *ws = mlp_static_scratch(c->device, &se);
  if (!ws) return hip_fail(c, se, "rate_mlp_train_step_static: static workspace");
  SGS_HIP(launch_mlp_train_step(c, theta, adam_m, adam_v, packed, X, target, rows, lr, step,
                                loss, grad_theta, ws, false),
          "rate_mlp_train_step_static");
  return SGS_OK;
}

sgs_status sgs_profile_enable(sgs_ctx *c, int32_t enable) {
  if (!c) return SGS_EINVAL;
  SGS_HIP(hipStreamSynchronize(c->stream), "profile sync");
  for (auto &r : c->prof_recs) {
    c->ev_free.push_back(r.a);
    c->ev_free.push_back(r.b);
  }
  c->prof_recs.clear();
  c->prof = enable != 0;
  return SGS_OK;
}

sgs_status sgs_profile_read(sgs_ctx *c, double *ms_total, int64_t *launches) {
  if (!c || !ms_total || !launches) return SGS_EINVAL;
  SGS_HIP(hipStreamSynchronize(c->stream), "profile sync");
  for (int g = 0; g < SGS_PROF_GROUPS; ++g) {
    ms_total[g] = 0.0;
    launches[g] = 0;
  }
  for (auto &r : c->prof_recs) {
    float ms = 0.0f;
    SGS_HIP(hipEventElapsedTime(&ms, r.a, r.b), "profile elapsed");
    ms_total[r.group] += ms;
    launches[r.group] += 1;
    c->ev_free.push_back(r.a);
    c->ev_free.push_back(r.b);
  }
  c->prof_recs.clear();
  return SGS_OK;
}

sgs_status sgs_copy_structure(sgs_ctx *c, uint32_t *tile_ids, uint32_t *vals, int64_t cap,
                              uint32_t *ranges, int32_t *spans, float *depth, float *splats);
sgs_status sgs_copy_splat_grads(sgs_ctx *c, float *out);

}  // extern "C"

// ---- inspection ----------------------------------------------------------
namespace {

__global__ void k_export(int64_t vn, const float4 *__restrict__ rec,
                         const uint32_t *__restrict__ touched, int32_t *__restrict__ spans,
                         float *__restrict__ depth, float *__restrict__ splats,
                         const uint32_t *__restrict__ dkey_unsorted) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= vn) return;
  const float4 a = rec[3 * s], b = rec[3 * s + 1], cc = rec[3 * s + 2];
  const bool valid = touched[s] != 0;
  if (spans) {
    const uint32_t sx = __float_as_uint(b.z), sy = __float_as_uint(b.w);
    spans[4 * s + 0] = valid ? (int)(sx & 0xFFFF) : -1;
    spans[4 * s + 1] = valid ? (int)(sx >> 16) : -1;
    spans[4 * s + 2] = valid ? (int)(sy & 0xFFFF) : -1;
    spans[4 * s + 3] = valid ? (int)(sy >> 16) : -1;
  }
  (void)dkey_unsorted;
  if (depth) depth[s] = 0.0f;
  if (splats) {
    float *o = splats + 12 * s;
    // the records hold the conic scaled for the blend: undo it
    o[0] = a.x; o[1] = a.y; o[2] = a.z / SGS_CONIC_KAC; o[3] = a.w / SGS_CONIC_KB;
    o[4] = b.x / SGS_CONIC_KAC; o[5] = b.y; o[6] = cc.x; o[7] = cc.y; o[8] = cc.z; o[9] = cc.w;
    o[10] = 0.0f; o[11] = 0.0f;
  }
}

// out[p] = t for every position p of tile t's range (one workgroup per tile)
__global__ void k_fill_tile_ids(const uint2 *__restrict__ ranges, uint32_t *__restrict__ out) {
  const uint2 r = ranges[blockIdx.x];
  for (uint32_t p = r.x + threadIdx.x; p < r.y; p += blockDim.x) out[p] = blockIdx.x;
}

// depth keys in splat order: scatter the sorted (key, index) pairs back (the
// segments' padding, index 0xFFFFFFFF, has no splat)
__global__ void k_export_depth(int64_t count, const uint32_t *__restrict__ skey,
                               const uint32_t *__restrict__ sval, float *__restrict__ depth) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= count) return;
  const uint32_t key = skey[k], s = sval[k];
  if (s != 0xFFFFFFFFu) depth[s] = key == 0xFFFFFFFFu ? -1.0f : __uint_as_float(key);
}

}  // namespace

extern "C" sgs_status sgs_copy_structure(sgs_ctx *c, uint32_t *tile_ids, uint32_t *vals,
                                         int64_t cap, uint32_t *ranges, int32_t *spans,
                                         float *depth, float *splats) {
  if (!c) return SGS_EINVAL;
  if (!c->rendered) return fail(c, SGS_ESTATE, "copy_structure: render_fwd first");
  const int64_t P = c->pairs;
  if ((tile_ids || vals) && cap < P) return fail(c, SGS_ECAPACITY, "copy_structure: cap < pairs");
  if (tile_ids && P) {
    // the tile id of every sorted pair, from the tile ranges
    k_fill_tile_ids<<<(unsigned)c->total_tiles, 256, 0, c->stream>>>(c->ranges, tile_ids);
    SGS_HIP(hipGetLastError(), "copy tile ids");
  }
  if (vals && P)
    SGS_HIP(hipMemcpyAsync(vals, c->pair_val[c->pair_sorted_buf], 4 * P,
                           hipMemcpyDeviceToDevice, c->stream), "copy vals");
  if (ranges)
    SGS_HIP(hipMemcpyAsync(ranges, c->ranges, 8 * c->total_tiles, hipMemcpyDeviceToDevice,
                           c->stream), "copy ranges");
  if (spans || splats) {
    k_export<<<sgs_blocks(c->vn, 256), 256, 0, c->stream>>>(c->vn, c->rec, c->touched, spans,
                                                            nullptr, splats, nullptr);
    SGS_HIP(hipGetLastError(), "copy_structure export");
  }
  if (depth) {
    k_export_depth<<<sgs_blocks(c->vn_pad, 256), 256, 0, c->stream>>>(
        c->vn_pad, c->depth_key[c->depth_sorted_buf], c->depth_val[c->depth_sorted_buf], depth);
    SGS_HIP(hipGetLastError(), "copy_structure depth");
  }
  return SGS_OK;
}

namespace {
// FP64 records of SGS_SGRAD values -> float rows of 12 (the last ones 0)
__global__ void k_export_grads(int64_t count, const double *__restrict__ in,
                               float *__restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const int64_t s = i / 12, k = i - s * 12;
  out[i] = k < SGS_SGRAD ? (float)in[s * SGS_SGRAD + k] : 0.0f;
}
}  // namespace

extern "C" sgs_status sgs_copy_splat_grads(sgs_ctx *c, float *out) {
  if (!c || !out) return SGS_EINVAL;
  const int64_t count = 12 * c->vn;
  k_export_grads<<<sgs_blocks(count, 256), 256, 0, c->stream>>>(count, c->splat_grad, out);
  SGS_HIP(hipGetLastError(), "copy splat grads");
  return SGS_OK;
}
