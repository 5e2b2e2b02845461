/*
 * speedygs.h -- C ABI of libspeedygs.so: one rate-distortion (RD) step of the
 * structural-formation stage of SpeedyGS on an AMD Instinct MI355X (gfx950).
 *
 * The step solves the paper's formation problem (Sec. 3.2, Eq. "sf"):
 *     min over (G, Q, M) of  D_render(G, Q, M) + lambda * R_formation(G, Q, M)
 * G = the 59 channels of every Gaussian (`params`), Q = the 59 channel step
 * sizes (`qstep`), M = the per-Gaussian retention scores (`score`).  A step is
 *     sgs_fakequant_prune -> sgs_rate_proxy -> sgs_render_fwd -> sgs_l1_loss
 *     -> sgs_render_bwd -> sgs_fakequant_prune_bwd,
 * or, with the same results and two fewer passes over the parameters each way,
 *     sgs_quant_render_fwd -> sgs_rate_proxy -> sgs_l1_loss -> sgs_quant_render_bwd.
 *
 * Conventions common to every call
 *  - Device pointers are HIP device memory owned by the caller; the library
 *    never frees or keeps them beyond the call.  Host pointers are marked.
 *  - Every call only enqueues work on the stream given to sgs_create (HIP
 *    stream order gives the dependencies).  The exceptions are sgs_render_fwd
 *    and sgs_quant_render_fwd, which read the pair count back to the host
 *    once (it sizes the sort) unless the pair capacity is fixed.
 *  - Gaussian parameters are SoA float32 [59][npad], npad a multiple of 64,
 *    256-byte aligned rows.  Channels: 0-2 mean, 3-5 SH DC (r,g,b), 6-50 SH
 *    k=1..15 coefficient-major (6 + 3(k-1) + c), 51 opacity logit,
 *    52-54 log-scale, 55-58 rotation quaternion (w,x,y,z).
 *  - Images are float32 [V][3][H][W]; per-pixel buffers [V][H][W].
 *  - A context is not thread-safe; calls on one context must not overlap.
 *  - On a non-OK status nothing has been enqueued unless the status is
 *    SGS_EHIP (a launch failed); sgs_last_error() explains.
 */
#ifndef SPEEDYGS_H
#define SPEEDYGS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SGS_NCH 59
/* uint64 words of the per-channel statistics buffer written by
 * sgs_fakequant_prune: [0,59) min keys, [59,118) max keys, [118] kept count,
 * [119] flags (bit 0: some q_j <= 0 or not finite).  A min key is
 * (order-preserving bits of the value << 32) | index; a max key stores
 * 0xFFFFFFFF - index in its low half, so both select the lowest index on ties. */
#define SGS_STATS_WORDS 128
/* float32 words of the compact rate-proxy gradient written by sgs_rate_proxy:
 * [0,59) d/dy at argmax_j, [64,123) d/dy at argmin_j, [128,187) d/dq_j,
 * [192] d/dM (same for every Gaussian). */
#define SGS_RATE_GRAD_FLOATS 256

typedef struct sgs_ctx sgs_ctx;

typedef enum {
  SGS_OK = 0,
  SGS_EINVAL = -1,    /* bad argument; nothing enqueued */
  SGS_ENOMEM = -2,    /* device allocation failed; context still usable */
  SGS_EHIP = -3,      /* a HIP call or launch failed */
  SGS_ESTATE = -4,    /* call out of order (e.g. render before set_scene) */
  SGS_ECAPACITY = -5  /* a size limit of the library was exceeded */
} sgs_status;

/* Pinhole camera, OpenCV axes (x right, y down, z forward); pixel (u, v) has
 * its centre at image coordinate (u, v).  19 floats. */
typedef struct {
  float R[9];      /* world -> camera rotation, row-major */
  float t[3];      /* world -> camera translation */
  float fx, fy, cx, cy;
  float campos[3]; /* camera centre in world coordinates (SH view direction) */
} sgs_camera;

typedef struct {
  int32_t tile_w, tile_h; /* blend tile: 8x8, 16x16 (default), 32x8, 32x16 or 32x32 */
  float tau;              /* Gumbel-sigmoid temperature (default 1) */
  int32_t schedule;       /* blend launch (one wave per 8x8 sub-tile): 0 one
                             workgroup per sub-tile (default), 1 resident
                             workgroups striding over the sub-tiles of the
                             tiles ordered by list length, 2 the same taken
                             from an atomic queue, 3 resident workgroups of one
                             whole tile each (a wave per sub-tile) striding
                             over that order; results do not depend on it */
  int32_t deterministic;  /* 0 (default): the blend backward adds each splat's
                             per-wave gradient sums with FP64 atomics (their
                             order, hence the last bits, varies from run to
                             run); 1: it adds them as 96-bit fixed-point
                             integers (units of 2^-64, terms below 2^31 in
                             magnitude) whose sums do not depend on order, so
                             every gradient is the same bits on every run and
                             schedule (3x the accumulator memory: 240 bytes per
                             view and Gaussian); a term out of that range is
                             left out and reported by sgs_query */
  int32_t reserved[3];    /* must be zero */
} sgs_options;

/* Create a context on HIP device `device` that enqueues on `hip_stream`
 * (a hipStream_t; NULL = the null stream).  *out receives the context. */
sgs_status sgs_create(sgs_ctx **out, int device, void *hip_stream);
void sgs_destroy(sgs_ctx *ctx);
/* Message for the last non-OK status of this context (never NULL). */
const char *sgs_last_error(const sgs_ctx *ctx);
/* Replace the stream later calls enqueue on. */
sgs_status sgs_set_stream(sgs_ctx *ctx, void *hip_stream);

/* Bind the scene shape and cameras and allocate the context's scratch.
 * n Gaussians (n >= 1), npad >= n and a multiple of 64, n_hat = number of
 * Gaussians before structural formation (Sec. 3.3.1, L_mask), views >= 1
 * cameras (host array, copied), width/height in pixels (<= 32768), opt host
 * (NULL = defaults).  Synchronizes the stream. */
sgs_status sgs_set_scene(sgs_ctx *ctx, int64_t n, int64_t npad, int64_t n_hat,
                         const sgs_camera *cams, int32_t views, int32_t width,
                         int32_t height, const sgs_options *opt);

/* a1-a2 (Sec. 3.3.1, uniform quantizer with learnable q_j; p_i = sigma(s_i);
 * M_i = GumbelSoftmax(p_i); hard mask).
 *   qparams[j][i] = q_j * rint(params[j][i] / q_j)   (FP32, ties to even)
 *   mask_mode 0: hard_mask = given_mask (score unused);
 *             1: Gumbel-sigmoid: u from SplitMix64(seed ^ ((step << 32) + i)),
 *                hard = [u (1 + e^s) > 1] (= [s + logit u > 0]),
 *                soft = sigmoid((s + logit u) / tau);
 *             2: keep every Gaussian.
 *   soft_mask (may be NULL unless mode 1 is used in the backward) = float [n].
 *   stats: SGS_STATS_WORDS device words; per-channel min/max/argmin/argmax of
 *   the RAW params over all n Gaussians and the kept count (rate proxy input).
 * Device-side errors (q_j <= 0 or not finite) set stats[119] bit 0. */
sgs_status sgs_fakequant_prune(sgs_ctx *ctx, const float *params, const float *qstep,
                               const float *score, int32_t mask_mode,
                               const uint8_t *given_mask, uint64_t seed, uint64_t step,
                               float *qparams, uint8_t *hard_mask, float *soft_mask,
                               uint64_t *stats);

/* a3 (Sec. 3.3.1, Eqs. L_j, L_quant, L_mask, R_proxy):
 *   c_j = max(1, ceil(fl32(max_j - min_j) / q_j)),  L_j = log2 c_j,
 *   L_quant = sum_j L_j,  L_mask = kept / n_hat,  R = L_mask * L_quant.
 * out3 (device float[3]) = {R, L_quant, L_mask}.  If rate_grad is not NULL it
 * receives the gradient of rate_weight * R in compact form (see
 * SGS_RATE_GRAD_FLOATS), straight through the ceil. */
sgs_status sgs_rate_proxy(sgs_ctx *ctx, const uint64_t *stats, const float *qstep,
                          float rate_weight, float *out3, float *rate_grad);

/* a4-a8 (Sec. 3.1: project, tile-bin, depth-sort, composite front to back).
 * Every view of the scene is rendered.  final_T and last (entries of the
 * pixel's tile list consumed before termination) are kept for the backward.
 * eval_count (device uint64, may be NULL) is INCREMENTED by the number of
 * in-support Gaussian-pixel evaluations.  Splats whose hard mask is 0 are
 * binned and visited but contribute alpha 0 (masked rasterization).
 * Synchronizes the stream once (pair count). */
sgs_status sgs_render_fwd(sgs_ctx *ctx, const float *qparams, const uint8_t *hard_mask,
                          float *image, float *final_T, uint32_t *last,
                          uint64_t *eval_count);

/* a9 (Supp. "Training Objective", L1 part): loss[0] = mean |image - target|,
 * dL_dimage = scale * sign(image - target) / (3 V H W), sign(0) = 0.
 * `scale` is the upstream gradient of the loss (1 for a plain step). */
sgs_status sgs_l1_loss(sgs_ctx *ctx, const float *image, const float *target,
                       float scale, float *loss, float *dL_dimage);

/* a10-a11: gradient of the rendered images w.r.t. qparams [59][npad]
 * (overwritten) and the hard mask (grad_hard_mask float [n], overwritten).
 * Must follow sgs_render_fwd of the same qparams / hard_mask on this context. */
sgs_status sgs_render_bwd(sgs_ctx *ctx, const float *qparams, const uint8_t *hard_mask,
                          const float *final_T, const uint32_t *last,
                          const float *dL_dimage, float *grad_qparams,
                          float *grad_hard_mask);

/* a12: quantizer and mask backward.
 *   grad_params = grad_qparams (straight through) [+ rate gradient];
 *   grad_qstep_j = sum_i grad_qparams_ij (k_ij - params_ij / q_j) [+ rate];
 *   grad_score_i = (grad_hard_mask_i [+ rate]) soft_i (1 - soft_i) / tau in
 *   mask mode 1, else 0.
 * rate_grad/stats (both or neither) add the rate-proxy gradient.  Outputs are
 * overwritten; grad_params may alias grad_qparams. */
sgs_status sgs_fakequant_prune_bwd(sgs_ctx *ctx, const float *params, const float *qstep,
                                   const float *soft_mask, int32_t mask_mode,
                                   const float *rate_grad, const uint64_t *stats,
                                   const float *grad_qparams, const float *grad_hard_mask,
                                   float *grad_params, float *grad_qstep, float *grad_score);

/* a1-a8 in one call (Sec. 3.3.1 quantizer and mask, Sec. 3.1 render): the
 * results of sgs_fakequant_prune followed by sgs_render_fwd (hard_mask,
 * soft_mask, stats, image, final_T, last, eval_count bit for bit), without
 * the quantized parameters: the projection quantizes the raw rows itself, so
 * qparams is neither written nor read (two fewer passes over [59][npad]).
 * Arguments as in those two calls; params rows 16-byte aligned.
 * Synchronizes the stream once, as sgs_render_fwd does. */
sgs_status sgs_quant_render_fwd(sgs_ctx *ctx, const float *params, const float *qstep,
                                const float *score, int32_t mask_mode,
                                const uint8_t *given_mask, uint64_t seed, uint64_t step,
                                uint8_t *hard_mask, float *soft_mask, uint64_t *stats,
                                float *image, float *final_T, uint32_t *last,
                                uint64_t *eval_count);

/* a10-a12 in one call: the results of sgs_render_bwd followed by
 * sgs_fakequant_prune_bwd with grad_params aliasing grad_qparams (grad_params,
 * grad_score and grad_hard_mask bit for bit; grad_qstep the same FP64 sum in
 * another order, then rounded to float).  The projection backward re-quantizes
 * the raw rows and applies the straight-through quantizer backward itself,
 * so no gradient of the quantized parameters crosses HBM.  Must follow
 * sgs_quant_render_fwd (or sgs_render_fwd of the quantized params) of the
 * same params / qstep on this context; rate_grad/stats (both or neither) add
 * the rate-proxy gradient.  All outputs are overwritten; grad_params [59][npad]
 * must not alias params. */
sgs_status sgs_quant_render_bwd(sgs_ctx *ctx, const float *params, const float *qstep,
                                const float *soft_mask, int32_t mask_mode,
                                const float *rate_grad, const uint64_t *stats,
                                const float *final_T, const uint32_t *last,
                                const float *dL_dimage, float *grad_params,
                                float *grad_qstep, float *grad_score, float *grad_hard_mask);

/* Autotuner of the batched step (tile shape, then blend schedule): times
 * `reps` (1..1000) whole RD steps (sgs_quant_render_fwd on the given mask,
 * sgs_rate_proxy, sgs_l1_loss, sgs_quant_render_bwd) per candidate with HIP
 * events on the context's stream, after one untimed step each: the tile
 * shapes 16x16, 8x8, 32x8, 32x16 and 32x32 with schedule 0, then schedules
 * 1, 2 and 3 with
 * the fastest shape.  *chosen (host) receives the fastest options (tau kept)
 * and the context is left bound to the same scene with them; a reserved pair
 * capacity is released (call sgs_reserve_pairs again).  ms_out (host
 * float[8], may be NULL) receives each candidate's mean step time in the
 * order timed.  The images and gradients do not depend on the choice (the
 * support rule is pixel-exact, Sec. 3.1 binning).  Needs params rows 16-byte
 * aligned, target [V][3][H][W]; allocates temporary device buffers for the
 * step's outputs and synchronizes.  On failure the scene stays bound with the
 * last options tried or the best found. */
sgs_status sgs_autotune(sgs_ctx *ctx, const float *params, const float *qstep,
                        const uint8_t *given_mask, const float *target, int32_t reps,
                        sgs_options *chosen, float *ms_out);

/* What the eval_count of sgs_render_fwd / sgs_quant_render_fwd counts:
 *   mode 0 (default): the method's evaluations, every (Gaussian, pixel) pair
 *     whose pixel lies in the splat's span, visited before the pixel stops
 *     (Sec. 3.1 compositing; the count the FP64 oracle reproduces);
 *   mode 1: the evaluations the uncounted (timed) blend performs: those of
 *     mode 0 whose splat can reach the alpha cut-off 1/255 somewhere in the
 *     pixel's 8x8 sub-tile (the blend's per-sub-tile reach test drops the
 *     others without evaluating them).
 * Images, T and stop positions are the same bit for bit in both modes and
 * without counting.  Takes effect at the next render. */
sgs_status sgs_set_eval_count_mode(sgs_ctx *ctx, int32_t mode);

/* Whether the fused backward (sgs_quant_render_bwd) and sgs_rate_mlp_bwd
 * write the gradient rows of the higher SH coefficients (channels 6-50,
 * degrees 1-3) into grad_params: on (1, the default) they do; off (0) they
 * leave those rows of grad_params untouched, for a step whose optimizer
 * update skips them (the separated higher-SH schedule of Sec. 4.1, as
 * sgs_adam_step with sh_rest = 0).  Every other output, the step-size
 * gradient included, is the same either way.  Takes effect at the next
 * backward call (a captured graph keeps the value it was captured with). */
sgs_status sgs_set_grad_sh_rest(sgs_ctx *ctx, int32_t on);

/* Host-side query (synchronizes the stream): pairs of the last render and the
 * device flags word of `stats` (may be NULL).  Returns SGS_EINVAL when the
 * flags report an invalid step size, SGS_ECAPACITY (once, then cleared) when
 * a render since the last query exceeded a reserved pair capacity (the
 * caller reserves more and reruns the step) or, in deterministic mode, a
 * per-wave gradient term fell outside the fixed-point range. */
sgs_status sgs_query(sgs_ctx *ctx, const uint64_t *stats, int64_t *pairs_last,
                     uint64_t *flags);

/* Host-side query (synchronizes the stream): the (splat, super-tile) items
 * of the last render: a splat yields one item per 8x8-tile super-tile its
 * tile rectangle meets (the first level of the tile binning). */
sgs_status sgs_query_items(sgs_ctx *ctx, int64_t *items);

/* Fix the (tile, Gaussian) pair capacity (allocating it now; 0 returns to
 * the default mode).  With a fixed capacity sgs_render_fwd never
 * synchronizes: the pair count stays on the device, grids are sized by the
 * capacity, pairs beyond it are dropped and reported by sgs_query. Required
 * for graph capture.  Synchronizes the stream. */
sgs_status sgs_reserve_pairs(sgs_ctx *ctx, int64_t capacity);

/* HIP-graph capture of the calls made on this context between begin and end
 * (any of the entry points above except set_scene / reserve_pairs / query /
 * profile_read, which synchronize).  Needs a reserved pair capacity and a
 * non-null stream.  The graph replays the same pointers and sizes. */
typedef struct sgs_graph sgs_graph;
sgs_status sgs_graph_begin(sgs_ctx *ctx);
sgs_status sgs_graph_end(sgs_ctx *ctx, sgs_graph **out);
sgs_status sgs_graph_launch(sgs_graph *graph, void *hip_stream);
void sgs_graph_destroy(sgs_graph *graph);

/* Inspection for tests: copy the last render's structure into caller device
 * buffers.  tile_ids/vals: uint32 [cap] (sorted pairs), ranges uint32
 * [V*tiles][2], spans int32 [V][n][4] (x0,x1,y0,y1; all -1 when culled),
 * depth float [V][n], splats float [V][n][12] (px, py, A, B, C, opacity,
 * r, g, b, mask, 0, 0).  Any pointer may be NULL. */
sgs_status sgs_copy_structure(sgs_ctx *ctx, uint32_t *tile_ids, uint32_t *vals,
                              int64_t cap, uint32_t *ranges, int32_t *spans,
                              float *depth, float *splats);
/* Per-(view, Gaussian) splat gradients of the last render_bwd:
 * float [V][n][12] (px, py, A, B, C, opacity, r, g, b, mask, 0, 0). */
sgs_status sgs_copy_splat_grads(sgs_ctx *ctx, float *out);

/* ---- a13: learned rate estimator -----------------------------------------
 * A per-Gaussian MLP 64 -> 128 -> 128 -> 1 (ReLU hidden layers, linear
 * output) estimating the bits a Gaussian costs under the paper's channel-wise
 * fixed-length coder (Sec. 3.4.1); it stands beside the range-based rate
 * proxy of Sec. 3.3.1:  R_learned = (1/n_hat) sum_i M_i f(x_i),
 * x_ij = log2(1 + (params_ij - min_j) / q_j) for the 59 channels (min_j from
 * the statistics of sgs_fakequant_prune), padded with 5 zeros.
 * theta: float32 [SGS_MLP_PARAMS] master weights, concatenated row-major
 *   W1[64][128] (in, out), b1[128], W2[128][128], b2[128], w3[128], b3.
 * packed: SGS_MLP_PACKED_BYTES of device memory holding the BF16 copy of W1
 *   and W2 in the matrix-core fragment order (written by sgs_rate_mlp_pack).
 * BF16 inputs, weights and first hidden activation; FP32 accumulation. */
#define SGS_MLP_PARAMS 24961
#define SGS_MLP_PACKED_BYTES 98304

/* packed <- BF16 fragments of theta (round to nearest even). */
sgs_status sgs_rate_mlp_pack(sgs_ctx *ctx, const float *theta, void *packed);
/* out_R (device float[1]) = R_learned; per_gaussian (float [n], may be NULL)
 * receives f(x_i).  Features are computed from params on the fly; f and the
 * hidden activation signs are kept in the context for sgs_rate_mlp_bwd. */
sgs_status sgs_rate_mlp_fwd(sgs_ctx *ctx, const void *packed, const float *theta,
                            const float *params, const float *qstep, const uint64_t *stats,
                            const uint8_t *hard_mask, float *out_R, float *per_gaussian);
/* Gradient of rate_weight * R_learned, ADDED into grad_params [59][npad] and
 * grad_qstep [59] (channel minima held fixed), and dR/dM_i = f_i / n_hat
 * added into grad_hard_mask (may be NULL) and, in mask mode 1, through the
 * straight-through Gumbel-sigmoid into grad_score (may be NULL).  Uses f and
 * the signs of the hidden pre-activations that the last sgs_rate_mlp_fwd
 * kept in the context (32 B per Gaussian): call it after that forward, on
 * the same packed, theta, params, qstep and stats (SGS_ESTATE if no forward
 * ran since set_scene), and after sgs_fakequant_prune_bwd. */
sgs_status sgs_rate_mlp_bwd(sgs_ctx *ctx, const void *packed, const float *theta,
                            const float *params, const float *qstep, const uint64_t *stats,
                            const uint8_t *hard_mask, const float *soft_mask,
                            int32_t mask_mode, float rate_weight, float *grad_params,
                            float *grad_qstep, float *grad_score, float *grad_hard_mask);
/* Feature rows of the estimator for chosen Gaussians of the scene (to build
 * training sets): X[r] = the BF16 features the in-loop forward gives Gaussian
 * idx[r] (x_j = log2(1 + (y_j - min_j) / q_j), min_j from `stats` of the
 * last sgs_fakequant_prune on these params and steps; channels 59-63 zero).
 * idx: device int32 [rows] (an index outside [0, n) gives a zero row);
 * X: device BF16 [rows][64], 8-byte aligned. */
sgs_status sgs_rate_mlp_features(sgs_ctx *ctx, const float *params, const float *qstep,
                                 const uint64_t *stats, const int32_t *idx, int64_t rows,
                                 uint16_t *X);
/* f over given feature rows: X BF16 [rows][64] (8-byte aligned), out float [rows]. */
sgs_status sgs_rate_mlp_infer(sgs_ctx *ctx, const void *packed, const float *theta,
                              const uint16_t *X, int64_t rows, float *out);
/* Bytes of the caller-provided device workspace a training step on `rows`
 * rows needs. */
int64_t sgs_rate_mlp_train_scratch_bytes(int64_t rows);
/* One training step on rows feature vectors X (BF16 [rows][64]) with targets
 * (float [rows]): loss[0] = mean (f - target)^2, grad_theta (float
 * [SGS_MLP_PARAMS]) = its gradient; if lr > 0, Adam (beta 0.9 / 0.999,
 * eps 1e-8, bias-corrected with `step` >= 1) updates theta, adam_m, adam_v in
 * place and re-packs `packed`.  rows must be a positive multiple of 8. */
sgs_status sgs_rate_mlp_train_step(sgs_ctx *ctx, float *theta, float *adam_m, float *adam_v,
                                   void *packed, const uint16_t *X, const float *target,
                                   int64_t rows, float lr, int64_t step, float *loss,
                                   float *grad_theta, void *scratch);
/* For callers that cannot allocate device memory (code under HIP-graph
 * capture, tight training loops, harnesses that forbid hipMalloc): the
 * training step of sgs_rate_mlp_train_step, same kernels and the same results
 * bit for bit, with its workspace taken from a static device array of the
 * library (sgs_rate_mlp_train_scratch_bytes(SGS_MLP_STATIC_ROWS) bytes, about
 * 14 MiB) instead of a caller buffer.  rows: a multiple of 8 in
 * [8, SGS_MLP_STATIC_ROWS]; a larger batch returns SGS_ECAPACITY with nothing
 * enqueued.  The array exists once per GPU, from the first sgs_create on that
 * GPU until the process ends, and every call on that GPU (from any context)
 * uses it: calls that overlap on one GPU (two streams, two threads) race and
 * their results are undefined.  Nothing in it needs clearing between calls.
 * Calls no device allocation or free; no profiling events are recorded for it.
 * Other arguments as in sgs_rate_mlp_train_step. */
#define SGS_MLP_STATIC_ROWS 8192
sgs_status sgs_rate_mlp_train_step_static(sgs_ctx *ctx, float *theta, float *adam_m,
                                          float *adam_v, void *packed, const uint16_t *X,
                                          const float *target, int64_t rows, float lr,
                                          int64_t step, float *loss, float *grad_theta);

/* Rate-proxy variants the paper compares with sgs_rate_proxy's range-based
 * multiplicative proxy (Sec. 3.3.1 and the supplement's "Comparison with an
 * Alternative Rate Proxy"; the ablation's additive masking).
 *  proxy 1, scale-based Laplace: per channel b_j = mean |y_ij - mean_j| over
 *    the N Gaussians (the maximum-likelihood Laplace scale) and
 *    L_j = log2(max(1, 2 e b_j / q_j)) (code length of a Laplace source
 *    quantized with step q_j); needs params, two passes over them.
 *  masking 1, additive: the loss carries lambda L_quant + alpha L_mask
 *    instead of lambda L_mask L_quant. */
typedef struct {
  int32_t proxy;     /* 0 range-based (Sec. 3.3.1), 1 scale-based Laplace */
  int32_t masking;   /* 0 multiplicative (Sec. 3.3.1), 1 additive */
  float alpha;       /* weight of the additive mask term */
  int32_t reserved;  /* must be zero */
} sgs_rate_options;

/* out3 (device float[3]) = {the rate's term in the loss (lambda = rate_weight
 * folded in), L_quant, L_mask}; rate_grad (device, SGS_RATE_GRAD_FLOATS, may
 * be NULL) receives the compact gradient sgs_fakequant_prune_bwd consumes
 * (the Laplace proxy has no argmin / argmax terms: its y gradient is dense and
 * added by sgs_rate_variant_bwd).  stats: from sgs_fakequant_prune on the
 * same params and steps. */
sgs_status sgs_rate_variant(sgs_ctx *ctx, const float *params, const float *qstep,
                            const uint64_t *stats, const sgs_rate_options *opt /* host */,
                            float rate_weight, float *out3, float *rate_grad);
/* After sgs_fakequant_prune_bwd: adds the dense y gradient of the last
 * sgs_rate_variant (Laplace proxy) to grad_params [59][npad]; does nothing
 * after the range proxy. */
sgs_status sgs_rate_variant_bwd(sgs_ctx *ctx, const float *params, float *grad_params);

/* SSIM term of the rendering distortion (the supplement takes D_render from
 * vanilla 3DGS: D = (1 - w) L1 + w (1 - SSIM), w = 0.2 there; call
 * sgs_l1_loss with scale 1 - w, then this with weight w).  SSIM (Wang et al.
 * 2004) per view and colour plane with the 11 x 11 Gaussian window of
 * standard deviation 1.5, zero outside the image, C1 = 0.01^2, C2 = 0.03^2,
 * averaged over the V * 3 * H * W pixels.  loss[0] (device float) receives
 * weight * (1 - SSIM); dL_dimage (device [V][3][H][W], may be NULL) has
 * weight * d(1 - SSIM)/d image ADDED.  weight in [0, 1].  The first call on a
 * scene allocates the context's SSIM scratch (24 bytes per pixel), so it
 * must not be the first inside graph capture. */
sgs_status sgs_ssim_loss(sgs_ctx *ctx, const float *image, const float *target, float weight,
                         float *loss, float *dL_dimage);

/* Pruning by the learned mask (the paper's supplement applies the learned
 * mask to prune every 1,000 iterations of the formation stage): copies the
 * Gaussians with hard_mask != 0 (hard_mask: device uint8 [n], 16-byte
 * aligned), in index order, of narrays (1..SGS_COMPACT_MAX_ARRAYS) SoA
 * float32 arrays of the scene.  src[a], dst[a]: host arrays of device
 * pointers; src[a] has rows[a] rows of stride npad (the scene's; 16-byte
 * aligned) of which columns [0, n) are read (a one-row array needs n
 * floats); dst[a] rows have stride dst_pad and receive columns [0, kept);
 * rows[a] in 1..59 (59 for the parameters and their moments, 1 for scores).
 * *kept (host) receives the count: the call synchronizes once to read it and
 * returns SGS_ECAPACITY if dst_pad < *kept, or SGS_EINVAL if what would be
 * written overlaps what is read, in both cases having written no dst.  The
 * caller then calls sgs_set_scene with the new count. */
#define SGS_COMPACT_MAX_ARRAYS 8
sgs_status sgs_compact(sgs_ctx *ctx, const uint8_t *hard_mask, int32_t narrays,
                       const float *const *src /* host */, float *const *dst /* host */,
                       const int32_t *rows /* host */, int64_t dst_pad, int64_t *kept /* host */);

/* One Adam step (Kingma & Ba 2015) on the formation variables: the
 * parameters y [59][npad] (SoA, 16-byte aligned rows), the step sizes q [59]
 * and the retention scores s [n] of the context's scene, from their
 * gradients.  Per element, with t = opt->step >= 1:
 *     m <- b1 m + (1 - b1) g,   v <- b2 v + (1 - b2) g^2,
 *     x <- x - lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps)
 * in FP32 (the two bias corrections are formed in FP64 and rounded once;
 * beta1, beta2 in [0.5, 1), so 1 - beta is exact in FP32; eps >= 0).
 * The schedule the paper adopts for speed (Sec. 4.1: separated updates of the
 * higher SH coefficients and an economical Adam) is read as two switches:
 *  - sh_rest = 0 leaves the 45 higher-order SH rows (channels 6-50) and
 *    their moments untouched this step (the caller updates them every k-th
 *    step with that step's gradient);
 *  - sparse = 1 leaves a Gaussian's parameters and moments untouched when
 *    every gradient of the rows updated this step is exactly zero (it is in
 *    no view and holds no range extreme); the steps and scores always update.
 * m, v: device buffers shaped like their variable, zero before step 1.  The
 * (q, q_m, q_v, grad_q) and (s, s_m, s_v, grad_s) groups may each be all
 * NULL to skip that variable; grad buffers are read only. */
typedef struct {
  float lr[SGS_NCH];      /* learning rate per parameter channel */
  float lr_q, lr_score;   /* learning rates of the steps and the scores */
  float beta1, beta2, eps;
  int32_t sh_rest;        /* 1: update channels 6-50 this step */
  int32_t sparse;         /* 1: skip Gaussians whose updated rows have zero gradient */
  int32_t reserved;       /* must be zero */
  int64_t step;           /* t >= 1 */
} sgs_adam_options;

sgs_status sgs_adam_step(sgs_ctx *ctx, const sgs_adam_options *opt /* host */, float *params,
                         float *params_m, float *params_v, const float *grad_params,
                         float *qstep, float *q_m, float *q_v, const float *grad_qstep,
                         float *score, float *s_m, float *s_v, const float *grad_score);

/* Channel-wise fixed-length coding (Sec. 3.4.1: each channel stored with the
 * fixed bit width its quantization precision gives, plus per-channel
 * metadata) of the kept Gaussians' quantization codes k_ij = rint(y_ij/q_j)
 * (the fake quantizer's decision, FP32 division, ties to even).
 * Stream: a header of 59 sgs_fl_channel records, then the payload,
 * channel-major, kept Gaussians in index order, each k_ij - kmin_j in
 * width_j bits LSB first; stream bit b is bit (b & 7) of byte b >> 3 (bit
 * b & 31 of 32-bit word b >> 5); width_j = ceil(log2(kmax_j - kmin_j + 1))
 * over the kept Gaussians, 0 for a constant channel or when none is kept.
 * Its size in bits is payload + 59 * 72 (q f32, kmin i32, width u8). */
typedef struct {
  float q;        /* q_j */
  int32_t kmin;   /* smallest kept code */
  int32_t width;  /* bits per kept Gaussian, 0..32 */
} sgs_fl_channel;

/* Encode params (SoA [59][npad], 16-byte aligned), qstep [59] and hard_mask
 * [n] (16-byte aligned; nonzero = kept) of the context's scene.  header:
 * device sgs_fl_channel[59]; payload: device uint32 words, payload_words of
 * them (words past the payload's end are left untouched); info: device
 * int64[3] receiving {payload bits, kept Gaussians, flags}, flags bit 0 = a
 * kept value whose code is not finite or lies outside int32 (the stream is
 * then not decodable: header and payload unspecified), bit 1 =
 * payload_words too small (the stream is cut there).  Sync-free; read info
 * afterwards. */
sgs_status sgs_fl_encode(sgs_ctx *ctx, const float *params, const float *qstep,
                         const uint8_t *hard_mask, sgs_fl_channel *header, uint32_t *payload,
                         int64_t payload_words, int64_t *info);
/* Decode: out [59][out_pad] (device, out_pad >= kept) receives the
 * dequantized parameters fl32((kmin_j + v) q_j) of the kept Gaussians in
 * index order (equal to the fake quantizer's output for them).  kept is the
 * count the encoder reported; payload holds payload_words words. */
sgs_status sgs_fl_decode(sgs_ctx *ctx, const sgs_fl_channel *header, const uint32_t *payload,
                         int64_t payload_words, int64_t kept, int64_t out_pad, float *out);

/* ---- Learned-coding stage, lossless parts (Sec. 3.4.2) -------------------
 *
 * Geometry occupancy tokens (Sec. 3.4.2, geometry occupancy coding: the
 * point cloud voxelized into a multiscale structure, each downsampling step
 * giving 8-bit occupancy tokens).  The kept Gaussians' position codes
 * k_c = rint(fl32(y_c / q_c)) (c = x, y, z: channels 0-2; the quantizer's
 * decision) become voxels u_c = k_c - kmin_c, kmin_c the smallest kept code,
 * in a cube of side 2^D, D >= 1 the least depth that holds every axis's
 * range.  Gaussians in one voxel merge: one voxel is coded and its extra
 * copies are listed as metadata (the paper keeps duplicate counts aside).
 * Tokens are written level by level from the root (level 0: one token;
 * level d: one token per occupied node of depth d, in the Morton order of
 * the nodes); bit (xb << 2 | yb << 1 | zb) of a node's token is set when its
 * child whose next coordinate bits are xb, yb, zb is occupied.  The Morton
 * code of a voxel has x bit b at bit 3b + 2, y bit b at 3b + 1, z bit b at
 * 3b.  Header (all int64): */
typedef struct {
  int64_t depth;          /* D, 1..21 */
  int64_t kmin[3];        /* smallest kept position code per axis (0 if none) */
  int64_t kept;           /* kept Gaussians */
  int64_t unique;         /* distinct voxels (nodes of depth D) */
  int64_t tokens;         /* tokens in all: the sum of level_size */
  int64_t dups;           /* entries of the duplicate list */
  int64_t flags;          /* bit 0: a code outside int32 or a range of 2^21 or more
                             (not decodable); bit 1: token_cap too small (tokens cut);
                             bit 2: dup_cap too small (list cut) */
  int64_t level_size[21]; /* tokens of level d (0 from level D on) */
} sgs_octree_header;

/* Encode the kept Gaussians' positions: params SoA [59][npad] (rows 0-2 are
 * read), qstep [>= 3], hard_mask [n] (nonzero = kept), all device; n <= npad,
 * n < 2^31.  Outputs (device, sync-free; read the header afterwards):
 * tokens [token_cap] (4-byte aligned, token_cap a multiple of 4; 21 n always
 * suffices); codes [n]: the distinct voxels' Morton codes, ascending (the
 * first `unique`); dup_index / dup_count [dup_cap]: the voxels holding more
 * than one kept Gaussian, ascending, with their copies beyond the first;
 * header: sgs_octree_header. */
sgs_status sgs_octree_encode(sgs_ctx *ctx, const float *params, int64_t npad, int64_t n,
                             const float *qstep, const uint8_t *hard_mask, uint8_t *tokens,
                             int64_t token_cap, uint64_t *codes, uint32_t *dup_index,
                             uint32_t *dup_count, int64_t dup_cap, sgs_octree_header *header);
/* Decode: header (HOST copy of the encoder's), tokens, dup_index /
 * dup_count and qstep (device) give codes [unique] (the distinct voxels'
 * codes, ascending) and xyz [3][out_pad] (out_pad >= kept): the decoded
 * positions fl32((u_c + kmin_c) q_c), voxels in code order, each followed by
 * its copies.  info: device int64[1], bit 0 set when the stream is
 * inconsistent (children that do not match the level sizes, an empty token,
 * duplicate entries out of order or not adding up to kept); outputs are then
 * unspecified but every write stays inside the buffers.  The header itself is
 * checked on the host (SGS_EINVAL). */
sgs_status sgs_octree_decode(sgs_ctx *ctx, const sgs_octree_header *header,
                             const uint8_t *tokens, const uint32_t *dup_index,
                             const uint32_t *dup_count, const float *qstep, uint64_t *codes,
                             float *xyz, int64_t out_pad, int64_t *info);

/* Entropy coder for byte streams (the paper codes the octree tokens with
 * p(t_i | t_{i-1}) and arithmetic coding; here the conditional model is a
 * count table carried with the stream, order 1: context = the previous
 * symbol of the same lane, 256 at a lane's start; or order 0: one context).
 * Model: for each context with counts c_s (K symbols present, N in all),
 * f_s = 1 + floor(c_s (4096 - K) / N) for present symbols, 0 otherwise, and
 * the most frequent symbol (the lowest on ties) takes 4096 - sum f.
 * freq: device uint16 [257][256] (rows of unused contexts 0).
 * Coder: range ANS with a 32-bit state in [2^16, 2^32), 16-bit words and
 * 12-bit frequencies (C(s, x) = floor(x / f_s) 4096 + cum_s + x mod f_s),
 * interleaved over 64 lanes: symbols [64 S b, 64 S (b + 1)) form block b,
 * lane l of it owns the run [64 S b + S l, 64 S b + S (l + 1)) (S =
 * lane_len); the decoder advances the 64 lanes together, one symbol each per
 * step, and after a step the lanes whose state is below 2^16 take the
 * block's next word, in lane order.  Block b's words start with the 64
 * lanes' final states (high half, low half), then its renormalization words
 * in that decoding order; block_off [blocks + 1] (int64, device) are the
 * blocks' word offsets.  n < 2^31; 1 <= lane_len <= 65536; order 0 or 1. */
int64_t sgs_ans_max_words(int64_t n, int32_t lane_len);  /* word capacity that always suffices */
/* Model of sym [n] (device) into freq; ideal_bits (device double, or null):
 * -sum_i log2(f / 4096) of the stream under the model (Eq. loss_geo's rate
 * with the count model's probabilities). */
sgs_status sgs_ans_model(sgs_ctx *ctx, const uint8_t *sym, int64_t n, int32_t order,
                         int32_t lane_len, uint16_t *freq, double *ideal_bits);
/* Encode: words [word_cap] (uint16, device), block_off [blocks + 1]; info:
 * device int64[2] = {words written in all, flags}: flags bit 0 a symbol of
 * frequency 0 in its context, bit 1 word_cap too small (cut), bit 2 a used
 * model row that does not sum to 4096. */
sgs_status sgs_ans_encode(sgs_ctx *ctx, const uint8_t *sym, int64_t n, int32_t order,
                          int32_t lane_len, const uint16_t *freq, uint16_t *words,
                          int64_t word_cap, int64_t *block_off, int64_t *info);
/* Decode n symbols into sym (device) from words [n_words] and block_off;
 * info: device int64[1], bit 0 a malformed stream (a block's words out of
 * range, run out or left over, a slot no symbol owns, a lane not back at
 * the initial state), bit 2 a bad model row. */
sgs_status sgs_ans_decode(sgs_ctx *ctx, const uint16_t *words, int64_t n_words,
                          const int64_t *block_off, int64_t n, int32_t order, int32_t lane_len,
                          const uint16_t *freq, uint8_t *sym, int64_t *info);

/* Several streams decoded in one launch (one wave per block of every
 * stream).  Each descriptor names one stream as sgs_ans_decode takes it;
 * info: device int64[count] of per-stream flags (as sgs_ans_decode's).  The
 * descriptors are read from host memory before the call returns (it
 * synchronizes the context's stream). */
typedef struct {
  const uint16_t *words;     /* device */
  int64_t n_words;
  const int64_t *block_off;  /* device [blocks + 1] */
  int64_t n;                 /* symbols */
  const uint16_t *freq;      /* device [257][256] */
  uint8_t *sym;              /* device [n], output */
  int32_t order;             /* 0 or 1 */
  int32_t lane_len;          /* 1 .. 65536 */
} sgs_ans_stream;
sgs_status sgs_ans_decode_multi(sgs_ctx *ctx, int32_t count, const sgs_ans_stream *streams,
                                int64_t *info);

/* Attributes (Sec. 3.4.2, autoregressive attribute coding): the kept
 * Gaussians are serialized in the Morton order of their voxels, and each
 * token a_i = [colour, opacity, scale, rotation] (channels 3-58) is coded
 * from its predecessor within a group of lane_len Gaussians (the groups
 * decode in parallel).  The paper's conditional model is a causal state
 * space model fed with the decoded attributes and positional embeddings;
 * here each channel takes one of two predictors (predictor [59], HOST bytes,
 * entries 3-58 used; null = 1 for all): 1, the previous token (the residual
 * of the fixed-length coder's value v = k - kmin against the group's
 * previous value, 0 for a group's first, zigzag-mapped: d >= 0 -> 2d,
 * d < 0 -> -2d - 1), or 0, no prediction (v itself).  The result's bytes are
 * entropy-coded as separate streams ("planes", most significant first): a
 * channel of width w bits (the fixed-length coder's, sgs_fl_encode) gives
 * ceil((w + 1) / 8) planes with predictor 1, ceil(w / 8) with 0, none for
 * w = 0.  Plane rows follow the channels in order.
 *
 * Morton order: perm [kept] (device int32) receives the kept Gaussians'
 * indices by voxel code (header: HOST copy of sgs_octree_encode's; codes:
 * its distinct voxel codes, device), Gaussians of one voxel by index. */
sgs_status sgs_morton_order(sgs_ctx *ctx, const float *params, int64_t npad, int64_t n,
                            const float *qstep, const uint8_t *hard_mask,
                            const sgs_octree_header *header, const uint64_t *codes,
                            int32_t *perm);
/* Plane rows of a fixed-length header (HOST sgs_fl_channel[59]) with the
 * given predictors. */
int64_t sgs_attr_plane_rows(const sgs_fl_channel *fl_header, const uint8_t *predictor);
/* Planes: planes [rows][kept] (device bytes) for the Gaussians perm [kept]
 * lists, in that order; fl_header: HOST copy of sgs_fl_encode's for the same
 * parameters, steps and mask. */
sgs_status sgs_attr_planes(sgs_ctx *ctx, const float *params, int64_t npad, const int32_t *perm,
                           int64_t kept, const sgs_fl_channel *fl_header,
                           const uint8_t *predictor, int32_t lane_len, uint8_t *planes);
/* Inverse: out [59][out_pad] (device, out_pad >= kept) rows 3-58 receive the
 * dequantized attributes fl32((kmin + v) q) in serialized order (rows 0-2,
 * the positions, are sgs_octree_decode's xyz). */
sgs_status sgs_attr_reconstruct(sgs_ctx *ctx, const uint8_t *planes, int64_t kept,
                                const sgs_fl_channel *fl_header, const uint8_t *predictor,
                                int32_t lane_len, float *out, int64_t out_pad);
/* Fourier positional embedding (Sec. 3.4.2): PE(mu) = W phi(mu) + b with
 * phi(mu) = [mu; sin(2 pi f_l mu); cos(2 pi f_l mu)], f_l = 2^l for l < L
 * (band-major, axis-minor: feature 3 + 3 l + c is sin of axis c in band l,
 * 3 + 3 L + 3 l + c its cosine), 3 + 6 L features.  xyz [3][pad] (device),
 * W [d][3 + 6L] and b [d] (device FP32), out [count][d] (device FP32, 16-byte
 * aligned).  1 <= L <= 16; d a multiple of 4, at most 64. */
sgs_status sgs_positional_embedding(sgs_ctx *ctx, const float *xyz, int64_t pad, int64_t count,
                                    int32_t L, int32_t d, const float *W, const float *b,
                                    float *out);

/* Kernel-group timing with HIP events recorded on the context's stream around
 * each group's launches (no extra synchronization inside a step).  Groups: */
enum {
  SGS_PROF_FAKEQUANT = 0,  /* a1-a3 quantize, mask, channel statistics */
  SGS_PROF_RATE = 1,       /* a3 rate proxy */
  SGS_PROF_PREPROCESS = 2, /* a4 projection */
  SGS_PROF_DEPTH_SORT = 3, /* a6 depth radix sort of the splats */
  SGS_PROF_SCAN = 4,       /* a5 pair and super-tile item offsets */
  SGS_PROF_DUPLICATE = 5,  /* a5 pair emission: every pair written at its place */
  SGS_PROF_TILE_SORT = 6,  /* a6 super-tile items sorted, per-tile pair counts */
  SGS_PROF_RANGES = 7,     /* a7 tile offsets and ranges */
  SGS_PROF_BLEND_FWD = 8,  /* a8 */
  SGS_PROF_L1 = 9,         /* a9 */
  SGS_PROF_GRAD_CLEAR = 10,/* a10 clearing of the splat-gradient accumulators */
  SGS_PROF_BLEND_BWD = 11, /* a10 */
  SGS_PROF_PREPROCESS_BWD = 12, /* a11 */
  SGS_PROF_FAKEQUANT_BWD = 13,  /* a12 */
  SGS_PROF_MLP_FWD = 14,   /* a13 learned rate, forward / inference */
  SGS_PROF_MLP_BWD = 15,   /* a13 learned rate, backward */
  SGS_PROF_MLP_TRAIN = 16, /* a13 training step */
  SGS_PROF_CODEC = 17,     /* fixed-length encode / decode */
  SGS_PROF_ADAM = 18,      /* optimizer step */
  SGS_PROF_SSIM = 19,      /* SSIM term of the distortion */
  SGS_PROF_OCTREE = 20,    /* octree tokens: encode / decode */
  SGS_PROF_ANS = 21,       /* entropy coder: model, encode, decode */
  SGS_PROF_GROUPS = 22
};
/* enable != 0 starts recording (and clears earlier records); 0 stops. */
sgs_status sgs_profile_enable(sgs_ctx *ctx, int32_t enable);
/* Synchronizes the stream, then returns per group the summed duration in ms
 * and the number of timed launches (host arrays of SGS_PROF_GROUPS entries)
 * and clears the records. */
sgs_status sgs_profile_read(sgs_ctx *ctx, double *ms_total, int64_t *launches);

#ifdef __cplusplus
}
#endif
#endif /* SPEEDYGS_H */
