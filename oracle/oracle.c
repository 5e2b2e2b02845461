/*
 * oracle.c -- plain, slow FP64 CPU oracle for one rate-distortion (RD) step of
 * SpeedyGS's structural-formation stage.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or
 * load this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code, header, table or constant generator
 * with the HIP library.
 *
 * What it computes (paper sections in brackets):
 *   - channel-wise uniform quantization with learnable step q_j
 *     [Sec. 3.3.1, quantized entropy passage and Eq. for L_j]; STE/LSQ backward;
 *   - retention score -> sigmoid -> Gumbel-sigmoid mask, hard mask
 *     [Sec. 3.3.1, Eqs. p_i and M_i, hard mask passage];
 *   - range-based quantization proxy L_j, L_quant, mask loss L_mask and
 *     R_proxy = L_mask * L_quant [Sec. 3.3.1, Eqs. L_j, L_quant, L_mask,
 *     R_proxy]; its gradient;
 *   - 3DGS projection + tile-based front-to-back alpha compositing
 *     [Sec. 3.1, Eq. G(x) and the compositing Eq.]; its hand-derived gradient;
 *   - L1 distortion [Supp. "Training Objective", L1 part];
 *   - channel-wise fixed-length code length [Sec. 3.4.1].
 *
 * Precision.  Continuous quantities are FP64.  Every discrete decision whose
 * outcome the GPU must reproduce bit for bit (quantization codes k, the hard
 * mask, culling, the pixel span of each splat, its tile rectangle and its depth
 * key, the ceil in L_j) is taken in IEEE FP32 with the fixed operation order
 * written out below, using only correctly rounded +, -, *, /, sqrt and the
 * exact rint/ceil/floor/ldexp/min/max.  Build with -ffp-contract=off.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define NCH 59
#define CH_MU 0
#define CH_DC 3
#define CH_REST 6
#define CH_OPA 51
#define CH_SCALE 52
#define CH_ROT 55
#define ORC_PI 3.14159265358979323846
#define ORC_LN2 0.69314718055994530942
#define NSPLATGRAD 10 /* px, py, A, B, C, opacity, r, g, b, mask */

/* blend constants (conventions; the paper does not state them) */
#define NEAR_PLANE 0.2f
#define DILATION 0.3
#define ALPHA_MAX 0.99
#define ALPHA_MIN (1.0 / 255.0)
#define T_MIN 1e-4
#define CLAMP_FOV 1.3

/* margins inside which an FP64 and an FP32 blend may take different
 * per-pair decisions; pixels touching them are reported, not compared */
#define MARGIN_REL 2e-5

typedef struct {
  float R[9], t[3], fx, fy, cx, cy, campos[3];
} orc_cam;

/* ------------------------------------------------------------------------ */
/* Counter-based uniforms: SplitMix64 (Steele, Lea, Flood, OOPSLA 2014).     */
/* ------------------------------------------------------------------------ */
static uint64_t splitmix64(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

/* u in (0,1), exactly representable in FP32: (23-bit integer + 1/2) / 2^23 */
float orc_uniform(uint64_t seed, uint64_t step, uint64_t i) {
  uint64_t h = splitmix64(seed ^ ((step << 32) + i));
  return ((float)(h >> 41) + 0.5f) * 0x1p-23f;
}

/* ------------------------------------------------------------------------ */
/* FP32 exponential for the decision layer.  Cody & Waite (1980) additive    */
/* range reduction x = n ln2 + r, |r| <= ln2/2, then the degree-7 Taylor     */
/* polynomial of e^r in Horner form, then scaling by 2^n.  Input is clamped  */
/* to [-80, 80] so every result is a normal float.                           */
/* ------------------------------------------------------------------------ */
float orc_exp_dl(float x) {
  if (x > 80.0f) x = 80.0f;
  if (x < -80.0f) x = -80.0f;
  const float log2e = 0x1.715476p+0f;  /* 1/ln 2 rounded to float */
  const float ln2_hi = 0x1.62e4p-1f;   /* ln 2 truncated to 16 bits */
  const float ln2_lo = 0x1.7f7d1cp-20f; /* ln 2 - ln2_hi rounded to float */
  float n = rintf(x * log2e);
  float r = (x - n * ln2_hi) - n * ln2_lo;
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

/* ------------------------------------------------------------------------ */
/* a1: fake quantization [Sec. 3.3.1: uniform quantization with step q_j].   */
/* k = rint(y/q) (FP32 division, round half to even), yhat = fl32(k*q).      */
/* ------------------------------------------------------------------------ */
void orc_fakequant(int64_t n, int64_t npad, const float *y, const float *q,
                   float *yhat, int32_t *kout) {
  for (int j = 0; j < NCH; ++j) {
    for (int64_t i = 0; i < n; ++i) {
      float kf = rintf(y[j * npad + i] / q[j]);
      /* the product of two floats is exact in FP64; rounding it once to
         float is the correctly rounded FP32 product */
      yhat[j * npad + i] = (float)((double)kf * (double)q[j]);
      if (kout) kout[j * npad + i] = (int32_t)kf;
    }
  }
}

/* ------------------------------------------------------------------------ */
/* a2: retention mask [Sec. 3.3.1: p_i = sigma(s_i), M_i = GumbelSoftmax,    */
/* hard mask].  Two-class Gumbel-softmax with class logits (log p, log(1-p)) */
/* equals sigma((s + l)/tau) with l = ln u - ln(1-u) logistic noise.  Hard   */
/* mask M = [s + l > 0], decided in FP32 as  u * (1 + e^s) > 1.             */
/* mode 0: given mask, 1: Gumbel, 2: keep all.                              */
/* ------------------------------------------------------------------------ */
void orc_mask(int64_t n, int mode, const uint8_t *given, const float *score,
              uint64_t seed, uint64_t step, double tau, uint8_t *mhat,
              double *msoft) {
  for (int64_t i = 0; i < n; ++i) {
    if (mode == 0) {
      mhat[i] = given[i] ? 1 : 0;
      msoft[i] = (double)mhat[i];
    } else if (mode == 2) {
      mhat[i] = 1;
      msoft[i] = 1.0;
    } else {
      float u = orc_uniform(seed, step, (uint64_t)i);
      float e = orc_exp_dl(score[i]);
      float lhs = u * (1.0f + e);
      mhat[i] = lhs > 1.0f ? 1 : 0;
      double l = log((double)u) - log(1.0 - (double)u);
      msoft[i] = 1.0 / (1.0 + exp(-((double)score[i] + l) / tau));
    }
  }
}

/* ------------------------------------------------------------------------ */
/* a3: rate proxy [Sec. 3.3.1, Eqs. L_j, L_quant, L_mask, R_proxy].          */
/* Range over the raw parameters of all N Gaussians; lowest index wins ties. */
/* c_j = ceil(fl32(fl32(max-min)/q_j)), at least 1; L_j = log2 c_j.          */
/* Gradient (straight through the ceil): dL_j/dR_j = 1/(c_j q_j ln2),        */
/* dL_j/dq_j = -R_j/(c_j q_j^2 ln2), zero when R_j = 0.                      */
/* out3 = {R, L_quant, L_mask}.  With lam != 0 the gradient of lam*R is      */
/* ADDED into gy (raw parameters), gq and gm (hard mask).                    */
/* ------------------------------------------------------------------------ */
void orc_rate_proxy(int64_t n, int64_t npad, const float *y, const float *q,
                    const uint8_t *mhat, int64_t n_hat, double lam,
                    double *out3, int32_t *argmin, int32_t *argmax,
                    double *cj, double *gy, double *gq, double *gm) {
  double Lq = 0.0;
  double dLdR[NCH], dLdq[NCH];
  for (int j = 0; j < NCH; ++j) {
    int64_t imin = 0, imax = 0;
    for (int64_t i = 1; i < n; ++i) {
      if (y[j * npad + i] < y[j * npad + imin]) imin = i;
      if (y[j * npad + i] > y[j * npad + imax]) imax = i;
    }
    argmin[j] = (int32_t)imin;
    argmax[j] = (int32_t)imax;
    float ymin = y[j * npad + imin], ymax = y[j * npad + imax];
    float Rf = ymax - ymin;
    float x = Rf / q[j];
    double c = 1.0;
    if (Rf > 0.0f) {
      float cf = ceilf(x);
      c = cf < 1.0f ? 1.0 : (double)cf;
    }
    cj[j] = c;
    Lq += log2(c);
    double R = (double)ymax - (double)ymin;
    if (R > 0.0) {
      dLdR[j] = 1.0 / (c * (double)q[j] * ORC_LN2);
      dLdq[j] = -R / (c * (double)q[j] * (double)q[j] * ORC_LN2);
    } else {
      dLdR[j] = 0.0;
      dLdq[j] = 0.0;
    }
  }
  int64_t kept = 0;
  for (int64_t i = 0; i < n; ++i) kept += mhat[i] ? 1 : 0;
  double Lm = (double)kept / (double)n_hat;
  out3[0] = Lm * Lq;
  out3[1] = Lq;
  out3[2] = Lm;
  if (lam != 0.0) {
    for (int j = 0; j < NCH; ++j) {
      if (gy) {
        gy[j * npad + argmax[j]] += lam * Lm * dLdR[j];
        gy[j * npad + argmin[j]] -= lam * Lm * dLdR[j];
      }
      if (gq) gq[j] += lam * Lm * dLdq[j];
    }
    if (gm)
      for (int64_t i = 0; i < n; ++i) gm[i] += lam * Lq / (double)n_hat;
  }
}

/* ------------------------------------------------------------------------ */
/* a12: quantizer + mask backward.  Straight-through: dy = dyhat.  Step size */
/* (learned step size quantization, Esser et al. 2020):                      */
/*   dq_j = sum_i dyhat_ij (k_ij - y_ij/q_j).                                */
/* Mask score (Gumbel mode only): ds_i = dM_i * Ms_i (1 - Ms_i) / tau.       */
/* Outputs are overwritten.                                                  */
/* ------------------------------------------------------------------------ */
void orc_fakequant_bwd(int64_t n, int64_t npad, const float *y, const float *q,
                       const double *gyhat, int mode, const double *msoft,
                       double tau, const double *gmhat, double *gy, double *gq,
                       double *gs) {
  for (int j = 0; j < NCH; ++j) {
    double acc = 0.0;
    for (int64_t i = 0; i < n; ++i) {
      double g = gyhat[j * npad + i];
      gy[j * npad + i] = g;
      float kf = rintf(y[j * npad + i] / q[j]);
      acc += g * ((double)kf - (double)y[j * npad + i] / (double)q[j]);
    }
    gq[j] = acc;
  }
  for (int64_t i = 0; i < n; ++i)
    gs[i] = (mode == 1) ? gmhat[i] * msoft[i] * (1.0 - msoft[i]) / tau : 0.0;
}

/* ------------------------------------------------------------------------ */
/* Decision layer of the projection (FP32, fixed operation order).          */
/* Outputs per (view, Gaussian): valid flag, depth t_z, projected mean,      */
/* radius r = ceil(3 sqrt(lambda_max)), inclusive pixel span [x0,x1]x[y0,y1] */
/* = pixels with |u - px| <= r and |v - py| <= r, and the tile count.        */
/* ------------------------------------------------------------------------ */
typedef struct {
  int valid;
  float tz, pxf, pyf;
  int r, x0, x1, y0, y1;
} dl_out;

static void dl_project(const float *p, int64_t npad, int64_t i,
                       const orc_cam *c, int W, int H, dl_out *o) {
  memset(o, 0, sizeof(*o));
  float mx = p[0 * npad + i], my = p[1 * npad + i], mz = p[2 * npad + i];
  float tx = ((c->R[0] * mx + c->R[1] * my) + c->R[2] * mz) + c->t[0];
  float ty = ((c->R[3] * mx + c->R[4] * my) + c->R[5] * mz) + c->t[1];
  float tz = ((c->R[6] * mx + c->R[7] * my) + c->R[8] * mz) + c->t[2];
  o->tz = tz;
  if (!(tz > NEAR_PLANE)) return;
  float qw = p[(CH_ROT + 0) * npad + i], qx = p[(CH_ROT + 1) * npad + i];
  float qy = p[(CH_ROT + 2) * npad + i], qz = p[(CH_ROT + 3) * npad + i];
  float qq = ((qw * qw + qx * qx) + qy * qy) + qz * qz;
  if (!(qq > 0.0f)) return;
  float qn = sqrtf(qq);
  qw = qw / qn; qx = qx / qn; qy = qy / qn; qz = qz / qn;
  float Rq[9];
  Rq[0] = 1.0f - 2.0f * (qy * qy + qz * qz);
  Rq[1] = 2.0f * (qx * qy - qw * qz);
  Rq[2] = 2.0f * (qx * qz + qw * qy);
  Rq[3] = 2.0f * (qx * qy + qw * qz);
  Rq[4] = 1.0f - 2.0f * (qx * qx + qz * qz);
  Rq[5] = 2.0f * (qy * qz - qw * qx);
  Rq[6] = 2.0f * (qx * qz - qw * qy);
  Rq[7] = 2.0f * (qy * qz + qw * qx);
  Rq[8] = 1.0f - 2.0f * (qx * qx + qy * qy);
  float S[3];
  for (int k = 0; k < 3; ++k) S[k] = orc_exp_dl(p[(CH_SCALE + k) * npad + i]);
  float M[9];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) M[a * 3 + b] = Rq[a * 3 + b] * S[b];
  float Sg[9];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b)
      Sg[a * 3 + b] = (M[a * 3 + 0] * M[b * 3 + 0] + M[a * 3 + 1] * M[b * 3 + 1]) +
                      M[a * 3 + 2] * M[b * 3 + 2];
  float limx = 1.3f * ((0.5f * (float)W) / c->fx);
  float limy = 1.3f * ((0.5f * (float)H) / c->fy);
  float ux = tx / tz, uy = ty / tz;
  float cux = fminf(limx, fmaxf(-limx, ux));
  float cuy = fminf(limy, fmaxf(-limy, uy));
  float J00 = c->fx / tz, J02 = -(c->fx * cux) / tz;
  float J11 = c->fy / tz, J12 = -(c->fy * cuy) / tz;
  float T0[3], T1[3];
  for (int b = 0; b < 3; ++b) {
    T0[b] = J00 * c->R[0 * 3 + b] + J02 * c->R[2 * 3 + b];
    T1[b] = J11 * c->R[1 * 3 + b] + J12 * c->R[2 * 3 + b];
  }
  float u[3], w[3];
  for (int a = 0; a < 3; ++a) {
    u[a] = (Sg[a * 3 + 0] * T0[0] + Sg[a * 3 + 1] * T0[1]) + Sg[a * 3 + 2] * T0[2];
    w[a] = (Sg[a * 3 + 0] * T1[0] + Sg[a * 3 + 1] * T1[1]) + Sg[a * 3 + 2] * T1[2];
  }
  float ca = ((T0[0] * u[0] + T0[1] * u[1]) + T0[2] * u[2]) + 0.3f;
  float cb = (T0[0] * w[0] + T0[1] * w[1]) + T0[2] * w[2];
  float cc = ((T1[0] * w[0] + T1[1] * w[1]) + T1[2] * w[2]) + 0.3f;
  float det = ca * cc - cb * cb;
  if (!(det > 0.0f)) return;
  float mid = 0.5f * (ca + cc);
  float disc = mid * mid - det;
  if (disc < 0.0f) disc = 0.0f;
  float lmax = mid + sqrtf(disc);
  float rf = ceilf(3.0f * sqrtf(lmax));
  float pxf = c->fx * ux + c->cx;
  float pyf = c->fy * uy + c->cy;
  o->pxf = pxf;
  o->pyf = pyf;
  float xlo = ceilf(pxf - rf), xhi = floorf(pxf + rf);
  float ylo = ceilf(pyf - rf), yhi = floorf(pyf + rf);
  if (xhi < 0.0f || xlo > (float)(W - 1) || yhi < 0.0f || ylo > (float)(H - 1)) return;
  o->x0 = xlo < 0.0f ? 0 : (int)xlo;
  o->x1 = xhi > (float)(W - 1) ? W - 1 : (int)xhi;
  o->y0 = ylo < 0.0f ? 0 : (int)ylo;
  o->y1 = yhi > (float)(H - 1) ? H - 1 : (int)yhi;
  o->r = rf > 1e9f ? 1000000000 : (int)rf;
  o->valid = 1;
}

/* Decision layer for all (view, Gaussian).  Arrays are [V][n]. */
void orc_decide(int64_t n, int64_t npad, const float *yhat, int32_t V,
                const float *cams, int32_t W, int32_t H, int32_t TW, int32_t TH,
                int32_t *valid, float *tz, float *pxy, int32_t *span,
                int32_t *radius, int32_t *tiles) {
  for (int v = 0; v < V; ++v) {
    const orc_cam *c = (const orc_cam *)(cams + 19 * v);
    for (int64_t i = 0; i < n; ++i) {
      dl_out o;
      dl_project(yhat, npad, i, c, W, H, &o);
      int64_t s = (int64_t)v * n + i;
      valid[s] = o.valid;
      tz[s] = o.tz;
      pxy[2 * s] = o.pxf;
      pxy[2 * s + 1] = o.pyf;
      span[4 * s + 0] = o.x0;
      span[4 * s + 1] = o.x1;
      span[4 * s + 2] = o.y0;
      span[4 * s + 3] = o.y1;
      radius[s] = o.r;
      tiles[s] = o.valid ? (o.x1 / TW - o.x0 / TW + 1) * (o.y1 / TH - o.y0 / TH + 1) : 0;
    }
  }
}

/* ------------------------------------------------------------------------ */
/* a5-a7: tile binning and the (tile, depth) order [Sec. 3.1: tile-based     */
/* rasterization, Gaussians sorted by depth].  Every (tile, Gaussian) pair   */
/* whose pixel span meets the tile is listed; pairs are ordered by global    */
/* tile id, then by the bits of t_z (positive floats order like their bits), */
/* then by Gaussian index.  ranges[t] = [first, end) of tile t.              */
/* ------------------------------------------------------------------------ */
typedef struct {
  uint64_t key;
  uint32_t val;
} pair_t;

static int pair_cmp(const void *a, const void *b) {
  const pair_t *x = (const pair_t *)a, *y = (const pair_t *)b;
  if (x->key != y->key) return x->key < y->key ? -1 : 1;
  if (x->val != y->val) return x->val < y->val ? -1 : 1;
  return 0;
}

int64_t orc_bin(int64_t n, int32_t V, const int32_t *valid, const float *tz,
                const int32_t *span, int32_t W, int32_t H, int32_t TW,
                int32_t TH, uint64_t *keys, uint32_t *vals, uint32_t *ranges) {
  int GW = (W + TW - 1) / TW, GH = (H + TH - 1) / TH;
  int64_t tiles_per_view = (int64_t)GW * GH;
  int64_t P = 0;
  for (int64_t s = 0; s < (int64_t)V * n; ++s)
    if (valid[s])
      P += (int64_t)(span[4 * s + 1] / TW - span[4 * s] / TW + 1) *
           (span[4 * s + 3] / TH - span[4 * s + 2] / TH + 1);
  if (!keys) return P;
  pair_t *pr = (pair_t *)malloc(sizeof(pair_t) * (size_t)(P > 0 ? P : 1));
  int64_t k = 0;
  for (int v = 0; v < V; ++v)
    for (int64_t i = 0; i < n; ++i) {
      int64_t s = (int64_t)v * n + i;
      if (!valid[s]) continue;
      uint32_t bits;
      memcpy(&bits, &tz[s], 4);
      for (int ty = span[4 * s + 2] / TH; ty <= span[4 * s + 3] / TH; ++ty)
        for (int tx = span[4 * s] / TW; tx <= span[4 * s + 1] / TW; ++tx) {
          uint64_t tile = (uint64_t)v * tiles_per_view + (uint64_t)ty * GW + tx;
          pr[k].key = (tile << 32) | bits;
          pr[k].val = (uint32_t)i;
          ++k;
        }
    }
  qsort(pr, (size_t)P, sizeof(pair_t), pair_cmp);
  for (int64_t t = 0; t < V * tiles_per_view; ++t) ranges[2 * t] = ranges[2 * t + 1] = 0;
  for (int64_t e = 0; e < P; ++e) {
    keys[e] = pr[e].key;
    vals[e] = pr[e].val;
    uint64_t t = pr[e].key >> 32;
    if (e == 0 || (pr[e - 1].key >> 32) != t) ranges[2 * t] = (uint32_t)e;
    ranges[2 * t + 1] = (uint32_t)(e + 1);
  }
  free(pr);
  return P;
}

/* ------------------------------------------------------------------------ */
/* Real spherical harmonics up to degree 3, orthonormal on the sphere with   */
/* the Condon-Shortley phase, index k = l^2 + l + m.  Built once from the    */
/* definitions: Legendre polynomials by Rodrigues' formula, associated       */
/* functions by differentiation, (x + iy)^m for the azimuth, and            */
/* K_l^m = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!).  Stored as polynomials in the  */
/* components of the unit direction: coef[k][a][b][c] x^a y^b z^c.           */
/* ------------------------------------------------------------------------ */
static double sh_coef[16][4][4][4];
static int sh_ready = 0;

static double fact(int k) {
  double f = 1.0;
  for (int i = 2; i <= k; ++i) f *= i;
  return f;
}
static double binom(int n, int k) { return fact(n) / (fact(k) * fact(n - k)); }

static void sh_build(void) {
  memset(sh_coef, 0, sizeof(sh_coef));
  for (int l = 0; l <= 3; ++l) {
    /* (z^2 - 1)^l, coefficients by power of z */
    double base[8] = {0};
    for (int k = 0; k <= l; ++k) base[2 * k] = binom(l, k) * ((l - k) % 2 ? -1.0 : 1.0);
    /* differentiate l times and divide by 2^l l!  ->  P_l */
    double P[8];
    memcpy(P, base, sizeof(P));
    for (int d = 0; d < l; ++d) {
      for (int e = 0; e < 7; ++e) P[e] = P[e + 1] * (e + 1);
      P[7] = 0.0;
    }
    for (int e = 0; e < 8; ++e) P[e] /= pow(2.0, l) * fact(l);
    for (int m = 0; m <= l; ++m) {
      /* (-1)^m d^m P_l / dz^m: associated Legendre without sin^m theta */
      double Pm[8];
      memcpy(Pm, P, sizeof(Pm));
      for (int d = 0; d < m; ++d) {
        for (int e = 0; e < 7; ++e) Pm[e] = Pm[e + 1] * (e + 1);
        Pm[7] = 0.0;
      }
      double sgn = (m % 2) ? -1.0 : 1.0;
      double K = sqrt((2.0 * l + 1.0) / (4.0 * ORC_PI) * fact(l - m) / fact(l + m));
      double norm = (m == 0) ? K : sqrt(2.0) * K;
      /* Re and Im of (x + iy)^m = sum_j C(m,j) x^(m-j) (iy)^j */
      for (int jj = 0; jj <= m; ++jj) {
        double bc = binom(m, jj);
        /* i^jj: jj%4 = 0 -> 1, 1 -> i, 2 -> -1, 3 -> -i */
        double re = 0.0, im = 0.0;
        switch (jj % 4) {
          case 0: re = 1.0; break;
          case 1: im = 1.0; break;
          case 2: re = -1.0; break;
          default: im = -1.0; break;
        }
        for (int e = 0; e <= l - m; ++e) {
          if (Pm[e] == 0.0) continue;
          int kp = l * l + l + m, kn = l * l + l - m;
          if (re != 0.0) sh_coef[kp][m - jj][jj][e] += norm * sgn * Pm[e] * bc * re;
          if (m > 0 && im != 0.0) sh_coef[kn][m - jj][jj][e] += norm * sgn * Pm[e] * bc * im;
        }
      }
    }
  }
  sh_ready = 1;
}

static double ipow(double x, int k) {
  double r = 1.0;
  for (int i = 0; i < k; ++i) r *= x;
  return r;
}

/* values and gradients (w.r.t. the direction components) of the 16 basis
   functions at direction d */
static void sh_eval(const double d[3], double Y[16], double dY[16][3]) {
  if (!sh_ready) sh_build();
  for (int k = 0; k < 16; ++k) {
    double v = 0.0, gx = 0.0, gy = 0.0, gz = 0.0;
    for (int a = 0; a < 4; ++a)
      for (int b = 0; b < 4; ++b)
        for (int c = 0; c < 4; ++c) {
          double co = sh_coef[k][a][b][c];
          if (co == 0.0) continue;
          v += co * ipow(d[0], a) * ipow(d[1], b) * ipow(d[2], c);
          if (a) gx += co * a * ipow(d[0], a - 1) * ipow(d[1], b) * ipow(d[2], c);
          if (b) gy += co * b * ipow(d[0], a) * ipow(d[1], b - 1) * ipow(d[2], c);
          if (c) gz += co * c * ipow(d[0], a) * ipow(d[1], b) * ipow(d[2], c - 1);
        }
    Y[k] = v;
    if (dY) {
      dY[k][0] = gx;
      dY[k][1] = gy;
      dY[k][2] = gz;
    }
  }
}

/* exported for the quadrature pin: basis values at n directions */
void orc_sh_basis(int64_t n, const double *dirs, double *Y) {
  for (int64_t i = 0; i < n; ++i) sh_eval(dirs + 3 * i, Y + 16 * i, NULL);
}

/* ------------------------------------------------------------------------ */
/* FP64 projection of one Gaussian into one view [Sec. 3.1].  Continuous    */
/* quantities only; the structure comes from the decision layer.           */
/*   Sigma = Rq diag(e^{2s}) Rq^T, t = W mu + t0,                            */
/*   J = [[fx/tz, 0, -fx cx(tx/tz)/tz], [0, fy/tz, -fy cy(ty/tz)/tz]]        */
/*   (cx, cy clamp the direction to 1.3x the half field of view),            */
/*   Sigma' = J W Sigma W^T J^T + 0.3 I,  conic = Sigma'^-1,                  */
/*   mean2D = (fx tx/tz + cx, fy ty/tz + cy),                                */
/*   colour = max(0, sum_k f_k Y_k(dir) + 1/2), dir = unit(mu - campos),     */
/*   opacity = sigmoid(o).                                                   */
/* ------------------------------------------------------------------------ */
typedef struct {
  double px, py, A, B, C, opa, col[3];
  int clampc[3];
} pj64;

typedef struct {
  /* intermediates kept for the backward pass */
  double mu[3], t[3], qh[4], qn, Rq[9], S[3], M[9], Sig[9];
  double ux, uy, cux, cuy, limx, limy;
  int clx, cly;
  double J00, J02, J11, J12, T0[3], T1[3], a, b, c, det;
  double dir[3], dist, Y[16], dY[16][3];
} pj64_tmp;

static void proj64(const double *p, int64_t npad, int64_t i, const orc_cam *c,
                   int W, int H, pj64 *o, pj64_tmp *m) {
  double Rc[9];
  for (int k = 0; k < 9; ++k) Rc[k] = c->R[k];
  double fx = c->fx, fy = c->fy;
  for (int k = 0; k < 3; ++k) m->mu[k] = p[k * npad + i];
  for (int a = 0; a < 3; ++a)
    m->t[a] = Rc[3 * a] * m->mu[0] + Rc[3 * a + 1] * m->mu[1] + Rc[3 * a + 2] * m->mu[2] + c->t[a];
  double q[4];
  for (int k = 0; k < 4; ++k) q[k] = p[(CH_ROT + k) * npad + i];
  m->qn = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  for (int k = 0; k < 4; ++k) m->qh[k] = q[k] / m->qn;
  double w = m->qh[0], x = m->qh[1], y = m->qh[2], z = m->qh[3];
  double *Rq = m->Rq;
  Rq[0] = 1 - 2 * (y * y + z * z); Rq[1] = 2 * (x * y - w * z); Rq[2] = 2 * (x * z + w * y);
  Rq[3] = 2 * (x * y + w * z); Rq[4] = 1 - 2 * (x * x + z * z); Rq[5] = 2 * (y * z - w * x);
  Rq[6] = 2 * (x * z - w * y); Rq[7] = 2 * (y * z + w * x); Rq[8] = 1 - 2 * (x * x + y * y);
  for (int k = 0; k < 3; ++k) m->S[k] = exp(p[(CH_SCALE + k) * npad + i]);
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) m->M[3 * a + b] = Rq[3 * a + b] * m->S[b];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      double s = 0;
      for (int k = 0; k < 3; ++k) s += m->M[3 * a + k] * m->M[3 * b + k];
      m->Sig[3 * a + b] = s;
    }
  double tz = m->t[2];
  m->limx = CLAMP_FOV * (0.5 * W / fx);
  m->limy = CLAMP_FOV * (0.5 * H / fy);
  m->ux = m->t[0] / tz;
  m->uy = m->t[1] / tz;
  m->clx = (m->ux < -m->limx || m->ux > m->limx);
  m->cly = (m->uy < -m->limy || m->uy > m->limy);
  m->cux = m->clx ? (m->ux < 0 ? -m->limx : m->limx) : m->ux;
  m->cuy = m->cly ? (m->uy < 0 ? -m->limy : m->limy) : m->uy;
  m->J00 = fx / tz; m->J02 = -fx * m->cux / tz;
  m->J11 = fy / tz; m->J12 = -fy * m->cuy / tz;
  for (int b = 0; b < 3; ++b) {
    m->T0[b] = m->J00 * Rc[b] + m->J02 * Rc[6 + b];
    m->T1[b] = m->J11 * Rc[3 + b] + m->J12 * Rc[6 + b];
  }
  double sa = 0, sb = 0, sc = 0;
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      sa += m->T0[a] * m->Sig[3 * a + b] * m->T0[b];
      sb += m->T0[a] * m->Sig[3 * a + b] * m->T1[b];
      sc += m->T1[a] * m->Sig[3 * a + b] * m->T1[b];
    }
  m->a = sa + DILATION; m->b = sb; m->c = sc + DILATION;
  m->det = m->a * m->c - m->b * m->b;
  o->A = m->c / m->det;
  o->B = -m->b / m->det;
  o->C = m->a / m->det;
  o->px = fx * m->ux + c->cx;
  o->py = fy * m->uy + c->cy;
  double ol = p[CH_OPA * npad + i];
  o->opa = 1.0 / (1.0 + exp(-ol));
  double v[3];
  for (int k = 0; k < 3; ++k) v[k] = m->mu[k] - (double)c->campos[k];
  m->dist = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
  for (int k = 0; k < 3; ++k) m->dir[k] = v[k] / m->dist;
  sh_eval(m->dir, m->Y, m->dY);
  for (int ch = 0; ch < 3; ++ch) {
    double s = 0.5;
    for (int k = 0; k < 16; ++k) {
      int chan = k == 0 ? CH_DC + ch : CH_REST + 3 * (k - 1) + ch;
      s += p[chan * npad + i] * m->Y[k];
    }
    o->clampc[ch] = s < 0.0;
    o->col[ch] = s < 0.0 ? 0.0 : s;
  }
}

/* Backward of proj64: g = d loss / d(px, py, A, B, C, opacity, r, g, b).
   Adds d loss / d p[.][i] into gp.  Matrix-form derivation:
     conic Q = Sigma'^-1:  dL/dSigma' = -Q G_Q Q,  G_Q = [[gA, gB/2],[gB/2, gC]]
     Sigma' = T Sig T^T:   dL/dT = 2 G T Sig,  dL/dSig = T^T G T
     Sig = M M^T:          dL/dM = 2 dL/dSig M
     M = Rq diag(S):       dL/dRq_ab = dL/dM_ab S_b,  dL/dS_b = sum_a dL/dM_ab Rq_ab
     qh = q/|q|:           dL/dq = (dL/dqh - qh (qh . dL/dqh)) / |q|                */
static void proj64_bwd(const double *p, int64_t npad, int64_t i,
                       const orc_cam *c, const pj64 *o, const pj64_tmp *m,
                       const double g[9], double *gp) {
  double fx = c->fx, fy = c->fy;
  double Rc[9];
  for (int k = 0; k < 9; ++k) Rc[k] = c->R[k];
  double gmu[3] = {0, 0, 0}, gt[3] = {0, 0, 0};
  /* opacity */
  gp[CH_OPA * npad + i] += g[5] * o->opa * (1.0 - o->opa);
  /* colour */
  double gdir[3] = {0, 0, 0};
  for (int ch = 0; ch < 3; ++ch) {
    if (o->clampc[ch]) continue;
    double gc = g[6 + ch];
    for (int k = 0; k < 16; ++k) {
      int chan = k == 0 ? CH_DC + ch : CH_REST + 3 * (k - 1) + ch;
      gp[chan * npad + i] += gc * m->Y[k];
      double f = p[chan * npad + i];
      for (int e = 0; e < 3; ++e) gdir[e] += gc * f * m->dY[k][e];
    }
  }
  double dd = gdir[0] * m->dir[0] + gdir[1] * m->dir[1] + gdir[2] * m->dir[2];
  for (int e = 0; e < 3; ++e) gmu[e] += (gdir[e] - m->dir[e] * dd) / m->dist;
  /* conic -> Sigma' */
  double Q[4] = {o->A, o->B, o->B, o->C};
  double GQ[4] = {g[2], 0.5 * g[3], 0.5 * g[3], g[4]};
  double QG[4], GS[4];
  for (int r = 0; r < 2; ++r)
    for (int s = 0; s < 2; ++s) QG[2 * r + s] = Q[2 * r] * GQ[s] + Q[2 * r + 1] * GQ[2 + s];
  for (int r = 0; r < 2; ++r)
    for (int s = 0; s < 2; ++s) GS[2 * r + s] = -(QG[2 * r] * Q[s] + QG[2 * r + 1] * Q[2 + s]);
  /* Sigma' = T Sig T^T (T rows T0, T1) */
  double T[6] = {m->T0[0], m->T0[1], m->T0[2], m->T1[0], m->T1[1], m->T1[2]};
  double gT[6], gSig[9];
  for (int r = 0; r < 2; ++r)
    for (int b = 0; b < 3; ++b) {
      double s = 0;
      for (int r2 = 0; r2 < 2; ++r2)
        for (int a = 0; a < 3; ++a) s += GS[2 * r + r2] * T[3 * r2 + a] * m->Sig[3 * a + b];
      gT[3 * r + b] = 2.0 * s;
    }
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      double s = 0;
      for (int r = 0; r < 2; ++r)
        for (int r2 = 0; r2 < 2; ++r2) s += T[3 * r + a] * GS[2 * r + r2] * T[3 * r2 + b];
      gSig[3 * a + b] = s;
    }
  /* Sig = M M^T */
  double gM[9];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      double s = 0;
      for (int k = 0; k < 3; ++k) s += gSig[3 * a + k] * m->M[3 * k + b];
      gM[3 * a + b] = 2.0 * s;
    }
  double gRq[9], gS[3] = {0, 0, 0};
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      gRq[3 * a + b] = gM[3 * a + b] * m->S[b];
      gS[b] += gM[3 * a + b] * m->Rq[3 * a + b];
    }
  for (int k = 0; k < 3; ++k) gp[(CH_SCALE + k) * npad + i] += gS[k] * m->S[k];
  /* rotation matrix of the unit quaternion (w, x, y, z) */
  double w = m->qh[0], x = m->qh[1], y = m->qh[2], z = m->qh[3];
  /* dRq_ab / d(w, x, y, z) */
  double D[9][4] = {
      {0, 0, -4 * y, -4 * z},         {-2 * z, 2 * y, 2 * x, -2 * w}, {2 * y, 2 * z, 2 * w, 2 * x},
      {2 * z, 2 * y, 2 * x, 2 * w},   {0, -4 * x, 0, -4 * z},         {-2 * x, -2 * w, 2 * z, 2 * y},
      {-2 * y, 2 * z, -2 * w, 2 * x}, {2 * x, 2 * w, 2 * z, 2 * y},   {0, -4 * x, -4 * y, 0}};
  double gqh[4] = {0, 0, 0, 0};
  for (int e = 0; e < 9; ++e)
    for (int k = 0; k < 4; ++k) gqh[k] += gRq[e] * D[e][k];
  double qd = gqh[0] * m->qh[0] + gqh[1] * m->qh[1] + gqh[2] * m->qh[2] + gqh[3] * m->qh[3];
  for (int k = 0; k < 4; ++k) gp[(CH_ROT + k) * npad + i] += (gqh[k] - m->qh[k] * qd) / m->qn;
  /* T = J Rc:  T0 = J00 Rc0 + J02 Rc2,  T1 = J11 Rc1 + J12 Rc2 */
  double gJ00 = 0, gJ02 = 0, gJ11 = 0, gJ12 = 0;
  for (int b = 0; b < 3; ++b) {
    gJ00 += gT[b] * Rc[b];
    gJ02 += gT[b] * Rc[6 + b];
    gJ11 += gT[3 + b] * Rc[3 + b];
    gJ12 += gT[3 + b] * Rc[6 + b];
  }
  double tx = m->t[0], ty = m->t[1], tz = m->t[2];
  gt[2] += gJ00 * (-fx / (tz * tz)) + gJ11 * (-fy / (tz * tz));
  if (!m->clx) {
    gt[0] += gJ02 * (-fx / (tz * tz));
    gt[2] += gJ02 * (2.0 * fx * tx / (tz * tz * tz));
  } else {
    gt[2] += gJ02 * (fx * m->cux / (tz * tz));
  }
  if (!m->cly) {
    gt[1] += gJ12 * (-fy / (tz * tz));
    gt[2] += gJ12 * (2.0 * fy * ty / (tz * tz * tz));
  } else {
    gt[2] += gJ12 * (fy * m->cuy / (tz * tz));
  }
  /* mean2D */
  gt[0] += g[0] * fx / tz;
  gt[2] += g[0] * (-fx * tx / (tz * tz));
  gt[1] += g[1] * fy / tz;
  gt[2] += g[1] * (-fy * ty / (tz * tz));
  /* t = Rc mu + t0 */
  for (int k = 0; k < 3; ++k) gmu[k] += Rc[k] * gt[0] + Rc[3 + k] * gt[1] + Rc[6 + k] * gt[2];
  for (int k = 0; k < 3; ++k) gp[k * npad + i] += gmu[k];
}

/* ------------------------------------------------------------------------ */
/* a8: per-pixel front-to-back compositing [Sec. 3.1, compositing Eq.]       */
/* over an ordered candidate list.  Per candidate j (in-support only):       */
/*   power = -(A dx^2 + C dy^2)/2 - B dx dy, d = pixel - mean2D;             */
/*   skip if power > 0;  alpha = min(0.99, opacity e^power);  skip if        */
/*   alpha < 1/255;  a~ = M alpha (masked rasterization);  stop, without     */
/*   blending j, if T (1 - a~) < 1e-4;  else C += c a~ T, T *= (1 - a~).     */
/* Returns the number of list entries consumed (the stop position, or the   */
/* list length) and the number of in-support evaluations.                   */
/* ------------------------------------------------------------------------ */
typedef struct {
  const pj64 *pj;      /* [V*n] FP64 projections */
  const int32_t *span; /* [V*n][4] */
  const double *mask;  /* [n] hard mask as a multiplier */
  int64_t n;
} blend_ctx;

typedef struct {
  int64_t j; /* list position */
  double alpha, at, T, G, opa;
  int clamped;
} blend_rec;

static int in_span(const int32_t *sp, int u, int v) {
  return u >= sp[0] && u <= sp[1] && v >= sp[2] && v <= sp[3];
}

static int64_t blend_pixel(const blend_ctx *bc, int view, int u, int v,
                           const uint32_t *list, int64_t cnt, double col[3],
                           double *Tout, int64_t *evals, int *margin,
                           blend_rec *recs, int64_t *nrec) {
  double T = 1.0;
  col[0] = col[1] = col[2] = 0.0;
  int64_t nr = 0;
  int64_t j;
  for (j = 0; j < cnt; ++j) {
    int64_t s = (int64_t)view * bc->n + list[j];
    if (!in_span(bc->span + 4 * s, u, v)) continue;
    ++*evals;
    const pj64 *g = &bc->pj[s];
    double dx = u - g->px, dy = v - g->py;
    double power = -0.5 * (g->A * dx * dx + g->C * dy * dy) - g->B * dx * dy;
    if (power > 0.0) continue;
    double G = exp(power);
    double raw = g->opa * G;
    if (fabs(raw / ALPHA_MAX - 1.0) < MARGIN_REL) *margin = 1;
    int clamped = raw > ALPHA_MAX;
    double alpha = clamped ? ALPHA_MAX : raw;
    if (fabs(alpha / ALPHA_MIN - 1.0) < MARGIN_REL) *margin = 1;
    if (alpha < ALPHA_MIN) continue;
    double at = bc->mask[list[j]] * alpha;
    double Tn = T * (1.0 - at);
    if (fabs(Tn / T_MIN - 1.0) < MARGIN_REL) *margin = 1;
    if (Tn < T_MIN) break;
    if (recs) {
      blend_rec *r = &recs[nr];
      r->j = j; r->alpha = alpha; r->at = at; r->T = T; r->G = G;
      r->opa = g->opa; r->clamped = clamped;
    }
    ++nr;
    for (int ch = 0; ch < 3; ++ch) col[ch] += g->col[ch] * at * T;
    T = Tn;
  }
  *Tout = T;
  if (nrec) *nrec = nr;
  return j;
}

static pj64 *project_all(int64_t n, int64_t npad, const double *p, int32_t V,
                         const float *cams, int W, int H, const int32_t *valid,
                         pj64_tmp *tmp_out) {
  pj64 *pj = (pj64 *)calloc((size_t)(V * n), sizeof(pj64));
  for (int v = 0; v < V; ++v) {
    const orc_cam *c = (const orc_cam *)(cams + 19 * v);
    for (int64_t i = 0; i < n; ++i) {
      int64_t s = (int64_t)v * n + i;
      if (!valid[s]) continue;
      pj64_tmp m;
      proj64(p, npad, i, c, W, H, &pj[s], tmp_out ? &tmp_out[s] : &m);
    }
  }
  return pj;
}

/* Binned forward over the tile lists of orc_bin.
   image [V][3][H][W], Tfinal/last/margin [V][H][W]. Returns total evals. */
int64_t orc_forward(int64_t n, int64_t npad, const double *p, const double *mask,
                    int32_t V, const float *cams, int32_t W, int32_t H,
                    int32_t TW, int32_t TH, const int32_t *valid,
                    const int32_t *span, const uint32_t *vals,
                    const uint32_t *ranges, double *image, double *Tfinal,
                    int32_t *last, uint8_t *margin) {
  pj64 *pj = project_all(n, npad, p, V, cams, W, H, valid, NULL);
  blend_ctx bc = {pj, span, mask, n};
  int GW = (W + TW - 1) / TW, GH = (H + TH - 1) / TH;
  int64_t evals = 0;
  for (int v = 0; v < V; ++v)
    for (int ty = 0; ty < GH; ++ty)
      for (int tx = 0; tx < GW; ++tx) {
        int64_t t = (int64_t)v * GW * GH + (int64_t)ty * GW + tx;
        uint32_t b = ranges[2 * t], e = ranges[2 * t + 1];
        for (int py = ty * TH; py < (ty + 1) * TH && py < H; ++py)
          for (int px = tx * TW; px < (tx + 1) * TW && px < W; ++px) {
            double col[3], T;
            int mg = 0;
            int64_t used = blend_pixel(&bc, v, px, py, vals + b, (int64_t)(e - b), col, &T,
                                       &evals, &mg, NULL, NULL);
            int64_t pix = (int64_t)py * W + px;
            for (int ch = 0; ch < 3; ++ch) image[((int64_t)v * 3 + ch) * H * W + pix] = col[ch];
            Tfinal[(int64_t)v * H * W + pix] = T;
            last[(int64_t)v * H * W + pix] = (int32_t)used;
            margin[(int64_t)v * H * W + pix] = (uint8_t)mg;
          }
      }
  free(pj);
  return evals;
}

/* Brute-force forward: every pixel walks ALL splats of its view in global
   (depth bits, index) order; the support rule alone selects candidates. */
static const float *g_sort_tz;
static int idx_cmp(const void *a, const void *b) {
  int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
  uint32_t bx, by;
  memcpy(&bx, &g_sort_tz[x], 4);
  memcpy(&by, &g_sort_tz[y], 4);
  if (bx != by) return bx < by ? -1 : 1;
  return x < y ? -1 : (x > y);
}

int64_t orc_forward_brute(int64_t n, int64_t npad, const double *p,
                          const double *mask, int32_t V, const float *cams,
                          int32_t W, int32_t H, const int32_t *valid,
                          const float *tz, const int32_t *span, double *image,
                          double *Tfinal) {
  pj64 *pj = project_all(n, npad, p, V, cams, W, H, valid, NULL);
  blend_ctx bc = {pj, span, mask, n};
  int64_t evals = 0;
  int64_t *ord = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
  uint32_t *list = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(n > 0 ? n : 1));
  for (int v = 0; v < V; ++v) {
    int64_t cnt = 0;
    for (int64_t i = 0; i < n; ++i)
      if (valid[(int64_t)v * n + i]) ord[cnt++] = i;
    g_sort_tz = tz + (int64_t)v * n;
    qsort(ord, (size_t)cnt, sizeof(int64_t), idx_cmp);
    for (int64_t k = 0; k < cnt; ++k) list[k] = (uint32_t)ord[k];
    for (int py = 0; py < H; ++py)
      for (int px = 0; px < W; ++px) {
        double col[3], T;
        int mg = 0;
        blend_pixel(&bc, v, px, py, list, cnt, col, &T, &evals, &mg, NULL, NULL);
        int64_t pix = (int64_t)py * W + px;
        for (int ch = 0; ch < 3; ++ch) image[((int64_t)v * 3 + ch) * H * W + pix] = col[ch];
        Tfinal[(int64_t)v * H * W + pix] = T;
      }
  }
  free(ord);
  free(list);
  free(pj);
  return evals;
}

/* ------------------------------------------------------------------------ */
/* a10 + a11: backward of the binned forward.  For each pixel the forward is */
/* replayed to list the blended candidates; then, with the colour seen      */
/* behind candidate i,  Bk_i = c_{i+1} a~_{i+1} + (1 - a~_{i+1}) Bk_{i+1}     */
/* (Bk after the last blended candidate = background = 0):                  */
/*   dC/dc_i = a~_i T_i,   dC/da~_i = T_i (c_i - Bk_i),                       */
/*   dL/dM_i = dL/da~_i alpha_i  (every blended candidate, masked or not),   */
/*   dL/dalpha_i = M_i dL/da~_i unless clamped at 0.99,                       */
/*   dalpha/dopacity = G,  dalpha/dpower = alpha,                            */
/*   dpower/dpx = A dx + B dy, dpower/dpy = B dx + C dy,                      */
/*   dpower/dA = -dx^2/2, dpower/dB = -dx dy, dpower/dC = -dy^2/2.            */
/* Then per (view, Gaussian) the projection backward, summed over views.    */
/* gparams [59][npad] and gmask [n] are overwritten; gsplat [V][n][10] (may */
/* be NULL) receives the per-view splat gradients.                          */
/* ------------------------------------------------------------------------ */
/* Reverse walk over the candidates one pixel blended (recs, nr from
 * blend_pixel), colour gradient gC of the pixel: adds every blended
 * candidate's splat-gradient terms into gs [view * n + i][NSPLATGRAD], or,
 * when only >= 0, only Gaussian `only`'s terms into gs [NSPLATGRAD]. */
static void pixel_backward(const blend_ctx *bc, int view, int px, int py, const uint32_t *list,
                           const blend_rec *recs, int64_t nr, const double gC[3],
                           int64_t only, double *gs) {
  const int64_t n = bc->n;
  double Bk[3] = {0.0, 0.0, 0.0};
  for (int64_t r = nr - 1; r >= 0; --r) {
    const blend_rec *br = &recs[r];
    int64_t i = list[br->j];
    int64_t s = (int64_t)view * n + i;
    const pj64 *g = &bc->pj[s];
    if (only < 0 || i == only) {
      double *gg = only < 0 ? gs + s * NSPLATGRAD : gs;
      double dat = 0.0;
      for (int ch = 0; ch < 3; ++ch) {
        gg[6 + ch] += gC[ch] * br->at * br->T;
        dat += gC[ch] * br->T * (g->col[ch] - Bk[ch]);
      }
      gg[9] += dat * br->alpha;
      double dalpha = bc->mask[i] * dat;
      if (!br->clamped) {
        gg[5] += dalpha * br->G;
        double dpow = dalpha * br->alpha;
        double dx = px - g->px, dy = py - g->py;
        gg[0] += dpow * (g->A * dx + g->B * dy);
        gg[1] += dpow * (g->B * dx + g->C * dy);
        gg[2] += dpow * (-0.5 * dx * dx);
        gg[3] += dpow * (-dx * dy);
        gg[4] += dpow * (-0.5 * dy * dy);
      }
    }
    for (int ch = 0; ch < 3; ++ch) Bk[ch] = g->col[ch] * br->at + (1.0 - br->at) * Bk[ch];
  }
}

void orc_backward(int64_t n, int64_t npad, const double *p, const double *mask,
                  int32_t V, const float *cams, int32_t W, int32_t H,
                  int32_t TW, int32_t TH, const int32_t *valid,
                  const int32_t *span, const uint32_t *vals,
                  const uint32_t *ranges, const double *dimage,
                  double *gparams, double *gmask, double *gsplat_out) {
  pj64 *pj = project_all(n, npad, p, V, cams, W, H, valid, NULL);
  blend_ctx bc = {pj, span, mask, n};
  double *gs = (double *)calloc((size_t)(V * n * NSPLATGRAD), sizeof(double));
  int GW = (W + TW - 1) / TW, GH = (H + TH - 1) / TH;
  int64_t maxlist = 1;
  for (int64_t t = 0; t < (int64_t)V * GW * GH; ++t)
    if (ranges[2 * t + 1] - ranges[2 * t] > maxlist) maxlist = ranges[2 * t + 1] - ranges[2 * t];
  blend_rec *recs = (blend_rec *)malloc(sizeof(blend_rec) * (size_t)maxlist);
  for (int v = 0; v < V; ++v)
    for (int ty = 0; ty < GH; ++ty)
      for (int tx = 0; tx < GW; ++tx) {
        int64_t t = (int64_t)v * GW * GH + (int64_t)ty * GW + tx;
        uint32_t b = ranges[2 * t], e = ranges[2 * t + 1];
        const uint32_t *list = vals + b;
        for (int py = ty * TH; py < (ty + 1) * TH && py < H; ++py)
          for (int px = tx * TW; px < (tx + 1) * TW && px < W; ++px) {
            double col[3], T;
            int64_t ev = 0, nr = 0;
            int mg = 0;
            blend_pixel(&bc, v, px, py, list, (int64_t)(e - b), col, &T, &ev, &mg, recs, &nr);
            int64_t pix = (int64_t)py * W + px;
            double gC[3];
            for (int ch = 0; ch < 3; ++ch) gC[ch] = dimage[((int64_t)v * 3 + ch) * H * W + pix];
            pixel_backward(&bc, v, px, py, list, recs, nr, gC, -1, gs);
          }
      }
  free(recs);
  memset(gparams, 0, sizeof(double) * (size_t)(NCH * npad));
  memset(gmask, 0, sizeof(double) * (size_t)n);
  for (int v = 0; v < V; ++v) {
    const orc_cam *c = (const orc_cam *)(cams + 19 * v);
    for (int64_t i = 0; i < n; ++i) {
      int64_t s = (int64_t)v * n + i;
      if (!valid[s]) continue;
      pj64 o;
      pj64_tmp m;
      proj64(p, npad, i, c, W, H, &o, &m);
      proj64_bwd(p, npad, i, c, &o, &m, gs + s * NSPLATGRAD, gparams);
      gmask[i] += gs[s * NSPLATGRAD + 9];
    }
  }
  if (gsplat_out) memcpy(gsplat_out, gs, sizeof(double) * (size_t)(V * n * NSPLATGRAD));
  free(gs);
  free(pj);
}

/* Number of (tile, Gaussian) pairs of every tile, from the pixel spans
 * (same rule as orc_bin, without materialising the pairs).  counts
 * [V*tiles] is overwritten. */
void orc_tile_counts(int64_t n, int32_t V, const int32_t *valid, const int32_t *span,
                     int32_t W, int32_t H, int32_t TW, int32_t TH, int64_t *counts) {
  int GW = (W + TW - 1) / TW, GH = (H + TH - 1) / TH;
  int64_t tpv = (int64_t)GW * GH;
  for (int64_t t = 0; t < V * tpv; ++t) counts[t] = 0;
  for (int v = 0; v < V; ++v)
    for (int64_t i = 0; i < n; ++i) {
      int64_t s = (int64_t)v * n + i;
      if (!valid[s]) continue;
      for (int ty = span[4 * s + 2] / TH; ty <= span[4 * s + 3] / TH; ++ty)
        for (int tx = span[4 * s] / TW; tx <= span[4 * s + 1] / TW; ++tx)
          counts[v * tpv + (int64_t)ty * GW + tx] += 1;
    }
}

/* The Gaussians listed for one tile, in (depth bits, index) order; returns
 * the count (out may be NULL to count only). */
int64_t orc_tile_list(int64_t n, int32_t view, int64_t tile_in_view, const int32_t *valid,
                      const float *tz, const int32_t *span, int32_t W, int32_t TW, int32_t TH,
                      uint32_t *out) {
  int GW = (W + TW - 1) / TW;
  int tx = (int)(tile_in_view % GW), ty = (int)(tile_in_view / GW);
  int X0 = tx * TW, X1 = X0 + TW - 1, Y0 = ty * TH, Y1 = Y0 + TH - 1;
  int64_t cnt = 0;
  for (int64_t i = 0; i < n; ++i) {
    int64_t s = (int64_t)view * n + i;
    if (!valid[s]) continue;
    const int32_t *sp = span + 4 * s;
    if (sp[0] <= X1 && sp[1] >= X0 && sp[2] <= Y1 && sp[3] >= Y0) {
      if (out) out[cnt] = (uint32_t)i;
      ++cnt;
    }
  }
  if (out) {
    g_sort_tz = tz + (int64_t)view * n;
    int64_t *tmp = (int64_t *)malloc(sizeof(int64_t) * (size_t)(cnt > 0 ? cnt : 1));
    for (int64_t k = 0; k < cnt; ++k) tmp[k] = out[k];
    qsort(tmp, (size_t)cnt, sizeof(int64_t), idx_cmp);
    for (int64_t k = 0; k < cnt; ++k) out[k] = (uint32_t)tmp[k];
    free(tmp);
  }
  return cnt;
}

/* Brute-force colour and transmittance of sampled pixels: each pixel walks
 * every valid splat of its view in global (depth bits, index) order and the
 * support rule alone selects candidates [Sec. 3.1, compositing equation].
 * pix [npix][3] = (view, u, v); out [npix][4] = (r, g, b, T), margin [npix]. */
int64_t orc_pixels_brute(int64_t n, int64_t npad, const double *p, const double *mask,
                         int32_t V, const float *cams, int32_t W, int32_t H,
                         const int32_t *valid, const float *tz, const int32_t *span,
                         int64_t npix, const int32_t *pix, double *out, uint8_t *margin) {
  int64_t evals = 0;
  int64_t *ord = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
  uint32_t *list = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(n > 0 ? n : 1));
  pj64 *pj = (pj64 *)calloc((size_t)n, sizeof(pj64));
  int64_t *vpix = (int64_t *)malloc(sizeof(int64_t) * (size_t)(npix > 0 ? npix : 1));
  int64_t *sat = (int64_t *)malloc(sizeof(int64_t) * (size_t)(W + 1) * (size_t)(H + 1));
  for (int v = 0; v < V; ++v) {
    int64_t nv = 0;
    for (int64_t k = 0; k < npix; ++k)
      if (pix[3 * k] == v) vpix[nv++] = k;
    if (!nv) continue;
    /* summed-area table of the view's sampled pixels: one lookup per span */
    for (int64_t k = 0; k < (int64_t)(W + 1) * (H + 1); ++k) sat[k] = 0;
    for (int64_t k = 0; k < nv; ++k)
      sat[(int64_t)(pix[3 * vpix[k] + 2] + 1) * (W + 1) + pix[3 * vpix[k] + 1] + 1] += 1;
    for (int y = 1; y <= H; ++y)
      for (int x = 1; x <= W; ++x)
        sat[(int64_t)y * (W + 1) + x] += sat[(int64_t)(y - 1) * (W + 1) + x] +
                                         sat[(int64_t)y * (W + 1) + x - 1] -
                                         sat[(int64_t)(y - 1) * (W + 1) + x - 1];
    const orc_cam *c = (const orc_cam *)(cams + 19 * v);
    int64_t cnt = 0;
    for (int64_t i = 0; i < n; ++i) {
      if (!valid[(int64_t)v * n + i]) continue;
      /* a splat whose span holds none of the sampled pixels is skipped by
         the support rule at every one of them: leave it out of the walk */
      const int32_t *sp = span + 4 * ((int64_t)v * n + i);
      int x0 = sp[0] < 0 ? 0 : sp[0], x1 = sp[1] >= W ? W - 1 : sp[1];
      int y0 = sp[2] < 0 ? 0 : sp[2], y1 = sp[3] >= H ? H - 1 : sp[3];
      if (x0 > x1 || y0 > y1) continue;
      int64_t inside = sat[(int64_t)(y1 + 1) * (W + 1) + x1 + 1] -
                       sat[(int64_t)y0 * (W + 1) + x1 + 1] -
                       sat[(int64_t)(y1 + 1) * (W + 1) + x0] + sat[(int64_t)y0 * (W + 1) + x0];
      if (!inside) continue;
      ord[cnt++] = i;
      pj64_tmp m;
      proj64(p, npad, i, c, W, H, &pj[i], &m);
    }
    g_sort_tz = tz + (int64_t)v * n;
    qsort(ord, (size_t)cnt, sizeof(int64_t), idx_cmp);
    for (int64_t k = 0; k < cnt; ++k) list[k] = (uint32_t)ord[k];
    /* blend_pixel indexes splats as view * n + i; give it a one-view table */
    blend_ctx bc = {pj, span + (int64_t)v * n * 4, mask, n};
    for (int64_t k = 0; k < npix; ++k) {
      if (pix[3 * k] != v) continue;
      double col[3], T;
      int mg = 0;
      blend_pixel(&bc, 0, pix[3 * k + 1], pix[3 * k + 2], list, cnt, col, &T, &evals, &mg,
                  NULL, NULL);
      out[4 * k] = col[0];
      out[4 * k + 1] = col[1];
      out[4 * k + 2] = col[2];
      out[4 * k + 3] = T;
      margin[k] = (uint8_t)mg;
    }
  }
  free(pj);
  free(vpix);
  free(sat);
  free(ord);
  free(list);
  return evals;
}

/* Splat and parameter gradients of chosen Gaussians by brute force over
 * their pixels [Sec. 3.1 compositing and its reverse pass]: in every view
 * where Gaussian i is not culled, each pixel of its span composites every
 * valid splat of that view whose span holds the pixel, in global (depth
 * bits, index) order, then walks back; only i's terms are summed.
 *   sel [nsel]: Gaussian indices; dimage [V][3][H][W] (NULL: only the
 *   margin flags are produced);
 *   gsplat [nsel][V][10] (px, py, A, B, C, opacity, r, g, b, mask; zero
 *   where culled); gparam [nsel][59]: the projection backward of those,
 *   summed over views; margin [V][H][W] (may be NULL) is set to 1 at every
 *   span pixel of a chosen Gaussian where a per-pair decision lies within
 *   the margin.  Returns the number of (view, pixel) walks. */
int64_t orc_splat_grads_sampled(int64_t n, int64_t npad, const double *p, const double *mask,
                                int32_t V, const float *cams, int32_t W, int32_t H,
                                const int32_t *valid, const float *tz, const int32_t *span,
                                int64_t nsel, const int64_t *sel, const double *dimage,
                                double *gsplat, double *gparam, uint8_t *margin) {
  int64_t walks = 0;
  int64_t *ord = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
  uint32_t *list = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(n > 0 ? n : 1));
  pj64 *pj = (pj64 *)calloc((size_t)n, sizeof(pj64));
  blend_rec *recs = (blend_rec *)malloc(sizeof(blend_rec) * (size_t)(n > 0 ? n : 1));
  if (gsplat) memset(gsplat, 0, sizeof(double) * (size_t)(nsel * V * NSPLATGRAD));
  if (gparam) memset(gparam, 0, sizeof(double) * (size_t)(nsel * NCH));
  for (int64_t q = 0; q < nsel; ++q) {
    const int64_t i = sel[q];
    double p1[NCH], gp1[NCH];
    for (int k = 0; k < NCH; ++k) {
      p1[k] = p[(int64_t)k * npad + i];
      gp1[k] = 0.0;
    }
    for (int v = 0; v < V; ++v) {
      const int64_t si = (int64_t)v * n + i;
      if (!valid[si]) continue;
      const orc_cam *c = (const orc_cam *)(cams + 19 * v);
      const int32_t *spi = span + 4 * si;
      int x0 = spi[0] < 0 ? 0 : spi[0], x1 = spi[1] >= W ? W - 1 : spi[1];
      int y0 = spi[2] < 0 ? 0 : spi[2], y1 = spi[3] >= H ? H - 1 : spi[3];
      if (x0 > x1 || y0 > y1) continue;
      /* every splat of the view whose span meets i's span, depth order */
      int64_t cnt = 0;
      for (int64_t k = 0; k < n; ++k) {
        const int64_t sk = (int64_t)v * n + k;
        if (!valid[sk]) continue;
        const int32_t *sp = span + 4 * sk;
        if (sp[1] < x0 || sp[0] > x1 || sp[3] < y0 || sp[2] > y1) continue;
        ord[cnt++] = k;
        pj64_tmp m;
        proj64(p, npad, k, c, W, H, &pj[k], &m);
      }
      g_sort_tz = tz + (int64_t)v * n;
      qsort(ord, (size_t)cnt, sizeof(int64_t), idx_cmp);
      for (int64_t k = 0; k < cnt; ++k) list[k] = (uint32_t)ord[k];
      blend_ctx bc = {pj, span + (int64_t)v * n * 4, mask, n};
      double gg[NSPLATGRAD] = {0};
      for (int py = y0; py <= y1; ++py)
        for (int px = x0; px <= x1; ++px) {
          double col[3], T;
          int64_t ev = 0, nr = 0;
          int mg = 0;
          blend_pixel(&bc, 0, px, py, list, cnt, col, &T, &ev, &mg, recs, &nr);
          ++walks;
          const int64_t pix = (int64_t)py * W + px;
          if (margin && mg) margin[(int64_t)v * H * W + pix] = 1;
          if (!dimage) continue;
          double gC[3];
          for (int ch = 0; ch < 3; ++ch) gC[ch] = dimage[((int64_t)v * 3 + ch) * H * W + pix];
          pixel_backward(&bc, 0, px, py, list, recs, nr, gC, i, gg);
        }
      if (!dimage) continue;
      if (gsplat)
        for (int k = 0; k < NSPLATGRAD; ++k) gsplat[(q * V + v) * NSPLATGRAD + k] = gg[k];
      pj64 o;
      pj64_tmp m;
      proj64(p1, 1, 0, c, W, H, &o, &m);
      proj64_bwd(p1, 1, 0, c, &o, &m, gg, gp1);
    }
    if (gparam)
      for (int k = 0; k < NCH; ++k) gparam[q * NCH + k] = gp1[k];
  }
  free(recs);
  free(pj);
  free(list);
  free(ord);
  return walks;
}

/* Projection only (FP64): fields px, py, A, B, C, opacity, r, g, b per
   (view, Gaussian) -> out [V][n][9]; invalid entries are left at zero. */
void orc_project64(int64_t n, int64_t npad, const double *p, int32_t V,
                   const float *cams, int32_t W, int32_t H, const int32_t *valid,
                   double *out) {
  pj64 *pj = project_all(n, npad, p, V, cams, W, H, valid, NULL);
  for (int64_t s = 0; s < (int64_t)V * n; ++s) {
    double *o = out + 9 * s;
    o[0] = pj[s].px; o[1] = pj[s].py; o[2] = pj[s].A; o[3] = pj[s].B; o[4] = pj[s].C;
    o[5] = pj[s].opa; o[6] = pj[s].col[0]; o[7] = pj[s].col[1]; o[8] = pj[s].col[2];
  }
  free(pj);
}

/* ------------------------------------------------------------------------ */
/* a9: L1 distortion [Supp. "Training Objective": the L1 part].             */
/* D = mean |C - target|;  dD/dC = sign(C - target) / count, sign(0) = 0.    */
/* ------------------------------------------------------------------------ */
double orc_l1(int64_t cnt, const double *img, const float *target, double *dimg) {
  double s = 0.0;
  for (int64_t k = 0; k < cnt; ++k) {
    double d = img[k] - (double)target[k];
    s += fabs(d);
    if (dimg) dimg[k] = (d > 0.0 ? 1.0 : (d < 0.0 ? -1.0 : 0.0)) / (double)cnt;
  }
  return s / (double)cnt;
}

/* ------------------------------------------------------------------------ */
/* Channel-wise fixed-length code length [Sec. 3.4.1].  Per channel j over  */
/* the kept Gaussians: K_j = kmax_j - kmin_j + 1, w_j = ceil(log2 K_j)       */
/* bits per code (0 when K_j = 1); header per channel (q_j f32, kmin_j i32,  */
/* w_j u8); bits = N_kept sum_j w_j + 59 * 72.                               */
/* kmin/kmax/width may be NULL.  Returns total bits.                         */
/* ------------------------------------------------------------------------ */
int64_t orc_fixed_length_bits(int64_t n, int64_t npad, const int32_t *k,
                              const uint8_t *mhat, int32_t *kmin_out,
                              int32_t *kmax_out, int32_t *width_out) {
  int64_t kept = 0;
  for (int64_t i = 0; i < n; ++i) kept += mhat[i] ? 1 : 0;
  int64_t bits = 0;
  for (int j = 0; j < NCH; ++j) {
    int64_t lo = 0, hi = 0;
    int first = 1;
    for (int64_t i = 0; i < n; ++i) {
      if (!mhat[i]) continue;
      int64_t v = k[j * npad + i];
      if (first || v < lo) lo = v;
      if (first || v > hi) hi = v;
      first = 0;
    }
    int64_t K = first ? 1 : hi - lo + 1;
    int w = 0;
    while (((int64_t)1 << w) < K) ++w;
    if (kmin_out) kmin_out[j] = (int32_t)lo;
    if (kmax_out) kmax_out[j] = (int32_t)hi;
    if (width_out) width_out[j] = w;
    bits += kept * w;
  }
  return bits + (int64_t)NCH * 72;
}

/* Pack/unpack of the fixed-length payload (kept Gaussians in index order,
   channel-major, LSB-first bit order); used to pin the code length by a
   round trip.  buf must hold ceil(bits/8) bytes (zeroed by the caller). */
void orc_fixed_length_pack(int64_t n, int64_t npad, const int32_t *k,
                           const uint8_t *mhat, const int32_t *kmin,
                           const int32_t *width, uint8_t *buf) {
  int64_t pos = 0;
  for (int j = 0; j < NCH; ++j)
    for (int64_t i = 0; i < n; ++i) {
      if (!mhat[i]) continue;
      uint64_t v = (uint64_t)((int64_t)k[j * npad + i] - kmin[j]);
      for (int b = 0; b < width[j]; ++b, ++pos)
        if ((v >> b) & 1) buf[pos >> 3] |= (uint8_t)(1u << (pos & 7));
    }
}

void orc_fixed_length_unpack(int64_t n, int64_t npad, const uint8_t *buf,
                             const uint8_t *mhat, const int32_t *kmin,
                             const int32_t *width, int32_t *k) {
  int64_t pos = 0;
  for (int j = 0; j < NCH; ++j)
    for (int64_t i = 0; i < n; ++i) {
      if (!mhat[i]) continue;
      uint64_t v = 0;
      for (int b = 0; b < width[j]; ++b, ++pos)
        if ((buf[pos >> 3] >> (pos & 7)) & 1) v |= (uint64_t)1 << b;
      k[j * npad + i] = (int32_t)((int64_t)v + kmin[j]);
    }
}

/* ------------------------------------------------------------------------ */
/* One RD step's render part (forward and backward) over a sample of tiles   */
/* [Sec. 3.1 compositing and its reverse pass]: the pixels of the chosen     */
/* tiles are composited and differentiated exactly as orc_forward /          */
/* orc_backward do, with the rest of the image left out (its dL/dC taken as  */
/* zero).  Each chosen tile's list (every valid splat of the view whose      */
/* span's tile rectangle holds the tile, in (depth bits, index) order) is    */
/* built by one pass over the splats; the splats of those lists are          */
/* projected once; gparams [59][npad] (overwritten) receives the projection  */
/* backward of their summed gradients; image [ntiles][3][TH][TW] the        */
/* chosen tiles' colours (pixels outside the image 0).  Tiles are            */
/* independent: built with OpenMP the tiles run in parallel and their        */
/* gradients are merged in tile order, so the result does not depend on the  */
/* thread count.  Returns the in-support evaluations of the forward.         */
/* ------------------------------------------------------------------------ */
static int u64_cmp(const void *a, const void *b) {
  uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
  return x < y ? -1 : (x > y);
}

int64_t orc_step_tiles_sampled(int64_t n, int64_t npad, const double *p, const double *mask,
                               int32_t V, const float *cams, int32_t W, int32_t H, int32_t TW,
                               int32_t TH, const int32_t *valid, const float *tz,
                               const int32_t *span, int64_t ntiles, const int64_t *tiles,
                               const double *dimage, double *image, double *gparams) {
  const int GW = (W + TW - 1) / TW, GH = (H + TH - 1) / TH;
  const int64_t tpv = (int64_t)GW * GH;
  if (!sh_ready) sh_build(); /* the SH tables, before any thread reads them */
  /* which chosen tile (index + 1) each global tile is, 0 = not chosen */
  int64_t *slot_of_tile = (int64_t *)calloc((size_t)(V * tpv), sizeof(int64_t));
  for (int64_t k = 0; k < ntiles; ++k) slot_of_tile[tiles[k]] = k + 1;
  /* lists: count, then fill (key = depth bits << 32 | index) */
  int64_t *cnt = (int64_t *)calloc((size_t)(ntiles + 1), sizeof(int64_t));
  for (int v = 0; v < V; ++v)
    for (int64_t i = 0; i < n; ++i) {
      const int64_t s = (int64_t)v * n + i;
      if (!valid[s]) continue;
      const int32_t *sp = span + 4 * s;
      for (int ty = sp[2] / TH; ty <= sp[3] / TH; ++ty)
        for (int tx = sp[0] / TW; tx <= sp[1] / TW; ++tx) {
          const int64_t k = slot_of_tile[(int64_t)v * tpv + (int64_t)ty * GW + tx];
          if (k) cnt[k - 1] += 1;
        }
    }
  int64_t *start = (int64_t *)malloc(sizeof(int64_t) * (size_t)(ntiles + 1));
  start[0] = 0;
  for (int64_t k = 0; k < ntiles; ++k) start[k + 1] = start[k] + cnt[k];
  const int64_t total = start[ntiles];
  uint64_t *keys = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(total > 0 ? total : 1));
  for (int64_t k = 0; k < ntiles; ++k) cnt[k] = 0;
  for (int v = 0; v < V; ++v)
    for (int64_t i = 0; i < n; ++i) {
      const int64_t s = (int64_t)v * n + i;
      if (!valid[s]) continue;
      const int32_t *sp = span + 4 * s;
      uint32_t zb;
      memcpy(&zb, &tz[s], 4);
      for (int ty = sp[2] / TH; ty <= sp[3] / TH; ++ty)
        for (int tx = sp[0] / TW; tx <= sp[1] / TW; ++tx) {
          const int64_t k = slot_of_tile[(int64_t)v * tpv + (int64_t)ty * GW + tx];
          if (k) keys[start[k - 1] + cnt[k - 1]++] = ((uint64_t)zb << 32) | (uint64_t)i;
        }
    }
  for (int64_t k = 0; k < ntiles; ++k)
    qsort(keys + start[k], (size_t)cnt[k], sizeof(uint64_t), u64_cmp);
  /* compact projection table of the listed splats: slot per (view, splat) */
  int32_t *pslot = (int32_t *)malloc(sizeof(int32_t) * (size_t)(V * n));
  for (int64_t s = 0; s < (int64_t)V * n; ++s) pslot[s] = -1;
  int64_t nused = 0;
  for (int64_t k = 0; k < ntiles; ++k) {
    const int v = (int)(tiles[k] / tpv);
    for (int64_t e = start[k]; e < start[k + 1]; ++e) {
      const int64_t s = (int64_t)v * n + (int64_t)(keys[e] & 0xFFFFFFFFu);
      if (pslot[s] < 0) pslot[s] = (int32_t)nused++;
    }
  }
  int64_t *used = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nused > 0 ? nused : 1));
  for (int64_t s = 0; s < (int64_t)V * n; ++s)
    if (pslot[s] >= 0) used[pslot[s]] = s;
  /* per-view tables indexed by Gaussian, as blend_pixel expects: the used
     splats' projections are placed at their Gaussian index of a view copy */
  pj64 *pjc = (pj64 *)calloc((size_t)(nused > 0 ? nused : 1), sizeof(pj64));
#pragma omp parallel for schedule(static)
  for (int64_t u = 0; u < nused; ++u) {
    const int64_t s = used[u];
    const int v = (int)(s / n);
    pj64_tmp m;
    proj64(p, npad, s - (int64_t)v * n, (const orc_cam *)(cams + 19 * v), W, H, &pjc[u], &m);
  }
  /* per-tile gradient sums of its list entries [start[k] + j][NSPLATGRAD] */
  double *tg = (double *)calloc((size_t)(total > 0 ? total : 1) * NSPLATGRAD, sizeof(double));
  int64_t evals = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : evals)
  for (int64_t k = 0; k < ntiles; ++k) {
    const int v = (int)(tiles[k] / tpv);
    const int64_t t = tiles[k] - (int64_t)v * tpv;
    const int tx = (int)(t % GW), ty = (int)(t / GW);
    const int64_t len = start[k + 1] - start[k];
    /* the tile's own view table: list position j holds Gaussian j */
    pj64 *pj = (pj64 *)malloc(sizeof(pj64) * (size_t)(len > 0 ? len : 1));
    int32_t *sp4 = (int32_t *)malloc(sizeof(int32_t) * 4 * (size_t)(len > 0 ? len : 1));
    double *mk = (double *)malloc(sizeof(double) * (size_t)(len > 0 ? len : 1));
    uint32_t *list = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(len > 0 ? len : 1));
    blend_rec *recs = (blend_rec *)malloc(sizeof(blend_rec) * (size_t)(len > 0 ? len : 1));
    double *gl = (double *)calloc((size_t)(len > 0 ? len : 1) * NSPLATGRAD, sizeof(double));
    for (int64_t j = 0; j < len; ++j) {
      const int64_t i = (int64_t)(keys[start[k] + j] & 0xFFFFFFFFu);
      const int64_t s = (int64_t)v * n + i;
      pj[j] = pjc[pslot[s]];
      memcpy(sp4 + 4 * j, span + 4 * s, 4 * sizeof(int32_t));
      mk[j] = mask[i];
      list[j] = (uint32_t)j;
    }
    blend_ctx bc = {pj, sp4, mk, len};
    for (int py = ty * TH; py < (ty + 1) * TH; ++py)
      for (int px = tx * TW; px < (tx + 1) * TW; ++px) {
        double *out = image ? image + k * 3 * TW * TH + (int64_t)(py - ty * TH) * TW + (px - tx * TW)
                            : NULL;
        if (px >= W || py >= H) {
          if (out) out[0] = out[TW * TH] = out[2 * TW * TH] = 0.0;
          continue;
        }
        double col[3], T;
        int64_t ev = 0, nr = 0;
        int mg = 0;
        blend_pixel(&bc, 0, px, py, list, len, col, &T, &ev, &mg, recs, &nr);
        evals += ev;
        if (out) {
          out[0] = col[0];
          out[TW * TH] = col[1];
          out[2 * TW * TH] = col[2];
        }
        const int64_t pix = (int64_t)py * W + px;
        double gC[3];
        for (int ch = 0; ch < 3; ++ch) gC[ch] = dimage[((int64_t)v * 3 + ch) * H * W + pix];
        pixel_backward(&bc, 0, px, py, list, recs, nr, gC, -1, gl);
      }
    memcpy(tg + start[k] * NSPLATGRAD, gl, sizeof(double) * (size_t)len * NSPLATGRAD);
    free(gl);
    free(recs);
    free(list);
    free(mk);
    free(sp4);
    free(pj);
  }
  /* merge in tile order into per-(view, splat) sums, then project back */
  double *gs = (double *)calloc((size_t)(nused > 0 ? nused : 1) * NSPLATGRAD, sizeof(double));
  for (int64_t k = 0; k < ntiles; ++k) {
    const int v = (int)(tiles[k] / tpv);
    for (int64_t e = start[k]; e < start[k + 1]; ++e) {
      const int64_t s = (int64_t)v * n + (int64_t)(keys[e] & 0xFFFFFFFFu);
      for (int c = 0; c < NSPLATGRAD; ++c) gs[pslot[s] * NSPLATGRAD + c] += tg[e * NSPLATGRAD + c];
    }
  }
  double *gpu = (double *)calloc((size_t)(nused > 0 ? nused : 1) * NCH, sizeof(double));
#pragma omp parallel for schedule(static)
  for (int64_t u = 0; u < nused; ++u) {
    const int64_t s = used[u];
    const int v = (int)(s / n);
    const int64_t i = s - (int64_t)v * n;
    double p1[NCH];
    for (int c = 0; c < NCH; ++c) p1[c] = p[(int64_t)c * npad + i];
    pj64 o;
    pj64_tmp m;
    const orc_cam *cam = (const orc_cam *)(cams + 19 * v);
    proj64(p1, 1, 0, cam, W, H, &o, &m);
    proj64_bwd(p1, 1, 0, cam, &o, &m, gs + u * NSPLATGRAD, gpu + u * NCH);
  }
  memset(gparams, 0, sizeof(double) * (size_t)(NCH * npad));
  for (int64_t u = 0; u < nused; ++u) {  /* (view, splat) order: fixed */
    const int64_t s = used[u];
    const int64_t i = s % n;
    for (int c = 0; c < NCH; ++c) gparams[(int64_t)c * npad + i] += gpu[u * NCH + c];
  }
  free(gpu);
  free(gs);
  free(tg);
  free(pjc);
  free(used);
  free(pslot);
  free(keys);
  free(start);
  free(cnt);
  free(slot_of_tile);
  return evals;
}
