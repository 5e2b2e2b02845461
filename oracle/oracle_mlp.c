/*
 * oracle_mlp.c -- FP64 oracle of the learned rate estimator: a per-Gaussian
 * MLP 64 -> 128 -> 128 -> 1 (59 features padded to 64, ReLU hidden layers,
 * linear output) that estimates the bits a Gaussian costs under the
 * channel-wise fixed-length coder of the paper [Sec. 3.4.1], placed beside
 * the range-based rate proxy [Sec. 3.3.1].
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.c).
 *
 * Arithmetic is FP64.  When `mirror` is non-zero the values the GPU feeds to
 * its BF16 matrix cores are rounded to BF16 (round to nearest, ties to even)
 * at the same points: inputs x, weights W1, W2, w3, the first hidden
 * activation h1, and, in the backward pass, dz2 and dz1.  With mirror = 0 the
 * same functions are plain FP64 (for finite-difference pins).
 *
 * Weights (row-major): W1[64][128] (in, out), b1[128], W2[128][128], b2[128],
 * w3[128], b3[1].
 *   z1 = x W1 + b1,  h1 = relu(z1),  z2 = h1 W2 + b2,  h2 = relu(z2),
 *   f = h2 . w3 + b3.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define MI 64
#define MH 128

/* Round to the nearest BF16 value (8 significant bits), ties to even.  Done
 * on the binary64 representation: keep 8 significant bits of the 53. */
double orc_bf16(double x) {
  if (x == 0.0 || !isfinite(x)) return x;
  int e;
  double m = frexp(x, &e); /* x = m 2^e, 0.5 <= |m| < 1 */
  double s = ldexp(m, 8);  /* 8 significant bits before the point */
  double r = nearbyint(s); /* current rounding mode: to nearest, ties to even */
  return ldexp(r, e - 8);
}

static double rb(double x, int mirror) { return mirror ? orc_bf16(x) : x; }

/* Features of one Gaussian: x_j = log2(1 + (y_j - m_j) / q_j) for the 59
 * channels (m_j the channel minimum), 0 for the 5 padding slots. */
void orc_mlp_features(int64_t n, int64_t npad, const float *y, const float *q,
                      const float *mmin, int mirror, double *X) {
  for (int64_t i = 0; i < n; ++i) {
    for (int j = 0; j < MI; ++j) {
      double v = 0.0;
      if (j < 59) {
        double u = ((double)y[j * npad + i] - (double)mmin[j]) / (double)q[j];
        v = log2(1.0 + u);
      }
      X[i * MI + j] = rb(v, mirror);
    }
  }
}

typedef struct {
  double W1[MI * MH], b1[MH], W2[MH * MH], b2[MH], w3[MH], b3;
} mlp_w;

static void load_w(const float *W1, const float *b1, const float *W2, const float *b2,
                   const float *w3, const float *b3, int mirror, mlp_w *w) {
  for (int k = 0; k < MI * MH; ++k) w->W1[k] = rb(W1[k], mirror);
  for (int k = 0; k < MH * MH; ++k) w->W2[k] = rb(W2[k], mirror);
  for (int k = 0; k < MH; ++k) {
    w->b1[k] = b1[k];
    w->b2[k] = b2[k];
    w->w3[k] = rb(w3[k], mirror);
  }
  w->b3 = b3[0];
}

/* one row: forward with intermediates */
static double row_fwd(const mlp_w *w, const double *x, int mirror, double *z1, double *h1,
                      double *z2, double *h2) {
  for (int o = 0; o < MH; ++o) {
    double s = w->b1[o];
    for (int k = 0; k < MI; ++k) s += x[k] * w->W1[k * MH + o];
    z1[o] = s;
    h1[o] = rb(s > 0.0 ? s : 0.0, mirror);
  }
  for (int o = 0; o < MH; ++o) {
    double s = w->b2[o];
    for (int k = 0; k < MH; ++k) s += h1[k] * w->W2[k * MH + o];
    z2[o] = s;
    h2[o] = s > 0.0 ? s : 0.0;
  }
  double f = w->b3;
  for (int k = 0; k < MH; ++k) f += h2[k] * w->w3[k];
  return f;
}

/* Forward over B rows of X [B][64] -> f [B]. */
void orc_mlp_forward(int64_t B, const double *X, const float *W1, const float *b1,
                     const float *W2, const float *b2, const float *w3, const float *b3,
                     int mirror, double *f) {
  mlp_w *w = (mlp_w *)malloc(sizeof(mlp_w));
  load_w(W1, b1, W2, b2, w3, b3, mirror, w);
  double z1[MH], h1[MH], z2[MH], h2[MH];
  for (int64_t i = 0; i < B; ++i) f[i] = row_fwd(w, X + i * MI, mirror, z1, h1, z2, h2);
  free(w);
}

/* Backward of  sum_i c_i f(x_i)  for given row weights c (the upstream
 * gradient df_i).  Outputs (any may be NULL) are overwritten:
 *   dW1 [64][128], db1 [128], dW2 [128][128], db2 [128], dw3 [128], db3 [1],
 *   dX [B][64].
 * Chain: dz2 = c w3 [z2 > 0];  dh1 = W2 dz2;  dz1 = dh1 [z1 > 0];
 *   dW2 = h1^T dz2,  dW1 = x^T dz1,  dX = dz1 W1^T,  dw3 = c h2. */
void orc_mlp_backward(int64_t B, const double *X, const float *W1, const float *b1,
                      const float *W2, const float *b2, const float *w3, const float *b3,
                      int mirror, const double *c, double *dW1, double *db1, double *dW2,
                      double *db2, double *dw3, double *db3, double *dX) {
  mlp_w *w = (mlp_w *)malloc(sizeof(mlp_w));
  load_w(W1, b1, W2, b2, w3, b3, mirror, w);
  double *gW1 = (double *)calloc(MI * MH, sizeof(double));
  double *gW2 = (double *)calloc(MH * MH, sizeof(double));
  double gb1[MH] = {0}, gb2[MH] = {0}, gw3[MH] = {0}, gb3 = 0.0;
  double z1[MH], h1[MH], z2[MH], h2[MH], dz2[MH], dz1[MH];
  for (int64_t i = 0; i < B; ++i) {
    const double *x = X + i * MI;
    row_fwd(w, x, mirror, z1, h1, z2, h2);
    double ci = c[i];
    gb3 += ci;
    for (int k = 0; k < MH; ++k) {
      gw3[k] += ci * h2[k];
      dz2[k] = rb(z2[k] > 0.0 ? ci * w->w3[k] : 0.0, mirror);
      gb2[k] += dz2[k];
    }
    for (int a = 0; a < MH; ++a)
      for (int b = 0; b < MH; ++b) gW2[a * MH + b] += h1[a] * dz2[b];
    for (int a = 0; a < MH; ++a) {
      double s = 0.0;
      for (int b = 0; b < MH; ++b) s += w->W2[a * MH + b] * dz2[b];
      dz1[a] = rb(z1[a] > 0.0 ? s : 0.0, mirror);
      gb1[a] += dz1[a];
    }
    for (int a = 0; a < MI; ++a)
      for (int b = 0; b < MH; ++b) gW1[a * MH + b] += x[a] * dz1[b];
    if (dX)
      for (int a = 0; a < MI; ++a) {
        double s = 0.0;
        for (int b = 0; b < MH; ++b) s += w->W1[a * MH + b] * dz1[b];
        dX[i * MI + a] = s;
      }
  }
  if (dW1) memcpy(dW1, gW1, sizeof(double) * MI * MH);
  if (dW2) memcpy(dW2, gW2, sizeof(double) * MH * MH);
  if (db1) memcpy(db1, gb1, sizeof(gb1));
  if (db2) memcpy(db2, gb2, sizeof(gb2));
  if (dw3) memcpy(dw3, gw3, sizeof(gw3));
  if (db3) db3[0] = gb3;
  free(gW1);
  free(gW2);
  free(w);
}

/* Adam (Kingma & Ba 2015) on a flat parameter vector, step t >= 1:
 *   m = b1 m + (1-b1) g,  v = b2 v + (1-b2) g^2,
 *   w -= lr (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps). */
void orc_adam(int64_t count, double *w, double *m, double *v, const double *g, double lr,
              double beta1, double beta2, double eps, int64_t t) {
  double c1 = 1.0 - pow(beta1, (double)t), c2 = 1.0 - pow(beta2, (double)t);
  for (int64_t k = 0; k < count; ++k) {
    m[k] = beta1 * m[k] + (1.0 - beta1) * g[k];
    v[k] = beta2 * v[k] + (1.0 - beta2) * g[k] * g[k];
    w[k] -= lr * (m[k] / c1) / (sqrt(v[k] / c2) + eps);
  }
}
