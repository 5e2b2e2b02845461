// One Adam step (Kingma & Ba 2015) on the formation variables: parameters
// [59][npad], the 59 step sizes and the n retention scores.  The paper's
// Sec. 4.1 adopts an economical optimizer schedule (separated updates of the
// higher SH coefficients, an efficient Adam); the two switches read from it
// are described with sgs_adam_step.
//
// Parameters: one thread per Gaussian reads the gradients of the rows
// updated this step (one coalesced row after another), decides whether the
// Gaussian is skipped (sparse mode: all of them exactly zero), then updates
// value, first and second moment of each row.  Every operation is FP32 in a
// fixed order (no contraction), so the result is reproducible.
#include "sgs_internal.h"

namespace {

constexpr int kAThreads = 256;
constexpr int kShRestLo = 6, kShRestHi = 50;  // channels of SH degrees 1-3

struct AdamConst {
  float b1, b2, omb1, omb2, bc1, bc2, eps;
};
struct AdamLr {
  float lr[SGS_NCH];
};

__device__ __forceinline__ void adam_update(float &x, float &m, float &v, float g, float lr,
                                            const AdamConst &c) {
  m = c.b1 * m + c.omb1 * g;
  v = c.b2 * v + c.omb2 * (g * g);
  const float mh = m / c.bc1;
  const float vh = v / c.bc2;
  x = x - lr * mh / (sqrtf(vh) + c.eps);
}

__device__ __forceinline__ bool row_updated(int j, int sh_rest) {
  return sh_rest || j < kShRestLo || j > kShRestHi;
}

__global__ void __launch_bounds__(kAThreads)
k_adam_params(int64_t n, int64_t npad, float *__restrict__ x, float *__restrict__ m,
              float *__restrict__ v, const float *__restrict__ g, AdamLr lr, AdamConst c,
              int sh_rest, int sparse) {
  const int64_t i = (int64_t)blockIdx.x * kAThreads + threadIdx.x;
  if (i >= n) return;
  float gr[SGS_NCH];
  bool any = false;
#pragma unroll
  for (int j = 0; j < SGS_NCH; ++j) {
    gr[j] = row_updated(j, sh_rest) ? g[j * npad + i] : 0.0f;
    any |= gr[j] != 0.0f;
  }
  if (sparse && !any) return;
#pragma unroll
  for (int j = 0; j < SGS_NCH; ++j) {
    if (!row_updated(j, sh_rest)) continue;
    const int64_t o = j * npad + i;
    float xv = x[o], mv = m[o], vv = v[o];
    adam_update(xv, mv, vv, gr[j], lr.lr[j], c);
    x[o] = xv;
    m[o] = mv;
    v[o] = vv;
  }
}

__global__ void __launch_bounds__(kAThreads)
k_adam_vec(int64_t n, float *__restrict__ x, float *__restrict__ m, float *__restrict__ v,
           const float *__restrict__ g, float lr, AdamConst c) {
  const int64_t i = (int64_t)blockIdx.x * kAThreads + threadIdx.x;
  if (i >= n) return;
  float xv = x[i], mv = m[i], vv = v[i];
  adam_update(xv, mv, vv, g[i], lr, c);
  x[i] = xv;
  m[i] = mv;
  v[i] = vv;
}

}  // namespace

hipError_t launch_adam(sgs_ctx *c, const sgs_adam_options *o, float *params, float *pm,
                       float *pv, const float *gp, float *q, float *qm, float *qv,
                       const float *gq, float *s, float *sm, float *sv, const float *gs) {
  SgsProfScope ps(c, SGS_PROF_ADAM);
  AdamConst k;
  k.b1 = o->beta1;
  k.b2 = o->beta2;
  k.omb1 = 1.0f - o->beta1;  // exact (Sterbenz) for beta in [0.5, 1)
  k.omb2 = 1.0f - o->beta2;
  k.bc1 = (float)(1.0 - pow((double)o->beta1, (double)o->step));
  k.bc2 = (float)(1.0 - pow((double)o->beta2, (double)o->step));
  k.eps = o->eps;
  AdamLr lr;
  for (int j = 0; j < SGS_NCH; ++j) lr.lr[j] = o->lr[j];
  const int64_t n = c->n;
  k_adam_params<<<sgs_blocks(n, kAThreads), kAThreads, 0, c->stream>>>(
      n, c->npad, params, pm, pv, gp, lr, k, o->sh_rest, o->sparse);
  if (q)
    k_adam_vec<<<1, kAThreads, 0, c->stream>>>(SGS_NCH, q, qm, qv, gq, o->lr_q, k);
  if (s)
    k_adam_vec<<<sgs_blocks(n, kAThreads), kAThreads, 0, c->stream>>>(n, s, sm, sv, gs,
                                                                      o->lr_score, k);
  return hipGetLastError();
}
