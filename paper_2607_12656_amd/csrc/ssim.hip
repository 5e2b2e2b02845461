// SSIM part of the rendering distortion (the supplement takes D_render from
// vanilla 3DGS: D = (1 - w) L1 + w (1 - SSIM)).  SSIM per image plane with
// the 11 x 11 Gaussian window of standard deviation 1.5, zero outside the
// image, C1 = 0.01^2, C2 = 0.03^2, averaged over all pixels.
//
// Forward: a 32 x 16 tile and its 5-pixel halo in LDS; separable window sums
// of x, y, x^2, y^2, xy (horizontal into LDS, then vertical), in FP64 (the
// products of two floats are exact there, and the variances s - m^2 cancel);
// per pixel S and the three maps G1 = dS/dmx, G2 = dS/dsxx, G3 = dS/dsxy
// (FP64, global), and per-block sums of S.
// Backward: the same separable sums of G1..G3 (the window is symmetric, so
// the adjoint of the sums is the same filter), then per pixel
//     dSSIM/dx = (w*G1 + 2 x (w*G2) + y (w*G3)) / N,
// and dL/dimage += -weight dSSIM/dx.  The G maps are kept in FP64: the three
// terms cancel where the image is flat.
#include <cmath>

#include "sgs_internal.h"

namespace {

constexpr int kSR = 5;                   // window radius
constexpr int kSTX = 32, kSTY = 16;      // output tile
constexpr int kSIX = kSTX + 2 * kSR, kSIY = kSTY + 2 * kSR;
constexpr int kSThreads = 256;
constexpr double kC1 = 0.01 * 0.01, kC2 = 0.03 * 0.03;

struct SsimWin {
  double w[2 * kSR + 1];
};

__global__ void __launch_bounds__(kSThreads)
k_ssim_fwd(int W, int H, const float *__restrict__ img, const float *__restrict__ tgt, SsimWin g,
           double *__restrict__ G, int64_t total, double *__restrict__ partial) {
  __shared__ float s_x[kSIY][kSIX], s_y[kSIY][kSIX];
  __shared__ double s_h[5][kSIY][kSTX];
  __shared__ double s_red[kSThreads / 64];
  const int64_t plane = blockIdx.z;
  const int64_t pix = (int64_t)W * H;
  const float *X = img + plane * pix, *Y = tgt + plane * pix;
  const int x0 = blockIdx.x * kSTX - kSR, y0 = blockIdx.y * kSTY - kSR;
  for (int i = threadIdx.x; i < kSIY * kSIX; i += kSThreads) {
    const int r = i / kSIX, c = i - r * kSIX, gx = x0 + c, gy = y0 + r;
    const bool in = gx >= 0 && gx < W && gy >= 0 && gy < H;
    s_x[r][c] = in ? X[(int64_t)gy * W + gx] : 0.0f;
    s_y[r][c] = in ? Y[(int64_t)gy * W + gx] : 0.0f;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kSIY * kSTX; i += kSThreads) {
    const int r = i / kSTX, c = i - r * kSTX;
    double a0 = 0, a1 = 0, a2 = 0, a3 = 0, a4 = 0;
#pragma unroll
    for (int k = 0; k <= 2 * kSR; ++k) {
      const double xv = s_x[r][c + k], yv = s_y[r][c + k], wk = g.w[k];
      a0 += wk * xv;
      a1 += wk * yv;
      a2 += wk * (xv * xv);
      a3 += wk * (yv * yv);
      a4 += wk * (xv * yv);
    }
    s_h[0][r][c] = a0;
    s_h[1][r][c] = a1;
    s_h[2][r][c] = a2;
    s_h[3][r][c] = a3;
    s_h[4][r][c] = a4;
  }
  __syncthreads();
  double ssum = 0.0;
  for (int i = threadIdx.x; i < kSTY * kSTX; i += kSThreads) {
    const int r = i / kSTX, c = i - r * kSTX;
    const int gx = blockIdx.x * kSTX + c, gy = blockIdx.y * kSTY + r;
    if (gx >= W || gy >= H) continue;
    double mx = 0, my = 0, sxx = 0, syy = 0, sxy = 0;
#pragma unroll
    for (int k = 0; k <= 2 * kSR; ++k) {
      const double wk = g.w[k];
      mx += wk * s_h[0][r + k][c];
      my += wk * s_h[1][r + k][c];
      sxx += wk * s_h[2][r + k][c];
      syy += wk * s_h[3][r + k][c];
      sxy += wk * s_h[4][r + k][c];
    }
    const double A = 2.0 * mx * my + kC1;
    const double B = 2.0 * (sxy - mx * my) + kC2;
    const double C = mx * mx + my * my + kC1;
    const double D = (sxx - mx * mx) + (syy - my * my) + kC2;
    const double CD = C * D;
    const double S = A * B / CD;
    ssum += S;
    // dS/dmx = S (2my/A - 2my/B - 2mx/C + 2mx/D), dS/dsxx = -S/D, dS/dsxy = 2S/B,
    // with S/A, S/B taken as B/CD, A/CD (finite where B crosses zero)
    const int64_t o = plane * pix + (int64_t)gy * W + gx;
    G[o] = 2.0 * my * (B - A) / CD + 2.0 * mx * S * (1.0 / D - 1.0 / C);
    G[total + o] = -S / D;
    G[2 * total + o] = 2.0 * A / CD;
  }
  ssum = sgs_wave_sum_d(ssum);
  if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = ssum;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < kSThreads / 64; ++w) t += s_red[w];
    partial[((int64_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x] = t;
  }
}

__global__ void k_ssim_finish(const double *__restrict__ partial, int64_t nb, int64_t total,
                              float weight, float *__restrict__ loss) {
  __shared__ double s_w[kSThreads / 64];
  double acc = 0.0;
  for (int64_t b = threadIdx.x; b < nb; b += kSThreads) acc += partial[b];
  acc = sgs_wave_sum_d(acc);
  if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < kSThreads / 64; ++w) t += s_w[w];
    loss[0] = (float)((double)weight * (1.0 - t / (double)total));
  }
}

__global__ void __launch_bounds__(kSThreads)
k_ssim_bwd(int W, int H, const float *__restrict__ img, const float *__restrict__ tgt, SsimWin g,
           const double *__restrict__ G, int64_t total, double scale, float *__restrict__ dimg) {
  __shared__ double s_g[3][kSIY][kSIX];
  __shared__ double s_h[3][kSIY][kSTX];
  const int64_t plane = blockIdx.z;
  const int64_t pix = (int64_t)W * H;
  const int x0 = blockIdx.x * kSTX - kSR, y0 = blockIdx.y * kSTY - kSR;
  for (int i = threadIdx.x; i < kSIY * kSIX; i += kSThreads) {
    const int r = i / kSIX, c = i - r * kSIX, gx = x0 + c, gy = y0 + r;
    const bool in = gx >= 0 && gx < W && gy >= 0 && gy < H;
    const int64_t o = plane * pix + (int64_t)gy * W + gx;
    s_g[0][r][c] = in ? G[o] : 0.0;
    s_g[1][r][c] = in ? G[total + o] : 0.0;
    s_g[2][r][c] = in ? G[2 * total + o] : 0.0;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kSIY * kSTX; i += kSThreads) {
    const int r = i / kSTX, c = i - r * kSTX;
    double a0 = 0, a1 = 0, a2 = 0;
#pragma unroll
    for (int k = 0; k <= 2 * kSR; ++k) {
      const double wk = g.w[k];
      a0 += wk * s_g[0][r][c + k];
      a1 += wk * s_g[1][r][c + k];
      a2 += wk * s_g[2][r][c + k];
    }
    s_h[0][r][c] = a0;
    s_h[1][r][c] = a1;
    s_h[2][r][c] = a2;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kSTY * kSTX; i += kSThreads) {
    const int r = i / kSTX, c = i - r * kSTX;
    const int gx = blockIdx.x * kSTX + c, gy = blockIdx.y * kSTY + r;
    if (gx >= W || gy >= H) continue;
    double f1 = 0, f2 = 0, f3 = 0;
#pragma unroll
    for (int k = 0; k <= 2 * kSR; ++k) {
      const double wk = g.w[k];
      f1 += wk * s_h[0][r + k][c];
      f2 += wk * s_h[1][r + k][c];
      f3 += wk * s_h[2][r + k][c];
    }
    const int64_t o = plane * pix + (int64_t)gy * W + gx;
    const double xv = img[o], yv = tgt[o];
    dimg[o] = (float)((double)dimg[o] + scale * (f1 + 2.0 * xv * f2 + yv * f3));
  }
}

}  // namespace

int64_t ssim_scratch_doubles(int64_t V, int64_t W, int64_t H) {
  const int64_t total = V * 3 * W * H;
  const int64_t nb = ((W + kSTX - 1) / kSTX) * ((H + kSTY - 1) / kSTY) * V * 3;
  return 3 * total + nb;
}

hipError_t launch_ssim(sgs_ctx *c, const float *image, const float *target, float weight,
                       float *loss, float *dimg) {
  SgsProfScope ps(c, SGS_PROF_SSIM);
  const int64_t total = (int64_t)c->V * 3 * c->W * c->H;
  if (ssim_scratch_doubles(c->V, c->W, c->H) > c->ssim_tmp_doubles) return hipErrorInvalidValue;
  SsimWin g;
  double sum = 0.0;
  for (int k = 0; k <= 2 * kSR; ++k) {
    const double u = (double)(k - kSR);
    g.w[k] = std::exp(-(u * u) / (2.0 * 1.5 * 1.5));
    sum += g.w[k];
  }
  for (int k = 0; k <= 2 * kSR; ++k) g.w[k] /= sum;
  const dim3 grid((c->W + kSTX - 1) / kSTX, (c->H + kSTY - 1) / kSTY, c->V * 3);
  const int64_t nb = (int64_t)grid.x * grid.y * grid.z;
  double *G = c->ssim_tmp, *partial = c->ssim_tmp + 3 * total;
  k_ssim_fwd<<<grid, kSThreads, 0, c->stream>>>(c->W, c->H, image, target, g, G, total, partial);
  k_ssim_finish<<<1, kSThreads, 0, c->stream>>>(partial, nb, total, weight, loss);
  if (dimg)
    k_ssim_bwd<<<grid, kSThreads, 0, c->stream>>>(c->W, c->H, image, target, g, G, total,
                                                  -(double)weight / (double)total, dimg);
  return hipGetLastError();
}
