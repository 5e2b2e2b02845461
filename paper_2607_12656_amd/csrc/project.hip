// Projection of every Gaussian into every view (paper Sec. 3.1: 3D Gaussians
// projected onto the image plane; view-dependent colour) and its backward.
// One thread per Gaussian reads the 59 parameter rows once (coalesced SoA)
// and loops over the views, so the parameters cross HBM once per step.
#include "sgs_internal.h"

namespace {

constexpr int kPThreads = 128;
constexpr int kPWaves = kPThreads / 64;

// The step sizes of the fused paths, once per block: q_j and rq_j = 1 / q_j
// (correctly rounded), rq_j NaN where it is not a normal float, so that the
// product test of sgs_rint_div fails there and the division decides.
__device__ __forceinline__ void load_quant_table(const float *__restrict__ q, float *s_q,
                                                 float *s_rq) {
  if (threadIdx.x < SGS_NCH) {
    const float qj = q[threadIdx.x];
    const float rq = __fdiv_rn(1.0f, qj);
    s_q[threadIdx.x] = qj;
    s_rq[threadIdx.x] = sgs_rq_ok(rq) ? rq : __int_as_float(0x7FC00000);
  }
  __syncthreads();
}

// Codes k_j = rint(fl32(v_j / q_j)) of one Gaussian's 59 raw values, decided
// from the products v_j rq_j (sgs_rint_div's rule; rq_j NaN sends channel j to
// the division), with the divisions, needed only near a tie, in one branch
// after all 59 products, so that the row's loads stay batched ahead of it.
__device__ __forceinline__ void quantize_row(const float (&v)[SGS_NCH], const float *s_q,
                                             const float *s_rq, float (&k)[SGS_NCH]) {
  bool slow = false;
#pragma unroll
  for (int j = 0; j < SGS_NCH; ++j) {
    const float t = v[j] * s_rq[j];
    k[j] = rintf(t);
    slow |= !sgs_product_decides(t, k[j]);
  }
  if (slow) {
#pragma unroll
    for (int j = 0; j < SGS_NCH; ++j)
      if (!sgs_product_decides(v[j] * s_rq[j], k[j])) k[j] = rintf(__fdiv_rn(v[j], s_q[j]));
  }
}

// Wave sums of 16 slots held by every lane, returned in lane L for slot
// L & 15: four exchange steps, each lane keeping the half of its slots that
// its lane bit selects and adding its partner's copy of that half (a
// transposing butterfly: 15 exchanges instead of 16 x 6), then two steps
// across the four 16-lane quarters.  The order of the additions is fixed.
// The slots are vector values, not an array: selecting between two array
// elements by a lane bit would be turned into a per-lane array index (a
// compare-and-select over every element).
typedef double sgs_d16 __attribute__((ext_vector_type(16)));
typedef double sgs_d8 __attribute__((ext_vector_type(8)));
typedef double sgs_d4 __attribute__((ext_vector_type(4)));
typedef double sgs_d2 __attribute__((ext_vector_type(2)));

template <typename H, int N>
__device__ __forceinline__ H exchange_half(H lo, H hi, int m) {
  const bool up = (threadIdx.x & m) != 0;
  const H send = up ? lo : hi;
  const H keep = up ? hi : lo;
  H r;
#pragma unroll
  for (int k = 0; k < N; ++k) r[k] = __shfl_xor(send[k], m, 64);
  return keep + r;
}

__device__ __forceinline__ double wave_transpose_sum16(sgs_d16 a) {
  const sgs_d8 b = exchange_half<sgs_d8, 8>(a.lo, a.hi, 8);
  const sgs_d4 c = exchange_half<sgs_d4, 4>(b.lo, b.hi, 4);
  const sgs_d2 d = exchange_half<sgs_d2, 2>(c.lo, c.hi, 2);
  const bool up = (threadIdx.x & 1) != 0;
  const double send = up ? d.x : d.y;
  const double keep = up ? d.y : d.x;
  const double e = keep + __shfl_xor(send, 1, 64);
  const double h = e + __shfl_xor(e, 16, 64);
  return h + __shfl_xor(h, 32, 64);
}

__device__ __forceinline__ void load_cam(const sgs_camera *cams, int v, SgsCam &cam) {
  const float *src = (const float *)(cams + v);
#pragma unroll
  for (int k = 0; k < 9; ++k) cam.R[k] = src[k];
#pragma unroll
  for (int k = 0; k < 3; ++k) cam.t[k] = src[9 + k];
  cam.fx = src[12];
  cam.fy = src[13];
  cam.cx = src[14];
  cam.cy = src[15];
#pragma unroll
  for (int k = 0; k < 3; ++k) cam.campos[k] = src[16 + k];
}

// Colour of one Gaussian seen from `cam`: sum_k f_k Y_k(dir) + 1/2, clamped at 0.
__device__ __forceinline__ void colour(const float *y, const SgsCam &cam, float col[3],
                                       bool clamped[3]) {
  float dx = y[0] - cam.campos[0], dy = y[1] - cam.campos[1], dz = y[2] - cam.campos[2];
  const float inv = 1.0f / sqrtf(dx * dx + dy * dy + dz * dz);
  dx *= inv; dy *= inv; dz *= inv;
  float Y[16];
  sgs_sh_basis(dx, dy, dz, Y);
#pragma unroll
  for (int ch = 0; ch < 3; ++ch) {
    float s = 0.5f;
#pragma unroll
    for (int k = 0; k < 16; ++k) s = fmaf(y[sgs_sh_channel(k, ch)], Y[k], s);
    clamped[ch] = s < 0.0f;
    col[ch] = clamped[ch] ? 0.0f : s;
  }
}

// QUANT: qp holds the raw rows and the kernel applies the quantizer itself
// (y_hat = rint(fl32(y / q)) q in FP32, the value the quantizer pass writes),
// so the quantized rows never cross HBM.
template <bool QUANT>
__global__ void __launch_bounds__(kPThreads)
k_preprocess(int64_t n, int64_t npad, int V, int W, int H, int TW, int TH,
             const sgs_camera *__restrict__ cams, const float *__restrict__ qp,
             const float *__restrict__ q, const uint8_t *__restrict__ hard,
             float4 *__restrict__ rec, uint32_t *__restrict__ depth_key,
             uint32_t *__restrict__ depth_val, uint32_t *__restrict__ touched,
             uint4 *__restrict__ bins, uint32_t *__restrict__ rect, int GW,
             int64_t tiles_per_view, int64_t vseg) {
  __shared__ float s_q[QUANT ? 64 : 1], s_rq[QUANT ? 64 : 1];
  if (QUANT) load_quant_table(q, s_q, s_rq);
  const int64_t i = (int64_t)blockIdx.x * kPThreads + threadIdx.x;
  if (i >= n) {
    // the padding of each view's depth segment: sorts after every splat of
    // the view and stands for no splat
    if (i < vseg)
      for (int v = 0; v < V; ++v) {
        const int64_t ps = (int64_t)v * vseg + i;
        depth_key[ps] = 0xFFFFFFFFu;
        depth_val[ps] = 0xFFFFFFFFu;
        rect[ps] = kNoRect;
      }
    return;
  }
  float y[SGS_NCH];
#pragma unroll
  for (int j = 0; j < SGS_NCH; ++j) y[j] = qp[j * npad + i];
  if (QUANT) {
    float k[SGS_NCH];
    quantize_row(y, s_q, s_rq, k);
#pragma unroll
    for (int j = 0; j < SGS_NCH; ++j) y[j] = k[j] * s_q[j];
  }
  const float m = hard[i] ? 1.0f : 0.0f;
  const float opa = 1.0f / (1.0f + __expf(-y[SGS_CH_OPA]));
  for (int v = 0; v < V; ++v) {
    SgsCam cam;
    load_cam(cams, v, cam);
    SgsProj p;
    sgs_project(y, cam, W, H, p);
    const int64_t s = (int64_t)v * n + i;
    const int64_t ps = (int64_t)v * vseg + i;  // its place in the depth segments
    depth_val[ps] = (uint32_t)s;
    if (!p.valid) {
      depth_key[ps] = 0xFFFFFFFFu;
      touched[s] = 0;
      rect[ps] = kNoRect;  // (an invalid splat's record is never read)
      rec[3 * s] = make_float4(0.f, 0.f, 0.f, 0.f);
      rec[3 * s + 1] = make_float4(0.f, 0.f, __int_as_float(-1), __int_as_float(-1));
      rec[3 * s + 2] = make_float4(0.f, 0.f, 0.f, 0.f);
      continue;
    }
    depth_key[ps] = __float_as_uint(p.tz);
    const int tw = p.x1 / TW - p.x0 / TW + 1, th = p.y1 / TH - p.y0 / TH + 1;
    touched[s] = (uint32_t)(tw * th);
    // binning record: first tile id, rectangle width in tiles, Gaussian, pairs
    // the tile rectangle in one word, which the depth sort carries along;
    // only a rectangle that does not fit it gets the full binning record
    // (first tile id, width in tiles, Gaussian, pairs), gathered later
    const uint32_t packed = sgs_pack_rect(p.x0 / TW, p.y0 / TH, tw, th);
    rect[ps] = packed;
    if (packed == kNoRect)
      bins[s] = make_uint4((uint32_t)(v * tiles_per_view) +
                               (uint32_t)((p.y0 / TH) * GW + p.x0 / TW),
                           (uint32_t)tw, (uint32_t)i, (uint32_t)(tw * th));
    const float A = p.c / p.det, B = -p.b / p.det, C = p.a / p.det;
    float col[3];
    bool cl[3];
    colour(y, cam, col, cl);
    const uint32_t sx = (uint32_t)p.x0 | ((uint32_t)p.x1 << 16);
    const uint32_t sy = (uint32_t)p.y0 | ((uint32_t)p.y1 << 16);
    // the conic scaled into the blend's exponent of 2 (SGS_CONIC_KAC / KB)
    rec[3 * s] = make_float4(p.px, p.py, A * SGS_CONIC_KAC, B * SGS_CONIC_KB);
    rec[3 * s + 1] = make_float4(C * SGS_CONIC_KAC, opa, __uint_as_float(sx), __uint_as_float(sy));
    rec[3 * s + 2] = make_float4(col[0], col[1], col[2], m);
  }
}

// Chain rule from the per-view splat gradients (px, py, A, B, C, opacity,
// r, g, b, mask) to the 59 channels, summed over views.
//
// FUSED: qp holds the raw rows; the kernel quantizes them as k_preprocess<true>
// does and also takes the quantizer's backward (Sec. 3.3.1, straight-through):
// the channel gradient it writes is the parameter gradient, and each block
// writes, per channel j, the FP64 sum over its Gaussians of g_ij (k_ij q_j -
// y_ij) (the learned-step gradient before the division by q_j; the residual
// is one fused multiply-add, exact, and its product with g exact in FP64) to
// partial[j * gridDim.x + block]; with gscore it also writes the score
// gradient (mask mode 1: (g_mask + rate term) s (1 - s) / tau, else 0).
template <bool FUSED>
__global__ void __launch_bounds__(kPThreads)
k_preprocess_bwd(int64_t n, int64_t npad, int V, int W, int H,
                 const sgs_camera *__restrict__ cams, const float *__restrict__ qp,
                 const float *__restrict__ q, const uint32_t *__restrict__ touched,
                 const double *__restrict__ sgrad, float *__restrict__ gout,
                 float *__restrict__ gmask, double *__restrict__ partial, int mode, float tau,
                 const float *__restrict__ soft, const float *__restrict__ rate_grad,
                 float *__restrict__ gscore, int sh_rows) {
  __shared__ float s_q[FUSED ? 64 : 1], s_rq[FUSED ? 64 : 1];
  // residuals k q - y of the block's Gaussians, kept for the end
  __shared__ float s_r[FUSED ? SGS_NCH : 1][kPThreads];
  __shared__ double s_part[FUSED ? kPWaves : 1][64];
  if (FUSED) load_quant_table(q, s_q, s_rq);
  const int64_t i = (int64_t)blockIdx.x * kPThreads + threadIdx.x;
  const bool live = i < n;
  if (!FUSED && !live) return;
  float y[SGS_NCH], g[SGS_NCH];
  const int64_t il = live ? i : 0;  // lanes past n load row entry 0, then drop it
#pragma unroll
  for (int j = 0; j < SGS_NCH; ++j) {
    const float v = qp[j * npad + il];
    y[j] = live ? v : 0.0f;
    g[j] = 0.0f;
  }
  if (FUSED) {
    float k[SGS_NCH];
    quantize_row(y, s_q, s_rq, k);
#pragma unroll
    for (int j = 0; j < SGS_NCH; ++j) {
      s_r[j][threadIdx.x] = fmaf(k[j], s_q[j], -y[j]);
      y[j] = k[j] * s_q[j];
    }
  }
  float gm = 0.0f;
  const float opa = 1.0f / (1.0f + __expf(-y[SGS_CH_OPA]));
  const int nv = live ? V : 0;
  // which of the first 32 views touch the splat, loaded together up front
  // (one wait instead of one per view before its record is read)
  uint32_t tmask = 0;
#pragma unroll 8
  for (int v = 0; v < min(nv, 32); ++v)
    tmask |= touched[(int64_t)v * n + i] != 0 ? 1u << v : 0u;
  for (int v = 0; v < nv; ++v) {
    const int64_t s = (int64_t)v * n + i;
    if (v < 32 ? ((tmask >> v) & 1u) == 0u : touched[s] == 0) continue;
    const double2 *gs = (const double2 *)(sgrad + s * SGS_SGRAD);
    const double2 h0 = gs[0], h1 = gs[1], h2 = gs[2], h3 = gs[3], h4 = gs[4];
    const float gpx = (float)h0.x, gpy = (float)h0.y, gA = (float)h1.x, gB = (float)h1.y;
    const float gC = (float)h2.x, gop = (float)h2.y;
    const float gcol[3] = {(float)h3.x, (float)h3.y, (float)h4.x};
    gm += (float)h4.y;
    SgsCam cam;
    load_cam(cams, v, cam);
    SgsProj p;
    sgs_project(y, cam, W, H, p);
    // opacity
    g[SGS_CH_OPA] += gop * opa * (1.0f - opa);
    // colour and view direction
    {
      float vx = y[0] - cam.campos[0], vy = y[1] - cam.campos[1], vz = y[2] - cam.campos[2];
      const float dist = sqrtf(vx * vx + vy * vy + vz * vz);
      const float inv = 1.0f / dist;
      const float dx = vx * inv, dy = vy * inv, dz = vz * inv;
      float Y[16], GY[16][3];
      sgs_sh_basis(dx, dy, dz, Y);
      sgs_sh_grad(dx, dy, dz, GY);
      float gd0 = 0.f, gd1 = 0.f, gd2 = 0.f;
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) {
        float raw = 0.5f;
#pragma unroll
        for (int k = 0; k < 16; ++k) raw = fmaf(y[sgs_sh_channel(k, ch)], Y[k], raw);
        if (raw < 0.0f) continue;
        const float gc = gcol[ch];
#pragma unroll
        for (int k = 0; k < 16; ++k) {
          const int chan = sgs_sh_channel(k, ch);
          g[chan] = fmaf(gc, Y[k], g[chan]);
          const float f = gc * y[chan];
          gd0 = fmaf(f, GY[k][0], gd0);
          gd1 = fmaf(f, GY[k][1], gd1);
          gd2 = fmaf(f, GY[k][2], gd2);
        }
      }
      const float dd = gd0 * dx + gd1 * dy + gd2 * dz;
      g[0] += (gd0 - dx * dd) * inv;
      g[1] += (gd1 - dy * dd) * inv;
      g[2] += (gd2 - dz * dd) * inv;
    }
    // conic (A, B, C) = (c, -b, a) / det  ->  Sigma' entries (a, b, c)
    const float a = p.a, b = p.b, c = p.c;
    const float id2 = 1.0f / (p.det * p.det);
    const float ga = (-c * c * gA + b * c * gB - b * b * gC) * id2;
    const float gb = (2.0f * b * c * gA - (a * c + b * b) * gB + 2.0f * a * b * gC) * id2;
    const float gc = (-b * b * gA + a * b * gB - a * a * gC) * id2;
    // a = T0 S T0^T, b = T0 S T1^T, c = T1 S T1^T
    const float *Sg = p.Sg;
    const float S[9] = {Sg[0], Sg[1], Sg[2], Sg[1], Sg[3], Sg[4], Sg[2], Sg[4], Sg[5]};
    float ST0[3], ST1[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      ST0[r] = S[3 * r] * p.T0[0] + S[3 * r + 1] * p.T0[1] + S[3 * r + 2] * p.T0[2];
      ST1[r] = S[3 * r] * p.T1[0] + S[3 * r + 1] * p.T1[1] + S[3 * r + 2] * p.T1[2];
    }
    float gT0[3], gT1[3], gS[9];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      gT0[r] = 2.0f * ga * ST0[r] + gb * ST1[r];
      gT1[r] = gb * ST0[r] + 2.0f * gc * ST1[r];
    }
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int q = 0; q < 3; ++q)
        gS[3 * r + q] = ga * p.T0[r] * p.T0[q] + 0.5f * gb * (p.T0[r] * p.T1[q] + p.T1[r] * p.T0[q]) +
                        gc * p.T1[r] * p.T1[q];
    // Sigma = M M^T  ->  dM = 2 dSigma M
    float gM[9];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int q = 0; q < 3; ++q)
        gM[3 * r + q] = 2.0f * (gS[3 * r] * p.M[q] + gS[3 * r + 1] * p.M[3 + q] +
                                gS[3 * r + 2] * p.M[6 + q]);
    // M = Rq diag(S)
    float gR[9];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      float acc = 0.0f;
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        gR[3 * r + q] = gM[3 * r + q] * p.S[q];
        acc += gM[3 * r + q] * p.Rq[3 * r + q];
      }
      g[SGS_CH_SCALE + q] += acc * p.S[q];
    }
    // rotation of the unit quaternion (w, x, y, z)
    {
      const float w = p.qh[0], x = p.qh[1], yq = p.qh[2], z = p.qh[3];
      const float gw = 2.0f * (-z * gR[1] + yq * gR[2] + z * gR[3] - x * gR[5] - yq * gR[6] + x * gR[7]);
      const float gx = 2.0f * (yq * gR[1] + z * gR[2] + yq * gR[3] - w * gR[5] + z * gR[6] + w * gR[7]) -
                       4.0f * x * (gR[4] + gR[8]);
      const float gy = 2.0f * (x * gR[1] + w * gR[2] + x * gR[3] + z * gR[5] - w * gR[6] + z * gR[7]) -
                       4.0f * yq * (gR[0] + gR[8]);
      const float gz = 2.0f * (-w * gR[1] + x * gR[2] + w * gR[3] + yq * gR[5] + x * gR[6] + yq * gR[7]) -
                       4.0f * z * (gR[0] + gR[4]);
      const float dot = gw * w + gx * x + gy * yq + gz * z;
      const float iq = 1.0f / p.qn;
      g[SGS_CH_ROT + 0] += (gw - w * dot) * iq;
      g[SGS_CH_ROT + 1] += (gx - x * dot) * iq;
      g[SGS_CH_ROT + 2] += (gy - yq * dot) * iq;
      g[SGS_CH_ROT + 3] += (gz - z * dot) * iq;
    }
    // T = J R_cam
    float gJ00 = 0.f, gJ02 = 0.f, gJ11 = 0.f, gJ12 = 0.f;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      gJ00 += gT0[q] * cam.R[q];
      gJ02 += gT0[q] * cam.R[6 + q];
      gJ11 += gT1[q] * cam.R[3 + q];
      gJ12 += gT1[q] * cam.R[6 + q];
    }
    const float tz = p.tz, itz = 1.0f / tz, itz2 = itz * itz;
    float gtx = 0.f, gty = 0.f, gtz = 0.f;
    gtz -= (gJ00 * cam.fx + gJ11 * cam.fy) * itz2;
    if (!p.clx) {
      gtx -= gJ02 * cam.fx * itz2;
      gtz += gJ02 * 2.0f * cam.fx * p.tx * itz2 * itz;
    } else {
      gtz -= gJ02 * p.J02 * itz;   // J02 = -fx u_clamped / tz
    }
    if (!p.cly) {
      gty -= gJ12 * cam.fy * itz2;
      gtz += gJ12 * 2.0f * cam.fy * p.ty * itz2 * itz;
    } else {
      gtz -= gJ12 * p.J12 * itz;
    }
    // projected mean
    gtx += gpx * cam.fx * itz;
    gty += gpy * cam.fy * itz;
    gtz -= (gpx * cam.fx * p.tx + gpy * cam.fy * p.ty) * itz2;
    // t = R mu + t0
#pragma unroll
    for (int k = 0; k < 3; ++k) g[k] += cam.R[k] * gtx + cam.R[3 + k] * gty + cam.R[6 + k] * gtz;
  }
  if (live) {
#pragma unroll
    for (int j = 0; j < SGS_NCH; ++j)
      if (sh_rows || j < SGS_CH_REST || j >= SGS_CH_REST_END) gout[j * npad + i] = g[j];
    gmask[i] = gm;
    if (FUSED && gscore) {
      float gs = 0.0f;
      if (mode == 1) {
        const float gg = gm + (rate_grad ? rate_grad[192] : 0.0f);
        const float sm = soft[i];
        gs = gg * sm * (1.0f - sm) / tau;
      }
      gscore[i] = gs;
    }
  }
  if (FUSED) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    // four groups of 16 channels (16 double slots each keep the registers
    // within budget)
#pragma unroll
    for (int grp = 0; grp < 4; ++grp) {
      sgs_d16 a;
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        const int j = 16 * grp + k;
        a[k] = j < SGS_NCH ? (double)g[j] * (double)s_r[j][threadIdx.x] : 0.0;
      }
      const double t = wave_transpose_sum16(a);
      if (lane < 16) s_part[wave][16 * grp + lane] = t;
    }
    __syncthreads();
    if (threadIdx.x < SGS_NCH) {
      double t = s_part[0][threadIdx.x];
#pragma unroll
      for (int w = 1; w < kPWaves; ++w) t += s_part[w][threadIdx.x];
      partial[(int64_t)threadIdx.x * gridDim.x + blockIdx.x] = t;
    }
  }
}

}  // namespace

int64_t proj_partial_doubles(int64_t n) { return (int64_t)SGS_NCH * sgs_blocks(n, kPThreads); }

hipError_t launch_preprocess(sgs_ctx *c, const float *qparams, const uint8_t *hard,
                             const float *q) {
  SgsProfScope ps(c, SGS_PROF_PREPROCESS);
  const int64_t nb = sgs_blocks(c->vseg, kPThreads);  // the padding's threads too
  if (q)
    k_preprocess<true><<<nb, kPThreads, 0, c->stream>>>(
        c->n, c->npad, c->V, c->W, c->H, c->TW, c->TH, c->d_cams, qparams, q, hard, c->rec,
        c->depth_key[0], c->depth_val[0], c->touched, c->bin_splat, c->depth_rect[0], c->GW,
        c->tiles_per_view, c->vseg);
  else
    k_preprocess<false><<<nb, kPThreads, 0, c->stream>>>(
        c->n, c->npad, c->V, c->W, c->H, c->TW, c->TH, c->d_cams, qparams, nullptr, hard,
        c->rec, c->depth_key[0], c->depth_val[0], c->touched, c->bin_splat, c->depth_rect[0],
        c->GW, c->tiles_per_view, c->vseg);
  return hipGetLastError();
}

hipError_t launch_preprocess_bwd(sgs_ctx *c, const float *qparams, float *grad_qparams,
                                 float *grad_mask) {
  SgsProfScope ps(c, SGS_PROF_PREPROCESS_BWD);
  k_preprocess_bwd<false><<<sgs_blocks(c->n, kPThreads), kPThreads, 0, c->stream>>>(
      c->n, c->npad, c->V, c->W, c->H, c->d_cams, qparams, nullptr, c->touched, c->splat_grad,
      grad_qparams, grad_mask, nullptr, 0, 1.0f, nullptr, nullptr, nullptr, 1);
  return hipGetLastError();
}

hipError_t launch_preprocess_bwd_fused(sgs_ctx *c, const float *params, const float *q,
                                       int mode, const float *soft, const float *rate_grad,
                                       float *grad_params, float *grad_mask, float *grad_score,
                                       double *partial, int64_t *nblocks) {
  SgsProfScope ps(c, SGS_PROF_PREPROCESS_BWD);
  const int64_t nb = sgs_blocks(c->n, kPThreads);
  if (proj_partial_doubles(c->n) > c->red_tmp_words) return hipErrorInvalidValue;
  *nblocks = nb;
  k_preprocess_bwd<true><<<nb, kPThreads, 0, c->stream>>>(
      c->n, c->npad, c->V, c->W, c->H, c->d_cams, params, q, c->touched, c->splat_grad,
      grad_params, grad_mask, partial, mode, c->tau, soft, rate_grad, grad_score,
      c->grad_sh_rest ? 1 : 0);
  return hipGetLastError();
}
