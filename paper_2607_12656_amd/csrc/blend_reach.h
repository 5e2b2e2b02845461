// Reach test of the blend (csrc/blend.hip): whether a splat can pass the
// alpha cut-off at any pixel centre of the 8x8 sub-tile whose first pixel
// is (sx0, sy0).  Plain float arithmetic, callable from host code too.
//
// The record holds the splat's exponent in base 2 as the quadratic
//   p2(dx, dy) = A' dx^2 + B' dx dy + C' dy^2,  dx = x - px, dy = y - py,
// and a pixel passes the cut-off only if p2 >= need = log2(1 / (255 o))
// (o the opacity).  With A' < 0 and C' < 0 the largest p2 over the
// rectangle of pixel centres is 0 when (px, py) lies inside; otherwise it
// lies on an edge, where p2 restricted to the edge is a concave parabola
// whose best point is clamped to the edge (this holds whether or not the
// whole form is definite).  The entry is kept when that largest value comes
// within a margin of `need`: 0.05 plus 2^-20 times the size of the terms
// over the rectangle, which bounds the rounding of the edge evaluation here
// and of the per-pixel evaluation in the blend (a needle splat's terms can
// reach 1e6 while their sum stays near `need`).  A form that is not
// negative along both axes, or any NaN, keeps the entry.
#ifndef SGS_BLEND_REACH_H
#define SGS_BLEND_REACH_H

#include <hip/hip_runtime.h>

__host__ __device__ inline bool sgs_may_reach(float px, float py, float Ap, float Bp, float Cp,
                                              float need, int sx0, int sy0) {
  if (!(Ap < 0.0f && Cp < 0.0f)) return true;
  const float x0 = (float)sx0 - px, x1 = x0 + 7.0f;
  const float y0 = (float)sy0 - py, y1 = y0 + 7.0f;
  if (x0 <= 0.0f && x1 >= 0.0f && y0 <= 0.0f && y1 >= 0.0f) return true;
  const float kx = -0.5f * Bp / Cp, ky = -0.5f * Bp / Ap;
  const auto p2 = [&](float dx, float dy) { return Ap * dx * dx + Cp * dy * dy + Bp * dx * dy; };
  const auto on_x = [&](float dx) { return p2(dx, fminf(fmaxf(kx * dx, y0), y1)); };
  const auto on_y = [&](float dy) { return p2(fminf(fmaxf(ky * dy, x0), x1), dy); };
  const float best = fmaxf(fmaxf(on_x(x0), on_x(x1)), fmaxf(on_y(y0), on_y(y1)));
  const float xm = fmaxf(fabsf(x0), fabsf(x1)), ym = fmaxf(fabsf(y0), fabsf(y1));
  const float mag = fabsf(Ap) * xm * xm + fabsf(Cp) * ym * ym + fabsf(Bp) * xm * ym;
  return !(best + 0.05f + mag * 0x1p-20f < need);
}

#endif  // SGS_BLEND_REACH_H
