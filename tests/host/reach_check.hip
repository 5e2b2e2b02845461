// Host check of the blend's reach test (sgs_may_reach): on random splats,
// needle-shaped ones included, and 8x8 sub-tiles placed along their major
// axis, an entry the test drops must fail the alpha cut-off at all 64 pixel
// centres when evaluated the way the blend evaluates a pair (the scaled
// quadratic with the same fused multiply-adds, then opacity 2^p2 against
// 1/255; a pixel within 1e-6 relative of the cut-off counts as passing).
// Prints "trials dropped violations"; exit status 0.
#include <math.h>
#include <stdio.h>
#include <stdint.h>

#include <random>

#include "../../paper_2607_12656_amd/csrc/blend_reach.h"

int main(int argc, char **argv) {
  const long trials = argc > 1 ? atol(argv[1]) : 200000;
  std::mt19937_64 rng(12345);
  std::uniform_real_distribution<double> U(0.0, 1.0);
  const double kac = -0.72134752044448170368, kb = -1.44269504088896340736;
  long dropped = 0, violations = 0;
  for (long t = 0; t < trials; ++t) {
    const double s1 = exp(log(0.5) + U(rng) * (log(2000.0) - log(0.5)));
    const double s2 = 0.3 + U(rng) * 4.7;
    const double th = U(rng) * 3.14159265358979323846;
    const double c = cos(th), s = sin(th);
    // covariance R diag(s1^2, s2^2) R^T + 0.3 I, then its inverse
    const double a = c * c * s1 * s1 + s * s * s2 * s2 + 0.3;
    const double b = c * s * (s1 * s1 - s2 * s2);
    const double d = s * s * s1 * s1 + c * c * s2 * s2 + 0.3;
    const double det = a * d - b * b;
    const double A = d / det, B = -b / det, C = a / det;
    const float Ap = (float)(kac * A), Bp = (float)(kb * B), Cp = (float)(kac * C);
    const float px = (float)(U(rng) * 2000.0), py = (float)(U(rng) * 2000.0);
    const float op = (float)(0.004 + U(rng) * 0.986);
    const float need = -log2f(255.0f * op);
    const double along = (U(rng) * 2.0 - 1.0) * 3.5 * s1;
    const double across = (U(rng) * 2.0 - 1.0) * (3.5 * s2 + 8.0);
    const double qx = px + along * c - across * s, qy = py + along * s + across * c;
    const int sx0 = (int)floor(qx) - (int)(U(rng) * 8.0);
    const int sy0 = (int)floor(qy) - (int)(U(rng) * 8.0);
    if (sgs_may_reach(px, py, Ap, Bp, Cp, need, sx0, sy0)) continue;
    ++dropped;
    bool any = false;
    for (int k = 0; k < 64 && !any; ++k) {
      const float dx = (float)(sx0 + (k & 7)) - px, dy = (float)(sy0 + (k >> 3)) - py;
      const float p2 = fmaf(Ap * dx, dx, fmaf(Cp * dy, dy, Bp * dx * dy));
      const float raw = op * exp2f(p2);
      any = !(p2 > 0.0f) && raw >= (1.0f / 255.0f) * (1.0f - 1e-6f);
    }
    if (any) ++violations;
  }
  printf("%ld %ld %ld\n", trials, dropped, violations);
  return 0;
}
