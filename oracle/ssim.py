"""FP64 oracle of the SSIM part of the rendering distortion.

TEST INFRASTRUCTURE ONLY (imported by ``tests/``).  Plain numpy, FP64.

The paper's supplement ("Training Objective") takes D_render from vanilla
3DGS: D = (1 - w) L1 + w (1 - SSIM), w = 0.2.  SSIM is Wang et al. (2004) with
Gaussian weights: per image plane, window weights g(u) g(v), g the 11-tap
Gaussian of standard deviation 1.5 normalised to sum 1, taken over the image
with zero outside it (so border windows see zeros), C1 = 0.01^2,
C2 = 0.03^2; the per-pixel index

    S = (2 mx my + C1)(2 sxy + C2) / ((mx^2 + my^2 + C1)(sx^2 + sy^2 + C2))

with mx = w*x, sx^2 = w*(x^2) - mx^2, sxy = w*(xy) - mx my, averaged over
every pixel of every plane.
"""
from __future__ import annotations

import numpy as np

C1 = 0.01 ** 2
C2 = 0.03 ** 2
RADIUS = 5
SIGMA = 1.5


def window() -> np.ndarray:
    u = np.arange(-RADIUS, RADIUS + 1, dtype=np.float64)
    g = np.exp(-(u * u) / (2.0 * SIGMA * SIGMA))
    return g / g.sum()


def filt(a: np.ndarray) -> np.ndarray:
    """Window-weighted sum around every pixel of the last two axes, zero
    outside the image: out[p] = sum_q g(p_row - q_row) g(p_col - q_col) a[q]."""
    a = np.asarray(a, np.float64)
    g = window()
    H, W = a.shape[-2:]
    pad = np.zeros(a.shape[:-2] + (H + 2 * RADIUS, W + 2 * RADIUS))
    pad[..., RADIUS:RADIUS + H, RADIUS:RADIUS + W] = a
    rows = np.zeros(a.shape[:-2] + (H + 2 * RADIUS, W))
    for k in range(2 * RADIUS + 1):
        rows += g[k] * pad[..., :, k:k + W]
    out = np.zeros(a.shape)
    for k in range(2 * RADIUS + 1):
        out += g[k] * rows[..., k:k + H, :]
    return out


def moments(x, y):
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    return filt(x), filt(y), filt(x * x), filt(y * y), filt(x * y)


def ssim_map(x, y) -> np.ndarray:
    mx, my, sxx, syy, sxy = moments(x, y)
    A = 2 * mx * my + C1
    B = 2 * (sxy - mx * my) + C2
    C = mx * mx + my * my + C1
    D = (sxx - mx * mx) + (syy - my * my) + C2
    return A * B / (C * D)


def ssim(x, y) -> float:
    return float(ssim_map(x, y).mean())


def ssim_grad(x, y) -> np.ndarray:
    """d mean(S) / d x.  With A, B, C, D as above, per pixel p
        dS/dmx = S (2 my / A - 2 my / B - 2 mx / C + 2 mx / D)
        dS/dsxx = -S / D,  dS/dsxy = 2 S / B   (sxx = w*(x^2), sxy = w*(xy))
    and each moment at p depends on x(q) through g(p - q):
        dmean/dx(q) = (1/N) [ (w * G1)(q) + 2 x(q) (w * G2)(q) + y(q) (w * G3)(q) ]
    (the window is symmetric, so the adjoint is the same filter, zero outside)."""
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    mx, my, sxx, syy, sxy = moments(x, y)
    A = 2 * mx * my + C1
    B = 2 * (sxy - mx * my) + C2
    C = mx * mx + my * my + C1
    D = (sxx - mx * mx) + (syy - my * my) + C2
    S = A * B / (C * D)
    G1 = S * (2 * my / A - 2 * my / B - 2 * mx / C + 2 * mx / D)
    G2 = -S / D
    G3 = 2 * S / B
    N = x.size
    return (filt(G1) + 2 * x * filt(G2) + y * filt(G3)) / N


def dssim_loss(x, y, weight: float = 0.2):
    """(weight * (1 - SSIM), its gradient with respect to x)."""
    return weight * (1.0 - ssim(x, y)), -weight * ssim_grad(x, y)
