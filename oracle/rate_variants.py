"""FP64 oracle of the rate-proxy variants the paper compares with its
range-based, multiplicative proxy.

TEST INFRASTRUCTURE ONLY (imported by ``tests/``).  Plain numpy in FP64 (the
range proxy's own terms come from the C oracle).

- Scale-based Laplace proxy (Sec. 3.3.1 and the supplement's "Comparison with
  an Alternative Rate Proxy"): each channel's centred values modelled as a
  zero-mean Laplace with scale b; its expected code length per value is
  log2(2 e b) (the mean of |y~| / (b ln 2) + log2(2b) when b is the mean
  absolute deviation, the maximum-likelihood scale), and after uniform
  quantization with step q the high-resolution result gives log2(2 e b / q).
  Reading: b_j = mean_i |y_ij - mean_j| over the N current Gaussians (masked
  ones included, as the range), L_j = log2(max(1, 2 e b_j / q_j)).
- Additive masking (the ablation's alternative): the loss carries
  lambda * L_quant + alpha * L_mask instead of lambda * L_mask * L_quant.
"""
from __future__ import annotations

import math

import numpy as np

NCH = 59
LN2 = math.log(2.0)


def laplace_quant(y, q, n):
    """Per-channel (L_j, b_j, mean_j, mean sign_j, active_j) and dL_quant/dy
    [59][npad], dL_quant/dq [59]."""
    y = np.asarray(y, np.float32)
    q64 = np.asarray(q, np.float32).astype(np.float64)
    yy = y[:, :n].astype(np.float64)
    mu = yy.mean(axis=1)
    dev = yy - mu[:, None]
    b = np.abs(dev).mean(axis=1)
    sbar = np.sign(dev).mean(axis=1)
    ratio = 2.0 * math.e * b / q64
    active = ratio > 1.0
    L = np.where(active, np.log2(np.where(active, ratio, 1.0)), 0.0)
    gy = np.zeros(y.shape)
    coef = np.where(active, 1.0 / (np.where(b > 0, b, 1.0) * LN2 * n), 0.0)
    gy[:, :n] = coef[:, None] * (np.sign(dev) - sbar[:, None])
    gq = np.where(active, -1.0 / (q64 * LN2), 0.0)
    return dict(L=L, b=b, mu=mu, sbar=sbar, active=active, gy=gy, gq=gq)


def range_quant(y, q, n):
    """The range proxy's L_quant and its gradient (from the C oracle with
    every Gaussian kept, so L_mask = 1 there)."""
    import oracle
    r = oracle.rate_proxy(y, q, np.ones(n, np.uint8), n, n, lam=1.0)
    return dict(Lq=r["Lq"], gy=r["gy"], gq=r["gq"], c=r["c"])


def rate_variant(y, q, mhat, n, n_hat, lam, proxy="range", masking="mult", alpha=0.0):
    """The rate's term in the loss and its gradients (y dense [59][npad], q,
    and the hard mask, one value per Gaussian)."""
    if proxy == "range":
        r = range_quant(y, q, n)
        Lq, gy, gq = r["Lq"], r["gy"], r["gq"]
    else:
        r = laplace_quant(y, q, n)
        Lq, gy, gq = float(r["L"].sum()), r["gy"], r["gq"]
    Lm = float(np.count_nonzero(np.asarray(mhat)[:n])) / n_hat
    if masking == "mult":
        term = lam * Lm * Lq
        fy = fq = lam * Lm
        gm = lam * Lq / n_hat
    else:
        term = lam * Lq + alpha * Lm
        fy = fq = lam
        gm = alpha / n_hat
    return dict(term=term, Lq=Lq, Lm=Lm, gy=fy * gy, gq=fq * gq, gm=gm, detail=r)
