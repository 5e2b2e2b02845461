"""Pins of the oracle's rate-proxy variants (CPU): the Laplace proxy's per
value code length against the entropy of quantized Laplace samples (the
high-resolution result it rests on), a two-valued channel in closed form, the
expectation form of the proxy, finite differences of its gradient, and the
additive masking combination."""
import math

import numpy as np

import oracle
from oracle import rate_variants as RV


def test_laplace_code_length_matches_quantized_entropy():
    """Samples of Laplace(0, b0), quantized with q << b0: the empirical
    entropy of the codes approaches log2(2 e b / q) (b the fitted scale)."""
    rng = np.random.default_rng(0)
    n = 2_000_000
    b0 = 0.05
    y = np.zeros((59, n), np.float32)
    y[0] = rng.laplace(0.0, b0, n)
    q = np.full(59, 1.0, np.float32)
    q[0] = b0 / 32
    r = RV.laplace_quant(y, q, n)
    k = np.rint(y[0].astype(np.float64) / q[0]).astype(np.int64)
    _, cnt = np.unique(k, return_counts=True)
    p = cnt / n
    H = -(p * np.log2(p)).sum()
    assert abs(r["L"][0] - H) < 0.01, (r["L"][0], H)
    assert abs(r["b"][0] - b0) < 2e-3 * b0 * 10


def test_two_valued_channel_closed_form_and_expectation_form():
    """Values -a, +a in equal numbers: mean 0, b = a, L = log2(2 e a / q);
    and log2(2 e b) equals the mean of |y~| / (b ln 2) + log2(2 b)."""
    n = 1000
    a = 0.3
    y = np.zeros((59, 1024), np.float32)
    y[:, :n] = np.where(np.arange(n) % 2 == 0, -a, a).astype(np.float32)
    q = np.full(59, 2.0 ** -6, np.float32)
    r = RV.laplace_quant(y, q, n)
    a32 = float(np.float32(a))
    assert np.allclose(r["b"], a32, rtol=1e-15)
    assert np.allclose(r["L"], math.log2(2 * math.e * a32 / 2.0 ** -6), rtol=1e-14)
    yt = y[0, :n].astype(np.float64) - r["mu"][0]
    b = r["b"][0]
    assert abs(np.mean(np.abs(yt) / (b * math.log(2)) + math.log2(2 * b))
               - math.log2(2 * math.e * b)) < 1e-12


def test_laplace_gradient_against_finite_differences():
    rng = np.random.default_rng(1)
    n, npad = 300, 320
    y = rng.normal(0, 0.2, (59, npad)).astype(np.float64)
    q = rng.uniform(2 ** -9, 2 ** -4, 59).astype(np.float32).astype(np.float64)
    q[5] = 10.0                               # an inactive channel (2 e b / q < 1)
    mhat = (rng.random(n) < 0.8).astype(np.uint8)

    def Lq(yv, qv):
        # the proxy in FP64 on FP64 inputs (the oracle casts to float32, so
        # evaluate the definition directly here for the perturbed points)
        yy = yv[:, :n]
        mu = yy.mean(axis=1)
        b = np.abs(yy - mu[:, None]).mean(axis=1)
        ratio = 2 * math.e * b / qv
        return np.where(ratio > 1, np.log2(np.maximum(ratio, 1)), 0).sum()

    r = RV.laplace_quant(y.astype(np.float32), q.astype(np.float32), n)
    y32 = y.astype(np.float32).astype(np.float64)
    h = 1e-7
    for (j, i) in [(0, 0), (7, 123), (58, 299), (5, 10), (30, 77)]:
        yp, ym = y32.copy(), y32.copy()
        yp[j, i] += h
        ym[j, i] -= h
        fd = (Lq(yp, q) - Lq(ym, q)) / (2 * h)
        assert abs(fd - r["gy"][j, i]) < 1e-6 * max(1.0, abs(fd)), (j, i, fd, r["gy"][j, i])
    for j in (0, 5, 40):
        qp, qm = q.copy(), q.copy()
        qp[j] *= 1 + 1e-7
        qm[j] *= 1 - 1e-7
        fd = (Lq(y32, qp) - Lq(y32, qm)) / (q[j] * 2e-7)
        assert abs(fd - r["gq"][j]) < 1e-5 * max(1.0, abs(fd)), (j, fd, r["gq"][j])
    assert r["gq"][5] == 0 and np.all(r["gy"][5] == 0)
    # multiplicative vs additive coupling
    lam, alpha = 0.7, 0.01
    m = RV.rate_variant(y.astype(np.float32), q.astype(np.float32), mhat, n, n, lam, "laplace")
    a = RV.rate_variant(y.astype(np.float32), q.astype(np.float32), mhat, n, n, lam, "laplace",
                        "add", alpha)
    Lm = mhat.sum() / n
    assert abs(m["term"] - lam * Lm * m["Lq"]) < 1e-12
    assert abs(a["term"] - (lam * a["Lq"] + alpha * Lm)) < 1e-12
    assert np.allclose(a["gy"], m["gy"] / Lm) and abs(a["gm"] - alpha / n) < 1e-18
    assert abs(m["gm"] - lam * m["Lq"] / n) < 1e-15


def test_range_proxy_with_additive_masking():
    sc_rng = np.random.default_rng(2)
    n, npad = 500, 512
    y = sc_rng.normal(0, 1, (59, npad)).astype(np.float32)
    q = np.full(59, 2.0 ** -6, np.float32)
    mhat = (sc_rng.random(n) < 0.5).astype(np.uint8)
    base = oracle.rate_proxy(y, q, mhat, n, n, lam=1.0)
    a = RV.rate_variant(y, q, mhat, n, n, 0.3, "range", "add", 0.02)
    assert abs(a["Lq"] - base["Lq"]) < 1e-12
    assert abs(a["term"] - (0.3 * base["Lq"] + 0.02 * base["Lm"])) < 1e-12
    # the range proxy's y gradient sits at the argmin / argmax only
    assert np.count_nonzero(a["gy"]) <= 2 * 59
