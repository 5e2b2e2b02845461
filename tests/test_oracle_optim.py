"""Pins of the oracle's optimizer step (CPU): torch's own Adam in FP64 (a
library implementation of Kingma & Ba's algorithm, written independently of
the oracle), the closed form of the first step, and what the two schedule
switches must leave untouched."""
import numpy as np
import pytest

import oracle

torch = pytest.importorskip("torch")


def _state(rng, n, npad):
    x = rng.normal(0, 1, (59, npad))
    g = rng.normal(0, 1, (59, npad)) * rng.choice([1e-3, 1.0, 30.0], (59, 1))
    return x, g


def test_matches_torch_adam_fp64_over_several_steps():
    rng = np.random.default_rng(0)
    n, npad = 300, 320
    x, _ = _state(rng, n, npad)
    lr = rng.uniform(1e-4, 1e-2, 59)
    ps = [torch.nn.Parameter(torch.tensor(x[j, :n].copy())) for j in range(59)]
    opt = torch.optim.Adam([{"params": [p], "lr": float(lr[j])} for j, p in enumerate(ps)],
                           betas=(0.9, 0.999), eps=1e-8)
    xo, m, v = x.copy(), np.zeros_like(x), np.zeros_like(x)
    for t in range(1, 8):
        g = rng.normal(0, 1, (59, npad)) * (10.0 ** rng.integers(-3, 2, (59, 1)))
        for j, p in enumerate(ps):
            p.grad = torch.tensor(g[j, :n].copy())
        opt.step()
        m_prev, v_prev = m, v
        xo, m, v = oracle.adam_params(xo, m, v, g, lr, t, n)
        ref = np.stack([p.detach().numpy() for p in ps])
        np.testing.assert_allclose(xo[:, :n], ref, rtol=1e-12, atol=1e-15)
        st = [opt.state[p] for p in ps]
        # torch forms the moments as m + (1 - b1)(g - m): the two agree to a
        # rounding of the terms (compounded over the steps), not of a result
        # that cancels
        scale_m = np.abs(m_prev[:, :n]) + np.abs(g[:, :n])
        scale_v = v_prev[:, :n] + g[:, :n] ** 2
        assert np.all(np.abs(m[:, :n] - np.stack([s["exp_avg"].numpy() for s in st]))
                      <= 1e-12 * scale_m)
        assert np.all(np.abs(v[:, :n] - np.stack([s["exp_avg_sq"].numpy() for s in st]))
                      <= 1e-12 * scale_v)
    assert np.array_equal(xo[:, n:], x[:, n:]), "padding columns untouched"


def test_first_step_closed_form():
    """From zero moments, step 1 moves every entry by lr * g / (|g| + eps)."""
    rng = np.random.default_rng(1)
    x = rng.normal(0, 1, 1000)
    g = rng.normal(0, 1, 1000) * 10.0 ** rng.integers(-6, 3, 1000)
    lr = 3e-3
    x1, m1, v1 = oracle.adam_vector(x, 0.0 * x, 0.0 * x, g, lr, 1, 0.9, 0.999, 1e-8)
    np.testing.assert_allclose(x1, x - lr * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    np.testing.assert_allclose(m1, 0.1 * g, rtol=1e-15)
    np.testing.assert_allclose(v1, 0.001 * g * g, rtol=1e-14)


def test_sh_rest_and_sparse_switches():
    rng = np.random.default_rng(2)
    n, npad = 200, 256
    x, g = _state(rng, n, npad)
    m = rng.normal(0, 0.1, (59, npad))
    v = m * m + rng.uniform(0, 0.01, (59, npad))
    dead = rng.random(n) < 0.2
    g[:, :n][:, dead] = 0.0
    only_sh = rng.random(n) < 0.1                 # gradient only in the SH rest rows
    g[:, :n][:, only_sh] = 0.0
    g[6:51, :n][:, only_sh] = 1.0
    lr = np.full(59, 1e-2)
    # sh_rest off: rows 6-50 bit-identical, other rows move
    x1, m1, v1 = oracle.adam_params(x, m, v, g, lr, 5, n, sh_rest=False)
    assert np.array_equal(x1[6:51], x[6:51]) and np.array_equal(m1[6:51], m[6:51])
    assert np.array_equal(v1[6:51], v[6:51])
    assert np.all(x1[:6, :n] != x[:6, :n])
    # sparse: dead Gaussians keep everything; with sh_rest off the SH-only ones too
    x2, m2, v2 = oracle.adam_params(x, m, v, g, lr, 5, n, sh_rest=False, sparse=True)
    skip = dead | only_sh
    for a, b in ((x2, x), (m2, m), (v2, v)):
        assert np.array_equal(a[:, :n][:, skip], b[:, :n][:, skip])
    assert np.all(x2[:6, :n][:, ~skip] != x[:6, :n][:, ~skip])
    # sparse with sh_rest on: the SH-only ones now update in every row
    x3, _, _ = oracle.adam_params(x, m, v, g, lr, 5, n, sh_rest=True, sparse=True)
    zero = dead & ~only_sh
    assert np.array_equal(x3[:, :n][:, zero], x[:, :n][:, zero])
    assert np.all(x3[6:51, :n][:, only_sh] != x[6:51, :n][:, only_sh])


def test_compact_against_a_plain_loop():
    """The oracle's compaction equals appending the kept columns one by one."""
    rng = np.random.default_rng(4)
    n, npad = 150, 192
    a = rng.normal(0, 1, (59, npad))
    b = rng.normal(0, 1, npad)
    mask = (rng.random(npad) < 0.6).astype(np.uint8) * rng.integers(1, 255, npad).astype(np.uint8)
    ca, cb = oracle.compact([a, b], mask, n)
    cols_a, vals_b = [], []
    for i in range(n):
        if mask[i]:
            cols_a.append(a[:, i])
            vals_b.append(b[i])
    assert np.array_equal(ca, np.stack(cols_a, axis=1)) and np.array_equal(cb, np.array(vals_b))
    assert ca.shape == (59, int((mask[:n] != 0).sum()))
    none = oracle.compact([a], np.zeros(npad, np.uint8), n)[0]
    assert none.shape == (59, 0)
