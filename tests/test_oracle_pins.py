"""Pins for the FP64 oracle: facts fixed by the paper or by mathematics, not by
the oracle's own formulas.  CPU only.

Each test names what it pins and the passage (paper section / equation) or the
textbook fact it follows.  A plausible slip in the oracle (a dropped term, a
wrong sign or index, a transposed operand) fails at least one of them.
"""
import math
import os

import numpy as np
import pytest

import synth
from synth import NCH, CH_DC, CH_REST, CH_OPA, CH_SCALE, CH_ROT

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------------------
# counter RNG and decision-layer exponential
# ---------------------------------------------------------------------------

def test_splitmix64_published_outputs(orc):
    """SplitMix64 from state 0 (published sequence) drives the Gumbel noise."""
    vals = [int(l, 16) for l in open(os.path.join(GOLDEN, "splitmix64_seed0.txt"))
            if l.startswith("0x")]
    gamma = 0x9E3779B97F4A7C15
    for k, h in enumerate(vals):
        seed = (k * gamma) % (1 << 64)
        u = orc.uniform(seed, 0, 0)
        assert u == ((h >> 41) + 0.5) * 2.0 ** -23


def test_exp_dl_accuracy(orc):
    """Cody-Waite + degree-7 Taylor exp: within 4 ulp of exp over [-80, 80]."""
    assert orc.exp_dl(0.0) == 1.0
    xs = np.concatenate([np.linspace(-80, 80, 4001), np.linspace(-8, 2, 2001)]).astype(np.float32)
    for x in xs:
        e = orc.exp_dl(float(x))
        ref = math.exp(float(x))
        assert abs(e - ref) <= 4 * np.spacing(np.float32(ref)), (x, e, ref)


# ---------------------------------------------------------------------------
# a1 / a12: quantizer (Sec. 3.3.1 uniform quantization with step q_j)
# ---------------------------------------------------------------------------

def test_quantizer_properties(orc):
    rng = np.random.default_rng(5)
    n = 1000
    y = rng.normal(0, 1, size=(NCH, 1024)).astype(np.float32)
    q = (2.0 ** rng.uniform(-9, -2, size=NCH)).astype(np.float32)
    yh, k = orc.fakequant(y, q, n)
    # error bounded by half a step (plus the one rounding of k*q)
    err = np.abs(yh[:, :n].astype(np.float64) - y[:, :n])
    bound = q[:, None].astype(np.float64) / 2 + np.spacing(np.abs(yh[:, :n]))
    assert np.all(err <= bound)
    # idempotent
    yh2, k2 = orc.fakequant(yh, q, n)
    assert np.array_equal(yh2[:, :n], yh[:, :n]) and np.array_equal(k2[:, :n], k[:, :n])
    # power-of-two step: reconstruction exact
    q2 = np.full(NCH, 2.0 ** -6, np.float32)
    yh3, k3 = orc.fakequant(y, q2, n)
    assert np.array_equal(yh3[:, :n].astype(np.float64), k3[:, :n] * 2.0 ** -6)
    # round half to even
    yt = np.zeros((NCH, 64), np.float32)
    yt[0, :4] = np.array([0.5, 1.5, 2.5, -0.5]) * 0.25
    _, kt = orc.fakequant(yt, np.full(NCH, 0.25, np.float32), 4)
    assert list(kt[0, :4]) == [0, 2, 2, 0]


def test_lsq_gradient_is_quantization_error_over_step(orc):
    """LSQ step gradient k - y/q equals (yhat - y)/q; STE passes dy unchanged."""
    rng = np.random.default_rng(6)
    n = 200
    y = rng.normal(0, 1, size=(NCH, 256)).astype(np.float32)
    q = np.full(NCH, 0.1, np.float32)
    yh, k = orc.fakequant(y, q, n)
    g = np.zeros((NCH, 256))
    g[:, :n] = rng.normal(size=(NCH, n))
    gy, gq, gs = orc.fakequant_bwd(y, q, g, 0, np.zeros(n), 1.0, np.zeros(n), n)
    assert np.array_equal(gy, g)
    ref = (g[:, :n] * (k[:, :n].astype(np.float64) - y[:, :n].astype(np.float64)
                       / q[:, None].astype(np.float64))).sum(1)
    err_form = (g[:, :n] * ((yh[:, :n].astype(np.float64) - y[:, :n]) / q[:, None])).sum(1)
    assert np.allclose(gq, ref, rtol=1e-12, atol=1e-12)
    assert np.allclose(gq, err_form, rtol=1e-5, atol=1e-6)
    # on-grid inputs (exact multiples of a power-of-two step) give no step gradient
    qp = np.full(NCH, 2.0 ** -4, np.float32)
    yg, _ = orc.fakequant(y, qp, n)
    gy2, gq2, _ = orc.fakequant_bwd(yg, qp, g, 0, np.zeros(n), 1.0, np.zeros(n), n)
    assert np.all(gq2 == 0.0)


# ---------------------------------------------------------------------------
# a2: retention mask (Sec. 3.3.1 p_i = sigma(s_i), M_i = GumbelSoftmax(p_i))
# ---------------------------------------------------------------------------

def test_mask_closed_form_and_frequency(orc):
    n = 200_000
    rng = np.random.default_rng(7)
    s = rng.normal(0.5, 1.5, size=n).astype(np.float32)
    mh, ms = orc.mask(n, 1, None, s, seed=11, step=3, tau=0.7)
    u = np.array([orc.uniform(11, 3, i) for i in range(2000)], np.float64)
    ell = np.log(u) - np.log1p(-u)
    z = s[:2000].astype(np.float64) + ell
    assert np.allclose(ms[:2000], 1 / (1 + np.exp(-z / 0.7)), rtol=1e-12)
    away = np.abs(z) > 1e-5
    assert np.array_equal(mh[:2000][away], (z[away] > 0).astype(np.uint8))
    # P(M=1) = sigma(s): compare the kept count to its expectation (4 sd)
    p = 1 / (1 + np.exp(-s.astype(np.float64)))
    assert abs(mh.sum() - p.sum()) < 4 * math.sqrt((p * (1 - p)).sum())
    # given / keep-all modes
    g = (rng.random(n) < 0.3).astype(np.uint8)
    mh0, ms0 = orc.mask(n, 0, g, s)
    assert np.array_equal(mh0, g) and np.array_equal(ms0, g.astype(float))
    mh2, _ = orc.mask(n, 2, None, s)
    assert mh2.all()
    # counter-based: the same (seed, step) reproduces, another step differs
    mh_again, _ = orc.mask(n, 1, None, s, seed=11, step=3, tau=0.7)
    assert np.array_equal(mh_again, mh)
    assert not np.array_equal(orc.mask(n, 1, None, s, seed=11, step=4)[0], mh)


# ---------------------------------------------------------------------------
# a3: rate proxy (Sec. 3.3.1 Eqs. L_j, L_quant, L_mask, R_proxy)
# ---------------------------------------------------------------------------

def _rate_scene(n=64):
    y = np.zeros((NCH, 64), np.float32)
    rng = np.random.default_rng(8)
    y[:, :n] = rng.uniform(-0.4, 0.4, size=(NCH, n))
    return y


def test_rate_proxy_hand_cases(orc):
    n = 64
    y = _rate_scene(n)
    y[0, 3], y[0, 7] = -0.5, 0.5           # range exactly 1
    y[1, :n] = 0.25                        # range 0
    y[2, 10], y[2, 20] = -0.5, 0.5         # range 1 with q = 0.3 -> ceil(3.33) = 4
    y[3, 5] = y[3, 9] = 0.9                # tied maxima: lowest index wins
    y[3, 2] = y[3, 30] = -0.9
    q = np.full(NCH, 2.0 ** -6, np.float32)
    q[2] = 0.3
    m = np.ones(n, np.uint8)
    m[:16] = 0
    r = orc.rate_proxy(y, q, m, n, n_hat=100)
    assert r["c"][0] == 64 and math.log2(r["c"][0]) == 6.0
    assert r["c"][1] == 1.0
    assert r["c"][2] == 4.0
    assert r["argmax"][3] == 5 and r["argmin"][3] == 2
    assert r["argmax"][0] == 7 and r["argmin"][0] == 3
    assert r["Lm"] == 48 / 100
    Lq = sum(math.log2(c) for c in r["c"])
    assert r["Lq"] == pytest.approx(Lq, rel=1e-15)
    assert r["R"] == pytest.approx(0.48 * Lq, rel=1e-15)


def test_rate_gradient_matches_smooth_proxy_at_integer_ratio(orc):
    """Where R_j/q_j is an integer the straight-through gradient equals the
    derivative of the smooth log2(R_j/q_j); masked-count gradient is L_quant/N_hat."""
    n = 64
    y = _rate_scene(n)
    y[:, 3], y[:, 7] = -0.5, 0.5
    q = np.full(NCH, 2.0 ** -6, np.float32)
    m = np.ones(n, np.uint8)
    lam = 0.7
    r = orc.rate_proxy(y, q, m, n, n_hat=n, lam=lam)
    Lm, Lq = r["Lm"], r["Lq"]
    h = 1e-7
    for j in (0, 17, 58):
        Rj, qj = 1.0, float(q[j])
        f = lambda R, qq: math.log2(R / qq)
        dR = (f(Rj + h, qj) - f(Rj - h, qj)) / (2 * h)
        dq = (f(Rj, qj + h * qj) - f(Rj, qj - h * qj)) / (2 * h * qj)
        assert r["gy"][j, 7] == pytest.approx(lam * Lm * dR, rel=1e-6)
        assert r["gy"][j, 3] == pytest.approx(-lam * Lm * dR, rel=1e-6)
        assert r["gq"][j] == pytest.approx(lam * Lm * dq, rel=1e-6)
    assert np.allclose(r["gm"], lam * Lq / n)
    assert np.count_nonzero(r["gy"]) == 2 * NCH


def test_high_resolution_quantization_entropy():
    """Supp. derivation: a Laplace(b) source quantized with step q << b has
    entropy close to log2(2 e b / q)."""
    rng = np.random.default_rng(9)
    b, q = 1.0, 0.05
    x = rng.laplace(0, b, size=2_000_000)
    k = np.rint(x / q).astype(np.int64)
    _, cnt = np.unique(k, return_counts=True)
    p = cnt / cnt.sum()
    H = -(p * np.log2(p)).sum()
    assert abs(H - math.log2(2 * math.e * b / q)) < 0.01


# ---------------------------------------------------------------------------
# SH basis (Sec. 3.1: view-dependent colour c_i; 48 colour channels)
# ---------------------------------------------------------------------------

def _sphere_quadrature(nt=24, nphi=48):
    xg, wg = np.polynomial.legendre.leggauss(nt)
    phi = (np.arange(nphi) + 0.5) * 2 * np.pi / nphi
    Z, PH = np.meshgrid(xg, phi, indexing="ij")
    W = np.repeat(wg[:, None], nphi, 1) * (2 * np.pi / nphi)
    S = np.sqrt(1 - Z ** 2)
    d = np.stack([S * np.cos(PH), S * np.sin(PH), Z], -1).reshape(-1, 3)
    return d, W.reshape(-1)


def test_sh_orthonormal_and_textbook_values(orc):
    d, w = _sphere_quadrature()
    Y = orc.sh_basis(d)
    G = (Y * w[:, None]).T @ Y
    assert np.allclose(G, np.eye(16), atol=1e-12)
    c1 = math.sqrt(3 / (4 * math.pi))
    Yx, Yy, Yz = orc.sh_basis(np.eye(3))
    assert Yx[0] == pytest.approx(1 / (2 * math.sqrt(math.pi)), rel=1e-15)
    # Condon-Shortley phase, index l^2 + l + m
    assert Yy[1] == pytest.approx(-c1) and Yz[2] == pytest.approx(c1) and Yx[3] == pytest.approx(-c1)
    for l in range(4):
        assert Yz[l * l + l] == pytest.approx(math.sqrt((2 * l + 1) / (4 * math.pi)), rel=1e-14)
    # addition theorem: sum_m Y_lm(d)^2 = (2l+1)/(4 pi) for every direction
    rng = np.random.default_rng(1)
    v = rng.normal(size=(50, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    Yr = orc.sh_basis(v)
    for l in range(4):
        s = (Yr[:, l * l:(l + 1) ** 2] ** 2).sum(1)
        assert np.allclose(s, (2 * l + 1) / (4 * math.pi), rtol=1e-13)


# ---------------------------------------------------------------------------
# Projection + compositing (Sec. 3.1 Eq. G(x) and the compositing equation)
# ---------------------------------------------------------------------------

def _empty_params(n):
    p = np.zeros((NCH, synth.pad64(n)), np.float32)
    p[CH_ROT, :n] = 1.0
    return p


def test_single_isotropic_gaussian_closed_form(orc):
    """On-axis isotropic Gaussian: Sigma' = ((f s / z)^2 + 0.3) I whatever the
    rotation; every pixel equals c * opacity * exp(-|d|^2 / (2 sigma'^2))."""
    W = H = 96
    cam = synth.camera_axis(W, H, 3.0)[None]
    p = _empty_params(1)
    s = 0.09
    p[CH_SCALE:CH_ROT, 0] = math.log(s)
    qrot = np.random.default_rng(3).normal(size=4)
    p[CH_ROT:, 0] = qrot / np.linalg.norm(qrot)
    p[0:3, 0] = (0.0, 0.0, 0.5)
    p[CH_OPA, 0] = 1.2
    p[CH_DC:CH_DC + 3, 0] = (0.3, -0.2, 0.1)
    st = orc.decide(p, 1, cam, W, H)
    assert st.valid[0, 0] == 1
    p64 = p.astype(np.float64)
    fw = orc.forward(p64, np.ones(1), 1, cam, W, H, st)
    f = float(cam[0, 12])
    z = 3.0 + float(p[2, 0])
    sig2 = (f * math.exp(float(p[CH_SCALE, 0])) / z) ** 2 + 0.3
    opa = 1 / (1 + math.exp(-float(p[CH_OPA, 0])))
    Y00 = 1 / (2 * math.sqrt(math.pi))
    col = np.maximum(p64[CH_DC:CH_DC + 3, 0] * Y00 + 0.5, 0)
    u, v = np.meshgrid(np.arange(W), np.arange(H))
    d2 = (u - W / 2) ** 2 + (v - H / 2) ** 2
    a = np.minimum(0.99, opa * np.exp(-0.5 * d2 / sig2))
    r = math.ceil(3 * math.sqrt(sig2))
    inside = (np.abs(u - W / 2) <= r) & (np.abs(v - H / 2) <= r) & (a >= 1 / 255)
    a = np.where(inside, a, 0.0)
    for ch in range(3):
        assert np.allclose(fw["image"][0, ch], col[ch] * a, atol=1e-12)
    assert np.allclose(fw["T"][0], 1 - a, atol=1e-12)
    assert st.radius[0, 0] == r
    # total alpha bracketed by the Gaussian's mass inside radius 3 sigma' and
    # inside the alpha cut-off radius (square span contains the first disk)
    tot = (fw["image"][0, 0] / col[0]).sum()
    unclamped = opa * 2 * math.pi * sig2
    rc2 = 2 * math.log(255 * opa)
    assert unclamped * (1 - math.exp(-4.5)) - 1e-6 <= tot <= unclamped * (1 - math.exp(-rc2 / 2)) + 1e-6


def _tiny(n=40, W=48, H=40, V=1, seed=0, logscale=-2.0):
    return synth.make_tiny(n, W, H, views=V, seed=seed, logscale_mu=logscale)


def test_decision_layer_agrees_with_fp64_projection(orc):
    """The FP32 decision layer (depth, mean, radius) agrees with the FP64
    projection: radius = ceil(3 sqrt(lambda_max(Sigma'))) from the FP64 conic."""
    sc = synth.make_scene("c1", n=2048)
    yh, _ = orc.fakequant(sc.params, sc.qstep, sc.n)
    st = orc.decide(yh, sc.n, sc.cams, sc.width, sc.height)
    pj = orc.project64(yh.astype(np.float64), sc.n, sc.cams, sc.width, sc.height, st)[0]
    ok = st.valid[0] == 1
    assert ok.sum() > 1500
    A, B, Cc = pj[ok, 2], pj[ok, 3], pj[ok, 4]
    # eigenvalues of Sigma' are reciprocals of those of the conic
    tr, det = A + Cc, A * Cc - B * B
    lmin_conic = tr / 2 - np.sqrt(np.maximum(tr * tr / 4 - det, 0))
    lmax = 1 / lmin_conic
    x = 3 * np.sqrt(lmax)
    clear = np.abs(x - np.rint(x)) > 1e-4
    assert np.array_equal(st.radius[0, ok][clear], np.ceil(x[clear]).astype(np.int32))
    assert np.allclose(st.pxy[0, ok, 0], pj[ok, 0], rtol=0, atol=1e-4)
    assert np.allclose(st.pxy[0, ok, 1], pj[ok, 1], rtol=0, atol=1e-4)


def test_compositing_invariants(orc):
    """Telescoping: with every colour 1, C = 1 - T_final; T stays in (0, 1];
    splats with hard mask 0 leave the image bitwise unchanged."""
    sc = _tiny(n=60)
    p = sc.params.copy()
    p[CH_DC:CH_DC + 3, :sc.n] = math.sqrt(math.pi)   # Y00 * sqrt(pi) + 1/2 = 1
    p[CH_REST:CH_OPA, :sc.n] = 0.0
    st = orc.decide(p, sc.n, sc.cams, sc.width, sc.height)
    fw = orc.forward(p.astype(np.float64), np.ones(sc.n), sc.n, sc.cams, sc.width, sc.height, st)
    assert fw["evals"] > 0
    for ch in range(3):
        assert np.allclose(fw["image"][0, ch], 1 - fw["T"][0], atol=1e-12)
    assert (fw["T"] > 0).all() and (fw["T"] <= 1).all()
    # add masked copies of other splats: image identical to the last bit
    extra = _tiny(n=30, seed=5)
    n2 = sc.n + extra.n
    p2 = np.zeros((NCH, synth.pad64(n2)), np.float32)
    p2[:, :sc.n] = p[:, :sc.n]
    p2[:, sc.n:n2] = extra.params[:, :extra.n]
    m2 = np.concatenate([np.ones(sc.n), np.zeros(extra.n)])
    st2 = orc.decide(p2, n2, sc.cams, sc.width, sc.height)
    assert st2.keys.size > st.keys.size
    fw2 = orc.forward(p2.astype(np.float64), m2, n2, sc.cams, sc.width, sc.height, st2)
    assert np.array_equal(fw2["image"], fw["image"]) and np.array_equal(fw2["T"], fw["T"])


@pytest.mark.parametrize("tile", [(8, 8), (16, 16), (32, 8)])
@pytest.mark.parametrize("V", [1, 2])
def test_brute_force_equals_binned(orc, tile, V):
    """Sec. 3.1: per-pixel compositing over ALL Gaussians in depth order (the
    definition) equals the tile-binned lists, for every tile shape."""
    sc = _tiny(n=48, W=45, H=37, V=V, seed=2)
    yh, _ = orc.fakequant(sc.params, sc.qstep, sc.n)
    m = sc.given_mask.astype(np.float64)
    st = orc.decide(yh, sc.n, sc.cams, sc.width, sc.height, *tile)
    p64 = yh.astype(np.float64)
    fb = orc.forward(p64, m, sc.n, sc.cams, sc.width, sc.height, st)
    br = orc.forward_brute(p64, m, sc.n, sc.cams, sc.width, sc.height, st)
    assert np.array_equal(fb["image"], br["image"]) and np.array_equal(fb["T"], br["T"])
    assert fb["evals"] == br["evals"] > 0
    # tile-shape independence of the image
    st16 = orc.decide(yh, sc.n, sc.cams, sc.width, sc.height, 16, 16)
    f16 = orc.forward(p64, m, sc.n, sc.cams, sc.width, sc.height, st16)
    assert np.array_equal(f16["image"], fb["image"])


def test_tile_lists_by_enumeration(orc):
    """Every (tile, Gaussian) pair whose pixel span meets the tile, ordered by
    (tile, depth, index): rebuilt here by a direct rectangle test."""
    sc = _tiny(n=64, W=70, H=50, V=2, seed=3)
    yh, _ = orc.fakequant(sc.params, sc.qstep, sc.n)
    TW, TH = 16, 8
    st = orc.decide(yh, sc.n, sc.cams, sc.width, sc.height, TW, TH)
    GW, GH = -(-sc.width // TW), -(-sc.height // TH)
    pairs = []
    for v in range(2):
        for t in range(GW * GH):
            tx, ty = t % GW, t // GW
            X0, X1, Y0, Y1 = tx * TW, min(tx * TW + TW, sc.width) - 1, ty * TH, min(ty * TH + TH, sc.height) - 1
            for i in range(sc.n):
                if not st.valid[v, i]:
                    continue
                x0, x1, y0, y1 = st.span[v, i]
                if x0 <= X1 and x1 >= X0 and y0 <= Y1 and y1 >= Y0:
                    pairs.append((v * GW * GH + t, int(st.tz[v, i].view(np.uint32)), i))
    pairs.sort()
    keys = np.array([(a << 32) | b for a, b, _ in pairs], np.uint64)
    vals = np.array([c for _, _, c in pairs], np.uint32)
    assert np.array_equal(st.keys, keys) and np.array_equal(st.vals, vals)
    for t in range(2 * GW * GH):
        b, e = st.ranges[t]
        sel = (keys >> np.uint64(32)) == t
        if sel.any():
            idx = np.nonzero(sel)[0]
            assert b == idx[0] and e == idx[-1] + 1
        else:
            assert b == e


def test_depth_ties_resolved_by_index_and_permutation_invariance(orc):
    W = H = 32
    cam = synth.camera_axis(W, H, 3.0)[None]
    p = _empty_params(2)
    for i, (x, col) in enumerate([(0.0, 1.0), (0.02, -1.0)]):
        p[0:3, i] = (x, 0.0, 0.0)     # same depth
        p[CH_SCALE:CH_ROT, i] = math.log(0.1)
        p[CH_OPA, i] = 2.0
        p[CH_DC, i] = col
    st = orc.decide(p, 2, cam, W, H)
    assert st.tz[0, 0] == st.tz[0, 1]
    a = orc.forward(p.astype(np.float64), np.ones(2), 2, cam, W, H, st)["image"]
    ps = p[:, [1, 0] + list(range(2, p.shape[1]))].copy()
    sts = orc.decide(ps, 2, cam, W, H)
    b = orc.forward(ps.astype(np.float64), np.ones(2), 2, cam, W, H, sts)["image"]
    # centre pixel: index 0 is in front, so its (red-heavy) colour dominates
    assert a[0, 0, 16, 16] > b[0, 0, 16, 16]
    # without ties a permutation of the inputs changes nothing
    sc = _tiny(n=30, seed=4)
    perm = np.random.default_rng(0).permutation(sc.n)
    pp = sc.params.copy()
    pp[:, :sc.n] = sc.params[:, perm]
    s1 = orc.decide(sc.params, sc.n, sc.cams, sc.width, sc.height)
    s2 = orc.decide(pp, sc.n, sc.cams, sc.width, sc.height)
    assert len(set(s1.tz[0][s1.valid[0] > 0].tolist())) == int(s1.valid[0].sum())
    i1 = orc.forward(sc.params.astype(np.float64), np.ones(sc.n), sc.n, sc.cams, sc.width, sc.height, s1)
    i2 = orc.forward(pp.astype(np.float64), np.ones(sc.n), sc.n, sc.cams, sc.width, sc.height, s2)
    assert np.array_equal(i1["image"], i2["image"])


# ---------------------------------------------------------------------------
# a10 / a11: analytic gradients against central finite differences
# ---------------------------------------------------------------------------

def _fd_check(orc, sc, n_gauss=8, seed=0):
    yh, _ = orc.fakequant(sc.params, sc.qstep, sc.n)
    st = orc.decide(yh, sc.n, sc.cams, sc.width, sc.height)
    p64 = yh.astype(np.float64)
    m = np.where(sc.given_mask > 0, 1.0, 0.0)
    rng = np.random.default_rng(seed)
    w = rng.normal(size=(sc.views, 3, sc.height, sc.width))
    gp, gm, _ = orc.backward(p64, m, sc.n, sc.cams, sc.width, sc.height, st, w)

    def loss(pp, mm):
        f = orc.forward(pp, mm, sc.n, sc.cams, sc.width, sc.height, st)
        return float((f["image"] * w).sum())

    gmax = max(np.abs(gp).max(), np.abs(gm).max())
    infl = np.abs(gp[:, :sc.n]).sum(0)
    cand = np.argsort(-infl)[:n_gauss]
    checked = skipped = 0
    worst = 0.0
    for i in cand:
        for j in list(range(NCH)) + ["mask"]:
            if j == "mask":
                x0 = m[i]
                hs = 1e-6
                def ev(d):
                    mm = m.copy(); mm[i] = x0 + d
                    return loss(p64, mm)
                g_an = gm[i]
            else:
                x0 = p64[j, i]
                hs = 1e-6 * max(1.0, abs(x0))
                def ev(d):
                    pp = p64.copy(); pp[j, i] = x0 + d
                    return loss(pp, m)
                g_an = gp[j, i]
            f1 = (ev(hs) - ev(-hs)) / (2 * hs)
            f2 = (ev(2 * hs) - ev(-2 * hs)) / (4 * hs)
            # FD round-off is ~1e-9 absolute here, so tiny entries are judged
            # against a floor of 1e-3 of the largest gradient
            scale = abs(f1) + 1e-3 * gmax
            if abs(f1 - f2) > 1e-5 * scale:
                skipped += 1          # a per-pair decision flips within +-2h
                continue
            checked += 1
            worst = max(worst, abs(f1 - g_an) / scale)
    return checked, skipped, worst


@pytest.mark.parametrize("V", [1, 2])
def test_backward_matches_finite_differences(orc, V):
    sc = _tiny(n=36, W=40, H=36, V=V, seed=6)
    checked, skipped, worst = _fd_check(orc, sc)
    assert checked >= 0.9 * (checked + skipped) and checked > 100
    assert worst < 1e-6, worst


def test_backward_with_clamped_direction_and_colour(orc):
    """Gaussians outside the 1.3x field-of-view clamp and with clamped colour."""
    sc = synth.make_tiny(30, 40, 32, seed=12, logscale_mu=-1.5, spread=1.6, dist=2.2)
    yh, _ = orc.fakequant(sc.params, sc.qstep, sc.n)
    st = orc.decide(yh, sc.n, sc.cams, sc.width, sc.height)
    pj = orc.project64(yh.astype(np.float64), sc.n, sc.cams, sc.width, sc.height, st)
    tz = st.tz[0]
    ux = np.abs(((sc.cams[0, 0:3] @ yh[0:3, :sc.n]) + sc.cams[0, 9]) / tz)
    assert (ux[st.valid[0] > 0] > 1.3 * 0.5 * sc.width / sc.cams[0, 12]).any()
    checked, skipped, worst = _fd_check(orc, sc, n_gauss=10, seed=2)
    assert checked > 100 and worst < 1e-6, worst


# ---------------------------------------------------------------------------
# a9: L1 distortion; Sec. 3.4.1 fixed-length code length
# ---------------------------------------------------------------------------

def test_l1_hand_case(orc):
    img = np.array([0.5, 0.5, 0.875, 0.375])
    tgt = np.array([0.25, 0.5, 1.0, 0.0], np.float32)
    D, d = orc.l1(img, tgt)
    assert D == (0.25 + 0 + 0.125 + 0.375) / 4
    assert list(d) == [0.25, 0.0, -0.25, 0.25]


def test_fixed_length_coder_hand_case_and_round_trip(orc):
    n = 5
    k = np.zeros((NCH, 64), np.int32)
    k[0, :n] = [3, -2, 5, 100, 0]     # kept: 3, -2, 5, 0 -> K = 8 -> 3 bits
    k[1, :n] = [7, 7, 7, 7, 7]        # K = 1 -> 0 bits
    k[2, :n] = [0, 1, 0, 1, 9]        # kept: 0, 1, 0, 9 -> K = 10 -> 4 bits
    m = np.array([1, 1, 1, 0, 1], np.uint8)
    bits, kmin, kmax, width = orc.fixed_length_bits(k, m, n)
    assert (width[0], width[1], width[2]) == (3, 0, 4)
    assert (kmin[0], kmax[0]) == (-2, 5)
    assert width[3:].sum() == 0
    assert bits == 4 * (3 + 0 + 4) + 59 * 72
    # payload bytes written out by hand from the stream definition (channel-
    # major, kept Gaussians in index order, k - kmin in w bits LSB first):
    # channel 0, w 3: 5, 0, 7, 2 -> bits 101 000 111 010; channel 2, w 4:
    # 0, 1, 0, 9 -> 0000 1000 0000 1001 (bit 0 first); bytes C5 05 01 09
    _, buf, bits2 = orc.fixed_length_roundtrip(k, m, n)
    assert bits2 - 59 * 72 == 28
    assert list(buf[:4]) == [0xC5, 0x05, 0x01, 0x09]
    assert not buf[4:].any()
    rng = np.random.default_rng(0)
    k2 = rng.integers(-300, 300, size=(NCH, 128)).astype(np.int32)
    m2 = (rng.random(100) < 0.7).astype(np.uint8)
    out, _, _ = orc.fixed_length_roundtrip(k2, m2, 100)
    kept = m2 > 0
    assert np.array_equal(out[:, :100][:, kept], k2[:, :100][:, kept])


def test_rd_step_composition(orc):
    """Total gradient = STE(render gradient) + lam * rate gradient."""
    sc = _tiny(n=40, seed=8)
    lam = 0.5
    r = orc.rd_step(sc.params, sc.qstep, sc.score, sc.given_mask, sc.cams, sc.width,
                    sc.height, sc.target, sc.n, sc.n_hat, lam)
    assert np.allclose(r["gy"], r["gyhat"] + r["rate"]["gy"])
    assert r["loss"] == pytest.approx(r["D"] + lam * r["rate"]["R"])
    assert np.all(r["gs"] == 0.0)    # given-mask mode: no score gradient
    r1 = orc.rd_step(sc.params, sc.qstep, sc.score, sc.given_mask, sc.cams, sc.width,
                     sc.height, sc.target, sc.n, sc.n_hat, lam, mask_mode=1, seed=3)
    ms = r1["msoft"]
    assert np.allclose(r1["gs"], r1["gmhat_total"] * ms * (1 - ms))


def test_sampled_oracle_helpers_agree_with_full_binning(orc):
    """Per-tile counts, single-tile lists and brute-force sampled pixels (the
    oracle's tools for full-size sampled parity) equal the full binning and
    the brute-force image."""
    sc = _tiny(n=80, W=70, H=50, V=2, seed=9)
    yh, _ = orc.fakequant(sc.params, sc.qstep, sc.n)
    st = orc.decide(yh, sc.n, sc.cams, sc.width, sc.height, 16, 8)
    lite = orc.decide(yh, sc.n, sc.cams, sc.width, sc.height, 16, 8, bin_pairs=False)
    assert lite.pairs == st.keys.size
    cnt = orc.tile_counts(lite, sc.n, 2, sc.width, sc.height)
    assert np.array_equal(cnt, (st.ranges[:, 1] - st.ranges[:, 0]).astype(np.int64))
    GW = -(-sc.width // 16)
    tpv = GW * (-(-sc.height // 8))
    for t in range(2 * tpv):
        b, e = st.ranges[t]
        lst = orc.tile_list(lite, sc.n, t // tpv, t % tpv, sc.width)
        assert np.array_equal(lst, st.vals[b:e])
    p64 = yh.astype(np.float64)
    m = sc.given_mask.astype(np.float64)
    full = orc.forward_brute(p64, m, sc.n, sc.cams, sc.width, sc.height, st)
    rng = np.random.default_rng(0)
    pix = np.stack([rng.integers(0, 2, 60), rng.integers(0, sc.width, 60),
                    rng.integers(0, sc.height, 60)], 1)
    out, _, _ = orc.pixels_brute(p64, m, sc.n, sc.cams, sc.width, sc.height, lite, pix)
    for k, (v, u, y) in enumerate(pix):
        assert np.array_equal(out[k, :3], full["image"][v, :, y, u])
        assert out[k, 3] == full["T"][v, y, u]
    # per-Gaussian gradients by brute force over span pixels = the full backward
    dimg = rng.normal(size=(2, 3, sc.height, sc.width))
    gp_full, gm_full, gs_full = orc.backward(p64, m, sc.n, sc.cams, sc.width, sc.height, st,
                                             dimg, want_splat=True)
    sel = np.array([0, 3, 17, 40, 41, 79])
    gs, gpar, margin = orc.splat_grads_sampled(p64, m, sc.n, sc.cams, sc.width, sc.height,
                                               lite, sel, dimg)
    fw = orc.forward(p64, m, sc.n, sc.cams, sc.width, sc.height, st)
    for q, i in enumerate(sel):
        scale = np.abs(gs_full[:, i]).max() + 1e-30
        assert np.abs(gs[q] - gs_full[:, i]).max() <= 1e-12 * scale
        pscale = np.abs(gp_full[:, i]).max() + 1e-30
        assert np.abs(gpar[q] - gp_full[:, i]).max() <= 1e-12 * pscale
        assert gs[q, :, 9].sum() == pytest.approx(gm_full[i], rel=1e-12, abs=1e-15)
        # margin flags: exactly the full forward's margin pixels inside the spans
        for v in range(2):
            if lite.valid[v, i]:
                x0, x1, y0, y1 = lite.span[v, i]
                x0, y0 = max(x0, 0), max(y0, 0)
                win = fw["margin"][v, y0:y1 + 1, x0:x1 + 1]
                assert np.array_equal(margin[v, y0:y1 + 1, x0:x1 + 1] | (win == 0), np.ones_like(win))


# ---------------------------------------------------------------------------
# Early termination (reading of Sec. 3.1's compositing with early stopping):
# a pixel stops BEFORE blending the candidate whose T (1 - alpha~) would fall
# below 1e-4; `last` is the list position of that candidate.
# ---------------------------------------------------------------------------

def _stack_scene(logits, masked, W=64, H=64):
    """Splats stacked on the optical axis (front to back in list order), each
    centred exactly on pixel (W/2, H/2), where its Gaussian factor is
    exactly 1 and alpha = sigmoid(logit); white colour (DC = sqrt(pi))."""
    n = len(logits)
    cam = synth.camera_axis(W, H, 3.0)[None]
    p = _empty_params(n)
    p[2, :n] = 0.05 * np.arange(n)                   # strictly increasing depth
    p[CH_SCALE:CH_ROT, :n] = math.log(0.03)
    p[CH_OPA, :n] = logits
    p[CH_DC:CH_DC + 3, :n] = math.sqrt(math.pi)
    m = np.array([0.0 if k in masked else 1.0 for k in range(n)])
    return p, m, cam, W, H


def _stop_closed_form(alpha_seq, mask):
    """Stop position and T of a pixel whose candidates have the given alpha
    and mask: for identical unmasked alphas the k-th candidate (0-based
    count of unmasked ones) is refused when (1 - alpha)^(k + 1) < 1e-4."""
    T = 1.0
    for j, (a, mk) in enumerate(zip(alpha_seq, mask)):
        if mk == 0.0:
            continue
        if T * (1.0 - a) < 1e-4:
            return j, T
        T *= 1.0 - a
    return len(alpha_seq), T


@pytest.mark.parametrize("logit,masked", [(1.375, ()), (0.5, ()), (1.375, (1, 4, 6))])
def test_termination_stack_closed_form(orc, logit, masked):
    n = 14
    p, m, cam, W, H = _stack_scene(np.full(n, logit, np.float32), masked)
    st = orc.decide(p, n, cam, W, H)
    assert (st.valid[0, :n] == 1).all()
    fw = orc.forward(p.astype(np.float64), m, n, cam, W, H, st)
    alpha = 1.0 / (1.0 + math.exp(-float(np.float32(logit))))
    # closed form: k unmasked splats are blended, k = floor(ln 1e-4 / ln(1 - alpha))
    k = math.floor(math.log(1e-4) / math.log(1.0 - alpha))
    assert k < n - len(masked)
    unmasked = [j for j in range(n) if j not in masked]
    stop_pos = unmasked[k]                           # the refused candidate's list position
    T_ref = (1.0 - alpha) ** k
    colour = float(np.float32(math.sqrt(math.pi))) / (2 * math.sqrt(math.pi)) + 0.5
    u = v = W // 2
    assert fw["last"][0, v, u] == stop_pos
    assert fw["T"][0, v, u] == pytest.approx(T_ref, rel=1e-12)
    for ch in range(3):
        assert fw["image"][0, ch, v, u] == pytest.approx(colour * (1 - T_ref), rel=1e-12)
    assert fw["margin"][0, v, u] == 0
    # the same stop from the step-by-step reading, as a cross-check of k
    pos, T2 = _stop_closed_form([alpha] * n, m)
    assert pos == stop_pos and T2 == pytest.approx(T_ref, rel=1e-12)


def test_termination_uses_candidate_alpha(orc):
    """Two alphas: eleven splats of alpha sigmoid(0) = 1/2 leave T = 2^-11;
    the twelfth (alpha 1/2) would give 2^-12 = 2.4e-4 >= 1e-4, so it is
    blended; the thirteenth is a high-opacity splat (logit 2.5, alpha 0.924)
    that would give 1.9e-5 < 1e-4: refused at position 12 with T = 2^-12,
    even though the splat after it (alpha 1/2) would pass on its own."""
    logits = np.array([0.0] * 12 + [2.5, 0.0], np.float32)
    p, m, cam, W, H = _stack_scene(logits, ())
    n = len(logits)
    st = orc.decide(p, n, cam, W, H)
    fw = orc.forward(p.astype(np.float64), m, n, cam, W, H, st)
    u = v = W // 2
    assert fw["last"][0, v, u] == 12
    assert fw["T"][0, v, u] == pytest.approx(2.0 ** -12, rel=1e-13)


# ---------------------------------------------------------------------------
# Projection and SH view direction under a rotated camera (Sec. 3.1): moving
# the scene and the camera by the same rigid rotation changes no pixel.
# ---------------------------------------------------------------------------

def _quat_matrix(q):
    """Textbook rotation matrix of the unit quaternion (w, x, y, z)."""
    w, x, y, z = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def _hamilton(a, b):
    aw, ax, ay, az = a
    bw, bx, by, bz = b
    return np.array([aw * bw - ax * bx - ay * by - az * bz,
                     aw * bx + ax * bw + ay * bz - az * by,
                     aw * by - ax * bz + ay * bw + az * bx,
                     aw * bz + ax * by - ay * bx + az * bw])


def _rotate_scene(orc, p64, n, cam, qw):
    """The scene and camera moved by the rotation Rw of unit quaternion qw:
    means Rw mu, orientations qw * q, SH coefficients re-fitted so that the
    colour seen along Rw d equals the old colour along d (degree <= 3 is a
    rotation-invariant space, so the least-squares fit is exact), camera
    R Rw^T with the same translation and centre Rw c."""
    Rw = _quat_matrix(qw)
    pr = p64.copy()
    pr[0:3, :n] = Rw @ p64[0:3, :n]
    for i in range(n):
        pr[CH_ROT:NCH, i] = _hamilton(qw, p64[CH_ROT:NCH, i])
    rng = np.random.default_rng(0)
    d = rng.normal(size=(400, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    Y, Yr = orc.sh_basis(d), orc.sh_basis(d @ Rw.T)
    for ch in range(3):
        rows = [CH_DC + ch] + [CH_REST + 3 * (k - 1) + ch for k in range(1, 16)]
        f = p64[rows, :n]
        fr, *_ = np.linalg.lstsq(Yr, Y @ f, rcond=None)
        pr[rows, :n] = fr
    cr = cam.astype(np.float64).copy()
    R = cam[0:9].astype(np.float64).reshape(3, 3)
    cr[0:9] = (R @ Rw.T).reshape(-1)
    cr[16:19] = Rw @ cam[16:19].astype(np.float64)
    return pr, cr, Rw


def test_rotated_scene_and_camera_render_identically(orc):
    """A ring camera (R != I) and a random 3D rotation of scene + camera: the
    FP64 projection records (mean, conic, opacity, colour with SH up to
    degree 3), the image, T and stop positions, and the gradients are
    invariant (mean gradients rotate with the scene).  A transposed
    world-to-camera rotation, a covariance conjugated the wrong way or an SH
    direction taken in camera coordinates breaks this."""
    sc = synth.make_tiny(50, 64, 48, views=2, seed=21, logscale_mu=-2.2)
    n, W, H = sc.n, sc.width, sc.height
    p64 = sc.params.astype(np.float64)
    p64[CH_REST:CH_OPA, :n] *= 0.8                  # keep colours mostly unclamped
    cam = sc.cams[1]                                # the ring camera at theta = pi
    assert not np.allclose(cam[0:9].reshape(3, 3), np.eye(3))
    st = orc.decide(p64.astype(np.float32), n, cam[None], W, H)
    qw = np.random.default_rng(4).normal(size=4)
    qw /= np.linalg.norm(qw)
    pr, cr, Rw = _rotate_scene(orc, p64, n, cam, qw)
    # the rotated camera record holds float32; rotate in FP64 and round once
    cr32 = cr.astype(np.float32)[None]
    a = orc.project64(p64, n, cam[None], W, H, st)[0]
    b = orc.project64(pr, n, cr32, W, H, st)[0]
    ok = st.valid[0] == 1
    assert ok.sum() > 30
    # camera entries rounded to FP32 move the projection by ~1e-7 relative
    assert np.allclose(b[ok, 0:2], a[ok, 0:2], rtol=0, atol=1e-4)
    for k in (2, 3, 4):
        scale = np.abs(a[ok, 2:5]).max(axis=1)
        assert (np.abs(b[ok, k] - a[ok, k]) <= 1e-5 * scale).all(), f"conic entry {k}"
    assert np.allclose(b[ok, 5], a[ok, 5], rtol=1e-15)
    assert np.allclose(b[ok, 6:9], a[ok, 6:9], rtol=0, atol=1e-6), "view-dependent colour"
    m = np.ones(n)
    fa = orc.forward(p64, m, n, cam[None], W, H, st)
    fb = orc.forward(pr, m, n, cr32, W, H, st)
    clean = (fa["margin"] == 0) & (fb["margin"] == 0)
    assert clean.mean() > 0.99
    assert np.abs(fb["image"] - fa["image"]).max(axis=1)[clean].max() < 1e-5
    assert np.array_equal(fb["last"][clean], fa["last"][clean])
    # gradients of the same image loss: mean gradients rotate, the rest match
    dimg = np.random.default_rng(5).normal(size=fa["image"].shape) * clean[:, None]
    ga, gma, _ = orc.backward(p64, m, n, cam[None], W, H, st, dimg)
    gb, gmb, _ = orc.backward(pr, m, n, cr32, W, H, st, dimg)
    gmax = np.abs(ga[0:3, :n]).max()
    assert np.abs(gb[0:3, :n] - Rw @ ga[0:3, :n]).max() <= 1e-3 * gmax
    for rows in ((CH_OPA,), tuple(range(CH_SCALE, CH_ROT))):
        r = list(rows)
        assert np.abs(gb[r, :n] - ga[r, :n]).max() <= 1e-3 * np.abs(ga[r, :n]).max()
    assert np.abs(gmb - gma).max() <= 1e-3 * np.abs(gma).max()
    # the FP32 decision layer on the rotated scene: the same spans almost everywhere
    st2 = orc.decide(pr.astype(np.float32), n, cr32, W, H)
    same = (st2.span[0] == st.span[0]).all(axis=1)
    assert same[ok].mean() >= 0.95
    assert np.abs(st2.pxy[0, ok] - st.pxy[0, ok]).max() < 1e-3


def test_sh_view_direction_sign(orc):
    """Only the degree-1 coefficient along z (index 2, Y_10 = sqrt(3/(4 pi)) z)
    is set: a Gaussian straight ahead of the axis camera is seen along +z
    (direction from the camera centre to the mean), so its colour is
    1/2 + f sqrt(3/(4 pi))."""
    W = H = 32
    cam = synth.camera_axis(W, H, 3.0)[None]
    p = _empty_params(1)
    p[CH_SCALE:CH_ROT, 0] = math.log(0.05)
    p[CH_OPA, 0] = 0.0
    f = 0.25
    p[CH_REST + 3 * (2 - 1) + 0, 0] = f               # red, coefficient k = 2
    st = orc.decide(p, 1, cam, W, H)
    pj = orc.project64(p.astype(np.float64), 1, cam, W, H, st)[0]
    assert pj[0, 6] == pytest.approx(0.5 + f * math.sqrt(3 / (4 * math.pi)), rel=1e-14)
    assert pj[0, 7] == pytest.approx(0.5, rel=1e-15) and pj[0, 8] == pytest.approx(0.5, rel=1e-15)


@pytest.mark.parametrize("parallel", [False, True])
def test_sampled_tile_step_equals_full_step_on_those_tiles(orc, parallel):
    """The CPU baseline's bounded sample (the render forward and backward over
    chosen tiles) computes exactly the full step restricted to them: the
    tiles' pixels equal the full forward's, and the parameter gradient equals
    the full backward's with dL/dC zero outside the chosen tiles; the OpenMP
    build gives the same bits as the serial one."""
    sc = _tiny(n=90, W=70, H=50, V=2, seed=14)
    yh, _ = orc.fakequant(sc.params, sc.qstep, sc.n)
    st = orc.decide(yh, sc.n, sc.cams, sc.width, sc.height, 16, 16)
    lite = orc.decide(yh, sc.n, sc.cams, sc.width, sc.height, 16, 16, bin_pairs=False)
    p64, m = yh.astype(np.float64), sc.given_mask.astype(np.float64)
    GW, GH = -(-sc.width // 16), -(-sc.height // 16)
    tiles = np.array([0, 3, GW * GH - 1, GW * GH + 5, 2 * GW * GH - 2])   # ragged ones too
    dimg = np.random.default_rng(2).normal(size=(2, 3, sc.height, sc.width))
    E, img, gp = orc.step_tiles_sampled(p64, m, sc.n, sc.cams, sc.width, sc.height, lite, tiles,
                                        dimg, parallel=parallel)
    fw = orc.forward(p64, m, sc.n, sc.cams, sc.width, sc.height, st)
    keep = np.zeros((2, sc.height, sc.width), bool)
    evals = 0
    for k, t in enumerate(tiles):
        v, tt = divmod(int(t), GW * GH)
        ty, tx = divmod(tt, GW)
        ys, xs = slice(ty * 16, min(ty * 16 + 16, sc.height)), slice(tx * 16, min(tx * 16 + 16, sc.width))
        keep[v, ys, xs] = True
        h, w = ys.stop - ys.start, xs.stop - xs.start
        assert np.array_equal(img[k, :, :h, :w], fw["image"][v, :, ys, xs])
        assert not img[k, :, h:, :].any() and not img[k, :, :, w:].any()
    gfull, _, _ = orc.backward(p64, m, sc.n, sc.cams, sc.width, sc.height, st,
                               dimg * keep[:, None], want_splat=False)
    assert np.abs(gp - gfull).max() <= 1e-12 * np.abs(gfull).max()
    assert E > 0
    if parallel:
        E1, img1, gp1 = orc.step_tiles_sampled(p64, m, sc.n, sc.cams, sc.width, sc.height, lite,
                                               tiles, dimg, parallel=False)
        assert E1 == E and np.array_equal(img1, img) and np.array_equal(gp1, gp)
