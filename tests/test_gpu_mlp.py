"""GPU parity of the learned rate estimator (BF16 MFMA kernels, through the C
ABI) against the FP64 oracle with BF16 mirroring, and a training run on the
GPU that shows what the learned estimate gains over the plain range proxy.

Bars (BF16 inputs/weights/activations, FP32 accumulation): outputs and
gradients within 1e-3 relative in L2.  Element-wise: the weight gradients of
a training step within 1e-3 relative on entries above 1 % of the largest
(each is a sum over the batch, where a single flipped rounding weighs
little); per-Gaussian outputs f (and the mask gradient f / N_hat) within
1e-2, because one BF16 rounding of a hidden activation can land on the other
side of a rounding midpoint in FP32 than in FP64, and one BF16 ulp is 0.4 %.
"""
import sys

import numpy as np
import pytest

import synth
from synth import NCH

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda", 0)


@pytest.fixture(scope="module")
def gctx(dev):
    from paper_2607_12656_amd import Context
    return Context(0)


@pytest.fixture(scope="module")
def mlp(orc):
    from oracle import mlp
    return mlp


def T(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def flat(w, mlp):
    return np.concatenate([w[k].reshape(-1) for k, _ in mlp.WEIGHT_SHAPES]).astype(np.float32)


def unflat(v, mlp):
    out, o = {}, 0
    for k, shape in mlp.WEIGHT_SHAPES:
        n = int(np.prod(shape))
        out[k] = v[o:o + n].reshape(shape)
        o += n
    return out


def to_bf16_bits(X):
    x32 = np.ascontiguousarray(X, np.float32)
    bits = x32.view(np.uint32)
    assert np.all((bits & 0xFFFF) == 0), "features must be BF16 values"
    return (bits >> 16).astype(np.uint16).view(np.int16)


def close(g, ref, name, tol=1e-3, ew_tol=1e-2):
    g = np.asarray(g, np.float64).ravel()
    ref = np.asarray(ref, np.float64).ravel()
    rel = np.linalg.norm(g - ref) / max(np.linalg.norm(ref), 1e-30)
    big = np.abs(ref) >= 1e-2 * np.abs(ref).max()
    ew = (np.abs(g - ref)[big] / np.abs(ref)[big]).max() if big.any() else 0.0
    _say(f"{name}: rel {rel:.2e} ew {ew:.2e}")
    assert rel <= tol, f"{name}: relative L2 {rel:.3e}"
    assert ew <= ew_tol, f"{name}: element-wise {ew:.3e}"


def random_weights(mlp, seed):
    w = mlp.init_weights(seed)
    rng = np.random.default_rng(seed + 100)
    for k in ("b1", "b2"):
        w[k] = rng.normal(0, 0.2, size=w[k].shape).astype(np.float32)
    w["b3"] = np.array([3.0], np.float32)
    return w


def scene_features(orc, mlp, seed, n=3000):
    sc = synth.make_tiny(n, 32, 32, seed=seed)
    q = synth.learnable_qsteps(seed + 7)
    mmin = mlp.channel_min(sc.params, sc.n)
    X = mlp.features(sc.params, q, mmin, sc.n, mirror=True)
    return sc, q, X


def test_mfma_inference_parity(orc, mlp, gctx, dev):
    _, _, X = scene_features(orc, mlp, 1, n=4000)
    X = X[:3998]                       # ragged: not a multiple of 32 rows
    w = random_weights(mlp, 2)
    theta = T(flat(w, mlp), dev)
    packed = torch.empty(98304 // 4, dtype=torch.int32, device=dev)
    gctx.rate_mlp_pack(theta, packed)
    Xb = T(to_bf16_bits(X), dev)
    out = torch.empty(X.shape[0], dtype=torch.float32, device=dev)
    gctx.rate_mlp_infer(packed, theta, Xb, X.shape[0], out)
    torch.cuda.synchronize()
    ref = mlp.forward(X, w, mirror=True)
    close(out.cpu().numpy(), ref, "f")


def test_mfma_training_gradient_parity(orc, mlp, gctx, dev):
    _, _, X = scene_features(orc, mlp, 3, n=4200)
    B = 4096
    X = X[:B]
    rng = np.random.default_rng(4)
    t = (rng.uniform(200, 400, size=B)).astype(np.float32)
    w = random_weights(mlp, 5)
    theta = T(flat(w, mlp), dev)
    packed = torch.empty(98304 // 4, dtype=torch.int32, device=dev)
    gctx.rate_mlp_pack(theta, packed)
    scratch = torch.empty(gctx.rate_mlp_train_scratch_bytes(B), dtype=torch.uint8, device=dev)
    loss = torch.empty(1, dtype=torch.float32, device=dev)
    g = torch.empty(24961, dtype=torch.float32, device=dev)
    gctx.rate_mlp_train_step(theta, None, None, packed, T(to_bf16_bits(X), dev), T(t, dev), B, 0.0,
                             1, loss, g, scratch)
    torch.cuda.synchronize()
    f = mlp.forward(X, w, mirror=True)
    ref_loss = float(((f - t) ** 2).mean())
    assert abs(float(loss.item()) - ref_loss) <= 1e-3 * ref_loss
    gr, _ = mlp.backward(X, w, mlp.mse_grad_weights(f, t), mirror=True)
    gg = unflat(g.cpu().numpy(), mlp)
    for k, _ in mlp.WEIGHT_SHAPES:
        close(gg[k], gr[k], f"d{k}", tol=1e-3, ew_tol=1e-3)


def test_learned_rate_in_loop_parity(orc, mlp, gctx, dev):
    """R_learned, f per Gaussian and the gradients to params / q / mask."""
    from paper_2607_12656_amd.rd import RDStep
    sc = synth.make_tiny(5000, 32, 32, seed=8)
    q = synth.learnable_qsteps(9)
    w = random_weights(mlp, 10)
    theta = T(flat(w, mlp), dev)
    packed = torch.empty(98304 // 4, dtype=torch.int32, device=dev)
    gctx.rate_mlp_pack(theta, packed)
    rd = RDStep(gctx, sc.n, sc.npad, sc.n_hat, sc.cams, sc.width, sc.height)
    params, qd = T(sc.params, dev), T(q, dev)
    gctx.fakequant_prune(params, qd, None, 0, T(sc.given_mask, dev), 0, 0, rd.qparams, rd.hard,
                         rd.soft, rd.stats)
    R = torch.empty(1, dtype=torch.float32, device=dev)
    fper = torch.empty(sc.n, dtype=torch.float32, device=dev)
    gctx.rate_mlp_fwd(packed, theta, params, qd, rd.stats, rd.hard, R, fper)
    gp = torch.zeros_like(params)
    gq = torch.zeros(NCH, dtype=torch.float32, device=dev)
    gm = torch.zeros(sc.n, dtype=torch.float32, device=dev)
    lam = 0.7
    gctx.rate_mlp_bwd(packed, theta, params, qd, rd.stats, rd.hard, rd.soft, 0, lam, gp, gq,
                      None, gm)
    torch.cuda.synchronize()
    ref = mlp.learned_rate(sc.params, q, sc.given_mask, sc.n, sc.n_hat, w, mirror=True,
                           weight=lam)
    assert abs(float(R.item()) - ref["R"]) <= 1e-3 * abs(ref["R"])
    close(fper.cpu().numpy(), ref["f"], "f in loop")
    close(gp.cpu().numpy()[:, :sc.n], ref["gy"][:, :sc.n], "grad params")
    close(gq.cpu().numpy(), ref["gq"], "grad q")
    close(gm.cpu().numpy(), ref["gm"], "grad mask")


def _training_set(orc, mlp, seeds, n=6000):
    """Feature rows of the kept Gaussians of several scenes, each labelled
    with its scene's fixed-length bits per kept Gaussian."""
    Xs, ts, scenes = [], [], []
    for s in seeds:
        sc = synth.make_tiny(n, 32, 32, seed=s, prune=0.1 + 0.3 * ((s * 37) % 10) / 10)
        q = synth.learnable_qsteps(s + 1000)
        bits, per = mlp.coder_targets(sc.params, q, sc.given_mask, sc.n)
        mmin = mlp.channel_min(sc.params, sc.n)
        X = mlp.features(sc.params, q, mmin, sc.n, mirror=True)
        kept = sc.given_mask > 0
        Xs.append(X[kept])
        ts.append(np.full(int(kept.sum()), per, np.float32))
        scenes.append((sc, q, bits))
    return np.concatenate(Xs), np.concatenate(ts), scenes


def test_training_on_gpu_and_gain_over_plain_proxy(orc, mlp, gctx, dev):
    """Train on coder bits of 24 scenes on the GPU; on 8 held-out scenes the
    learned total-bit estimate sum_kept f(x_i) beats the plain proxy's
    N_kept * L_quant against the exact fixed-length bits."""
    X, t, _ = _training_set(orc, mlp, range(100, 124))
    rng = np.random.default_rng(0)
    w = mlp.init_weights(42)
    w["b3"] = np.array([float(t.mean())], np.float32)
    theta = T(flat(w, mlp), dev)
    m = torch.zeros_like(theta)
    v = torch.zeros_like(theta)
    packed = torch.empty(98304 // 4, dtype=torch.int32, device=dev)
    gctx.rate_mlp_pack(theta, packed)
    B = 65536
    scratch = torch.empty(gctx.rate_mlp_train_scratch_bytes(B), dtype=torch.uint8, device=dev)
    loss = torch.empty(1, dtype=torch.float32, device=dev)
    g = torch.empty(24961, dtype=torch.float32, device=dev)
    Xb_all = T(to_bf16_bits(X), dev)
    t_all = T(t, dev)
    losses = []
    for step in range(1, 401):
        idx = torch.from_numpy(rng.integers(0, X.shape[0], size=B)).to(dev)
        xb = Xb_all[idx].contiguous()
        tb = t_all[idx].contiguous()
        gctx.rate_mlp_train_step(theta, m, v, packed, xb, tb, B, 1e-3, step, loss, g, scratch)
        if step % 50 == 0 or step == 1:
            losses.append(float(loss.item()))
    _say("training loss", losses)
    assert losses[-1] < 0.2 * losses[0]
    # held-out scenes
    _, _, held = _training_set(orc, mlp, range(500, 508))
    err_l, err_p = [], []
    from paper_2607_12656_amd.rd import RDStep
    for sc, q, bits in held:
        rd = RDStep(gctx, sc.n, sc.npad, sc.n_hat, sc.cams, sc.width, sc.height)
        params, qd = T(sc.params, dev), T(q, dev)
        gctx.fakequant_prune(params, qd, None, 0, T(sc.given_mask, dev), 0, 0, rd.qparams,
                             rd.hard, rd.soft, rd.stats)
        gctx.rate_proxy(rd.stats, qd, 0.0, rd.rate3)
        R = torch.empty(1, dtype=torch.float32, device=dev)
        gctx.rate_mlp_fwd(packed, theta, params, qd, rd.stats, rd.hard, R, None)
        torch.cuda.synchronize()
        est_l = float(R.item()) * sc.n_hat
        est_p = float(rd.rate3[0].item()) * sc.n_hat
        err_l.append(abs(est_l - bits) / bits)
        err_p.append(abs(est_p - bits) / bits)
    _say(f"held-out rate-estimate error: learned {np.mean(err_l):.4f}, plain {np.mean(err_p):.4f}")
    assert np.mean(err_l) < np.mean(err_p)


def test_feature_rows_match_oracle(orc, mlp, gctx, dev):
    """sgs_rate_mlp_features: the BF16 rows the in-loop forward uses, for chosen
    Gaussians (out-of-range indices give zero rows).  FP32 evaluation vs the
    FP64 features rounded once to BF16: equal, except where the FP64 value lies
    within FP32 rounding of a BF16 rounding boundary (then one BF16 ulp)."""
    from paper_2607_12656_amd.rd import RDStep
    _say("[gpu] mlp features")
    sc = synth.make_tiny(5000, 32, 32, seed=12)
    q = synth.learnable_qsteps(13)
    rd = RDStep(gctx, sc.n, sc.npad, sc.n_hat, sc.cams, sc.width, sc.height)
    params, qd = T(sc.params, dev), T(q, dev)
    gctx.fakequant_prune(params, qd, None, 0, T(sc.given_mask, dev), 0, 0, rd.qparams, rd.hard,
                         rd.soft, rd.stats)
    rng = np.random.default_rng(3)
    idx = rng.integers(0, sc.n, 3001).astype(np.int32)
    idx[[5, 77, 3000]] = [-1, sc.n, sc.n + 9]
    X = torch.full((3001, 64), 0x7FFF, dtype=torch.int16, device=dev)
    gctx.rate_mlp_features(params, qd, rd.stats, T(idx, dev), 3001, X)
    torch.cuda.synchronize()
    got = X.cpu().numpy().view(np.uint16)
    mmin = mlp.channel_min(sc.params, sc.n)
    ok = (idx >= 0) & (idx < sc.n)
    assert np.all(got[~ok] == 0), "zero rows for out-of-range indices"
    ref64 = mlp.features(sc.params, q, mmin, sc.n, mirror=False)[idx[ok]]
    refb = mlp.features(sc.params, q, mmin, sc.n, mirror=True)[idx[ok]]
    ref_bits = (refb.astype(np.float32).view(np.uint32) >> 16).astype(np.uint16)
    g = got[ok]
    diff = g != ref_bits
    assert diff.mean() < 1e-3, f"{diff.sum()} of {diff.size} features differ"
    gv = (g.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
    rv = refb.astype(np.float64)
    ulp = np.abs(rv) * 2.0 ** -7
    assert np.all(np.abs(gv - rv)[diff] <= ulp[diff] * 1.01), "more than one BF16 ulp"
    mid = (gv + rv) / 2
    assert np.all(np.abs(ref64[diff] - mid[diff]) <= 1e-5 * np.abs(ref64[diff]) + 1e-30), \
        "a differing feature is not at a BF16 rounding boundary"
    assert np.all(g[:, 59:] == 0)


def test_learned_rate_backward_skips_higher_sh_rows(mlp, gctx, dev):
    """The learned-rate backward with the higher-SH gradient rows off leaves
    those rows of grad_params untouched and adds into every other row as with
    them on; the step-size and mask gradients are unchanged."""
    from paper_2607_12656_amd.rd import RDStep
    sc = synth.make_tiny(4000, 32, 32, seed=31)
    q = synth.learnable_qsteps(32)
    theta = T(flat(random_weights(mlp, 33), mlp), dev)
    packed = torch.empty(98304 // 4, dtype=torch.int32, device=dev)
    gctx.rate_mlp_pack(theta, packed)
    rd = RDStep(gctx, sc.n, sc.npad, sc.n_hat, sc.cams, sc.width, sc.height)
    params, qd = T(sc.params, dev), T(q, dev)
    gctx.fakequant_prune(params, qd, None, 0, T(sc.given_mask, dev), 0, 0, rd.qparams, rd.hard,
                         rd.soft, rd.stats)
    R = torch.empty(1, dtype=torch.float32, device=dev)
    gctx.rate_mlp_fwd(packed, theta, params, qd, rd.stats, rd.hard, R, None)
    g0 = torch.randn(params.shape, generator=torch.Generator().manual_seed(34)).to(dev)
    outs = []
    try:
        for on in (True, False):
            gp = g0.clone()
            gq = torch.zeros(NCH, dtype=torch.float32, device=dev)
            gm = torch.zeros(sc.n, dtype=torch.float32, device=dev)
            gctx.set_grad_sh_rest(on)
            gctx.rate_mlp_bwd(packed, theta, params, qd, rd.stats, rd.hard, rd.soft, 0, 0.7,
                              gp, gq, None, gm)
            torch.cuda.synchronize()
            outs.append([x.cpu().numpy().copy() for x in (gp, gq, gm)])
    finally:
        gctx.set_grad_sh_rest(True)
    (pa, qa, ma), (pb, qb, mb) = outs
    n, rest = sc.n, np.r_[6:51]
    keep = np.setdiff1d(np.arange(pa.shape[0]), rest)
    init = g0.cpu().numpy()
    assert np.array_equal(pa[keep, :n].view(np.uint32), pb[keep, :n].view(np.uint32))
    assert np.array_equal(pb[rest, :n].view(np.uint32), init[rest, :n].view(np.uint32))
    assert not np.array_equal(pa[rest, :n], init[rest, :n]), "rows were not added to"
    assert np.array_equal(ma.view(np.uint32), mb.view(np.uint32))
    d = np.abs(qa.astype(np.float64) - qb).max()
    assert d <= 1e-6 * np.abs(qa).max(), f"grad q {d:.3e}"
