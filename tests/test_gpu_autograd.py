"""The torch.autograd wrappers (FormationStep, Render) over the C ABI:
gradients of (D + lam R) and of a torch image loss against the FP64 oracle's
gradient and against central finite differences of the oracle's forward;
the guard against a backward that follows another forward; and the
autotuner's choice among tile shapes and blend schedules."""
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


def T(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def rel_close(g, ref, tol=1e-3, name=""):
    g = np.asarray(g, np.float64).ravel()
    ref = np.asarray(ref, np.float64).ravel()
    rel = np.linalg.norm(g - ref) / max(np.linalg.norm(ref), 1e-30)
    big = np.abs(ref) >= 1e-2 * np.abs(ref).max()
    ew = (np.abs(g - ref)[big] / np.abs(ref)[big]).max() if big.any() else 0.0
    _say(f"{name}: rel {rel:.2e} ew {ew:.2e}")
    assert rel <= tol and ew <= tol, f"{name}: rel {rel:.3e} ew {ew:.3e}"


def _clean_scene(orc, mode, lam, seeds=range(40, 80)):
    """First seeded scene whose oracle step has no margin pixel and no colour
    within 1e-4 of its target (each side may then use its own L1 gradient)."""
    for seed in seeds:
        sc = synth.make_tiny(120, 56, 40, views=2, seed=seed)
        s = orc.rd_step(sc.params, sc.qstep, sc.score, sc.given_mask, sc.cams, sc.width,
                        sc.height, sc.target, sc.n, sc.n_hat, lam, mask_mode=mode, seed=77,
                        step=3)
        if not s["fw"]["margin"].any() and not (np.abs(s["fw"]["image"] - sc.target) <= 1e-4).any():
            return sc, s
    pytest.fail("no clean scene")


@pytest.mark.parametrize("mode", [0, 1])
def test_formation_step_autograd_matches_oracle(orc, gctx, dev, mode):
    """(D + lam R).backward() through FormationStep equals the oracle's
    gradient of the same loss (straight-through quantizer, learned step
    size, Gumbel-sigmoid score gradient in mode 1)."""
    from paper_2607_12656_amd.autograd import FormationStep
    from paper_2607_12656_amd.rd import RDStep
    lam = 0.5
    sc, s = _clean_scene(orc, mode, lam)
    rd = RDStep(gctx, sc.n, sc.npad, sc.n_hat, sc.cams, sc.width, sc.height)
    params = T(sc.params, dev).requires_grad_(True)
    q = T(sc.qstep, dev).requires_grad_(True)
    score = T(sc.score, dev).requires_grad_(mode == 1)
    D, R, img = FormationStep.apply(params, q, score, rd, T(sc.target, dev), mode,
                                    T(sc.given_mask, dev), 77, 3)
    assert abs(float(D.detach()) - s["D"]) <= 1e-6 * s["D"]
    assert abs(float(R.detach()) - s["rate"]["R"]) <= 1e-6 * abs(s["rate"]["R"])
    (D + lam * R).backward()
    torch.cuda.synchronize()
    rel_close(params.grad.cpu().numpy()[:, :sc.n], s["gy"][:, :sc.n], name="d/dparams")
    rel_close(q.grad.cpu().numpy(), s["gq"], name="d/dq")
    if mode == 1:
        rel_close(score.grad.cpu().numpy(), s["gs"], name="d/dscore")
    # D alone: the rate weight is then 0 in the backward
    params.grad = None
    D2, R2, _ = FormationStep.apply(params, q, score, rd, T(sc.target, dev), mode,
                                    T(sc.given_mask, dev), 77, 3)
    D2.backward()
    torch.cuda.synchronize()
    gyhat = s["gyhat"][:, :sc.n]
    rel_close(params.grad.cpu().numpy()[:, :sc.n], gyhat, name="dD/dparams")


def test_render_autograd_matches_oracle_and_finite_differences(orc, gctx, dev):
    """Render with a torch image loss sum(w * image): the gradient w.r.t. the
    quantized parameters against the oracle's backward and against central
    differences of the oracle's FP64 forward (structure held fixed, entries
    whose difference quotient is not stable under halving h skipped)."""
    from paper_2607_12656_amd.autograd import Render
    from paper_2607_12656_amd.rd import RDStep
    sc = synth.make_tiny(40, 48, 40, views=1, seed=61)
    yh, _ = orc.fakequant(sc.params, sc.qstep, sc.n)
    st = orc.decide(yh, sc.n, sc.cams, sc.width, sc.height)
    p64 = yh.astype(np.float64)
    m64 = sc.given_mask.astype(np.float64)
    wimg = np.random.default_rng(3).normal(size=(1, 3, sc.height, sc.width))
    fw = orc.forward(p64, m64, sc.n, sc.cams, sc.width, sc.height, st)
    assert not fw["margin"].any()
    rd = RDStep(gctx, sc.n, sc.npad, sc.n_hat, sc.cams, sc.width, sc.height)
    qp = T(yh, dev).requires_grad_(True)
    img = Render.apply(qp, T(sc.given_mask, dev), rd)
    loss = (img * T(wimg.astype(np.float32), dev)).sum()
    loss.backward()
    torch.cuda.synchronize()
    assert np.abs(img.detach().cpu().numpy() - fw["image"]).max() <= 1e-4
    g = qp.grad.cpu().numpy()
    gref, gm, _ = orc.backward(p64, m64, sc.n, sc.cams, sc.width, sc.height, st, wimg)
    rel_close(g[:, :sc.n], gref[:, :sc.n], name="d/dqparams vs oracle")
    rel_close(rd.grad_mask.cpu().numpy(), gm, name="d/dmask vs oracle")

    def L(p):
        return float((orc.forward(p, m64, sc.n, sc.cams, sc.width, sc.height, st)["image"]
                      * wimg).sum())
    rng = np.random.default_rng(5)
    checked = 0
    gmax = np.abs(gref[:, :sc.n]).max()
    for _ in range(120):
        j, i = int(rng.integers(0, NCH)), int(rng.integers(0, sc.n))
        if not st.valid[0, i]:
            continue
        h = 1e-6 * max(1.0, abs(p64[j, i]))
        def ev(d):
            pp = p64.copy()
            pp[j, i] += d
            return L(pp)
        f1 = (ev(h) - ev(-h)) / (2 * h)
        f2 = (ev(2 * h) - ev(-2 * h)) / (4 * h)
        scale = abs(f1) + 1e-3 * gmax
        if abs(f1 - f2) > 1e-5 * scale:
            continue
        checked += 1
        assert abs(g[j, i] - f1) <= 1e-3 * scale, (j, i, g[j, i], f1)
    assert checked >= 60
    _say(f"render FD: {checked} entries")


def test_backward_after_another_forward_raises(orc, gctx, dev):
    from paper_2607_12656_amd.autograd import FormationStep, Render
    from paper_2607_12656_amd.rd import RDStep
    sc = synth.make_tiny(40, 32, 32, seed=62)
    rd = RDStep(gctx, sc.n, sc.npad, sc.n_hat, sc.cams, sc.width, sc.height)
    params = T(sc.params, dev).requires_grad_(True)
    q = T(sc.qstep, dev).requires_grad_(True)
    args = (T(sc.score, dev), rd, T(sc.target, dev), 0, T(sc.given_mask, dev), 0, 0)
    D1, _, _ = FormationStep.apply(params, q, *args)
    D2, _, _ = FormationStep.apply(params, q, *args)
    with pytest.raises(RuntimeError, match="another forward"):
        D1.backward()
    D2.backward()                       # the latest forward still differentiates
    assert params.grad is not None
    qp = T(sc.params, dev).requires_grad_(True)
    img1 = Render.apply(qp, T(sc.given_mask, dev), rd)
    Render.apply(qp, T(sc.given_mask, dev), rd)
    with pytest.raises(RuntimeError, match="another forward"):
        img1.sum().backward()


def test_autotuner_choice_and_cache(orc, gctx, dev, tmp_path):
    """The tuner times every tile shape, then every schedule with the best
    shape, returns the fastest, caches it, and the chosen configuration
    renders the same image as the default one (the support rule makes the
    image independent of the choice)."""
    from paper_2607_12656_amd import autotune
    from paper_2607_12656_amd.rd import RDStep
    sc = synth.make_tiny(400, 150, 90, views=2, seed=11)
    params, q = T(sc.params, dev), T(sc.qstep, dev)
    score, mask, target = T(sc.score, dev), T(sc.given_mask, dev), T(sc.target, dev)

    def step(rd):
        rd.forward(params, q, score, target, 0.5, 0, mask, 0, 0, count_evals=False)
        rd.backward(params, q, 0)

    cache = str(tmp_path / "tune.json")
    res = autotune.tune(gctx, sc.n, sc.npad, sc.n_hat, sc.cams, sc.width, sc.height, step,
                        reps=2, cache_path=cache)
    assert res["tile"] in autotune.CANDIDATES and res["schedule"] in autotune.SCHEDULES
    assert len(res["ms"]) == len(autotune.CANDIDATES) + len(autotune.SCHEDULES) - 1
    best = f"{res['tile'][0]}x{res['tile'][1]}/{res['schedule']}"
    assert res["ms"][best] == min(res["ms"].values())
    again = autotune.tune(gctx, sc.n, sc.npad, sc.n_hat, sc.cams, sc.width, sc.height, step,
                          reps=2, cache_path=cache)
    assert again["cached"] and again["tile"] == res["tile"] and again["schedule"] == res["schedule"]
    imgs = []
    for tile, sched in ((res["tile"], res["schedule"]), ((16, 16), "tile")):
        rd = RDStep(gctx, sc.n, sc.npad, sc.n_hat, sc.cams, sc.width, sc.height, tile=tile,
                    schedule=sched)
        step(rd)
        torch.cuda.synchronize()
        imgs.append(rd.image.cpu().numpy())
    assert np.array_equal(imgs[0], imgs[1])


def test_native_autotuner(orc, gctx, dev):
    """sgs_autotune: eight candidates timed (five tile shapes, then three more
    schedules with the fastest shape), the fastest chosen, the context left
    bound with it, and that binding renders the image the oracle renders."""
    from paper_2607_12656_amd import autotune
    sc = synth.make_tiny(400, 150, 90, views=2, seed=11)
    params, q = T(sc.params, dev), T(sc.qstep, dev)
    mask, target = T(sc.given_mask, dev), T(sc.target, dev)
    gctx.set_scene(sc.n, sc.npad, sc.n_hat, sc.cams, sc.width, sc.height)
    res = autotune.tune_native(gctx, params, q, mask, target, sc.n, sc.views, sc.width,
                               sc.height, reps=2)
    ms = res["ms"]
    assert len(ms) == 8 and all(v > 0 for v in ms.values())
    best = f"{res['tile'][0]}x{res['tile'][1]}/{res['schedule']}"
    assert ms[best] == min(ms.values())
    # the context is bound with the choice: a step renders the oracle's image
    n, V, W, H = sc.n, sc.views, sc.width, sc.height
    e = lambda *s_, dt=torch.float32: torch.empty(*s_, dtype=dt, device=dev)
    hard, soft, stats = e(n, dt=torch.uint8), e(n), e(128, dt=torch.int64)
    img, fT, last = e(V, 3, H, W), e(V, H, W), e(V, H, W, dt=torch.int32)
    gctx.quant_render_fwd(params, q, None, 0, mask, 0, 0, hard, soft, stats, img, fT, last, None)
    torch.cuda.synchronize()
    yh, _ = orc.fakequant(sc.params, sc.qstep, n)
    st = orc.decide(yh, n, sc.cams, W, H, res["tile"][0], res["tile"][1])
    fw = orc.forward(yh.astype(np.float64), sc.given_mask.astype(np.float64), n, sc.cams, W, H,
                     st)
    ok = fw["margin"] == 0
    assert np.abs(img.cpu().numpy() - fw["image"]).max(axis=1)[ok].max() <= 1e-4
