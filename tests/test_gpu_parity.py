"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the
same seeded inputs.

Bars: structure (codes k, hard mask, culling, spans, depth keys, sorted tile
lists, ranges, per-pixel stop positions) bit-exact; pixels within 1e-4
absolute outside margin pixels (where FP32 and FP64 may take a different
per-pair decision: alpha within 2e-5 relative of 1/255 or 0.99, or T within
2e-5 relative of 1e-4); margin pixels at most 1e-3 of all pixels, and margin
pixels whose value or stop position actually differs at most 1e-5 of them;
the L1 gradient dL/dC element-wise within 1e-6 relative wherever |C - target|
> 1e-4; gradients within 1e-3 relative (per tensor in L2, and element-wise on
entries above 1 % of the tensor's largest); rate scalars within 1e-6
relative.

Every forward is run twice: with the evaluation count (which keeps every
in-span list entry) and without it (the timed path, which drops the entries
that cannot reach the alpha cut-off in a sub-tile); the two must give the
same image, transmittance and stop positions bit for bit, and both are
compared with the oracle.  Both backward passes take the oracle's own L1
gradient, zeroed at the oracle's margin pixels (no oracle input comes from
the GPU).
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
    sys.stdout.flush()


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


def grad_close(g, ref, tol=1e-3, name=""):
    g = np.asarray(g, np.float64).ravel()
    ref = np.asarray(ref, np.float64).ravel()
    nr = np.linalg.norm(ref)
    rel = np.linalg.norm(g - ref) / max(nr, 1e-30)
    big = np.abs(ref) >= 1e-2 * np.abs(ref).max() if ref.size else np.zeros(0, bool)
    ew = (np.abs(g - ref)[big] / np.abs(ref)[big]).max() if big.any() else 0.0
    if rel > tol or ew > tol:
        e = np.where(big, np.abs(g - ref) / np.maximum(np.abs(ref), 1e-30), 0.0)
        worst = np.argsort(-e)[:5]
        _say(f"{name}: rel {rel:.3e} ew {ew:.3e} max|ref| {np.abs(ref).max():.3e}; worst "
             + ", ".join(f"[{k}] {g[k]:.6e} vs {ref[k]:.6e}" for k in worst))
    assert rel <= tol, f"{name}: relative L2 error {rel:.3e}"
    assert ew <= tol, f"{name}: element-wise relative error {ew:.3e}"
    return rel, ew


def run_pair(orc, gctx, dev, sc, tile=(16, 16), lam=0.5, mode=0, seed=0, step=0,
             schedule="tile", fused=False):
    """GPU step and oracle step on the same inputs.  The GPU forward runs with
    and without the evaluation count (bit-identical results required).  Both
    backward passes get the same dL/dimage: the oracle's L1 gradient with the
    oracle's margin pixels zeroed, so no gradient depends on a decision FP32
    and FP64 may take differently at a kink (alpha clamp, alpha cut-off,
    termination).  fused: the GPU step runs quant_render_fwd /
    quant_render_bwd (the quantized rows and their gradient are then not
    materialized)."""
    from paper_2607_12656_amd.rd import RDStep
    _say(f"[gpu] {sc.name} tile={tile} schedule={schedule} mode={mode} n={sc.n} V={sc.views}"
         f" fused={fused}")
    rd = RDStep(gctx, sc.n, sc.npad, sc.n_hat, sc.cams, sc.width, sc.height, tile=tile,
                schedule=schedule, fused=fused)
    params, q, score = T(sc.params, dev), T(sc.qstep, dev), T(sc.score, dev)
    mask, target = T(sc.given_mask, dev), T(sc.target, dev)
    rd.forward(params, q, score, target, lam, mode, mask, seed, step)
    torch.cuda.synchronize()
    counted = [x.cpu().numpy().view(np.uint32) for x in (rd.image, rd.final_T, rd.last)]
    rd.forward(params, q, score, target, lam, mode, mask, seed, step, count_evals=False)
    torch.cuda.synchronize()
    timed = [x.cpu().numpy().view(np.uint32) for x in (rd.image, rd.final_T, rd.last)]
    for name, a, b in zip(("image", "T", "last"), counted, timed):
        assert np.array_equal(a, b), f"{name}: counting and timed forward differ"
    s = orc.rd_forward(sc.params, sc.qstep, sc.score, sc.given_mask, sc.cams, sc.width,
                       sc.height, sc.target, sc.n, sc.n_hat, lam, mask_mode=mode, seed=seed,
                       step=step, TW=tile[0], TH=tile[1])
    l1_oracle = s["dimage"].copy()
    dimage = (s["dimage"] * (s["fw"]["margin"] == 0)[:, None, :, :]).astype(np.float32)
    g = gpu_backward(gctx, dev, sc, rd, params, q, mode, tile, dimage)
    g["dimage_l1"] = rd.dimage.cpu().numpy()
    r = orc.rd_backward(s, dimage.astype(np.float64))
    r["l1_grad"] = l1_oracle
    return g, r


def check_l1(g, r, sc):
    """L1 loss within 1e-6 and dL/dC element by element (value and scale),
    off pixels where |C - target| <= 1e-4 (the sign may flip there) and off
    margin pixels."""
    assert abs(g["loss"] - r["D"]) <= 1e-6 * r["D"], f"L1 {g['loss']} vs {r['D']}"
    ok = (r["fw"]["margin"] == 0)[:, None, :, :]
    far = (np.abs(r["fw"]["image"] - sc.target) > 1e-4) & ok
    ref = r["l1_grad"]
    err = np.abs(g["dimage_l1"].astype(np.float64) - ref)[far]
    assert far.mean() > 0.99
    assert (err <= 1e-6 * np.abs(ref[far])).all(), f"dL/dC max error {err.max():.3e}"


def gpu_backward(gctx, dev, sc, rd, params, q, mode, tile, dimage):
    d_in = T(dimage.astype(np.float32), dev)
    gp = torch.empty_like(params)
    rd.backward(params, q, mode, grad_params=gp, dimage=d_in)
    torch.cuda.synchronize()
    P, flags = gctx.query(rd.stats)
    out = dict(rd=rd, P=P)
    tile_ids = torch.empty(max(P, 1), dtype=torch.int32, device=dev)
    vals = torch.empty(max(P, 1), dtype=torch.int32, device=dev)
    ranges = torch.empty(rd.V * (-(-sc.width // tile[0])) * (-(-sc.height // tile[1])), 2,
                         dtype=torch.int32, device=dev)
    spans = torch.empty(rd.V, sc.n, 4, dtype=torch.int32, device=dev)
    depth = torch.empty(rd.V, sc.n, dtype=torch.float32, device=dev)
    splats = torch.empty(rd.V, sc.n, 12, dtype=torch.float32, device=dev)
    gctx.copy_structure(tile_ids, vals, max(P, 1), ranges, spans, depth, splats)
    sgrad = torch.empty(rd.V, sc.n, 12, dtype=torch.float32, device=dev)
    gctx.copy_splat_grads(sgrad)
    torch.cuda.synchronize()
    c = lambda x: x.cpu().numpy()
    out.update(qparams=None if rd.fused else c(rd.qparams), hard=c(rd.hard), soft=c(rd.soft),
               stats=c(rd.stats).view(np.uint64), rate3=c(rd.rate3), rate_grad=c(rd.rate_grad),
               image=c(rd.image), T=c(rd.final_T), last=c(rd.last).view(np.uint32),
               evals=int(c(rd.evals)[0]), loss=float(c(rd.loss)[0]), dimage=c(rd.dimage),
               gq_render=None if rd.fused else c(rd.grad_qparams), gmask=c(rd.grad_mask),
               gparams=c(gp),
               gq=c(rd.grad_q), gscore=c(rd.grad_score),
               tile_ids=c(tile_ids)[:P].view(np.uint32), vals=c(vals)[:P].view(np.uint32),
               ranges=c(ranges).view(np.uint32), spans=c(spans), depth=c(depth),
               splats=c(splats), sgrad=c(sgrad))
    return out


def check_structure(g, r, sc):
    n = sc.n
    if g["qparams"] is not None:
        assert np.array_equal(g["qparams"][:, :n], r["yhat"][:, :n]), "quantized parameters"
    assert np.array_equal(g["hard"], r["mhat"]), "hard mask"
    st = r["st"]
    valid = st.valid > 0
    gvalid = g["spans"][..., 0] >= 0
    assert np.array_equal(gvalid, valid), "culling"
    assert np.array_equal(g["spans"][valid], st.span[valid]), "pixel spans"
    assert np.array_equal(g["depth"][valid].view(np.uint32), st.tz[valid].view(np.uint32)), "depth"
    assert g["P"] == st.keys.size, f"pair count {g['P']} vs {st.keys.size}"
    assert np.array_equal(g["tile_ids"].astype(np.uint64), st.keys >> np.uint64(32)), "tile ids"
    assert np.array_equal(g["vals"], st.vals), "sorted Gaussian indices"
    assert np.array_equal(g["ranges"], st.ranges), "tile ranges"


def check_stats(g, r, sc):
    s = g["stats"]
    rate = r["rate"]
    imin = (s[:NCH] & np.uint64(0xFFFFFFFF)).astype(np.int64)
    imax = 0xFFFFFFFF - (s[NCH:2 * NCH] & np.uint64(0xFFFFFFFF)).astype(np.int64)
    assert np.array_equal(imin, rate["argmin"]) and np.array_equal(imax, rate["argmax"])
    assert int(s[118]) == int(r["mhat"].sum())
    assert int(s[119]) == 0
    R, Lq, Lm = g["rate3"]
    assert abs(R - rate["R"]) <= 1e-6 * abs(rate["R"])
    assert abs(Lq - rate["Lq"]) <= 1e-6 * abs(rate["Lq"])
    assert abs(Lm - rate["Lm"]) <= 1e-6 * abs(rate["Lm"])


def check_image(g, r):
    ok = r["fw"]["margin"] == 0
    frac = 1 - ok.mean()
    perr = np.maximum(np.abs(g["image"] - r["fw"]["image"]).max(axis=1),
                      np.abs(g["T"] - r["fw"]["T"]))
    err = perr[ok].max()
    assert err <= 1e-4, f"pixel / transmittance error {err:.3e}"
    same_last = g["last"] == r["fw"]["last"].astype(np.uint32)
    assert same_last[ok].all(), "stop positions"
    assert frac <= 1e-3, f"margin pixels {frac:.2e}"
    # margin pixels that really took another decision
    moved = ~ok & ((perr > 1e-4) | ~same_last)
    assert moved.sum() <= 1e-5 * ok.size, f"{moved.sum()} margin pixels differ"
    if not (~ok).any():
        assert g["evals"] == r["fw"]["evals"]
    g["margin_moved"] = int(moved.sum())
    return err, frac


TINY = [
    dict(n=48, W=45, H=37, V=1, seed=2),
    dict(n=64, W=70, H=50, V=2, seed=3),
    dict(n=200, W=96, H=80, V=1, seed=4, logscale=-2.5),
    # large splats: tile rectangles of 512 tiles and more take the backward's
    # replica records (folded into the splat's record after the blend)
    dict(n=60, W=640, H=480, V=2, seed=5, logscale=-1.8, big=True),
    # dense: one super-tile's chunk of items holds several times the pairs the
    # pair scatter stages in LDS at once (its tiles are taken in groups)
    dict(n=1500, W=128, H=128, V=1, seed=7, logscale=-1.4, dense=True),
    # three views: the view bits of the super-tile ids leave ids with no view
    # (view 3), and the depth order's segments are padded (n not a multiple
    # of 2048)
    dict(n=300, W=150, H=100, V=3, seed=12),
]
BIG_TILES = 512   # the library's large-splat threshold (tiles per rectangle)
L2_OUT = 12288    # pairs the library's pair scatter stages in LDS at once


@pytest.mark.parametrize("tile", [(16, 16), (8, 8), (32, 8), (32, 16), (32, 32)])
@pytest.mark.parametrize("cfg", range(len(TINY)))
def test_tiny_scenes_full_step(orc, gctx, dev, tile, cfg):
    c = TINY[cfg]
    sc = synth.make_tiny(c["n"], c["W"], c["H"], views=c["V"], seed=c["seed"],
                         logscale_mu=c.get("logscale", -2.0))
    g, r = run_pair(orc, gctx, dev, sc, tile=tile)
    check_structure(g, r, sc)
    check_stats(g, r, sc)
    check_image(g, r)
    check_l1(g, r, sc)
    if c.get("big") and tile[0] * tile[1] <= 256:  # (the case is sized for 256-pixel tiles)
        sp = g["spans"].reshape(-1, 4).astype(np.int64)
        sp = sp[sp[:, 0] >= 0]
        tiles = ((sp[:, 1] // tile[0] - sp[:, 0] // tile[0] + 1) *
                 (sp[:, 3] // tile[1] - sp[:, 2] // tile[1] + 1))
        assert (tiles >= BIG_TILES).sum() >= 3, "no large splats in the large-splat case"
        assert (tiles < BIG_TILES).sum() >= 3, "no small splats in the large-splat case"
    if c.get("dense") and tile[0] * tile[1] <= 512:  # (sized for tiles of at most 512 pixels)
        # a super-tile (8 x 8 tiles) with twice the pairs the LDS array holds:
        # its items (at most 2048) make at most two chunks of 1024, so one of
        # them holds more pairs than the array
        assert sc.n <= 2048
        gw, gh = -(-sc.width // tile[0]), -(-sc.height // tile[1])
        r0 = g["ranges"].reshape(-1, 2).astype(np.int64)
        per = (r0[:, 1] - r0[:, 0]).reshape(sc.views, gh, gw)
        st_pairs = max(int(per[v, y:y + 8, x:x + 8].sum()) for v in range(sc.views)
                       for y in range(0, gh, 8) for x in range(0, gw, 8))
        assert st_pairs > 2 * L2_OUT, "dense case not dense"
    # render backward fed the same dL/dimage
    grad_close(g["gq_render"][:, :sc.n], r["gyhat"][:, :sc.n], name="grad qparams")
    grad_close(g["gmask"], r["gmhat"], name="grad mask")
    grad_close(g["gparams"][:, :sc.n], r["gy"][:, :sc.n], name="grad params")
    grad_close(g["gq"], r["gq"], name="grad qstep")
    # the exported per-(view, Gaussian) splat gradients (the records the
    # sampled full-size test compares) against the oracle's
    _, _, gs = orc.backward(r["p64"], r["m64"], sc.n, sc.cams, sc.width, sc.height, r["st"],
                            r["dimage"], want_splat=True)
    for k, name in enumerate(("px", "py", "A", "B", "C", "opacity", "r", "g", "b", "mask")):
        grad_close(g["sgrad"][..., k], gs[..., k], name=f"splat grad {name}")


def test_projection_records(orc, gctx, dev):
    sc = synth.make_scene("c1")
    g, r = run_pair(orc, gctx, dev, sc)
    pj = orc.project64(r["yhat"].astype(np.float64), sc.n, sc.cams, sc.width, sc.height, r["st"])
    ok = r["st"].valid > 0
    sp = g["splats"][ok]
    ref = pj[ok]
    assert np.allclose(sp[:, 0:2], ref[:, 0:2], rtol=0, atol=2e-4)
    for k in (2, 3, 4):
        scale = np.abs(ref[:, 2:5]).max(axis=1)
        assert (np.abs(sp[:, k] - ref[:, k]) <= 1e-5 * scale + 1e-7).all(), f"conic {k}"
    assert np.allclose(sp[:, 5], ref[:, 5], atol=1e-6)
    assert np.allclose(sp[:, 6:9], ref[:, 6:9], atol=2e-6)


def test_c1_full_step(orc, gctx, dev):
    """4,096 Gaussians, 128x128: the small measured configuration, lam = 2.5e-5
    and lam = 1 (rate gradients visible)."""
    sc = synth.make_scene("c1")
    for lam in (2.5e-5, 1.0):
        g, r = run_pair(orc, gctx, dev, sc, lam=lam)
        check_structure(g, r, sc)
        check_stats(g, r, sc)
        err, frac = check_image(g, r)
        check_l1(g, r, sc)
        _say(f"c1 lam={lam}: pixel err {err:.2e}, margin {frac:.2e}, P={g['P']}, E={g['evals']}")
        grad_close(g["gparams"][:, :sc.n], r["gy"][:, :sc.n], name="grad params")
        grad_close(g["gq"], r["gq"], name="grad qstep")
        grad_close(g["gmask"], r["gmhat"], name="grad mask")


def test_eval_count_modes(orc, gctx, dev):
    """Mode 0 counts the method's evaluations (the oracle's count); mode 1 the
    evaluations the timed blend performs after its reach test (no more than
    mode 0); images, T and stop positions are the same bits in every mode."""
    from paper_2607_12656_amd.rd import RDStep
    sc = synth.make_scene("c1")
    rd = RDStep(gctx, sc.n, sc.npad, sc.n_hat, sc.cams, sc.width, sc.height, fused=True)
    params, q, score = T(sc.params, dev), T(sc.qstep, dev), T(sc.score, dev)
    mask, target = T(sc.given_mask, dev), T(sc.target, dev)
    outs, counts = [], []
    for mode in (0, 1, None):
        if mode is not None:
            gctx.set_eval_count_mode(mode)
        rd.evals.zero_()
        rd.forward(params, q, score, target, 0.5, 0, mask, 0, 0, count_evals=mode is not None)
        torch.cuda.synchronize()
        counts.append(int(rd.evals.item()))
        outs.append([x.cpu().numpy().view(np.uint32) for x in (rd.image, rd.final_T, rd.last)])
    gctx.set_eval_count_mode(0)
    s = orc.rd_forward(sc.params, sc.qstep, sc.score, sc.given_mask, sc.cams, sc.width,
                       sc.height, sc.target, sc.n, sc.n_hat, 0.5)
    assert counts[0] == s["fw"]["evals"]
    assert 0 < counts[1] <= counts[0] and counts[2] == 0
    _say(f"c1 evaluations: {counts[0]} in span, {counts[1]} after the reach test")
    for o in outs[1:]:
        for a, b in zip(outs[0], o):
            assert np.array_equal(a, b)
    from paper_2607_12656_amd import SgsError
    with pytest.raises(SgsError):
        gctx.set_eval_count_mode(2)


@pytest.mark.parametrize("fused", [False, True])
def test_end_to_end_each_side_own_l1_gradient(orc, gctx, dev, fused):
    """The whole step with nothing shared but the inputs: each side takes its
    own L1 gradient into its own backward.  Scenes are drawn (seeds in a
    fixed order) until one has no margin pixel and no colour within 1e-4 of
    its target, where the two sides could legitimately differ."""
    from paper_2607_12656_amd.rd import RDStep
    lam = 0.5
    for seed in range(40, 60):
        sc = synth.make_tiny(120, 56, 40, views=2, seed=seed)
        s = orc.rd_step(sc.params, sc.qstep, sc.score, sc.given_mask, sc.cams, sc.width,
                        sc.height, sc.target, sc.n, sc.n_hat, lam)
        near = np.abs(s["fw"]["image"] - sc.target) <= 1e-4
        if s["fw"]["margin"].any() or near.any():
            continue
        break
    else:
        pytest.fail("no seed without margin pixels and near-target colours")
    _say(f"[gpu] end-to-end seed {seed} fused={fused}")
    rd = RDStep(gctx, sc.n, sc.npad, sc.n_hat, sc.cams, sc.width, sc.height, fused=fused)
    params, q, score = T(sc.params, dev), T(sc.qstep, dev), T(sc.score, dev)
    mask, target = T(sc.given_mask, dev), T(sc.target, dev)
    rd.forward(params, q, score, target, lam, 0, mask, 0, 0, count_evals=False)
    gp = torch.empty_like(params)
    rd.backward(params, q, 0, grad_params=gp)
    torch.cuda.synchronize()
    assert abs(float(rd.loss.item()) - s["D"]) <= 1e-6 * s["D"]
    assert np.abs(rd.image.cpu().numpy() - s["fw"]["image"]).max() <= 1e-4
    grad_close(gp.cpu().numpy()[:, :sc.n], s["gy"][:, :sc.n], name="grad params")
    grad_close(rd.grad_q.cpu().numpy(), s["gq"], name="grad qstep")
    grad_close(rd.grad_mask.cpu().numpy(), s["gmhat"], name="grad mask")


@pytest.mark.parametrize("schedule", ["stride", "queue", "block"])
@pytest.mark.parametrize("tile", [(16, 16), (8, 8), (32, 8)])
def test_persistent_schedules(orc, gctx, dev, tile, schedule):
    """Resident-workgroup blend schedules (tiles ordered by list length) give
    the same structure, image and gradients as the oracle; two views."""
    sc = synth.make_tiny(400, 150, 90, views=2, seed=11)
    g, r = run_pair(orc, gctx, dev, sc, tile=tile, schedule=schedule)
    check_structure(g, r, sc)
    check_image(g, r)
    check_l1(g, r, sc)
    grad_close(g["gparams"][:, :sc.n], r["gy"][:, :sc.n], name="grad params")
    grad_close(g["gmask"], r["gmhat"], name="grad mask")


def test_gumbel_mask_mode(orc, gctx, dev):
    sc = synth.make_tiny(300, 64, 48, seed=9)
    for step in (0, 7):
        g, r = run_pair(orc, gctx, dev, sc, mode=1, seed=1234, step=step)
        assert np.array_equal(g["hard"], r["mhat"])
        assert np.allclose(g["soft"], r["msoft"], atol=2e-6)
        check_structure(g, r, sc)
        check_image(g, r)
        check_l1(g, r, sc)
        grad_close(g["gscore"], r["gs"], name="grad score")
    # keep-all mode
    g, _ = run_pair(orc, gctx, dev, sc, mode=2)
    assert g["hard"].all()


FUSED_CASES = [
    dict(kind="tiny", cfg=0),
    dict(kind="tiny", cfg=1),
    dict(kind="tiny", cfg=2, tile=(8, 8)),
    dict(kind="c1", lam=1.0),
    dict(kind="gumbel", mode=1, step=7),
    dict(kind="gumbel", mode=2),
    dict(kind="two_views", schedule="stride", tile=(32, 8)),
    dict(kind="two_views", schedule="block", tile=(16, 16)),
]


@pytest.mark.parametrize("case", range(len(FUSED_CASES)))
def test_fused_step_matches_oracle(orc, gctx, dev, case):
    """quant_render_fwd / quant_render_bwd (quantizer inside the projection and
    its backward) against the oracle: structure, statistics, image and every
    gradient, mask modes 0-2, several tile shapes and schedules."""
    c = FUSED_CASES[case]
    kind = c["kind"]
    if kind == "tiny":
        t = TINY[c["cfg"]]
        sc = synth.make_tiny(t["n"], t["W"], t["H"], views=t["V"], seed=t["seed"],
                             logscale_mu=t.get("logscale", -2.0))
    elif kind == "c1":
        sc = synth.make_scene("c1")
    elif kind == "gumbel":
        sc = synth.make_tiny(300, 64, 48, seed=9)
    else:
        sc = synth.make_tiny(400, 150, 90, views=2, seed=11)
    mode = c.get("mode", 0)
    g, r = run_pair(orc, gctx, dev, sc, tile=c.get("tile", (16, 16)), lam=c.get("lam", 0.5),
                    mode=mode, seed=1234 if mode == 1 else 0, step=c.get("step", 0),
                    schedule=c.get("schedule", "tile"), fused=True)
    check_structure(g, r, sc)
    check_stats(g, r, sc)
    check_image(g, r)
    check_l1(g, r, sc)
    if mode == 1:
        assert np.allclose(g["soft"], r["msoft"], atol=2e-6)
        grad_close(g["gscore"], r["gs"], name="grad score")
    elif mode == 2:
        assert g["hard"].all()
    grad_close(g["gparams"][:, :sc.n], r["gy"][:, :sc.n], name="grad params")
    grad_close(g["gq"], r["gq"], name="grad qstep")
    grad_close(g["gmask"], r["gmhat"], name="grad mask")


def test_fakequant_bwd_isolated(orc, gctx, dev):
    """Same upstream gradient on both sides: STE copy, LSQ step gradient,
    rate-gradient scatter."""
    from paper_2607_12656_amd.rd import RDStep
    sc = synth.make_tiny(5000, 32, 32, seed=5)
    rng = np.random.default_rng(1)
    gyh = np.zeros((NCH, sc.npad), np.float32)
    gyh[:, :sc.n] = rng.normal(size=(NCH, sc.n))
    rd = RDStep(gctx, sc.n, sc.npad, sc.n_hat, sc.cams, sc.width, sc.height)
    params, q = T(sc.params, dev), T(sc.qstep, dev)
    gctx.fakequant_prune(params, q, None, 0, T(sc.given_mask, dev), 0, 0, rd.qparams, rd.hard,
                         rd.soft, rd.stats)
    lam = 0.3
    gctx.rate_proxy(rd.stats, q, lam, rd.rate3, rd.rate_grad)
    gin = T(gyh, dev)
    gm = torch.zeros(sc.n, device=dev)
    gp = torch.empty_like(params)
    gctx.fakequant_prune_bwd(params, q, rd.soft, 0, rd.rate_grad, rd.stats, gin, gm, gp,
                             rd.grad_q, rd.grad_score)
    torch.cuda.synchronize()
    rate = orc.rate_proxy(sc.params, sc.qstep, sc.given_mask, sc.n, sc.n_hat, lam)
    gy, gq, _ = orc.fakequant_bwd(sc.params, sc.qstep, gyh.astype(np.float64), 0,
                                  np.zeros(sc.n), 1.0, np.zeros(sc.n), sc.n)
    gy = gy + rate["gy"]
    gq = gq + rate["gq"]
    grad_close(gp.cpu().numpy()[:, :sc.n], gy[:, :sc.n], tol=1e-6, name="grad params")
    grad_close(rd.grad_q.cpu().numpy(), gq, tol=1e-5, name="grad qstep")


def test_invalid_step_size_flag(gctx, dev):
    from paper_2607_12656_amd import SgsError
    from paper_2607_12656_amd.rd import RDStep
    sc = synth.make_tiny(100, 32, 32, seed=6)
    rd = RDStep(gctx, sc.n, sc.npad, sc.n_hat, sc.cams, sc.width, sc.height)
    q = sc.qstep.copy()
    q[7] = 0.0
    gctx.fakequant_prune(T(sc.params, dev), T(q, dev), None, 0, T(sc.given_mask, dev), 0, 0,
                         rd.qparams, rd.hard, rd.soft, rd.stats)
    with pytest.raises(SgsError):
        gctx.query(rd.stats)


def test_full_size_1m_workload(orc, gctx, dev):
    """The measured configuration (1M Gaussians, 1297x840, 16x16 tiles, the
    bench's launch configuration): every pair, pixel and gradient against the
    oracle (about 10 s of oracle time)."""
    sc = synth.make_scene("c2")
    g, r = run_pair(orc, gctx, dev, sc, lam=2.5e-5)
    check_structure(g, r, sc)
    check_stats(g, r, sc)
    err, frac = check_image(g, r)
    check_l1(g, r, sc)
    _say(f"c2: pixel err {err:.2e}, margin {frac:.2e}, P={g['P']}, E={g['evals']}")
    grad_close(g["gq_render"][:, :sc.n], r["gyhat"][:, :sc.n], name="grad qparams")
    grad_close(g["gmask"], r["gmhat"], name="grad mask")
    grad_close(g["gq"], r["gq"], name="grad qstep")


def test_full_size_1m_workload_fused(orc, gctx, dev):
    """The benchmark's step (fused entry points, whole-tile blend schedule,
    16x16 tiles) at 1M Gaussians, 1297x840: every pair, pixel and gradient
    against the oracle."""
    sc = synth.make_scene("c2")
    g, r = run_pair(orc, gctx, dev, sc, lam=2.5e-5, schedule="block", fused=True)
    check_structure(g, r, sc)
    check_stats(g, r, sc)
    err, frac = check_image(g, r)
    check_l1(g, r, sc)
    _say(f"c2 fused: pixel err {err:.2e}, margin {frac:.2e}, P={g['P']}, E={g['evals']}")
    grad_close(g["gparams"][:, :sc.n], r["gy"][:, :sc.n], name="grad params")
    grad_close(g["gmask"], r["gmhat"], name="grad mask")
    grad_close(g["gq"], r["gq"], name="grad qstep")


@pytest.fixture(scope="module")
def c3_case(orc):
    """The 3M x 8-view scene, its quantized parameters and the oracle's
    decision layer (culling, spans, depths; no pair list)."""
    sc = synth.make_scene("c3")
    yh, _ = orc.fakequant(sc.params, sc.qstep, sc.n)
    lite = orc.decide(yh, sc.n, sc.cams, sc.width, sc.height, 16, 16, bin_pairs=False)
    return sc, yh, lite


def test_full_size_3m_8views_gradients_sampled(orc, gctx, dev, c3_case):
    """Gradients at 3M Gaussians x 8 views of 1600x1060 (the bench's launch
    configuration, the timed forward path): 24 Gaussians (20 kept, 4
    pruned), each with its splat gradients in every view summed by the
    oracle over every pixel of its span (each pixel composited by brute
    force over the view's splats in depth order), the projection backward
    summed over views, and the mask gradient.  The upstream gradient is a
    seeded +-1/(3VHW) pattern (the L1 gradient's shape), zeroed at the
    oracle's margin pixels inside those spans on both sides."""
    from paper_2607_12656_amd.rd import RDStep
    sc, yh, lite = c3_case
    n, V, W, H = sc.n, sc.views, sc.width, sc.height
    _say(f"[gpu] c3 gradients n={n} V={V} {W}x{H}")
    rng = np.random.default_rng(17)
    valid = lite.valid > 0
    nvalid = valid.sum(0)
    rmax = np.where(valid, lite.radius, 0).max(0)
    ok = (nvalid >= 4) & (rmax >= 2) & (rmax <= 10)
    kept = sc.given_mask > 0
    sel = np.concatenate([rng.choice(np.flatnonzero(ok & kept), 20, replace=False),
                          rng.choice(np.flatnonzero(ok & ~kept), 4, replace=False)])
    p64 = yh.astype(np.float64)
    m64 = sc.given_mask.astype(np.float64)
    _, _, margin = orc.splat_grads_sampled(p64, m64, n, sc.cams, W, H, lite, sel)
    drng = np.random.default_rng(23)
    d = np.where(drng.random((V, 3, H, W), dtype=np.float32) < 0.5, -1.0, 1.0).astype(np.float32)
    d *= np.float32(1.0 / (3 * V * W * H))
    d *= (margin == 0)[:, None, :, :]
    _say(f"c3 gradients: {int(margin.sum())} margin pixels in the chosen spans")

    rd = RDStep(gctx, n, sc.npad, sc.n_hat, sc.cams, W, H, tile=(16, 16))
    gctx.reserve_pairs(lite.pairs + lite.pairs // 8 + 4096)
    params, q, score = T(sc.params, dev), T(sc.qstep, dev), T(sc.score, dev)
    mask, target = T(sc.given_mask, dev), T(sc.target, dev)
    rd.forward(params, q, score, target, 2.5e-5, 0, mask, 0, 0, count_evals=False)
    gp = torch.empty_like(params)
    rd.backward(params, q, 0, grad_params=gp, dimage=T(d, dev))
    del gp
    sg = torch.empty(V, n, 12, dtype=torch.float32, device=dev)
    gctx.copy_splat_grads(sg)
    sel_t = torch.from_numpy(sel).to(dev)
    g_splat = sg[:, sel_t, :10].cpu().numpy().transpose(1, 0, 2)     # [k][V][10]
    del sg
    g_param = rd.grad_qparams[:, sel_t].cpu().numpy().T              # [k][59]
    g_mask = rd.grad_mask[sel_t].cpu().numpy()
    torch.cuda.synchronize()
    gs, gpar, _ = orc.splat_grads_sampled(p64, m64, n, sc.cams, W, H, lite, sel,
                                          d.astype(np.float64))
    culled = ~valid[:, sel].T
    assert not g_splat[culled].any(), "culled (view, Gaussian) with a gradient"
    for k, name in enumerate(("px", "py", "A", "B", "C", "opacity", "r", "g", "b", "mask")):
        grad_close(g_splat[..., k], gs[..., k], name=f"splat grad {name}")
    grad_close(g_param, gpar, name="grad qparams (render)")
    grad_close(g_mask, gs[..., 9].sum(1), name="grad mask (render)")
    _say(f"c3 gradients: {len(sel)} Gaussians over {int(valid[:, sel].sum())} (view, Gaussian) "
         f"spans agree")


def test_full_size_3m_8views_sampled(orc, gctx, dev, c3_case):
    """3M Gaussians x 8 views of 1600x1060 in the bench's launch configuration
    (16x16 tiles, reserved pair capacity, about 5.5e8 pairs).  Full check of
    what the oracle can afford at this size: quantized parameters, hard mask,
    rate scalars, every (view, Gaussian)'s culling, span and depth, the pair
    count and every tile's range; sampled checks of the rest: the sorted lists
    of 24 tiles (the heaviest, the ragged bottom row, random ones) and the
    colour and transmittance of 24 pixels per view by brute force."""
    from paper_2607_12656_amd.rd import RDStep
    sc, yh, lite = c3_case
    n, V, W, H = sc.n, sc.views, sc.width, sc.height
    lam = 2.5e-5
    _say(f"[gpu] c3 n={n} V={V} {W}x{H}")
    cnt = orc.tile_counts(lite, n, V, W, H)
    assert cnt.sum() == lite.pairs

    rd = RDStep(gctx, n, sc.npad, sc.n_hat, sc.cams, W, H, tile=(16, 16))
    gctx.reserve_pairs(lite.pairs + lite.pairs // 8 + 4096)
    params, q, score = T(sc.params, dev), T(sc.qstep, dev), T(sc.score, dev)
    mask, target = T(sc.given_mask, dev), T(sc.target, dev)
    rd.forward(params, q, score, target, lam, 0, mask, 0, 0)
    torch.cuda.synchronize()
    P, _ = gctx.query(rd.stats)
    assert P == lite.pairs, f"pair count {P} vs {lite.pairs}"

    assert np.array_equal(rd.qparams[:, :n].cpu().numpy(), yh[:, :n]), "quantized parameters"
    assert np.array_equal(rd.hard.cpu().numpy(), sc.given_mask), "hard mask"
    rp = orc.rate_proxy(sc.params, sc.qstep, sc.given_mask, n, sc.n_hat)
    R, Lq, Lm = rd.rate3.cpu().numpy()
    for a, b in ((R, rp["R"]), (Lq, rp["Lq"]), (Lm, rp["Lm"])):
        assert abs(a - b) <= 1e-6 * abs(b)

    GW, GH = -(-W // 16), -(-H // 16)
    tile_ids = torch.empty(P, dtype=torch.int32, device=dev)
    vals = torch.empty(P, dtype=torch.int32, device=dev)
    ranges = torch.empty(V * GW * GH, 2, dtype=torch.int32, device=dev)
    spans = torch.empty(V, n, 4, dtype=torch.int32, device=dev)
    depth = torch.empty(V, n, dtype=torch.float32, device=dev)
    splats = torch.empty(V, n, 12, dtype=torch.float32, device=dev)
    gctx.copy_structure(tile_ids, vals, P, ranges, spans, depth, splats)
    torch.cuda.synchronize()
    del splats

    valid = lite.valid > 0
    gsp = spans.cpu().numpy()
    assert np.array_equal(gsp[..., 0] >= 0, valid), "culling"
    assert np.array_equal(gsp[valid], lite.span[valid]), "pixel spans"
    del gsp
    assert np.array_equal(depth.cpu().numpy()[valid].view(np.uint32),
                          lite.tz[valid].view(np.uint32)), "depth"

    rg = ranges.cpu().numpy().astype(np.int64)
    nz = cnt > 0
    start = np.concatenate([[0], np.cumsum(cnt)[:-1]])
    assert np.array_equal(rg[nz, 0], start[nz]) and np.array_equal(rg[nz, 1] - rg[nz, 0], cnt[nz]), \
        "tile ranges"
    assert (rg[~nz, 0] == rg[~nz, 1]).all(), "empty tiles"

    rng = np.random.default_rng(7)
    tpv = GW * GH
    heavy = int(np.argmax(cnt))
    bottom = [v * tpv + (GH - 1) * GW + tx for v, tx in ((0, 0), (3, GW // 2), (7, GW - 1))]
    pick = [heavy] + [t for t in bottom if cnt[t] > 0] + list(rng.choice(np.flatnonzero(nz), 20,
                                                                        replace=False))
    for t in pick:
        b, e = int(rg[t, 0]), int(rg[t, 1])
        assert (tile_ids[b:e] == t).all().item(), f"tile ids of tile {t}"
        got = vals[b:e].cpu().numpy().view(np.uint32)
        ref = orc.tile_list(lite, n, t // tpv, t % tpv, W)
        assert np.array_equal(got, ref), f"sorted list of tile {t} ({e - b} pairs)"
    _say(f"c3: P={P}, heaviest tile {heavy} with {cnt[heavy]} pairs, {len(pick)} tile lists equal")
    del tile_ids, vals

    per = 24
    hv, ht = heavy // tpv, heavy % tpv
    px = []
    for v in range(V):
        u = rng.integers(0, W, per)
        y = rng.integers(0, H, per)
        u[:2], y[:2] = (0, W - 1), (H - 1, H - 1)          # corners of the ragged row
        if v == hv:                                        # inside the heaviest tile
            u[2:6] = (ht % GW) * 16 + rng.integers(0, 16, 4)
            y[2:6] = np.minimum((ht // GW) * 16 + rng.integers(0, 16, 4), H - 1)
        px.append(np.stack([np.full(per, v), u, y], 1))
    px = np.concatenate(px)
    out, mg, _ = orc.pixels_brute(yh.astype(np.float64), sc.given_mask.astype(np.float64), n,
                                  sc.cams, W, H, lite, px)
    img = rd.image.cpu().numpy()
    Tg = rd.final_T.cpu().numpy()
    ok = mg == 0
    # about 3.5e-4 of the pixels are margin pixels at this size (71 in-span
    # evaluations per pixel): expect none or one among these 192
    assert (~ok).sum() <= 2, f"too many margin pixels ({(~ok).sum()})"
    g = np.concatenate([img[px[:, 0], :, px[:, 2], px[:, 1]], Tg[px[:, 0], px[:, 2], px[:, 1]][:, None]], 1)
    err = np.abs(g - out)[ok].max()
    _say(f"c3: {ok.sum()} sampled pixels, max error {err:.2e}")
    assert err <= 1e-4, f"sampled pixel error {err:.3e}"
    # the L1 gradient at the sampled pixels: sign(C - target) / (3 V H W)
    # from the brute-force colours, wherever |C - target| > 1e-4
    dg = rd.dimage.cpu().numpy()[px[:, 0], :, px[:, 2], px[:, 1]].astype(np.float64)
    tg = sc.target[px[:, 0], :, px[:, 2], px[:, 1]].astype(np.float64)
    diff = out[:, :3] - tg
    far = (np.abs(diff) > 1e-4) & ok[:, None]
    ref = np.sign(diff) / (3.0 * V * W * H)
    assert (np.abs(dg - ref)[far] <= 1e-6 * np.abs(ref[far])).all(), "L1 gradient"
