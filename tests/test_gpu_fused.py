"""The fused step entry points (quant_render_fwd / quant_render_bwd) against
the separate calls (fakequant_prune -> render_fwd, render_bwd ->
fakequant_prune_bwd) on the same inputs: every output bit for bit, except
the step-size gradient, the same FP64 sum added in another order and then
rounded to float (within 1e-6 of the largest entry).  The separate calls are
themselves checked against the oracle in test_gpu_parity.py, and so is the
fused path there."""
import sys

import numpy as np
import pytest

import synth

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


def one_step(rd, params, q, score, mask, target, lam, mode, seed, step):
    rd.evals.zero_()
    gp = torch.empty_like(params)
    rd.forward(params, q, score, target, lam, mode, mask, seed, step)
    rd.backward(params, q, mode, grad_params=gp)
    torch.cuda.synchronize()
    c = lambda x: x.cpu().numpy().copy()
    return dict(hard=c(rd.hard), soft=c(rd.soft), stats=c(rd.stats), rate3=c(rd.rate3),
                image=c(rd.image), T=c(rd.final_T), last=c(rd.last), evals=c(rd.evals),
                loss=c(rd.loss), gparams=c(gp), gmask=c(rd.grad_mask), gq=c(rd.grad_q),
                gscore=c(rd.grad_score))


CASES = [
    dict(scene="c1", lam=1.0),
    dict(scene="tiny2", lam=0.5, tile=(8, 8), schedule="queue"),
    dict(scene="gumbel", lam=0.5, mode=1, step=3),
    dict(scene="gumbel", lam=0.5, mode=2),
    dict(scene="c2", lam=2.5e-5, schedule="stride"),
    dict(scene="c2", lam=2.5e-5, schedule="block"),
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_fused_equals_separate_calls(gctx, dev, case):
    from paper_2607_12656_amd.rd import RDStep
    c = CASES[case]
    if c["scene"] == "tiny2":
        sc = synth.make_tiny(700, 130, 70, views=2, seed=21)
    elif c["scene"] == "gumbel":
        sc = synth.make_tiny(900, 96, 64, seed=22)
    else:
        sc = synth.make_scene(c["scene"])
    mode = c.get("mode", 0)
    _say(f"[gpu] fused vs separate: {sc.name} n={sc.n} V={sc.views} mode={mode}")
    rd = RDStep(gctx, sc.n, sc.npad, sc.n_hat, sc.cams, sc.width, sc.height,
                tile=c.get("tile", (16, 16)), schedule=c.get("schedule", "tile"))
    params, q, score = T(sc.params, dev), T(sc.qstep, dev), T(sc.score, dev)
    mask, target = T(sc.given_mask, dev), T(sc.target, dev)
    args = (params, q, score, mask, target, c["lam"], mode, 77, c.get("step", 0))
    rd.fused = False
    a = one_step(rd, *args)
    rd.fused = True
    b = one_step(rd, *args)
    for k in ("hard", "soft", "stats", "rate3", "image", "T", "last", "evals", "loss", "gmask",
              "gscore"):
        assert np.array_equal(a[k].view(np.uint8), b[k].view(np.uint8)), k
    n = sc.n
    assert np.array_equal(a["gparams"][:, :n].view(np.uint32),
                          b["gparams"][:, :n].view(np.uint32)), "grad params"
    gq_a, gq_b = a["gq"].astype(np.float64), b["gq"].astype(np.float64)
    tol = 1e-6 * np.abs(gq_a).max()
    assert np.abs(gq_a - gq_b).max() <= tol, f"grad qstep {np.abs(gq_a - gq_b).max():.3e}"
    # the fused path repeats exactly
    b2 = one_step(rd, *args)
    for k in b:
        assert np.array_equal(b[k].view(np.uint8), b2[k].view(np.uint8)), f"repeat {k}"


def test_fused_backward_without_rate_terms(gctx, dev):
    """rate_grad / stats omitted (the learned-rate path adds its own): the
    fused backward equals render_bwd + fakequant_prune_bwd without them."""
    from paper_2607_12656_amd.rd import RDStep
    sc = synth.make_tiny(1500, 120, 90, seed=23)
    rd = RDStep(gctx, sc.n, sc.npad, sc.n_hat, sc.cams, sc.width, sc.height)
    params, q, score = T(sc.params, dev), T(sc.qstep, dev), T(sc.score, dev)
    mask, target = T(sc.given_mask, dev), T(sc.target, dev)
    c = gctx
    outs = []
    for fused in (False, True):
        gp = torch.empty_like(params)
        gq = torch.empty_like(q)
        gs = torch.empty_like(score)
        gm = torch.empty(sc.n, dtype=torch.float32, device=dev)
        if fused:
            c.quant_render_fwd(params, q, score, 1, None, 5, 9, rd.hard, rd.soft, rd.stats,
                               rd.image, rd.final_T, rd.last)
            c.l1_loss(rd.image, target, rd.loss, rd.dimage)
            c.quant_render_bwd(params, q, rd.soft, 1, None, None, rd.final_T, rd.last,
                               rd.dimage, gp, gq, gs, gm)
        else:
            c.fakequant_prune(params, q, score, 1, None, 5, 9, rd.qparams, rd.hard, rd.soft,
                              rd.stats)
            c.render_fwd(rd.qparams, rd.hard, rd.image, rd.final_T, rd.last)
            c.l1_loss(rd.image, target, rd.loss, rd.dimage)
            c.render_bwd(rd.qparams, rd.hard, rd.final_T, rd.last, rd.dimage, rd.grad_qparams,
                         gm)
            c.fakequant_prune_bwd(params, q, rd.soft, 1, None, None, rd.grad_qparams, gm, gp,
                                  gq, gs)
        torch.cuda.synchronize()
        outs.append([x.cpu().numpy().copy() for x in (rd.image, gp, gq, gs, gm)])
    (ia, pa, qa, sa, ma), (ib, pb, qb, sb, mb) = outs
    assert np.array_equal(ia, ib)
    assert np.array_equal(pa[:, :sc.n].view(np.uint32), pb[:, :sc.n].view(np.uint32))
    assert np.array_equal(sa.view(np.uint32), sb.view(np.uint32))
    assert np.array_equal(ma.view(np.uint32), mb.view(np.uint32))
    assert np.abs(qa.astype(np.float64) - qb).max() <= 1e-6 * np.abs(qa).max()


def test_fused_entry_validation(gctx, dev):
    from paper_2607_12656_amd import SgsError
    from paper_2607_12656_amd.rd import RDStep
    sc = synth.make_tiny(100, 32, 32, seed=6)
    rd = RDStep(gctx, sc.n, sc.npad, sc.n_hat, sc.cams, sc.width, sc.height)
    params, q = T(sc.params, dev), T(sc.qstep, dev)
    mask = T(sc.given_mask, dev)
    with pytest.raises(SgsError):   # mode 0 needs the given mask
        gctx.quant_render_fwd(params, q, None, 0, None, 0, 0, rd.hard, rd.soft, rd.stats,
                              rd.image, rd.final_T, rd.last)
    gctx.quant_render_fwd(params, q, None, 0, mask, 0, 0, rd.hard, rd.soft, rd.stats,
                          rd.image, rd.final_T, rd.last)
    with pytest.raises(SgsError):   # grad_params may not alias params
        gctx.quant_render_bwd(params, q, rd.soft, 0, None, None, rd.final_T, rd.last,
                              rd.dimage, params, rd.grad_q, rd.grad_score, rd.grad_mask)
    with pytest.raises(SgsError):   # rate_grad without stats
        gctx.quant_render_bwd(params, q, rd.soft, 0, rd.rate_grad, None, rd.final_T, rd.last,
                              rd.dimage, rd.grad_qparams, rd.grad_q, rd.grad_score,
                              rd.grad_mask)
    torch.cuda.synchronize()


ORDER_CASES = [
    dict(tile=(16, 16), views=1, schedule="block"),   # 3,933 tiles
    dict(tile=(16, 16), views=2, schedule="queue"),   # 7,866 tiles
    dict(tile=(8, 8), views=1, schedule="block"),     # 15,594 tiles
    dict(tile=(8, 8), views=1, schedule="stride"),
]


@pytest.mark.parametrize("case", range(len(ORDER_CASES)))
def test_length_ordered_schedules_match_per_tile(gctx, dev, case):
    """The persistent blend schedules walk tiles in list-length order; every
    tile is still blended exactly once, so image, T and stop index equal
    those of the one-workgroup-per-tile schedule bit for bit, and the
    gradients (FP64 sums in another order) agree closely, on grids of
    thousands of tiles."""
    from paper_2607_12656_amd.rd import RDStep
    c = ORDER_CASES[case]
    sc = synth.make_tiny(6000, 1100, 900, views=c["views"], seed=31)
    _say(f"[gpu] tile order: tile={c['tile']} V={sc.views} schedule={c['schedule']}")
    params, q, score = T(sc.params, dev), T(sc.qstep, dev), T(sc.score, dev)
    mask, target = T(sc.given_mask, dev), T(sc.target, dev)
    outs = []
    for schedule in ("tile", c["schedule"]):
        rd = RDStep(gctx, sc.n, sc.npad, sc.n_hat, sc.cams, sc.width, sc.height,
                    tile=c["tile"], schedule=schedule)
        rd.fused = True
        outs.append(one_step(rd, params, q, score, mask, target, 0.5, 0, 5, 0))
    a, b = outs
    for k in ("image", "T", "last", "evals", "hard"):
        assert np.array_equal(a[k].view(np.uint8), b[k].view(np.uint8)), k
    n = sc.n
    ga, gb = a["gparams"][:, :n].astype(np.float64), b["gparams"][:, :n].astype(np.float64)
    assert np.linalg.norm(ga - gb) <= 1e-5 * np.linalg.norm(ga)
    assert np.linalg.norm(a["gmask"] - b["gmask"]) <= 1e-5 * np.linalg.norm(a["gmask"])


def test_fused_backward_skips_higher_sh_rows(gctx, dev):
    """With the higher-SH gradient rows switched off (a step whose Adam update
    skips channels 6-50), the fused backward leaves those rows of grad_params
    as they were and writes every other output bit for bit as with them on;
    the step-size gradient still takes all channels."""
    from paper_2607_12656_amd.rd import RDStep
    sc = synth.make_tiny(1500, 120, 90, seed=24)
    rd = RDStep(gctx, sc.n, sc.npad, sc.n_hat, sc.cams, sc.width, sc.height)
    params, q, score = T(sc.params, dev), T(sc.qstep, dev), T(sc.score, dev)
    target = T(sc.target, dev)
    c = gctx
    c.quant_render_fwd(params, q, score, 1, None, 5, 9, rd.hard, rd.soft, rd.stats, rd.image,
                       rd.final_T, rd.last)
    c.rate_proxy(rd.stats, q, 0.5, rd.rate3, rd.rate_grad)
    c.l1_loss(rd.image, target, rd.loss, rd.dimage)
    sentinel = -1234.5
    outs = []
    try:
        for on in (True, False):
            gp = torch.full_like(params, sentinel)
            gq, gs = torch.empty_like(q), torch.empty_like(score)
            gm = torch.empty(sc.n, dtype=torch.float32, device=dev)
            c.set_grad_sh_rest(on)
            c.quant_render_bwd(params, q, rd.soft, 1, rd.rate_grad, rd.stats, rd.final_T,
                               rd.last, rd.dimage, gp, gq, gs, gm)
            torch.cuda.synchronize()
            outs.append([x.cpu().numpy().copy() for x in (gp, gq, gs, gm)])
    finally:
        c.set_grad_sh_rest(True)
    (pa, qa, sa, ma), (pb, qb, sb, mb) = outs
    n, rest = sc.n, np.r_[6:51]
    keep = np.setdiff1d(np.arange(pa.shape[0]), rest)
    assert np.array_equal(pa[keep, :n].view(np.uint32), pb[keep, :n].view(np.uint32))
    assert np.all(pb[rest, :n] == np.float32(sentinel)), "higher-SH rows were written"
    assert not np.any(pa[rest, :n] == np.float32(sentinel)), "higher-SH rows were skipped"
    for a, b in ((qa, qb), (sa, sb), (ma, mb)):
        assert np.array_equal(a.view(np.uint32), b.view(np.uint32))
