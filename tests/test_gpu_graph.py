"""Device-side pair count, capacity overflow and HIP-graph capture of whole
RD steps (forward + backward), through the C ABI."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda", 0)


def T(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def _setup(dev, sc, stream, tile=(16, 16)):
    from paper_2607_12656_amd import Context
    from paper_2607_12656_amd.rd import RDStep
    ctx = Context(0, stream=stream)
    rd = RDStep(ctx, sc.n, sc.npad, sc.n_hat, sc.cams, sc.width, sc.height, tile=tile)
    ins = dict(params=T(sc.params, dev), q=T(sc.qstep, dev), score=T(sc.score, dev),
               mask=T(sc.given_mask, dev), target=T(sc.target, dev))
    return ctx, rd, ins


def _step(rd, ins, lam=0.5, gp=None):
    rd.forward(ins["params"], ins["q"], ins["score"], ins["target"], lam, 0, ins["mask"], 0, 0,
               count_evals=False)
    return rd.backward(ins["params"], ins["q"], 0, grad_params=gp)


def _snap(rd, gp):
    return dict(image=rd.image.cpu().numpy().copy(), last=rd.last.cpu().numpy().copy(),
                gp=gp.cpu().numpy().copy(), gq=rd.grad_q.cpu().numpy().copy(),
                loss=float(rd.loss.item()))


def _grads_close(a, b, tol=1e-5):
    for k in ("gp", "gq"):
        d = np.linalg.norm(a[k] - b[k]) / max(np.linalg.norm(b[k]), 1e-30)
        assert d <= tol, (k, d)


@pytest.mark.parametrize("name", ["tiny", "c1"])
def test_fixed_capacity_matches_default_mode(dev, name):
    sc = synth.make_scene("c1") if name == "c1" else synth.make_tiny(200, 96, 80, seed=4)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        ctx, rd, ins = _setup(dev, sc, stream)
        gp = torch.empty_like(ins["params"])
        _step(rd, ins, gp=gp)
        stream.synchronize()
        ref = _snap(rd, gp)
        P, _ = ctx.query()
        ctx.reserve_pairs(P + 100)
        _step(rd, ins, gp=gp)
        P2, _ = ctx.query()
        got = _snap(rd, gp)
    assert P2 == P
    assert np.array_equal(got["image"], ref["image"]) and np.array_equal(got["last"], ref["last"])
    _grads_close(got, ref)


def test_capacity_overflow_is_reported(dev):
    from paper_2607_12656_amd import SgsError
    sc = synth.make_tiny(200, 96, 80, seed=4)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        ctx, rd, ins = _setup(dev, sc, stream)
        gp = torch.empty_like(ins["params"])
        _step(rd, ins, gp=gp)
        P, _ = ctx.query()
        ref = _snap(rd, gp)
        ctx.reserve_pairs(P // 2)
        _step(rd, ins, gp=gp)
        with pytest.raises(SgsError) as e:
            ctx.query()
        assert e.value.status == -5
        ctx.reserve_pairs(P)
        _step(rd, ins, gp=gp)
        ctx.query()
        got = _snap(rd, gp)
    assert np.array_equal(got["image"], ref["image"])


@pytest.mark.parametrize("fused", [False, True])
@pytest.mark.parametrize("tile", [(16, 16), (8, 8)])
def test_graph_replays_match_eager(dev, tile, fused):
    sc = synth.make_scene("c1")
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        ctx, rd, ins = _setup(dev, sc, stream, tile=tile)
        rd.fused = fused
        gp = torch.empty_like(ins["params"])
        _step(rd, ins, gp=gp)
        P, _ = ctx.query()
        ctx.reserve_pairs(P + P // 4)
        _step(rd, ins, gp=gp)
        stream.synchronize()
        ref = _snap(rd, gp)
        ctx.graph_begin()
        _step(rd, ins, gp=gp)
        g = ctx.graph_end()
        for rep in range(3):
            # eager work of the program between replays
            rd.image.zero_()
            gp.fill_(123.0)
            junk = torch.randn(1 << 16, device=dev).sum()
            stream.synchronize()
            g.launch(stream)
            stream.synchronize()
            got = _snap(rd, gp)
            assert np.array_equal(got["image"], ref["image"]), rep
            assert np.array_equal(got["last"], ref["last"]), rep
            assert got["loss"] == ref["loss"]
            _grads_close(got, ref)
            del junk
        ctx.query()
        g.close()
