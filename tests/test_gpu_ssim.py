"""GPU SSIM term (sgs_ssim_loss) against the FP64 oracle: the loss, and the
gradient it adds to dL/dimage (FP64 inside, one rounding to FP32 when added),
on ragged tile edges, two views and the 1297x840 image; identity and the
optional gradient output."""
import sys

import numpy as np
import pytest

import synth
from oracle import ssim as S

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


def run(gctx, dev, V, W, H, seed, weight=0.2, same=False):
    sc = synth.make_tiny(500, W, H, views=V, seed=seed)
    gctx.set_scene(sc.n, sc.npad, sc.n_hat, sc.cams, sc.width, sc.height)
    rng = np.random.default_rng(seed)
    x = rng.random((V, 3, H, W)).astype(np.float32)
    # a smooth part, so flat regions (where the gradient terms cancel) occur
    x[..., : H // 2, :] = 0.25 + 0.01 * x[..., : H // 2, :]
    y = x.copy() if same else rng.random((V, 3, H, W)).astype(np.float32)
    d0 = (rng.normal(0, 1e-7, x.shape)).astype(np.float32)
    dimg = T(d0, dev)
    loss = torch.empty(1, dtype=torch.float32, device=dev)
    gctx.ssim_loss(T(x, dev), T(y, dev), weight, loss, dimg)
    torch.cuda.synchronize()
    # the library receives the weight as a float32
    lref, gref = S.dssim_loss(x.astype(np.float64), y.astype(np.float64),
                              float(np.float32(weight)))
    lg = float(loss.item())
    assert abs(lg - lref) <= 1e-6 * max(abs(lref), 1e-6), (lg, lref)
    got = dimg.cpu().numpy().astype(np.float64)
    ref = d0.astype(np.float64) + gref
    bound = 0.5 * np.spacing(np.abs(ref).astype(np.float32)).astype(np.float64) * 1.01 \
        + 1e-9 * max(np.abs(gref).max(), 1e-30)
    bad = np.abs(got - ref) > bound
    assert not bad.any(), f"{bad.sum()} gradient entries off, worst {np.abs(got - ref).max():.3e}"
    return lg, gref


@pytest.mark.parametrize("V,W,H", [(1, 70, 37), (2, 64, 48), (1, 33, 17)])
def test_ssim_small(gctx, dev, V, W, H):
    _say(f"[gpu] ssim V={V} {W}x{H}")
    run(gctx, dev, V, W, H, seed=V * 100 + W)


def test_ssim_identity_and_options(gctx, dev):
    _say("[gpu] ssim identity")
    lg, g = run(gctx, dev, 1, 40, 30, seed=3, same=True)
    assert abs(lg) < 1e-6 and np.abs(g).max() < 1e-12
    run(gctx, dev, 1, 40, 30, seed=4, weight=0.0)
    sc = synth.make_tiny(500, 40, 30, seed=5)
    gctx.set_scene(sc.n, sc.npad, sc.n_hat, sc.cams, sc.width, sc.height)
    x = torch.rand(1, 3, 30, 40, device=dev)
    loss = torch.empty(1, dtype=torch.float32, device=dev)
    gctx.ssim_loss(x, x.flip(-1).contiguous(), 0.2, loss, None)     # loss only
    torch.cuda.synchronize()
    xs = x.cpu().numpy().astype(np.float64)
    assert abs(float(loss.item()) - 0.2 * (1 - S.ssim(xs, xs[..., ::-1]))) < 1e-6


def test_ssim_1297x840(gctx, dev):
    _say("[gpu] ssim 1297x840")
    run(gctx, dev, 1, 1297, 840, seed=11)
