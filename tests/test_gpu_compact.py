"""GPU pruning by the learned mask (sgs_compact) against the oracle's
compaction, bit-exact: several arrays at once, ragged chunks, nothing / all /
the first and last kept, nonzero mask values other than 1, columns past the
kept count untouched, and the capacity check (nothing written)."""
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
SENT = np.float32(-12345.5)


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


def run(gctx, dev, sc, mask, rng, dst_pad=None):
    gctx.set_scene(sc.n, sc.npad, sc.n_hat, sc.cams, sc.width, sc.height)
    arrays = [rng.normal(0, 1, (59, sc.npad)).astype(np.float32) for _ in range(3)]
    arrays += [rng.normal(0, 1, sc.npad).astype(np.float32) for _ in range(3)]
    kept_ref = int((mask[:sc.n] != 0).sum())
    pad = dst_pad if dst_pad is not None else max(64, -(-kept_ref // 64) * 64)
    src = [T(a, dev) for a in arrays]
    dst = [torch.full((59, pad) if a.ndim == 2 else (pad,), float(SENT), device=dev)
           for a in arrays]
    kept = gctx.compact(T(mask, dev), list(zip(src, dst)), pad)
    torch.cuda.synchronize()
    assert kept == kept_ref
    ref = oracle.compact(arrays, mask, sc.n)
    for d, r in zip(dst, ref):
        d = d.cpu().numpy()
        assert np.array_equal(d[..., :kept], r), "compacted values"
        assert np.all(d[..., kept:] == SENT), "columns past the kept count written"
    return kept


@pytest.mark.parametrize("n", [300, 4096, 2 * 4096 + 77])
def test_compact_random_masks(gctx, dev, n):
    _say(f"[gpu] compact n={n}")
    sc = synth.make_tiny(n, 32, 32, seed=40 + n % 7)
    rng = np.random.default_rng(n)
    mask = np.zeros(sc.npad, np.uint8)
    mask[:n] = (rng.random(n) < 0.7) * rng.integers(1, 256, n)
    run(gctx, dev, sc, mask, rng)


def test_compact_edge_masks(gctx, dev):
    _say("[gpu] compact edges")
    sc = synth.make_tiny(4096 + 33, 32, 32, seed=47)
    rng = np.random.default_rng(1)
    n = sc.n
    none = np.zeros(sc.npad, np.uint8)
    assert run(gctx, dev, sc, none, rng) == 0
    allk = np.zeros(sc.npad, np.uint8)
    allk[:n] = 1
    assert run(gctx, dev, sc, allk, rng) == n
    ends = np.zeros(sc.npad, np.uint8)
    ends[[0, n - 1]] = [200, 3]
    assert run(gctx, dev, sc, ends, rng) == 2


def test_compact_capacity_checked(gctx, dev):
    from paper_2607_12656_amd._lib import SgsError
    sc = synth.make_tiny(1000, 32, 32, seed=48)
    gctx.set_scene(sc.n, sc.npad, sc.n_hat, sc.cams, sc.width, sc.height)
    mask = np.zeros(sc.npad, np.uint8)
    mask[:500] = 1
    src = torch.zeros(59, sc.npad, device=dev)
    dst = torch.full((59, 256), float(SENT), device=dev)
    with pytest.raises(SgsError):
        gctx.compact(T(mask, dev), [(src, dst)], 256)
    torch.cuda.synchronize()
    assert torch.all(dst == float(SENT)).item(), "nothing written on a capacity error"
    with pytest.raises(SgsError):
        gctx.compact(T(mask, dev), [(src, src)], sc.npad)       # overlapping buffers


def test_compact_full_size_1m(gctx, dev):
    _say("[gpu] compact 1M")
    sc = synth.make_scene("c2")
    rng = np.random.default_rng(5)
    run(gctx, dev, sc, sc.given_mask, rng)
