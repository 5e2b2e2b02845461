"""GPU Adam step (sgs_adam_step) against the FP64 oracle on the same FP32
state: every updated entry within an a-priori bound on FP32 rounding,
derived from the reference's own terms; every skipped entry (SH rows off,
sparse Gaussians, padding columns) bit-identical."""
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
U = 2.0 ** -24
B1, B2, EPS = np.float32(0.9), np.float32(0.999), np.float32(1e-8)


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


def state(rng, shape, zero_cols=None):
    x = rng.normal(0, 1, shape).astype(np.float32)
    m = rng.normal(0, 0.1, shape).astype(np.float32)
    v = (m.astype(np.float64) ** 2 + rng.uniform(0, 0.01, shape)).astype(np.float32)
    scale = 10.0 ** rng.integers(-4, 2, shape[:-1] + (1,)) if len(shape) == 2 else 1.0
    g = (rng.normal(0, 1, shape) * scale).astype(np.float32)
    g[rng.random(shape) < 0.02] = 0.0
    if zero_cols is not None:
        g[..., zero_cols] = 0.0
    return x, m, v, g


def bounds(x, m, v, g, lr, t):
    """FP64 reference and a bound on |FP32 evaluation - reference| per entry:
    the moment sums carry 3u of their terms; bias corrections, square root,
    eps sum, product and quotient add about 9u of the update, the final
    subtraction u of the result (u = 2^-24); doubled for safety."""
    x64, m64, v64, g64 = (a.astype(np.float64) for a in (x, m, v, g))
    lr = np.asarray(lr, np.float64)
    b1, b2 = float(B1), float(B2)
    bc1, bc2 = 1.0 - b1 ** t, 1.0 - b2 ** t
    m1 = b1 * m64 + (1 - b1) * g64
    v1 = b2 * v64 + (1 - b2) * g64 * g64
    den = np.sqrt(v1 / bc2) + float(EPS)
    upd = lr * (m1 / bc1) / den
    x1 = x64 - upd
    em = 3 * U * (b1 * np.abs(m64) + (1 - b1) * np.abs(g64))
    ev = 3 * U * (b2 * v64 + (1 - b2) * g64 * g64)
    ex = lr * (em / bc1) / den + 9 * U * np.abs(upd) + U * np.abs(x1)
    return (x1, m1, v1), (2 * ex, 2 * em, 2 * ev)


def check(name, got, ref, bound, where):
    for a, r, b, lab in zip(got, ref, bound, ("x", "m", "v")):
        d = np.abs(a[where].astype(np.float64) - r[where])
        bad = d > b[where]
        assert not bad.any(), (f"{name} {lab}: {bad.sum()} entries over the bound, worst "
                               f"{(d / np.maximum(b[where], 1e-300)).max():.2f}x")


def run_case(gctx, dev, sc, rng, t, sh_rest, sparse, with_q=True, with_s=True):
    n, npad = sc.n, sc.npad
    gctx.set_scene(sc.n, sc.npad, sc.n_hat, sc.cams, sc.width, sc.height)
    dead = rng.random(n) < 0.15
    x, m, v, g = state(rng, (59, npad), zero_cols=np.flatnonzero(dead))
    lr = rng.uniform(1e-4, 1e-2, 59).astype(np.float32)
    q, qm, qv, gq = state(rng, (59,))
    s, sm, sv, gs = state(rng, (n,))
    bufs = [T(a, dev) for a in (x, m, v, g, q, qm, qv, gq, s, sm, sv, gs)]
    gctx.adam_step([float(a) for a in lr], t, *bufs[:4],
                   *(bufs[4:8] if with_q else [None] * 4), *(bufs[8:12] if with_s else [None] * 4),
                   lr_q=2e-3, lr_score=5e-2, beta1=float(B1), beta2=float(B2), eps=float(EPS),
                   sh_rest=sh_rest, sparse=sparse)
    torch.cuda.synchronize()
    out = [b.cpu().numpy() for b in bufs]
    # parameters
    rows = np.ones(59, bool)
    if not sh_rest:
        rows[6:51] = False
    skip_col = np.zeros(npad, bool)
    skip_col[n:] = True
    if sparse:
        skip_col[:n] |= ~np.any(g[rows, :n] != 0, axis=0)
    upd = rows[:, None] & ~skip_col[None, :]
    ref, bnd = bounds(x, m, v, g, lr[:, None], t)
    check(f"params t={t} sh_rest={sh_rest} sparse={sparse}", out[:3], ref, bnd, upd)
    for a, b in zip(out[:3], (x, m, v)):
        assert np.array_equal(a[~upd], b[~upd]), "skipped parameter entries changed"
    if with_q:
        ref, bnd = bounds(q, qm, qv, gq, 2e-3, t)
        check("steps", out[4:7], ref, bnd, np.ones(59, bool))
    else:
        assert np.array_equal(out[4], q)
    if with_s:
        ref, bnd = bounds(s, sm, sv, gs, 5e-2, t)
        check("scores", out[8:11], ref, bnd, np.ones(n, bool))
    else:
        assert np.array_equal(out[8], s)
    assert np.array_equal(out[3], g) and np.array_equal(out[7], gq) and np.array_equal(out[11], gs)
    return upd.sum()


@pytest.mark.parametrize("t", [1, 7, 1000])
@pytest.mark.parametrize("sh_rest,sparse", [(1, 0), (0, 0), (1, 1), (0, 1)])
def test_adam_matches_oracle_small(gctx, dev, t, sh_rest, sparse):
    _say(f"[gpu] adam n=5000 t={t} sh_rest={sh_rest} sparse={sparse}")
    sc = synth.make_tiny(5000, 64, 48, seed=31)
    rng = np.random.default_rng(100 + t + 10 * sh_rest + 20 * sparse)
    run_case(gctx, dev, sc, rng, t, bool(sh_rest), bool(sparse))


def test_adam_optional_groups(gctx, dev):
    _say("[gpu] adam optional groups")
    sc = synth.make_tiny(777, 64, 48, seed=32)
    rng = np.random.default_rng(7)
    run_case(gctx, dev, sc, rng, 3, True, True, with_q=False, with_s=False)
    run_case(gctx, dev, sc, rng, 4, False, False, with_q=True, with_s=False)


def test_adam_full_size_1m(gctx, dev):
    _say("[gpu] adam 1M")
    sc = synth.make_scene("c2")
    rng = np.random.default_rng(9)
    k = run_case(gctx, dev, sc, rng, 25, False, True)
    assert k > 0


def test_adam_option_checks(gctx, dev):
    from paper_2607_12656_amd._lib import SgsError
    sc = synth.make_tiny(300, 64, 48, seed=33)
    gctx.set_scene(sc.n, sc.npad, sc.n_hat, sc.cams, sc.width, sc.height)
    z = torch.zeros(59, sc.npad, device=dev)
    q = torch.zeros(59, device=dev)
    with pytest.raises(SgsError):
        gctx.adam_step(1e-3, 0, z, z.clone(), z.clone(), z.clone())          # step 0
    with pytest.raises(SgsError):
        gctx.adam_step(1e-3, 1, z, z.clone(), z.clone(), z.clone(), beta1=1.0)
    with pytest.raises(SgsError):
        gctx.adam_step(1e-3, 1, z, z.clone(), z.clone(), z.clone(), q, q.clone())  # partial group
