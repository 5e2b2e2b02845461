"""The formation iteration on the GPU (RD step on the Gumbel-sigmoid mask,
Adam) and pruning by the learned mask: the compacted parameters, moments and
scores equal the oracle's compaction bit for bit, and rendering the
survivors with every Gaussian kept gives the image the masked scene gave
(masked splats change nothing, and compaction keeps the index order that
breaks depth ties), bit for bit."""
import sys

import numpy as np
import pytest

import oracle
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


def render(f, mode):
    c, rd = f.ctx, f.rd
    c.fakequant_prune(f.params, f.q, f.score, mode, None, f.seed, f.k, rd.qparams, rd.hard,
                      rd.soft, rd.stats)
    c.render_fwd(rd.qparams, rd.hard, rd.image, rd.final_T, rd.last, None)
    torch.cuda.synchronize()
    return rd.image.cpu().numpy().copy(), rd.hard.cpu().numpy().copy()


@pytest.mark.parametrize("views", [1, 2])
def test_iterate_then_prune(gctx, dev, views):
    from paper_2607_12656_amd.formation import Formation
    from paper_2607_12656_amd.rd import RDStep
    _say(f"[gpu] formation + prune, views={views}")
    sc = synth.make_tiny(6000, 64, 48, views=views, seed=51)
    rd = RDStep(gctx, sc.n, sc.npad, sc.n_hat, sc.cams, sc.width, sc.height)
    p, q, s = T(sc.params, dev), T(sc.qstep, dev), T(sc.score, dev)
    f = Formation(rd, p, q, s, T(sc.target, dev), 2.5e-5, mask_mode=1, seed=9)
    p_init = sc.params.copy()
    for _ in range(6):
        f.iterate()
    torch.cuda.synchronize()
    assert np.all(np.isfinite(f.params.cpu().numpy()))
    assert not np.array_equal(f.params.cpu().numpy(), p_init), "Adam moved nothing"
    img_masked, hard = render(f, 1)
    before = [a.cpu().numpy().copy() for a in (f.params, f.pm, f.pv, f.score, f.sm, f.sv)]
    kept = f.prune()
    assert kept == int((hard[:sc.n] != 0).sum()) and 0 < kept < sc.n
    after = [a.cpu().numpy() for a in (f.params, f.pm, f.pv, f.score, f.sm, f.sv)]
    for b, a in zip(before, after):
        ref = oracle.compact([b], hard, sc.n)[0]
        assert np.array_equal(a[..., :kept], ref)
    img_kept, hard2 = render(f, 2)
    assert np.all(hard2[:kept] == 1)
    assert np.array_equal(img_kept, img_masked), \
        f"max |diff| {np.abs(img_kept - img_masked).max()}"
    for _ in range(3):
        f.iterate()
    torch.cuda.synchronize()
    assert np.all(np.isfinite(f.params.cpu().numpy()[:, :kept]))


def test_learned_rate_iterations_run(gctx, dev):
    from paper_2607_12656_amd.formation import Formation
    from paper_2607_12656_amd.rate_train import RateTrainer
    from paper_2607_12656_amd.rd import RDStep
    _say("[gpu] formation learned")
    sc = synth.make_tiny(8000, 64, 48, seed=52)
    rd = RDStep(gctx, sc.n, sc.npad, sc.n_hat, sc.cams, sc.width, sc.height)
    p, q, s = T(sc.params, dev), T(sc.qstep, dev), T(sc.score, dev)
    tr = RateTrainer(gctx, rd, p, s, sc.given_mask, seed=1, scenes=16)
    theta, packed, losses = tr.train(steps=60, scenes_per_batch=8, rows_per_scene=1024)
    assert losses[-1] < losses[0]
    el, ep = tr.held_out_errors(theta, packed, scenes=4)
    _say(f"held-out error learned {el:.4f} plain {ep:.4f}")
    assert np.isfinite(el) and np.isfinite(ep)
    f = Formation(rd, p, q, s, T(sc.target, dev), 2.5e-5, mask_mode=1, seed=3,
                  mlp=(packed, theta))
    for _ in range(4):
        f.iterate()
    torch.cuda.synchronize()
    assert np.isfinite(float(f.R_learned.item())) and float(f.R_learned.item()) > 0
    assert np.all(np.isfinite(f.params.cpu().numpy()[:, :sc.n]))


def test_learned_rate_fallback_rule(orc, gctx, dev):
    """The learned estimate drives the iteration while its error against the
    exact coder bits is not larger than the plain proxy's, and the plain
    proxy's gradient drives it after a check that finds it larger.  Two
    estimators with zero weights and a constant output: f = B / kept (exact:
    N_hat R_learned = B) and f = 3 B / kept (error 2)."""
    from oracle import mlp as omlp
    from paper_2607_12656_amd._lib import MLP_PACKED_BYTES, MLP_PARAMS
    from paper_2607_12656_amd.formation import Formation
    from paper_2607_12656_amd.rd import RDStep
    sc = synth.make_tiny(3000, 48, 40, seed=52)
    bits, per = omlp.coder_targets(sc.params, sc.qstep, sc.given_mask, sc.n)
    lam = 0.5
    grads = {}
    for name, b3 in (("exact", per), ("bad", 3.0 * per), ("plain", None)):
        rd = RDStep(gctx, sc.n, sc.npad, sc.n_hat, sc.cams, sc.width, sc.height)
        mlp = None
        if b3 is not None:
            theta = torch.zeros(MLP_PARAMS, dtype=torch.float32, device=dev)
            theta[-1] = b3
            packed = torch.empty(MLP_PACKED_BYTES // 4, dtype=torch.int32, device=dev)
            gctx.rate_mlp_pack(theta, packed)
            mlp = (packed, theta)
        f = Formation(rd, T(sc.params, dev), T(sc.qstep, dev), T(sc.score, dev),
                      T(sc.target, dev), lam, mask_mode=0, given_mask=T(sc.given_mask, dev),
                      mlp=mlp, check_every=4)
        B, kept, e_plain, e_learn = f.rate_errors()
        assert B == bits and kept == int(sc.given_mask.sum())
        f.iterate()                     # k = 0: the check runs first
        torch.cuda.synchronize()
        grads[name] = rd.grad_q.cpu().numpy().copy()
        if name == "exact":
            assert e_learn <= 1e-6 and f.use_learned
        elif name == "bad":
            assert abs(e_learn - 2.0) <= 1e-6 and not f.use_learned
            assert f.checks[-1][3] is False
        _say(f"{name}: plain error {e_plain:.4f}, learned {e_learn}")
    # fallen back: the step-size gradient is the plain iteration's (up to the
    # order of the render gradient's atomic sums); with the exact estimator
    # (zero weights: no rate gradient to q) it is not
    scale = np.abs(grads["plain"]).max()
    assert np.abs(grads["bad"] - grads["plain"]).max() <= 1e-5 * scale
    assert np.abs(grads["exact"] - grads["plain"]).max() > 1e-2 * scale
