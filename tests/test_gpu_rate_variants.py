"""GPU rate-proxy variants (sgs_rate_variant / _bwd) against the FP64 oracle:
the loss term, L_quant, L_mask, the compact gradient the quantizer backward
consumes, the Laplace proxy's dense y gradient, and the whole rate gradient
after sgs_fakequant_prune_bwd (no render gradient), at a ragged size and at
1M Gaussians."""
import sys

import numpy as np
import pytest

import oracle
import synth
from oracle import rate_variants as RV

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


def rel(a, b, tol, what):
    assert abs(a - b) <= tol * max(abs(b), 1e-30), f"{what}: {a} vs {b}"


def run(gctx, dev, sc, q, proxy, masking, lam=0.7, alpha=0.013):
    from paper_2607_12656_amd.rd import RDStep
    rd = RDStep(gctx, sc.n, sc.npad, sc.n_hat, sc.cams, sc.width, sc.height)
    params, qd, mask = T(sc.params, dev), T(q, dev), T(sc.given_mask, dev)
    gctx.fakequant_prune(params, qd, None, 0, mask, 0, 0, rd.qparams, rd.hard, rd.soft, rd.stats)
    out3 = torch.empty(3, dtype=torch.float32, device=dev)
    rg = torch.full((256,), 7.0, dtype=torch.float32, device=dev)
    gctx.rate_variant(params, qd, rd.stats, lam, out3, rg, proxy, masking, alpha)
    # the whole rate gradient: quantizer backward with a zero render gradient
    zero_g = torch.zeros_like(params)
    zero_m = torch.zeros(sc.n, dtype=torch.float32, device=dev)
    gp = torch.empty_like(params)
    gq = torch.empty(59, dtype=torch.float32, device=dev)
    gs = torch.empty(sc.n, dtype=torch.float32, device=dev)
    gctx.fakequant_prune_bwd(params, qd, rd.soft, 0, rg, rd.stats, zero_g, zero_m, gp, gq, gs)
    gctx.rate_variant_bwd(params, gp)
    torch.cuda.synchronize()
    ref = RV.rate_variant(sc.params, q, sc.given_mask, sc.n, sc.n_hat, lam, proxy, masking, alpha)
    o = out3.cpu().numpy()
    rel(o[0], ref["term"], 1e-5, "loss term")
    rel(o[1], ref["Lq"], 1e-5, "L_quant")
    rel(o[2], ref["Lm"], 1e-6, "L_mask")
    r = rg.cpu().numpy()
    assert np.allclose(r[128:187], ref["gq"], rtol=1e-5, atol=1e-12), "compact q terms"
    rel(r[192], ref["gm"], 1e-5, "mask term")
    got = gp.cpu().numpy()[:, :sc.n].astype(np.float64)
    want = ref["gy"][:, :sc.n]
    scale = np.abs(want).max()
    assert np.all(np.abs(got - want) <= 1e-5 * np.abs(want) + 1e-6 * scale), \
        f"y gradient: worst {np.abs(got - want).max():.3e} of {scale:.3e}"
    # the step gradient = the rate's (the LSQ term is zero with a zero render gradient)
    assert np.allclose(gq.cpu().numpy(), ref["gq"], rtol=1e-5, atol=1e-12), "grad q"
    return o


@pytest.mark.parametrize("proxy,masking", [("range", "add"), ("laplace", "mult"),
                                           ("laplace", "add"), ("range", "mult")])
def test_rate_variants_small(gctx, dev, proxy, masking):
    _say(f"[gpu] rate variant {proxy} {masking}")
    sc = synth.make_tiny(9000, 32, 32, seed=61)
    q = synth.learnable_qsteps(62)
    q[5] = 50.0                        # a channel below one Laplace code bit (clamped)
    run(gctx, dev, sc, q, proxy, masking)


def test_laplace_full_size_1m(gctx, dev):
    _say("[gpu] laplace 1M")
    sc = synth.make_scene("c2")
    o = run(gctx, dev, sc, sc.qstep, "laplace", "mult", lam=2.5e-5)
    _say(f"laplace proxy at 1M: L_quant {o[1]:.3f} bits, L_mask {o[2]:.3f}")
