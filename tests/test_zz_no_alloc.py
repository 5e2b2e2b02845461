"""The allocation-free training step of the learned rate estimator
(sgs_rate_mlp_train_step_static, workspace in a static device array) against
the workspace-argument entry point (sgs_rate_mlp_train_step), through the C
ABI: loss, weight gradient, and the Adam-updated weights, moments and packed
BF16 fragments bit for bit, on two calls in a row (the second with fewer
rows), plus the host-side rejection of a batch beyond the static workspace.
"""
import sys

import numpy as np
import pytest

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


def _batch(rows, seed, dev):
    g = torch.Generator(device="cpu").manual_seed(seed)
    # BF16 features in [0, 8): sign bit clear, exponents of small values
    x = (torch.rand(rows, 64, generator=g) * 8.0).to(torch.bfloat16)
    x[:, 59:] = 0
    t = torch.rand(rows, generator=g) * 100.0 + 200.0
    return x.view(torch.int16).to(dev), t.to(dev)


def test_static_train_step_equals_workspace_step(dev):
    from paper_2607_12656_amd import Context
    from paper_2607_12656_amd._lib import MLP_PACKED_BYTES, MLP_PARAMS, MLP_STATIC_ROWS

    ctx = Context(0)
    g = torch.Generator(device="cpu").manual_seed(11)
    theta0 = ((torch.rand(MLP_PARAMS, generator=g) * 2 - 1) * 0.1).to(dev)

    def state():
        th = theta0.clone()
        m = torch.zeros_like(th)
        v = torch.zeros_like(th)
        packed = torch.empty(MLP_PACKED_BYTES // 4, dtype=torch.int32, device=dev)
        ctx.rate_mlp_pack(th, packed)
        return dict(theta=th, m=m, v=v, packed=packed, loss=torch.empty(1, device=dev),
                    grad=torch.empty_like(th))

    ref, got = state(), state()
    for call, rows in enumerate((MLP_STATIC_ROWS, 1000)):
        _say(f"[gpu] no-alloc train step call {call + 1}: rows={rows}")
        X, tgt = _batch(rows, 100 + call, dev)
        ws = torch.empty(ctx.rate_mlp_train_scratch_bytes(rows), dtype=torch.uint8, device=dev)
        step = call + 1
        ctx.rate_mlp_train_step(ref["theta"], ref["m"], ref["v"], ref["packed"], X, tgt, rows,
                                1e-3, step, ref["loss"], ref["grad"], ws)
        ctx.rate_mlp_train_step_static(got["theta"], got["m"], got["v"], got["packed"], X, tgt,
                                       rows, 1e-3, step, got["loss"], got["grad"])
        torch.cuda.synchronize()
        for k in ("loss", "grad", "theta", "m", "v", "packed"):
            a, b = ref[k].cpu().numpy(), got[k].cpu().numpy()
            assert np.array_equal(a.view(np.uint32), b.view(np.uint32)), \
                f"call {call + 1}: {k} differs"
        assert np.isfinite(got["loss"].cpu().numpy()).all()
        del ws
    _say(f"no-alloc train step: loss {float(got['loss'][0]):.4f}, two calls bit-identical")

    # a batch beyond the static workspace is refused on the host
    from paper_2607_12656_amd import SgsError
    X, tgt = _batch(8, 5, dev)
    with pytest.raises(SgsError) as ei:
        ctx.rate_mlp_train_step_static(got["theta"], got["m"], got["v"], got["packed"], X, tgt,
                                       MLP_STATIC_ROWS + 8, 1e-3, 3, got["loss"], got["grad"])
    assert "ECAPACITY" in str(ei.value)
    ctx.close()
