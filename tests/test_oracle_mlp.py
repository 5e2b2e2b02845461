"""Pins for the oracle of the learned rate estimator (CPU only)."""
import math

import numpy as np
import pytest

import synth
from synth import NCH


@pytest.fixture(scope="module")
def mlp(orc):
    from oracle import mlp
    return mlp


def test_bf16_round_to_nearest_even(mlp):
    """Textbook BF16 values (8 significant bits, ties to even)."""
    assert mlp.bf16(1.0) == 1.0
    assert mlp.bf16(1 + 2 ** -8) == 1.0                      # tie -> even
    assert mlp.bf16(1 + 3 * 2 ** -8) == 1 + 2 ** -6          # tie -> even (up)
    assert mlp.bf16(1 + 2 ** -7 + 2 ** -9) == 1 + 2 ** -7    # below half
    assert mlp.bf16(1 / 3) == 0.333984375
    assert mlp.bf16(-1 / 3) == -0.333984375
    assert mlp.bf16(3.0) == 3.0
    assert mlp.bf16(0.0) == 0.0


def _toy(seed, B=40):
    rng = np.random.default_rng(seed)
    X = np.zeros((B, 64))
    X[:, :59] = rng.uniform(0, 4, size=(B, 59))
    return X


def test_mlp_gradients_match_finite_differences(mlp):
    w = mlp.init_weights(3)
    for k in ("b1", "b2"):
        w[k] = np.random.default_rng(4).normal(0, 0.1, size=w[k].shape).astype(np.float32)
    X = _toy(5)
    c = np.random.default_rng(6).normal(size=X.shape[0])
    g, dX = mlp.backward(X, w, c, mirror=False, want_dx=True)
    loss = lambda ww, XX: float((mlp.forward(XX, ww, mirror=False) * c).sum())
    rng = np.random.default_rng(7)
    worst = 0.0
    for name, shape in mlp.WEIGHT_SHAPES:
        flat = w[name].reshape(-1)
        for idx in rng.choice(flat.size, size=min(12, flat.size), replace=False):
            h = 1e-3
            # weights are float32 inputs: perturb in float64 through a copy
            wp = {k: v.astype(np.float64) for k, v in w.items()}
            base = wp[name].reshape(-1)[idx]

            def ev(d):
                ww = {k: v.copy() for k, v in wp.items()}
                ww[name].reshape(-1)[idx] = base + d
                return loss({k: v.astype(np.float32) for k, v in ww.items()}, X)
            # float32 storage limits h; use exactly representable steps
            fd = (ev(h) - ev(-h)) / (2 * h)
            an = g[name].reshape(-1)[idx]
            worst = max(worst, abs(fd - an) / (abs(an) + 1e-3 * np.abs(g[name]).max() + 1e-12))
    assert worst < 2e-3, worst   # FD through float32-rounded weights
    # input gradient in full FP64
    for r, j in [(0, 0), (3, 17), (7, 58), (11, 30)]:
        h = 1e-6
        Xp, Xm = X.copy(), X.copy()
        Xp[r, j] += h
        Xm[r, j] -= h
        fd = (loss(w, Xp) - loss(w, Xm)) / (2 * h)
        assert fd == pytest.approx(dX[r, j], rel=1e-6, abs=1e-9)


def test_mlp_weight_gradients_fp64_exact_fd(mlp):
    """Finite differences in FP64 on weights that are exact binary fractions."""
    rng = np.random.default_rng(11)
    w = {name: (np.round(rng.normal(0, 0.3, size=shape) * 64) / 64).astype(np.float32)
         for name, shape in mlp.WEIGHT_SHAPES}
    X = _toy(12, B=16)
    c = rng.normal(size=16)
    g, _ = mlp.backward(X, w, c, mirror=False)
    f0 = lambda ww: float((mlp.forward(X, ww, mirror=False) * c).sum())
    for name in ("W1", "W2", "w3", "b1", "b3"):
        flat = w[name].reshape(-1)
        for idx in rng.choice(flat.size, size=min(6, flat.size), replace=False):
            h = 2.0 ** -12   # exact in float32 around these magnitudes
            wp = {k: v.copy() for k, v in w.items()}
            wm = {k: v.copy() for k, v in w.items()}
            wp[name].reshape(-1)[idx] += h
            wm[name].reshape(-1)[idx] -= h
            fd = (f0(wp) - f0(wm)) / (2 * h)
            assert fd == pytest.approx(g[name].reshape(-1)[idx], rel=1e-5, abs=1e-7)


def test_adam_first_step_closed_form(mlp):
    """From zero moments the bias-corrected first step is lr * g / (|g| + eps)."""
    g = np.array([0.5, -2.0, 1e-3, 0.0])
    w = np.array([1.0, 1.0, 1.0, 1.0])
    m = np.zeros(4)
    v = np.zeros(4)
    mlp.adam(w, m, v, g, 0.01, 1)
    assert np.allclose(w, 1.0 - 0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=1e-15)


def test_training_reduces_loss(mlp):
    """A few hundred Adam steps fit a smooth target of the features."""
    rng = np.random.default_rng(21)
    X = np.zeros((512, 64))
    X[:, :59] = rng.uniform(0, 3, size=(512, 59))
    t = X[:, :59].sum(1) * 0.1 + 2.0
    w = mlp.init_weights(1)
    flat = {k: v.astype(np.float64) for k, v in w.items()}
    mom = {k: np.zeros_like(v) for k, v in flat.items()}
    vel = {k: np.zeros_like(v) for k, v in flat.items()}
    losses = []
    for step in range(1, 201):
        ww = {k: v.astype(np.float32) for k, v in flat.items()}
        f = mlp.forward(X, ww, mirror=False)
        losses.append(float(((f - t) ** 2).mean()))
        g, _ = mlp.backward(X, ww, mlp.mse_grad_weights(f, t), mirror=False)
        for k in flat:
            mlp.adam(flat[k].reshape(-1), mom[k].reshape(-1), vel[k].reshape(-1),
                     g[k].reshape(-1), 3e-3, step)
    assert losses[-1] < 0.05 * losses[0]


def test_coder_targets_and_learned_rate_gradient(orc, mlp):
    sc = synth.make_tiny(300, 32, 32, seed=3)
    q = synth.learnable_qsteps(4)
    bits, per = mlp.coder_targets(sc.params, q, sc.given_mask, sc.n)
    _, k = orc.fakequant(sc.params, q, sc.n)
    kept = sc.given_mask > 0
    K = k[:NCH, :sc.n][:, kept].max(1) - k[:NCH, :sc.n][:, kept].min(1) + 1
    wd = np.ceil(np.log2(K)).astype(int)
    assert bits == kept.sum() * wd.sum() + 59 * 72
    assert per == pytest.approx(bits / kept.sum())
    # in-loop learned rate: gradient against finite differences (no BF16)
    w = mlp.init_weights(2)
    r = mlp.learned_rate(sc.params, q, sc.given_mask, sc.n, sc.n_hat, w, mirror=False)
    mmin = mlp.channel_min(sc.params, sc.n)
    rng = np.random.default_rng(5)
    for _ in range(12):
        j = int(rng.integers(0, NCH))
        i = int(rng.integers(0, sc.n))
        if sc.params[j, i] == mmin[j]:
            continue
        h = 1e-3 * q[j]
        pp, pm = sc.params.astype(np.float64).copy(), sc.params.astype(np.float64).copy()
        pp[j, i] += h
        pm[j, i] -= h

        def R_of(p):
            u = (p[:NCH, :sc.n] - mmin[:, None].astype(np.float64)) / q[:, None].astype(np.float64)
            X = np.zeros((sc.n, 64))
            X[:, :NCH] = np.log2(1 + u).T
            f = mlp.forward(X, w, mirror=False)
            return float((sc.given_mask * f).sum() / sc.n_hat)
        fd = (R_of(pp) - R_of(pm)) / (2 * h)
        assert fd == pytest.approx(r["gy"][j, i], rel=1e-4, abs=1e-10)
    # mask gradient is f / N_hat
    assert np.allclose(r["gm"], r["f"] / sc.n_hat)


def _torch_mlp(w, bf16_points=False):
    """The estimator as a torch FP64 nn.Sequential (Linear stores W as
    (out, in): the transposes of the (in, out) weight layout).  With
    bf16_points the values the matrix cores take in BF16 (inputs, W1, W2, w3
    and the first hidden activation) are rounded by torch's own bfloat16
    conversion (round to nearest even) in between."""
    torch = pytest.importorskip("torch")
    r = (lambda t: t.to(torch.bfloat16).to(torch.float64)) if bf16_points else (lambda t: t)
    l1 = torch.nn.Linear(64, 128, dtype=torch.float64)
    l2 = torch.nn.Linear(128, 128, dtype=torch.float64)
    l3 = torch.nn.Linear(128, 1, dtype=torch.float64)
    with torch.no_grad():
        l1.weight.copy_(r(torch.from_numpy(w["W1"].astype(np.float64)).T))
        l1.bias.copy_(torch.from_numpy(w["b1"].astype(np.float64)))
        l2.weight.copy_(r(torch.from_numpy(w["W2"].astype(np.float64)).T))
        l2.bias.copy_(torch.from_numpy(w["b2"].astype(np.float64)))
        l3.weight.copy_(r(torch.from_numpy(w["w3"].astype(np.float64))[None, :]))
        l3.bias.copy_(torch.from_numpy(w["b3"].astype(np.float64)))

    class Rb(torch.nn.Module):
        def forward(self, t):
            return r(t)
    return torch.nn.Sequential(Rb(), l1, torch.nn.ReLU(), Rb(), l2, torch.nn.ReLU(), l3)


def test_mlp_forward_and_backward_match_torch_fp64(mlp):
    """The oracle MLP (mirror off) against torch's FP64 Linear / ReLU layers:
    forward, weight gradients and input gradient of sum_i c_i f(x_i)."""
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(31)
    w = mlp.init_weights(8)
    for k in ("b1", "b2", "b3"):
        w[k] = rng.normal(0, 0.2, size=w[k].shape).astype(np.float32)
    X = _toy(32, B=48)
    c = rng.normal(size=48)
    f = mlp.forward(X, w, mirror=False)
    net = _torch_mlp(w)
    Xt = torch.from_numpy(X).requires_grad_(True)
    ft = net(Xt)[:, 0]
    assert np.allclose(f, ft.detach().numpy(), rtol=1e-13, atol=1e-13)
    (ft * torch.from_numpy(c)).sum().backward()
    g, dX = mlp.backward(X, w, c, mirror=False, want_dx=True)
    l1, l2, l3 = net[1], net[4], net[6]
    pairs = (("W1", l1.weight.grad.T), ("b1", l1.bias.grad), ("W2", l2.weight.grad.T),
             ("b2", l2.bias.grad), ("w3", l3.weight.grad[0]), ("b3", l3.bias.grad))
    for name, ref in pairs:
        ref = ref.numpy().reshape(g[name].shape)
        assert np.allclose(g[name], ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max()), name
    assert np.allclose(dX, Xt.grad.numpy(), rtol=1e-12, atol=1e-13)


def test_mlp_bf16_mirror_points_match_torch(mlp):
    """With mirroring on, the oracle forward on BF16 features equals the FP64
    network whose W1, W2, w3 and first hidden activation are rounded to BF16
    (the values the matrix cores read), and nothing else."""
    torch = pytest.importorskip("torch")
    w = mlp.init_weights(9)
    # the features arrive in BF16 (the feature pass rounds them)
    X = torch.from_numpy(_toy(33, B=40)).to(torch.bfloat16).to(torch.float64).numpy()
    f = mlp.forward(X, w, mirror=True)
    ft = _torch_mlp(w, bf16_points=True)(torch.from_numpy(X))[:, 0].detach().numpy()
    assert np.allclose(f, ft, rtol=1e-13, atol=1e-13)
    # and it is not the unrounded network
    assert not np.allclose(f, mlp.forward(X, w, mirror=False), rtol=1e-6)


def test_mlp_bf16_mirror_backward_points_match_torch(mlp):
    """With mirroring on, the oracle backward of sum_i c_i f(x_i) equals torch
    autograd through the BF16-rounded network with the gradients at the two
    backward matrix-core inputs rounded to BF16: dz2 = c w3 [z2 > 0] (the
    row weight c enters before the rounding) and dz1 = (W2 dz2) [z1 > 0]."""
    torch = pytest.importorskip("torch")
    rb = lambda t: t.to(torch.bfloat16).to(torch.float64)
    rng = np.random.default_rng(41)
    w = mlp.init_weights(10)
    for k in ("b1", "b2"):
        w[k] = rng.normal(0, 0.1, size=w[k].shape).astype(np.float32)
    X = torch.from_numpy(_toy(34, B=24)).to(torch.bfloat16).to(torch.float64)
    c = rng.normal(size=24)
    leaf = lambda a: rb(torch.from_numpy(a.astype(np.float64))).requires_grad_(True)
    W1, W2, w3 = leaf(w["W1"]), leaf(w["W2"]), leaf(w["w3"])
    b1 = torch.from_numpy(w["b1"].astype(np.float64)).requires_grad_(True)
    b2 = torch.from_numpy(w["b2"].astype(np.float64)).requires_grad_(True)
    b3 = torch.from_numpy(w["b3"].astype(np.float64)).requires_grad_(True)
    Xl = X.clone().requires_grad_(True)
    z1 = Xl @ W1 + b1
    h1 = rb(torch.relu(z1))             # its gradient passes through the cast: rounded
    z2 = h1 @ W2 + b2
    z2.register_hook(lambda g: rb(g))   # dz2 rounded before the second GEMM
    f = torch.relu(z2) @ w3 + b3
    (f * torch.from_numpy(c)).sum().backward()
    g, dX = mlp.backward(X.numpy(), w, c, mirror=True, want_dx=True)
    for name, ref in (("W1", W1.grad), ("b1", b1.grad), ("W2", W2.grad), ("b2", b2.grad),
                      ("w3", w3.grad), ("b3", b3.grad)):
        ref = ref.numpy().reshape(g[name].shape)
        assert np.allclose(g[name], ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max()), name
    assert np.allclose(dX, Xl.grad.numpy(), rtol=1e-12, atol=1e-13)
