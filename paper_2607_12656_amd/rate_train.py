"""Training of the learned rate estimator on the GPU against the exact bits
of the channel-wise fixed-length coder (paper Sec. 3.4.1), for one scene.

A training "scene" is the given parameters and retention mask with its own
per-channel steps q_j = 2^U[-9,-3]; its target is the coder's bits per kept
Gaussian (payload + 59 x 72 header bits, over the kept count), the same for
each of its kept Gaussians.  A batch takes ``rows_per_scene`` random kept
Gaussians from each of ``scenes_per_batch`` scenes; their feature rows come
from ``sgs_rate_mlp_features``, the step from ``sgs_rate_mlp_train_step``
(MSE, Adam).  Every arithmetic step runs in the library's kernels; the host
draws the random numbers and moves indices and targets.
"""
from __future__ import annotations

import numpy as np

from ._lib import MLP_PACKED_BYTES, MLP_PARAMS, NCH, STATS_WORDS

# theta layout: W1 [64][128], b1 [128], W2 [128][128], b2 [128], w3 [128], b3 [1]
_SHAPES = (("W1", (64, 128)), ("b1", (128,)), ("W2", (128, 128)), ("b2", (128,)),
           ("w3", (128,)), ("b3", (1,)))


def he_uniform(seed: int, b3: float = 0.0) -> np.ndarray:
    """He-uniform weights (bound sqrt(6 / fan_in)), zero hidden biases, output
    bias b3; float32 [24961]."""
    rng = np.random.default_rng(seed)
    parts = []
    for name, shape in _SHAPES:
        if name == "b3":
            parts.append(np.full(shape, b3, np.float32))
        elif name.startswith("b"):
            parts.append(np.zeros(shape, np.float32))
        else:
            lim = np.sqrt(6.0 / shape[0])
            parts.append(rng.uniform(-lim, lim, shape).astype(np.float32))
    theta = np.concatenate([p.ravel() for p in parts])
    assert theta.size == MLP_PARAMS
    return theta


def coder_bits(ctx, params, qstep, hard, payload, info, hdr) -> tuple[int, int]:
    """Exact fixed-length bits (payload + header) and kept count; synchronizes."""
    ctx.fl_encode(params, qstep, hard, hdr, payload, payload.numel(), info)
    v = info.cpu().numpy()
    if v[2] != 0:
        raise RuntimeError(f"fixed-length coder flags {int(v[2])}")
    return int(v[0]) + NCH * 72, int(v[1])


class RateTrainer:
    def __init__(self, ctx, rd, params, score, given_mask_host: np.ndarray, seed: int = 0,
                 scenes: int = 64):
        import torch
        self.torch, self.ctx, self.rd = torch, ctx, rd
        dev = rd.dev
        self.dev = dev
        n = rd.n
        self.params, self.score = params, score
        self.kept_idx = np.flatnonzero(given_mask_host[:n]).astype(np.int32)
        mask = torch.from_numpy(np.ascontiguousarray(given_mask_host[:n], np.uint8)).to(dev)
        self.mask = mask
        rng = np.random.default_rng(seed)
        self.rng = rng
        payload = torch.empty(n * NCH + 64, dtype=torch.int32, device=dev)
        info = torch.empty(3, dtype=torch.int64, device=dev)
        hdr = torch.empty((NCH, 3), dtype=torch.int32, device=dev)
        self.q, self.stats, self.target = [], [], []
        for _ in range(scenes):
            q = torch.from_numpy((2.0 ** rng.uniform(-9, -3, NCH)).astype(np.float32)).to(dev)
            stats = torch.empty(STATS_WORDS, dtype=torch.int64, device=dev)
            ctx.fakequant_prune(params, q, score, 0, mask, 0, 0, rd.qparams, rd.hard, rd.soft,
                                stats)
            bits, kept = coder_bits(ctx, params, q, rd.hard, payload, info, hdr)
            self.q.append(q)
            self.stats.append(stats)
            self.target.append(bits / kept)
        del payload

    def train(self, steps: int = 400, scenes_per_batch: int = 16, rows_per_scene: int = 4096,
              lr: float = 1e-3, seed: int = 42):
        """Returns (theta, packed, [loss at steps 1, 50, 100, ...])."""
        torch, ctx, dev = self.torch, self.ctx, self.dev
        B = scenes_per_batch * rows_per_scene
        theta = torch.from_numpy(he_uniform(seed, float(np.mean(self.target)))).to(dev)
        m, v = torch.zeros_like(theta), torch.zeros_like(theta)
        g = torch.empty_like(theta)
        packed = torch.empty(MLP_PACKED_BYTES // 4, dtype=torch.int32, device=dev)
        ctx.rate_mlp_pack(theta, packed)
        scratch = torch.empty(ctx.rate_mlp_train_scratch_bytes(B), dtype=torch.uint8,
                              device=dev)
        loss = torch.empty(1, dtype=torch.float32, device=dev)
        X = torch.empty((B, 64), dtype=torch.int16, device=dev)
        losses = []
        for step in range(1, steps + 1):
            pick = self.rng.choice(len(self.q), scenes_per_batch, replace=False)
            idx = self.rng.choice(self.kept_idx, (scenes_per_batch, rows_per_scene))
            idx_d = torch.from_numpy(np.ascontiguousarray(idx, np.int32)).to(dev)
            t = np.repeat(np.asarray([self.target[s] for s in pick], np.float32),
                          rows_per_scene)
            t_d = torch.from_numpy(t).to(dev)
            for k, s in enumerate(pick):
                r0 = k * rows_per_scene
                ctx.rate_mlp_features(self.params, self.q[s], self.stats[s], idx_d[k],
                                      rows_per_scene, X[r0:r0 + rows_per_scene])
            ctx.rate_mlp_train_step(theta, m, v, packed, X, t_d, B, lr, step, loss, g, scratch)
            if step == 1 or step % 50 == 0:
                losses.append(float(loss.item()))
        return theta, packed, losses

    def held_out_errors(self, theta, packed, scenes: int = 8, seed: int = 7):
        """Mean |estimate - bits| / bits of the learned and plain rate terms on
        fresh steps (N_hat R against the coder's exact bits)."""
        torch, ctx, rd, dev = self.torch, self.ctx, self.rd, self.dev
        rng = np.random.default_rng(seed)
        n = rd.n
        payload = torch.empty(n * NCH + 64, dtype=torch.int32, device=dev)
        info = torch.empty(3, dtype=torch.int64, device=dev)
        hdr = torch.empty((NCH, 3), dtype=torch.int32, device=dev)
        R = torch.empty(1, dtype=torch.float32, device=dev)
        mask = self.mask
        el, ep = [], []
        for _ in range(scenes):
            q = torch.from_numpy((2.0 ** rng.uniform(-9, -3, NCH)).astype(np.float32)).to(dev)
            ctx.fakequant_prune(self.params, q, self.score, 0, mask, 0, 0, rd.qparams, rd.hard,
                                rd.soft, rd.stats)
            ctx.rate_proxy(rd.stats, q, 0.0, rd.rate3)
            ctx.rate_mlp_fwd(packed, theta, self.params, q, rd.stats, rd.hard, R, None)
            bits, _ = coder_bits(ctx, self.params, q, rd.hard, payload, info, hdr)
            el.append(abs(float(R.item()) * rd.n_hat - bits) / bits)
            ep.append(abs(float(rd.rate3[0].item()) * rd.n_hat - bits) / bits)
        return float(np.mean(el)), float(np.mean(ep))
