"""The structural-formation iteration on the GPU (paper Sec. 3.3): one RD
step on the Gumbel-sigmoid (or given) mask, the plain rate proxy or the
learned estimator in the loop, L1 or (with ``ssim_weight``) vanilla 3DGS's
L1 + SSIM distortion, then one Adam step on the parameters, the
step sizes and the retention scores (Sec. 4.1 adopts an economical Adam
schedule with separated updates of the higher SH coefficients; read here as
``sh_every`` and ``sparse``).

Only library calls are issued; nothing here computes, and an iteration never
synchronizes with the host.  ``prune`` applies the learned mask (the
supplement prunes with it every 1,000 iterations of the formation stage):
the Gaussians whose current hard mask is 0 leave the scene, with their
moments, and the step is rebuilt for the survivors (one synchronization).

With the learned estimator in the loop the plain proxy is still evaluated
every iteration; ``check_rate`` (every ``check_every`` iterations when that
is set, one synchronization each) compares both estimates with the exact
bits of the channel-wise fixed-length coder (Sec. 3.4.1) and, while the
learned estimate's relative error is the larger, the plain proxy's gradient
drives the iteration instead (the proxy is the fallback and the judge).

The learning rates are vanilla 3DGS's defaults
(Kerbl et al. 2023; the paper builds on vanilla 3DGS, Sec. 4.1): mean 1.6e-4,
DC colour 2.5e-3, higher SH 2.5e-3 / 20, opacity 2.5e-2, log-scale 5e-3,
rotation 1e-3; the step sizes and scores take rates the paper does not
state (``lr_q``, ``lr_score``).
"""
from __future__ import annotations

from .rd import RDStep

LR_3DGS = ([1.6e-4] * 3 + [2.5e-3] * 3 + [2.5e-3 / 20] * 45 + [2.5e-2] + [5e-3] * 3
           + [1e-3] * 4)
assert len(LR_3DGS) == 59


class Formation:
    """Iterate the formation objective D + lam R on device tensors in place.

    params [59][npad], qstep [59], score [n] (float32, device) are updated by
    every ``iterate``; target is the image stack the L1 distortion compares
    with.  ``mlp = (packed, theta)`` puts the learned estimator in the loop
    (its forward and its backward from the saved activation signs); otherwise the plain proxy supplies
    the rate gradient: the paper's range-based multiplicative proxy, or with
    ``proxy="laplace"`` / ``masking="add"`` (weight ``alpha``) the variants its
    ablations compare."""

    def __init__(self, rd: RDStep, params, qstep, score, target, lam: float,
                 mask_mode: int = 1, given_mask=None, seed: int = 0, mlp=None,
                 lr=LR_3DGS, lr_q: float = 1e-4, lr_score: float = 1e-2,
                 sh_every: int = 16, sparse: bool = True, ssim_weight: float = 0.0,
                 proxy: str = "range", masking: str = "mult", alpha: float = 0.0,
                 check_every: int = 0):
        torch = rd.torch
        self.rd, self.ctx = rd, rd.ctx
        self.params, self.q, self.score, self.target = params, qstep, score, target
        self.lam, self.mask_mode, self.given, self.seed = lam, mask_mode, given_mask, seed
        self.mlp = mlp
        self.lr, self.lr_q, self.lr_score = list(lr), lr_q, lr_score
        self.sh_every, self.sparse, self.ssim_weight = sh_every, sparse, ssim_weight
        self.proxy, self.masking, self.alpha = proxy, masking, alpha
        self.variant = (proxy, masking) != ("range", "mult")
        z = lambda a: torch.zeros_like(a)
        self.pm, self.pv = z(params), z(params)
        self.qm, self.qv = z(qstep), z(qstep)
        self.sm, self.sv = z(score), z(score)
        self.R_learned = torch.zeros(1, dtype=torch.float32, device=rd.dev)
        self.k = 0
        self.check_every = check_every
        self.use_learned = mlp is not None
        self.checks = []               # (iteration, plain error, learned error, learned used)
        self._coder = None

    def _state_tensors(self):
        return (self.params, self.q, self.score, self.pm, self.pv, self.qm, self.qv, self.sm,
                self.sv)

    def snapshot(self):
        """Copies of the iterated tensors and the iteration count."""
        return [t.clone() for t in self._state_tensors()], self.k

    def restore(self, snap):
        """Back to a snapshot, in place (buffers keep their addresses, so
        captured graphs stay valid)."""
        tensors, k = snap
        for dst, src in zip(self._state_tensors(), tensors):
            dst.copy_(src)
        self.k = k

    def rate_errors(self):
        """Plain proxy and learned estimate (if any) of the current state
        against the exact fixed-length coder bits B: returns (B, kept,
        |N_hat R_plain - B| / B, |N_hat R_learned - B| / B or None).
        Synchronizes."""
        torch = self.rd.torch
        c, rd = self.ctx, self.rd
        p, q, s = self.params, self.q, self.score
        if self._coder is None:
            words = rd.n * 59 + 64            # 32 bits per code at most
            dev = rd.dev
            self._coder = (torch.empty((59, 3), dtype=torch.int32, device=dev),
                           torch.empty(words, dtype=torch.int32, device=dev),
                           torch.empty(3, dtype=torch.int64, device=dev))
        hdr, payload, info = self._coder
        c.fakequant_prune(p, q, s, self.mask_mode, self.given, self.seed, self.k, rd.qparams,
                          rd.hard, rd.soft, rd.stats)
        c.rate_proxy(rd.stats, q, 0.0, rd.rate3, None)
        if self.mlp is not None:
            packed, theta = self.mlp
            c.rate_mlp_fwd(packed, theta, p, q, rd.stats, rd.hard, self.R_learned, None)
        c.fl_encode(p, q, rd.hard, hdr, payload, payload.numel(), info)
        v = info.cpu().numpy()
        if v[2] != 0:
            raise RuntimeError(f"fixed-length coder flags {int(v[2])}")
        bits = int(v[0]) + 59 * 72
        e_plain = abs(float(rd.rate3[0].item()) * rd.n_hat - bits) / bits
        e_learn = None
        if self.mlp is not None:
            e_learn = abs(float(self.R_learned[0].item()) * rd.n_hat - bits) / bits
        return bits, int(v[1]), e_plain, e_learn

    def check_rate(self):
        """The fallback rule: the learned estimate drives the iteration until a
        check finds its error larger than the plain proxy's."""
        bits, kept, e_plain, e_learn = self.rate_errors()
        if self.mlp is not None:
            self.use_learned = e_learn <= e_plain
        self.checks.append((self.k, e_plain, e_learn, self.use_learned))
        return e_plain, e_learn

    def iterate(self, count_evals: bool = False):
        if self.check_every and self.mlp is not None and self.k % self.check_every == 0:
            self.check_rate()
        c, rd, k, mm = self.ctx, self.rd, self.k, self.mask_mode
        p, q, s = self.params, self.q, self.score
        learned = self.mlp is not None and self.use_learned
        # quantizer, mask and render in one call (the quantized rows stay in
        # registers); the rate terms read the statistics it leaves
        c.quant_render_fwd(p, q, s, mm, self.given, self.seed, k, rd.hard, rd.soft, rd.stats,
                           rd.image, rd.final_T, rd.last, rd.evals if count_evals else None)
        if learned:
            packed, theta = self.mlp
            c.rate_proxy(rd.stats, q, 0.0, rd.rate3, None)      # evaluated, not followed
            c.rate_mlp_fwd(packed, theta, p, q, rd.stats, rd.hard, self.R_learned, None)
        elif self.variant:      # the Laplace proxy or additive masking
            c.rate_variant(p, q, rd.stats, self.lam, rd.rate3, rd.rate_grad, self.proxy,
                           self.masking, self.alpha)
        else:
            c.rate_proxy(rd.stats, q, self.lam, rd.rate3, rd.rate_grad)
        w = self.ssim_weight
        c.l1_loss(rd.image, self.target, rd.loss, rd.dimage, 1.0 - w)
        if w > 0.0:
            c.ssim_loss(rd.image, self.target, w, rd.loss_ssim, rd.dimage)
        # the higher-SH gradient rows only in the steps whose update takes them
        sh_rest = k % self.sh_every == 0
        c.set_grad_sh_rest(sh_rest)
        c.quant_render_bwd(p, q, rd.soft, mm, None if learned else rd.rate_grad,
                           None if learned else rd.stats, rd.final_T, rd.last, rd.dimage,
                           rd.grad_qparams, rd.grad_q, rd.grad_score, rd.grad_mask)
        if learned:
            c.rate_mlp_bwd(packed, theta, p, q, rd.stats, rd.hard, rd.soft, mm, self.lam,
                           rd.grad_qparams, rd.grad_q, rd.grad_score, None)
        elif self.variant:
            c.rate_variant_bwd(p, rd.grad_qparams)
        c.adam_step(self.lr, k + 1, p, self.pm, self.pv, rd.grad_qparams, q, self.qm, self.qv,
                    rd.grad_q, s, self.sm, self.sv, rd.grad_score, lr_q=self.lr_q,
                    lr_score=self.lr_score, sh_rest=sh_rest, sparse=self.sparse)
        c.set_grad_sh_rest(True)
        self.k += 1

    def prune(self, pair_capacity: int = 0) -> int:
        """Keep the Gaussians the mask keeps now (the hard mask of a fresh
        decision at the current step); returns the new count.  N_hat (the
        count before formation) is unchanged.  pair_capacity > 0 reserves that
        pair capacity for the rebuilt scene."""
        torch = self.rd.torch
        c, rd = self.ctx, self.rd
        p, q, s = self.params, self.q, self.score
        c.fakequant_prune(p, q, s, self.mask_mode, self.given, self.seed, self.k, rd.qparams,
                          rd.hard, rd.soft, rd.stats)
        npad = rd.npad
        new = [torch.empty_like(a) for a in (p, self.pm, self.pv, s, self.sm, self.sv)]
        old = (p, self.pm, self.pv, s, self.sm, self.sv)
        kept = c.compact(rd.hard, list(zip(old, new)), npad)
        (self.params, self.pm, self.pv, self.score, self.sm, self.sv) = new
        if self.given is not None:   # every survivor was kept by the given mask
            self.given = torch.ones(npad, dtype=torch.uint8, device=rd.dev)
        self.rd = RDStep(c, kept, npad, rd.n_hat, rd.cams, rd.W, rd.H, tile=rd.tile,
                         tau=rd.tau, schedule=rd.schedule, deterministic=rd.deterministic)
        if pair_capacity > 0:
            c.reserve_pairs(pair_capacity)
        return kept

