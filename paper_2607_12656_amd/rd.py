"""One RD step of the structural-formation stage on the GPU.

``RDStep`` owns the device buffers of a step (torch tensors, used only as
memory) and issues the C-ABI calls in order:

    fakequant_prune -> rate_proxy -> render_fwd -> l1_loss
    -> render_bwd -> fakequant_prune_bwd

or, with ``fused=True`` (the same results; the quantized rows are neither
written nor read back):

    quant_render_fwd -> rate_proxy -> l1_loss -> quant_render_bwd

Every arithmetic step runs in libspeedygs's HIP kernels; nothing here
computes.  The loss is D_render + lam * R_proxy (paper Sec. 3.3.2, total loss).
D_render is the L1 distortion, or with ``ssim_weight`` = w > 0 vanilla
3DGS's (1 - w) L1 + w (1 - SSIM), which the supplement's training objective
follows (w = 0.2 there).
"""
from __future__ import annotations

import numpy as np

from ._lib import NCH, RATE_GRAD_FLOATS, STATS_WORDS, Context


class RDStep:
    def __init__(self, ctx: Context, n: int, npad: int, n_hat: int, cams: np.ndarray,
                 width: int, height: int, tile=(16, 16), tau: float = 1.0,
                 schedule: str = "tile", fused: bool = False, deterministic: bool = False):
        import torch
        self.torch = torch
        self.ctx = ctx
        self.fused = fused
        dev = torch.device("cuda", ctx.device)
        self.dev = dev
        V = cams.shape[0]
        self.n, self.npad, self.n_hat, self.V, self.W, self.H = n, npad, n_hat, V, width, height
        self.cams, self.tile, self.tau, self.schedule = cams, tile, tau, schedule
        self.deterministic = deterministic
        ctx.set_scene(n, npad, n_hat, cams, width, height, tile=tile, tau=tau,
                      schedule=schedule, deterministic=deterministic)
        f32, u8, i32, i64 = torch.float32, torch.uint8, torch.int32, torch.int64
        e = lambda *s, dt=f32: torch.empty(*s, dtype=dt, device=dev)
        self.qparams = e(NCH, npad)
        self.hard = e(n, dt=u8)
        self.soft = e(n)
        self.stats = e(STATS_WORDS, dt=i64)
        self.rate3 = e(3)
        self.rate_grad = e(RATE_GRAD_FLOATS)
        self.image = e(V, 3, height, width)
        self.final_T = e(V, height, width)
        self.last = e(V, height, width, dt=i32)
        self.evals = torch.zeros(1, dtype=i64, device=dev)
        self.loss = e(1)
        self.loss_ssim = torch.zeros(1, dtype=f32, device=dev)
        self.dimage = e(V, 3, height, width)
        self.grad_qparams = e(NCH, npad)
        self.grad_mask = e(n)
        self.grad_q = e(NCH)
        self.grad_score = e(n)
        # forwards issued on this step's buffers (and context): a backward
        # must follow the forward it differentiates, with no other in between
        self.generation = 0

    def forward(self, params, qstep, score, target, lam: float, mask_mode: int = 0,
                given_mask=None, seed: int = 0, step: int = 0, count_evals: bool = True,
                loss_scale: float = 1.0, ssim_weight: float = 0.0):
        c = self.ctx
        ev = self.evals if count_evals else None
        self.generation += 1
        if self.fused:
            c.quant_render_fwd(params, qstep, score, mask_mode, given_mask, seed, step,
                               self.hard, self.soft, self.stats, self.image, self.final_T,
                               self.last, ev)
            c.rate_proxy(self.stats, qstep, lam, self.rate3, self.rate_grad)
        else:
            c.fakequant_prune(params, qstep, score, mask_mode, given_mask, seed, step,
                              self.qparams, self.hard, self.soft, self.stats)
            c.rate_proxy(self.stats, qstep, lam, self.rate3, self.rate_grad)
            c.render_fwd(self.qparams, self.hard, self.image, self.final_T, self.last, ev)
        c.l1_loss(self.image, target, self.loss, self.dimage, loss_scale * (1.0 - ssim_weight))
        if ssim_weight > 0.0:
            c.ssim_loss(self.image, target, loss_scale * ssim_weight, self.loss_ssim, self.dimage)

    def backward(self, params, qstep, mask_mode: int = 0, grad_params=None, dimage=None):
        """Gradients of loss = D + lam R.  grad_params defaults to an in-place
        reuse of the render gradient buffer (straight-through aliasing)."""
        c = self.ctx
        gp = self.grad_qparams if grad_params is None else grad_params
        if self.fused:
            c.quant_render_bwd(params, qstep, self.soft, mask_mode, self.rate_grad, self.stats,
                               self.final_T, self.last,
                               self.dimage if dimage is None else dimage, gp, self.grad_q,
                               self.grad_score, self.grad_mask)
            return gp
        c.render_bwd(self.qparams, self.hard, self.final_T, self.last,
                     self.dimage if dimage is None else dimage, self.grad_qparams,
                     self.grad_mask)
        c.fakequant_prune_bwd(params, qstep, self.soft, mask_mode, self.rate_grad, self.stats,
                              self.grad_qparams, self.grad_mask, gp, self.grad_q,
                              self.grad_score)
        return gp

    def step(self, params, qstep, score, target, lam, mask_mode=0, given_mask=None, seed=0,
             step=0, count_evals=True, grad_params=None):
        self.forward(params, qstep, score, target, lam, mask_mode, given_mask, seed, step,
                     count_evals)
        return self.backward(params, qstep, mask_mode, grad_params)
