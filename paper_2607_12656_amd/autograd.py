"""torch.autograd wrappers over the C ABI.

``FormationStep``: (params, qstep, score) -> (D_render, R_proxy, image); its
backward runs render_bwd, the rate-proxy gradient and the quantizer's
straight-through / learned-step-size backward in the library's kernels.  The
upstream gradients of D and R become the scale of dL/dimage and the weight of
the rate gradient, so ``(D + lam * R).backward()`` gives the gradient of the
paper's structural-formation loss (Sec. 3.3.2).

``Render``: (qparams, hard_mask) -> image for callers with their own image
loss; the gradient w.r.t. the hard mask is left in ``rd.grad_mask``.

Both keep no per-pair state: the backward re-walks the tile lists of the
forward (alpha and T recomputed from the per-pixel final T and stop
position).  Those lists, records and per-pixel buffers belong to the
``RDStep`` (and its context), so a backward must follow its own forward with
no other forward on that ``RDStep`` in between; otherwise it raises instead of
differentiating the wrong scene.
"""
from __future__ import annotations

import torch

from .rd import RDStep


def _check_current(ctx, rd: RDStep):
    if rd.generation != ctx.generation:
        raise RuntimeError(
            "backward after another forward on the same RDStep: the tile lists and "
            "per-pixel state of this forward were overwritten (run backward before the "
            "next forward, or use one RDStep per pending graph)")


class FormationStep(torch.autograd.Function):
    @staticmethod
    def forward(ctx, params, qstep, score, rd: RDStep, target, mask_mode: int, given_mask,
                seed: int, step: int):
        rd.forward(params, qstep, score, target, 0.0, mask_mode, given_mask, seed, step,
                   count_evals=False)
        ctx.rd, ctx.target, ctx.mask_mode = rd, target, mask_mode
        ctx.generation = rd.generation
        ctx.save_for_backward(params, qstep)
        image = rd.image.clone()
        ctx.mark_non_differentiable(image)
        return rd.loss.clone().reshape(()), rd.rate3[0].clone(), image

    @staticmethod
    def backward(ctx, gD, gR, _gimg):
        params, qstep = ctx.saved_tensors
        rd: RDStep = ctx.rd
        _check_current(ctx, rd)
        gd = 0.0 if gD is None else float(gD)
        gr = 0.0 if gR is None else float(gR)
        c = rd.ctx
        c.l1_loss(rd.image, ctx.target, rd.loss, rd.dimage, gd)
        c.rate_proxy(rd.stats, qstep, gr, rd.rate3, rd.rate_grad)
        gp = torch.empty_like(params)
        rd.backward(params, qstep, ctx.mask_mode, grad_params=gp)
        gs = rd.grad_score.clone() if ctx.mask_mode == 1 else None
        return gp, rd.grad_q.clone(), gs, None, None, None, None, None, None


class Render(torch.autograd.Function):
    @staticmethod
    def forward(ctx, qparams, hard_mask, rd: RDStep):
        c = rd.ctx
        rd.generation += 1
        c.render_fwd(qparams, hard_mask, rd.image, rd.final_T, rd.last, None)
        ctx.rd = rd
        ctx.generation = rd.generation
        ctx.save_for_backward(qparams, hard_mask)
        return rd.image.clone()

    @staticmethod
    def backward(ctx, gimg):
        qparams, hard_mask = ctx.saved_tensors
        rd: RDStep = ctx.rd
        _check_current(ctx, rd)
        g = torch.empty_like(qparams)
        rd.ctx.render_bwd(qparams, hard_mask, rd.final_T, rd.last, gimg.contiguous(), g,
                          rd.grad_mask)
        return g, None, None
