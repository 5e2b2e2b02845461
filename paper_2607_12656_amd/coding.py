"""Host logic of the learned-coding stage's attribute half (paper Sec. 3.4.2):
the per-channel choice of the attribute predictor.  Every number comes from
library calls (`sgs_attr_planes`, `sgs_ans_model`); this module only adds up
each channel's ideal code length under both predictors and keeps the
smaller, the way the paper's per-scene coder adapts its model to the
scene's own attributes."""
from __future__ import annotations

import numpy as np

NCH = 59


def plane_channels(ctx, fl, predictor):
    """Channel of every plane row, in row order."""
    widths = [fl[j].width for j in range(NCH)]
    out = []
    for j in range(3, NCH):
        w = widths[j]
        if w == 0:
            continue
        p = 1 if predictor is None else int(predictor[j])
        out += [j] * ((w + 8) // 8 if p else (w + 7) // 8)
    return out


def channel_bits(ctx, torch, params, npad, perm, kept, fl, S, predictor, dev):
    """Ideal order-0 code length of each channel's planes (dict j -> bits)."""
    rows = ctx.attr_plane_rows(fl, predictor)
    bits = {j: 0.0 for j in range(3, NCH)}
    if rows == 0 or kept == 0:
        return bits
    planes = torch.empty((rows, kept), dtype=torch.uint8, device=dev)
    ctx.attr_planes(params, npad, perm, kept, fl, S, planes, predictor)
    freq = torch.empty(257 * 256, dtype=torch.int16, device=dev)
    ib = torch.empty(rows, dtype=torch.float64, device=dev)
    for t in range(rows):
        ctx.ans_model(planes[t], kept, 0, S, freq, ib[t:t + 1])
    v = ib.cpu().numpy()
    for t, j in enumerate(plane_channels(ctx, fl, predictor)):
        bits[j] += float(v[t])
    return bits


def choose_predictors(ctx, params, npad, perm, kept, fl, S):
    """Per channel 1 (previous-token prediction) where its planes' ideal bits
    are fewer than without prediction, else 0.  Returns (predictor [59]
    uint8, bits with the choice, bits with prediction everywhere)."""
    import torch
    dev = params.device
    p0 = np.zeros(NCH, np.uint8)
    p1 = np.ones(NCH, np.uint8)
    b0 = channel_bits(ctx, torch, params, npad, perm, kept, fl, S, p0, dev)
    b1 = channel_bits(ctx, torch, params, npad, perm, kept, fl, S, p1, dev)
    pred = np.ones(NCH, np.uint8)
    for j in range(3, NCH):
        pred[j] = 1 if b1[j] < b0[j] else 0
    chosen = sum(b1[j] if pred[j] else b0[j] for j in range(3, NCH))
    return pred, chosen, sum(b1.values())
