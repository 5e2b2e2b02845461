"""Host logic of the learned-coding stage (paper Sec. 3.4.2).

- The per-channel choice of the attribute predictor: every number comes
  from library calls (`sgs_attr_planes`, `sgs_ans_model`); this module only
  adds up each channel's ideal code length under both predictors and keeps
  the smaller, the way the paper's per-scene coder adapts its model to the
  scene's own attributes.
- The stream as bytes: `encode_scene` runs the library's encoders and packs
  their outputs (headers, model tables, rANS words) into one byte string;
  `decode_scene` unpacks it and runs the library's decoders.  Packing and
  unpacking are marshalling only."""
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


# ---------------------------------------------------------------------------
# The stream as bytes: a container of everything the decoder needs
# ---------------------------------------------------------------------------
# Layout (little-endian):
#   b"SGSC", u16 version, u16 lane length S
#   geometry: the octree header (30 x i64), q of the position channels
#     (3 x f32), the duplicate list (dups x (u32 voxel, u32 copies)), the
#     token stream (order-1 model, then the stream)
#   attributes: per channel 3-58 q (f32), kmin (i32), width (u8); the
#     predictor bits (56 bits in 7 bytes); one stream per plane row (order-0
#     model, then the stream)
# A model: u8 order, for order 1 the 257-bit map of the contexts in use
# (33 bytes); per context in use u16 K, then K x (u8 symbol, u16 f - 1).
# A stream: u32 blocks, the blocks' word counts (u32 each), the words (u16).
MAGIC = b"SGSC"
VERSION = 1
CTX = 257


def pack_model(freq, order: int) -> bytes:
    f = np.asarray(freq, np.uint16).reshape(CTX, 256)
    out = bytearray([order])
    rows = range(CTX) if order else [0]
    if order:
        used = np.array([f[x].any() for x in range(CTX)], np.uint8)
        out += np.packbits(np.concatenate([used, np.zeros(264 - CTX, np.uint8)]),
                           bitorder="little").tobytes()
        rows = [x for x in range(CTX) if used[x]]
    for x in rows:
        s = np.nonzero(f[x])[0]
        out += np.uint16(s.size).tobytes()
        rec = np.zeros(s.size, dtype=[("s", "u1"), ("f", "<u2")])
        rec["s"] = s
        rec["f"] = f[x][s] - 1
        out += rec.tobytes()
    return bytes(out)


def unpack_model(buf, pos: int):
    order = buf[pos]
    pos += 1
    f = np.zeros((CTX, 256), np.uint16)
    if order:
        used = np.unpackbits(np.frombuffer(buf, np.uint8, 33, pos), bitorder="little")[:CTX]
        pos += 33
        rows = np.nonzero(used)[0]
    else:
        rows = [0]
    for x in rows:
        k = int(np.frombuffer(buf, "<u2", 1, pos)[0])
        pos += 2
        rec = np.frombuffer(buf, dtype=[("s", "u1"), ("f", "<u2")], count=k, offset=pos)
        pos += 3 * k
        f[x][rec["s"]] = rec["f"].astype(np.uint16) + 1
    return f, int(order), pos


def pack_stream(words, block_off) -> bytes:
    off = np.asarray(block_off, np.int64)
    cnt = np.diff(off).astype("<u4")
    return (np.uint32(cnt.size).tobytes() + cnt.tobytes() +
            np.asarray(words, np.uint16)[:int(off[-1]) if off.size else 0].astype("<u2").tobytes())


def unpack_stream(buf, pos: int):
    nb = int(np.frombuffer(buf, "<u4", 1, pos)[0])
    pos += 4
    cnt = np.frombuffer(buf, "<u4", nb, pos).astype(np.int64)
    pos += 4 * nb
    off = np.concatenate([[0], np.cumsum(cnt)]).astype(np.int64)
    total = int(off[-1])
    words = np.frombuffer(buf, "<u2", total, pos).copy()
    pos += 2 * total
    return words, off, pos


def _coded(ctx, torch, sym, n, order, S, dev):
    """Model and stream of one symbol stream (device), read back."""
    freq = torch.empty(CTX * 256, dtype=torch.int16, device=dev)
    ctx.ans_model(sym, n, order, S, freq)
    cap = ctx.ans_max_words(n, S)
    nb = (n + 64 * S - 1) // (64 * S)
    words = torch.empty(max(cap, 1), dtype=torch.int16, device=dev)[:cap]
    off = torch.empty(nb + 1, dtype=torch.int64, device=dev)
    info = torch.empty(2, dtype=torch.int64, device=dev)
    ctx.ans_encode(sym, n, order, S, freq, words, off, info)
    inf = info.cpu().numpy()
    if inf[1] != 0:
        raise RuntimeError(f"entropy coder flags {int(inf[1])}")
    w = words.cpu().numpy().view(np.uint16)[:int(inf[0])]
    return pack_model(freq.cpu().numpy().view(np.uint16), order) + \
        pack_stream(w, off.cpu().numpy())


def encode_scene(ctx, params, npad: int, n: int, qstep, hard_mask, lane_len: int = 256):
    """The kept Gaussians of a scene as one byte string (geometry and
    attributes of the learned-coding stage).  ctx's scene must be the one
    `params` belongs to (the fixed-length coder's pass reads its sizes).
    Returns (bytes, sizes by part)."""
    import torch
    from ._lib import OCTREE_HEADER_WORDS
    dev = params.device
    S = lane_len
    cap = (21 * n + 3) // 4 * 4
    tokens = torch.empty(cap, dtype=torch.uint8, device=dev)
    codes = torch.empty(n, dtype=torch.int64, device=dev)
    di = torch.empty(n, dtype=torch.int32, device=dev)
    dc = torch.empty(n, dtype=torch.int32, device=dev)
    hdr = torch.empty(OCTREE_HEADER_WORDS, dtype=torch.int64, device=dev)
    ctx.octree_encode(params, npad, n, qstep, hard_mask, tokens, codes, di, dc, hdr)
    h = hdr.cpu().numpy()
    if h[8] != 0:
        raise RuntimeError(f"octree flags {int(h[8])}")
    T, kept, dups = int(h[6]), int(h[4]), int(h[7])
    out = bytearray(MAGIC + np.uint16(VERSION).tobytes() + np.uint16(S).tobytes())
    out += h.astype("<i8").tobytes()
    out += qstep[:3].cpu().numpy().astype("<f4").tobytes()
    dl = np.stack([di[:dups].cpu().numpy(), dc[:dups].cpu().numpy()], axis=1).astype("<u4")
    out += dl.tobytes()
    sizes = {"header": len(out)}
    geo = _coded(ctx, torch, tokens, T, 1, S, dev)
    out += geo
    sizes["geometry_stream"] = len(geo)
    # attributes
    fh = torch.empty((NCH, 3), dtype=torch.int32, device=dev)
    payload = torch.empty(NCH * n + 64, dtype=torch.int32, device=dev)
    finfo = torch.empty(3, dtype=torch.int64, device=dev)
    ctx.fl_encode(params, qstep, hard_mask, fh, payload, payload.numel(), finfo)
    fhn = fh.cpu().numpy()
    fl = ctx.fl_header_host(fhn)
    perm = torch.empty(max(kept, 1), dtype=torch.int32, device=dev)
    ctx.morton_order(params, npad, n, qstep, hard_mask, ctx.octree_header(h), codes, perm)
    pred, _, _ = choose_predictors(ctx, params, npad, perm, kept, fl, S)
    a0 = len(out)
    rec = np.zeros(NCH - 3, dtype=[("q", "<f4"), ("kmin", "<i4"), ("w", "u1")])
    rec["q"] = fhn[3:, 0].view(np.float32)
    rec["kmin"] = fhn[3:, 1]
    rec["w"] = fhn[3:, 2]
    out += rec.tobytes()
    out += np.packbits(pred[3:], bitorder="little").tobytes()
    rows = ctx.attr_plane_rows(fl, pred)
    if rows and kept:
        planes = torch.empty((rows, kept), dtype=torch.uint8, device=dev)
        ctx.attr_planes(params, npad, perm, kept, fl, S, planes, pred)
        for t in range(rows):
            out += _coded(ctx, torch, planes[t], kept, 0, S, dev)
    sizes["attributes"] = len(out) - a0
    sizes["total"] = len(out)
    return bytes(out), sizes


def decode_scene(ctx, data: bytes, dev):
    """Decode encode_scene's bytes: scene rows [59][kept] (float32, device):
    positions (octree), then colour, opacity, scale and rotation, the kept
    Gaussians in Morton order; every arithmetic step in the library."""
    import torch
    from ._lib import OCTREE_HEADER_WORDS, sgs_fl_channel
    buf = memoryview(data)
    if bytes(buf[:4]) != MAGIC:
        raise ValueError("not a SpeedyGS coding-stage stream")
    ver, S = np.frombuffer(buf, "<u2", 2, 4)
    if ver != VERSION:
        raise ValueError(f"stream version {ver}")
    S = int(S)
    pos = 8
    h = np.frombuffer(buf, "<i8", OCTREE_HEADER_WORDS, pos).copy()
    pos += 8 * OCTREE_HEADER_WORDS
    qpos = np.frombuffer(buf, "<f4", 3, pos).copy()
    pos += 12
    T, m, kept, dups = int(h[6]), int(h[5]), int(h[4]), int(h[7])
    dl = np.frombuffer(buf, "<u4", 2 * dups, pos).reshape(dups, 2).copy()
    pos += 8 * dups
    t_ = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    # geometry
    f, order, pos = unpack_model(buf, pos)
    words, off, pos = unpack_stream(buf, pos)
    tokens = torch.empty(max(T, 1), dtype=torch.uint8, device=dev)
    info = torch.zeros(2, dtype=torch.int64, device=dev)
    w_dev = t_(words.view(np.int16)) if words.size else torch.zeros(1, dtype=torch.int16,
                                                                     device=dev)
    ctx.ans_decode(w_dev, words.size, t_(off), T, order, S, t_(f.view(np.int16)), tokens, info)
    out = torch.empty((NCH, max(kept, 1)), dtype=torch.float32, device=dev)
    codes = torch.empty(max(m, 1), dtype=torch.int64, device=dev)
    qd = torch.zeros(NCH, dtype=torch.float32, device=dev)
    qd[:3] = t_(qpos)
    di = t_(dl[:, 0].astype(np.int32)) if dups else None
    dc = t_(dl[:, 1].astype(np.int32)) if dups else None
    oinfo = torch.zeros(1, dtype=torch.int64, device=dev)
    if kept:
        ctx.octree_decode(ctx.octree_header(h), tokens, di, dc, qd, codes, out[:3], max(kept, 1),
                          oinfo)
    # attributes
    rec = np.frombuffer(buf, dtype=[("q", "<f4"), ("kmin", "<i4"), ("w", "u1")], count=NCH - 3,
                        offset=pos)
    pos += 9 * (NCH - 3)
    pred = np.ones(NCH, np.uint8)
    pred[3:] = np.unpackbits(np.frombuffer(buf, np.uint8, 7, pos), bitorder="little")[:NCH - 3]
    pos += 7
    fl = (sgs_fl_channel * NCH)()
    for j in range(3, NCH):
        fl[j].q, fl[j].kmin, fl[j].width = float(rec["q"][j - 3]), int(rec["kmin"][j - 3]), \
            int(rec["w"][j - 3])
    rows = ctx.attr_plane_rows(fl, pred)
    planes = torch.empty((max(rows, 1), max(kept, 1)), dtype=torch.uint8, device=dev)
    streams, keep = [], []
    for t in range(rows):
        f, order, pos = unpack_model(buf, pos)
        words, off, pos = unpack_stream(buf, pos)
        d = dict(words=t_(words.view(np.int16)) if words.size else
                 torch.zeros(1, dtype=torch.int16, device=dev),
                 n_words=words.size, block_off=t_(off), n=kept, freq=t_(f.view(np.int16)),
                 sym=planes[t], order=order, lane_len=S)
        streams.append(d)
    minfo = torch.zeros(max(rows, 1), dtype=torch.int64, device=dev)
    if rows and kept:
        ctx.ans_decode_multi(streams, minfo)
    if kept:
        ctx.attr_reconstruct(planes, kept, fl, S, out, max(kept, 1), pred)
    flags = int(info[0].item()) | int(oinfo.item()) | int(minfo.abs().sum().item())
    if flags:
        raise RuntimeError(f"damaged stream (flags {flags})")
    if pos != len(data):
        raise ValueError("trailing bytes after the stream")
    return out[:, :kept]
