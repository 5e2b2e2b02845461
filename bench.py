#!/usr/bin/env python
"""Benchmark of one RD step (forward + backward) of SpeedyGS's structural
formation on one MI355X.

Default workload (the measured configuration): plain rate proxy, 1,000,000
Gaussians (clustered: 3-component mixture), one 1297x840 camera on the
radius-4 ring, learned per-channel steps initialised to 2^-6, 20 % pruned by
a given mask, L1 distortion against a seeded random target, lambda 2.5e-5,
16x16 tiles.  `--workload c3`: 3,000,000 Gaussians, 8 views of 1600x1060,
tile shape from the autotuner.  Inputs are synthetic (seeded) and resident
in HBM before the timed region.

A step = fake-quantize + mask + channel statistics, rate proxy, projection,
depth sort, pair emission, tile sort, ranges, blend, L1, blend backward,
projection backward, quantizer/mask backward (all in libspeedygs kernels).
The pair capacity is reserved once, so a step never synchronizes.

Prints one JSON line: ms/step and Gaussian-pixel evaluations per second
(E / step time, E = in-support (Gaussian, pixel) evaluations of the forward,
the set the backward re-walks) over K replays of the step captured in a HIP
graph; the same step enqueued eagerly, with the roofline of the dominant
kernel group (HIP events recorded on the library's stream around every kernel
group over that run); the learned-rate
step (MLP in the loop, forward + recompute backward) timed beside it, the
MLP's training / inference throughput, the fixed-length encode / decode of
the kept Gaussians (Sec. 3.4.1), the SSIM term of the distortion, the
Laplace rate proxy beside the range proxy, and the FP64 oracle timed on the
host as a CPU baseline.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X published peaks
HBM_PEAK_GBS = 8000.0
FP32_VECTOR_PEAK_TFLOPS = 157.3
BF16_MFMA_PEAK_TFLOPS = 2500.0

# Algorithmic work per unit of each kernel group.
NCH = 59
FLOP_PER_EVAL_FWD = 24     # offsets 2, quadratic form 9, exp 2, alpha/T 5, colour 6
FLOP_PER_EVAL_BWD = 60     # alpha recompute 15, T and dalpha 12, 10 gradients 23, back colour 10
MLP_FLOP_PER_ROW = 2 * (64 * 128 + 128 * 128 + 128)


def group_work(g: str, n: int, V: int, P: int, E: int, W: int, H: int):
    """(bound, algorithmic amount per launch, unit) of one kernel group."""
    pix = V * W * H
    # the step runs the fused entry points: the quantizer pass reads the rows
    # for the rate statistics only, the projections quantize in registers,
    # and the projection backward applies the quantizer's backward
    if g == "fakequant":
        return "hbm", n * (NCH * 4 + 1 + 1 + 4), "B"
    if g == "preprocess":
        return "hbm", n * (NCH * 4 + 1) + V * n * (48 + 12), "B"
    if g in ("depth_sort", "scan"):
        return "hbm", V * n * 16, "B"
    if g == "duplicate":
        return "hbm", V * n * 12 + P * 8, "B"
    if g == "tile_sort":
        return "hbm", P * 16, "B"
    if g == "ranges":
        return "hbm", P * 4, "B"
    if g == "blend_fwd":
        return "alu", E * FLOP_PER_EVAL_FWD, "FLOP"
    if g == "l1":
        return "hbm", pix * 3 * 12, "B"
    if g == "grad_clear":
        return "hbm", V * n * 48, "B"
    if g == "blend_bwd":
        return "alu", E * FLOP_PER_EVAL_BWD, "FLOP"
    if g == "preprocess_bwd":
        return "hbm", n * (NCH * 4 * 2 + 4 + 4) + V * n * 48, "B"
    if g == "fakequant_bwd":     # the step-size partials of the projection backward
        return "hbm", NCH * 8 * -(-n // 128), "B"
    return "hbm", 0, "B"


def roofline(g, ms, n, V, P, E, W, H):
    bound, amount, unit = group_work(g, n, V, P, E, W, H)
    dur = ms * 1e-3
    if unit == "B":
        achieved, peak, ru = amount / dur / 1e9, HBM_PEAK_GBS, "GB/s"
    else:
        achieved, peak, ru = amount / dur / 1e12, FP32_VECTOR_PEAK_TFLOPS, "TFLOP/s"
    return {"bound": bound, "kernel": g, "achieved": round(achieved, 3), "peak": peak,
            "unit": ru, "frac": round(achieved / peak, 5), "traffic": None,
            "algorithmic_per_launch": amount, "avg_launch_ms": round(ms, 4)}


def cpu_baseline(sc, lam):
    """The FP64 oracle, as it stands, on the same workload: one full step
    (forward + backward) on the same scene and camera, single-threaded."""
    import oracle
    t0 = time.perf_counter()
    r = oracle.rd_step(sc.params, sc.qstep, sc.score, sc.given_mask, sc.cams, sc.width,
                       sc.height, sc.target, sc.n, sc.n_hat, lam)
    dt = time.perf_counter() - t0
    E = r["fw"]["evals"]
    return {"value": E / dt, "unit": "Gaussian-pixel evals/s", "cores": 1, "kind": "oracle",
            "sample": f"one full RD step (fwd+bwd) of the measured workload, "
                      f"{E} evals in {dt:.1f} s, single thread",
            "s_per_step": round(dt, 3)}


def bench_formation(args, sc, ctx, rd, stream, dev, t, tile, schedule, tune):
    """Full formation iterations at 3M Gaussians x 8 views: RD step on the
    Gumbel-sigmoid mask, learned rate in the loop (forward + recompute
    backward), Adam on (y, q, s); the same iterations with the plain proxy.
    Both start from the same scene; every iteration counts its evaluations.
    Ends with the rate-estimate error of each rate term against the exact
    bits of the fixed-length coder on the final state."""
    import numpy as np
    import torch

    from paper_2607_12656_amd.formation import Formation
    from paper_2607_12656_amd.rate_train import RateTrainer

    lam = 2.5e-5
    K, W = args.steps, args.warmup
    p0, q0, s0, target = t(sc.params), t(sc.qstep), t(sc.score), t(sc.target)
    # the estimator, trained on this scene's own coder bits (GPU only)
    t0 = time.perf_counter()
    trainer = RateTrainer(ctx, rd, p0, s0, sc.given_mask, seed=3, scenes=64)
    theta, packed, losses = trainer.train(steps=400)
    err_l, err_p = trainer.held_out_errors(theta, packed)
    train_s = time.perf_counter() - t0
    del trainer
    rd.forward(p0, q0, s0, target, lam, 1, None, 5, 0, count_evals=False)
    P, _ = ctx.query()
    ctx.reserve_pairs(P + P // 2 + 4096)       # the scene moves; the count is checked after
    runs = {}
    for name, mlp in (("learned", (packed, theta)), ("plain", None)):
        p, q, s = p0.clone(), q0.clone(), s0.clone()
        f = Formation(rd, p, q, s, target, lam, mask_mode=1, seed=5, mlp=mlp)
        for _ in range(W):
            f.iterate()
        torch.cuda.synchronize()
        rd.evals.zero_()
        ctx.profile_enable(True)
        t0 = time.perf_counter()
        for _ in range(K):
            f.iterate(count_evals=True)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        prof = ctx.profile_read()
        ctx.profile_enable(False)
        pairs, _ = ctx.query()                 # raises if the reserved capacity overflowed
        E = int(rd.evals.item())
        # the final state: plain proxy, learned estimate and the coder's exact bits
        c = ctx
        c.fakequant_prune(p, q, s, 1, None, 5, f.k, rd.qparams, rd.hard, rd.soft, rd.stats)
        c.rate_proxy(rd.stats, q, 0.0, rd.rate3, None)
        c.rate_mlp_fwd(packed, theta, p, q, rd.stats, rd.hard, f.R_learned, None)
        words = sc.n * NCH + 64
        hdr = torch.empty((NCH, 3), dtype=torch.int32, device=dev)
        payload = torch.empty(words, dtype=torch.int32, device=dev)
        info = torch.empty(3, dtype=torch.int64, device=dev)
        c.fl_encode(p, q, rd.hard, hdr, payload, words, info)
        torch.cuda.synchronize()
        bits = int(info[0].item()) + NCH * 72
        r_plain = float(rd.rate3[0].item()) * sc.n_hat
        r_learn = float(f.R_learned[0].item()) * sc.n_hat
        kernels = {g: round(tot / cnt, 4) for g, (tot, cnt) in prof.items() if cnt}
        runs[name] = {"ms_per_step": round(dt * 1e3 / K, 4), "value": round(E / dt, 1),
                      "evals": E, "pairs_last": pairs, "kept_last": int(info[1].item()),
                      "coder_bits_last": bits,
                      "plain_proxy_error": round(abs(r_plain - bits) / bits, 4),
                      "learned_error": round(abs(r_learn - bits) / bits, 4),
                      "kernel_ms": kernels}
        del payload
    L = runs["learned"]
    dom = max(L["kernel_ms"], key=L["kernel_ms"].get)
    roof = roofline(dom, L["kernel_ms"][dom], sc.n, sc.views, L["pairs_last"],
                    L["evals"] // K, sc.width, sc.height)
    line = {
        "metric": "RD-step ms/iter & Gaussian-pixel evals/s (fwd+bwd), learned vs plain rate",
        "value": L["value"], "unit": "Gaussian-pixel evals/s", "n_gpus": 1, "steps": K,
        "warmup": W, "ms_per_step": L["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"c5: full formation iteration, {sc.n} Gaussians (clustered), "
                               f"{sc.views} views {sc.width}x{sc.height}, Gumbel-sigmoid mask, "
                               f"learned rate in the loop (forward + recompute backward), "
                               f"Adam on parameters / steps / scores (higher SH every 16th, "
                               f"sparse), lambda {lam}, {K} iterations, tile "
                               f"{tile[0]}x{tile[1]}",
                   "gaussians": sc.n, "views": sc.views, "width": sc.width,
                   "height": sc.height, "tile": f"{tile[0]}x{tile[1]}", "schedule": schedule,
                   "mlp_weights": "trained on the GPU on this scene's fixed-length coder "
                                  "bits (64 step vectors 2^U[-9,-3], 400 steps of 65,536 "
                                  "rows)"},
        "mlp_training": {"seconds": round(train_s, 2), "loss": [round(v, 2) for v in losses],
                         "held_out_error_learned": round(err_l, 4),
                         "held_out_error_plain": round(err_p, 4)},
        "roofline": roof,
        "learned": L, "plain": runs["plain"],
        "learned_over_plain_time": round(L["ms_per_step"] / runs["plain"]["ms_per_step"], 4),
    }
    if tune is not None:
        line["autotune_ms"] = tune["ms"]
    return line


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default 20; 1000 iterations for c5)")
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="c2", choices=("c2", "c3", "c5"),
                    help="c2: 1M Gaussians, 1 view; c3: 3M Gaussians, 8 views; c5: the full "
                         "formation iteration at 3M x 8 views (learned rate in the loop, "
                         "Gumbel-sigmoid mask, Adam), learned vs plain rate")
    ap.add_argument("--tile", default=None, help="16x16 | 8x8 | 32x8 | auto")
    ap.add_argument("--schedule", default=None, choices=("tile", "stride", "queue", "block"),
                    help="blend launch schedule when --tile names a shape (default: block "
                         "on the 1M workload, the fastest there, else tile)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip graph / learned / MLP / codec / SSIM / rate-variant legs")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run one plain 256 MiB device copy first (scale for HBM counters)")
    ap.add_argument("--traffic", default=os.path.join(ROOT, "profiles", "traffic.json"),
                    help="rocprofv3 HBM bytes per launch (used only while the kernel source "
                         "is unchanged since the counters were taken)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the step runs on one GPU; --gpus must be 1 (sharding "
                                   "over GPUs is not implemented)"}))
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    from paper_2607_12656_amd import Context
    from paper_2607_12656_amd.rd import RDStep

    if args.steps is None:
        args.steps = 1000 if args.workload == "c5" else 20
    sc = synth.make_scene("c3" if args.workload == "c5" else args.workload)
    lam = 2.5e-5
    dev = torch.device("cuda", 0)
    stream = torch.cuda.Stream(dev)
    torch.cuda.set_stream(stream)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    params, q, score = t(sc.params), t(sc.qstep), t(sc.score)
    mask, target = t(sc.given_mask), t(sc.target)
    ctx = Context(0, stream=stream)
    if args.calibrate_copy:
        src = torch.ones(64 << 20, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    def plain_step(rd, count=False):
        # the fused entry points (quant_render_fwd / quant_render_bwd): the
        # quantized rows and their gradient never cross HBM
        rd.fused = True
        rd.forward(params, q, score, target, lam, 0, mask, 0, 0, count_evals=count)
        rd.backward(params, q, 0)

    tile_choice = args.tile or ("16x16" if args.workload == "c2" else "auto")
    tune = None
    if tile_choice == "auto":
        from paper_2607_12656_amd import autotune
        tune = autotune.tune(ctx, sc.n, sc.npad, sc.n_hat, sc.cams, sc.width, sc.height,
                             plain_step, reps=2)
        tile, schedule = tune["tile"], tune["schedule"]
    else:
        tile = tuple(int(v) for v in tile_choice.split("x"))
        schedule = args.schedule or ("block" if args.workload == "c2" else "tile")
    rd = RDStep(ctx, sc.n, sc.npad, sc.n_hat, sc.cams, sc.width, sc.height, tile=tile,
                schedule=schedule)
    if args.workload == "c5":
        print(json.dumps(bench_formation(args, sc, ctx, rd, stream, dev, t, tile, schedule,
                                         tune)), flush=True)
        return

    # evaluation count and pair count of one step (deterministic)
    rd.evals.zero_()
    plain_step(rd, count=True)
    torch.cuda.synchronize()
    E = int(rd.evals.item())
    P, _ = ctx.query()
    ctx.reserve_pairs(P + P // 8 + 4096)      # no host synchronization inside a step
    for _ in range(args.warmup):
        plain_step(rd)
    ctx.query()
    torch.cuda.synchronize()
    ctx.profile_enable(True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plain_step(rd)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = ctx.profile_read()
    ctx.profile_enable(False)
    ctx.query()                                # raises if the capacity overflowed
    ms = (t1 - t0) * 1e3 / args.steps          # eager: the host enqueues every call
    kernels = {g: round(tot / cnt, 4) for g, (tot, cnt) in prof.items() if cnt}
    # the timed steps: the whole step captured once in a HIP graph and
    # replayed K times between synchronizations (no host work inside)
    ctx.graph_begin()
    plain_step(rd)
    graph = ctx.graph_end()
    for _ in range(max(args.warmup, 2)):
        graph.launch(stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        graph.launch(stream)
    torch.cuda.synchronize()
    gms = (time.perf_counter() - t0) * 1e3 / args.steps
    ctx.query()
    graph.close()
    value = E / (gms * 1e-3)
    dom = max(kernels, key=kernels.get)
    roof = roofline(dom, kernels[dom], sc.n, sc.views, P, E, sc.width, sc.height)
    if args.traffic and os.path.exists(args.traffic):
        import hashlib
        tr = json.load(open(args.traffic))
        ent = tr.get(f"{args.workload}:{dom}")
        if ent:
            # the counters hold while the kernel's sources are unchanged
            h = hashlib.sha256()
            for f in ent.get("kernel_files", [ent.get("kernel_file")]):
                h.update(open(os.path.join(ROOT, f), "rb").read())
            cur = h.hexdigest()[:16]
            if cur == ent["kernel_sha256_16"]:
                roof["traffic"] = ent["bytes_per_launch"]
                roof["traffic_source"] = ent["source"] + " (profiles/hbm_traffic_*.md)"

    line = {
        "metric": "RD-step ms/iter & Gaussian-pixel evals/s (fwd+bwd), learned vs plain rate",
        "value": round(value, 1), "unit": "Gaussian-pixel evals/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(gms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: plain RD step, {sc.n} Gaussians (clustered), "
                               f"{sc.views} view(s) {sc.width}x{sc.height}, 20% pruned, "
                               f"lambda 2.5e-5, tile {tile[0]}x{tile[1]}",
                   "gaussians": sc.n, "views": sc.views, "width": sc.width,
                   "height": sc.height, "tile": f"{tile[0]}x{tile[1]}", "schedule": schedule, "pairs": P,
                   "evals_per_step": E},
        "roofline": roof,
        "kernel_ms": kernels,
        "timing": "HIP-graph replays of the whole step; eager_ms_per_step: the same calls "
                  "enqueued by the host each step (kernel_ms, roofline: HIP events in that run)",
        "eager_ms_per_step": round(ms, 4),
        "eager_value": round(E / (ms * 1e-3), 1),
    }
    if tune is not None:
        line["autotune_ms"] = tune["ms"]

    if not args.no_extras:
        # learned rate in the loop: MLP forward + recompute backward replace
        # the range proxy's gradient; the proxy is still evaluated (forward)
        theta = torch.empty(24961, dtype=torch.float32, device=dev)
        gen = torch.Generator(device="cpu").manual_seed(7)
        theta.copy_((torch.rand(24961, generator=gen) * 2 - 1) * 0.2)
        packed = torch.empty(98304 // 4, dtype=torch.int32, device=dev)
        ctx.rate_mlp_pack(theta, packed)
        Rl = torch.empty(1, dtype=torch.float32, device=dev)

        def learned_step():
            c = ctx
            c.quant_render_fwd(params, q, score, 0, mask, 0, 0, rd.hard, rd.soft, rd.stats,
                               rd.image, rd.final_T, rd.last)
            c.rate_proxy(rd.stats, q, 0.0, rd.rate3, None)
            c.rate_mlp_fwd(packed, theta, params, q, rd.stats, rd.hard, Rl, None)
            c.l1_loss(rd.image, target, rd.loss, rd.dimage)
            c.quant_render_bwd(params, q, rd.soft, 0, None, None, rd.final_T, rd.last, rd.dimage,
                               rd.grad_qparams, rd.grad_q, rd.grad_score, rd.grad_mask)
            c.rate_mlp_bwd(packed, theta, params, q, rd.stats, rd.hard, rd.soft, 0, lam,
                           rd.grad_qparams, rd.grad_q, rd.grad_score, None)

        for _ in range(args.warmup):
            learned_step()
        torch.cuda.synchronize()
        ctx.profile_enable(True)
        t0 = time.perf_counter()
        for _ in range(args.steps):
            learned_step()
        torch.cuda.synchronize()
        lms = (time.perf_counter() - t0) * 1e3 / args.steps
        lprof = ctx.profile_read()
        ctx.profile_enable(False)
        ctx.query()
        lk = {g: round(tot / cnt, 4) for g, (tot, cnt) in lprof.items() if cnt}
        mf = lk.get("mlp_fwd", 0.0)
        line["learned_rate"] = {
            "ms_per_step": round(lms, 4), "value": round(E / (lms * 1e-3), 1),
            "mlp_fwd_ms": mf, "mlp_bwd_ms": lk.get("mlp_bwd", 0.0),
            "mlp_fwd_tflops": round(sc.n * MLP_FLOP_PER_ROW / (mf * 1e-3) / 1e12, 2) if mf else None,
            "plain_ms_per_step": round(ms, 4), "timing": "eager, both"}

        # MLP alone: one training step on 65,536 rows, inference over 3M rows
        B = 65536
        Xtr = torch.randint(0, 1 << 14, (B, 64), dtype=torch.int16, device=dev)
        ttr = torch.rand(B, device=dev) * 100 + 200
        m_ = torch.zeros_like(theta)
        v_ = torch.zeros_like(theta)
        g_ = torch.empty_like(theta)
        lo = torch.empty(1, device=dev)
        scratch = torch.empty(ctx.rate_mlp_train_scratch_bytes(B), dtype=torch.uint8, device=dev)
        th2 = theta.clone()
        for s in range(1, 4):
            ctx.rate_mlp_train_step(th2, m_, v_, packed, Xtr, ttr, B, 1e-4, s, lo, g_, scratch)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for s in range(4, 4 + args.steps):
            ctx.rate_mlp_train_step(th2, m_, v_, packed, Xtr, ttr, B, 1e-4, s, lo, g_, scratch)
        torch.cuda.synchronize()
        tms = (time.perf_counter() - t0) * 1e3 / args.steps
        Ni = 3_000_000
        Xin = torch.randint(0, 1 << 14, (Ni, 64), dtype=torch.int16, device=dev)
        fo = torch.empty(Ni, device=dev)
        ctx.rate_mlp_pack(theta, packed)
        ctx.rate_mlp_infer(packed, theta, Xin, Ni, fo)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            ctx.rate_mlp_infer(packed, theta, Xin, Ni, fo)
        torch.cuda.synchronize()
        ims = (time.perf_counter() - t0) * 1e3 / args.steps
        line["mlp"] = {
            "train_step_ms_65536_rows": round(tms, 4),
            "train_tflops": round(3 * B * MLP_FLOP_PER_ROW / (tms * 1e-3) / 1e12, 2),
            "infer_ms_3M_rows": round(ims, 4),
            "infer_tflops": round(Ni * MLP_FLOP_PER_ROW / (ims * 1e-3) / 1e12, 2),
            "infer_mfma_frac": round(Ni * MLP_FLOP_PER_ROW / (ims * 1e-3) / 1e12
                                     / BF16_MFMA_PEAK_TFLOPS, 4)}
        del Xin, fo, Xtr, scratch

        # fixed-length coding of the kept Gaussians (the pruned step's mask)
        rd.forward(params, q, score, target, lam, 0, mask, 0, 0)
        words = sc.n * NCH + 64                 # 32 bits per code at most
        hdr = torch.empty((NCH, 3), dtype=torch.int32, device=dev)
        payload = torch.empty(words, dtype=torch.int32, device=dev)
        info = torch.empty(3, dtype=torch.int64, device=dev)
        ctx.fl_encode(params, q, rd.hard, hdr, payload, words, info)
        torch.cuda.synchronize()
        bits, kept, flags = (int(v) for v in info.cpu())
        pad = (kept + 63) // 64 * 64
        out = torch.empty((NCH, max(pad, 64)), dtype=torch.float32, device=dev)
        pw = (bits + 31) // 32 + 1
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        for _ in range(3):
            ctx.fl_encode(params, q, rd.hard, hdr, payload, words, info)
            ctx.fl_decode(hdr, payload, pw, kept, max(pad, 64), out)
        ev[0].record(stream)
        for _ in range(args.steps):
            ctx.fl_encode(params, q, rd.hard, hdr, payload, words, info)
        ev[1].record(stream)
        for _ in range(args.steps):
            ctx.fl_decode(hdr, payload, pw, kept, max(pad, 64), out)
        ev[2].record(stream)
        torch.cuda.synchronize()
        ems = ev[0].elapsed_time(ev[1]) / args.steps
        dms = ev[1].elapsed_time(ev[2]) / args.steps
        enc_bytes = sc.n * NCH * 4 + sc.n + bits / 8          # params + mask in, payload out
        dec_bytes = bits / 8 + kept * NCH * 4                   # payload in, parameters out
        line["codec"] = {
            "kept": kept, "payload_bits": bits, "header_bits": NCH * 72, "flags": flags,
            "bits_per_kept_gaussian": round(bits / max(kept, 1), 2),
            "encode_ms": round(ems, 4), "decode_ms": round(dms, 4),
            "encode_gbs": round(enc_bytes / (ems * 1e-3) / 1e9, 1),
            "decode_gbs": round(dec_bytes / (dms * 1e-3) / 1e9, 1),
            "encode_hbm_frac": round(enc_bytes / (ems * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "decode_hbm_frac": round(dec_bytes / (dms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
        del payload, out

        # SSIM term of the distortion (forward + gradient) on the step's image
        lss = torch.empty(1, dtype=torch.float32, device=dev)
        for _ in range(3):
            ctx.ssim_loss(rd.image, target, 0.2, lss, rd.dimage)
        ev[0].record(stream)
        for _ in range(args.steps):
            ctx.ssim_loss(rd.image, target, 0.2, lss, rd.dimage)
        ev[1].record(stream)
        torch.cuda.synchronize()
        sms = ev[0].elapsed_time(ev[1]) / args.steps
        npx = sc.views * 3 * sc.width * sc.height
        line["ssim"] = {"ms": round(sms, 4), "pixels": npx,
                        "gpix_per_s": round(npx / (sms * 1e-3) / 1e9, 2)}

        # rate-proxy variants: the range proxy from the quantizer's statistics
        # against the scale-based Laplace proxy (two passes + dense backward)
        def time_rate(proxy):
            for _ in range(3):
                ctx.rate_variant(params, q, rd.stats, lam, rd.rate3, rd.rate_grad, proxy)
                ctx.rate_variant_bwd(params, rd.grad_qparams)
            ev[0].record(stream)
            for _ in range(args.steps):
                ctx.rate_variant(params, q, rd.stats, lam, rd.rate3, rd.rate_grad, proxy)
                ctx.rate_variant_bwd(params, rd.grad_qparams)
            ev[1].record(stream)
            torch.cuda.synchronize()
            return ev[0].elapsed_time(ev[1]) / args.steps
        line["rate_variants"] = {"range_ms": round(time_rate("range"), 4),
                                 "laplace_fwd_bwd_ms": round(time_rate("laplace"), 4)}

    if not args.no_cpu_baseline and args.workload == "c2":
        line["cpu_baseline"] = cpu_baseline(sc, lam)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
