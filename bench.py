#!/usr/bin/env python
"""Benchmark of SpeedyGS's structural-formation step on one MI355X.

Default workload (``--workload c5``): the full formation iteration at
3,000,000 Gaussians (clustered: 3-component mixture) rendered in 8 views of
1600x1060 on a radius-4 ring, Gumbel-sigmoid retention mask, L1 distortion
against a seeded random target, lambda 2.5e-5, the learned rate estimator in
the loop (MLP forward + backward from the saved activation signs; the range proxy evaluated beside
it; every 100 iterations both checked against the coder's exact bits, the
plain proxy's gradient taking over while the learned estimate's error is the
larger) and Adam on (parameters, step sizes, scores) so the scene evolves.  The
same iterations with the plain range proxy are timed beside it.  Tile shape
and blend schedule come from the library's autotuner; the estimator is
trained first on the GPU on this scene's exact fixed-length coder bits.

A step = one iteration: fake-quantize + mask + channel statistics and
projection (one call), rate proxy, learned rate forward, depth sort, pair
emission, tile sort, ranges, blend, L1, blend backward, projection and
quantizer backward, learned rate backward, Adam; all in libspeedygs
kernels, no host synchronization.  Timed region: K iterations replayed from
HIP graphs, one graph per iteration of a 16-iteration period (the higher-SH
update period), launched in turn; their Gumbel-noise step and Adam step
count repeat with that period.  The evaluation counts and per-kernel times
come from re-runs of the same K iterations from the same starting state
(restored in place), outside the timed region.

Prints one JSON line.  ``value`` = E / t: Gaussian-pixel evaluations per
second, E = the method's evaluations (in-span (Gaussian, pixel) pairs before
the pixel stops) summed over the K iterations of the learned run.  Also:
the plain-proxy run, both runs enqueued eagerly, the RD step alone (forward
+ backward, graph-replayed), the rate-estimate errors against the exact coder
bits, the roofline of the dominant kernel group, the 1M-Gaussian single-view
step (``c2``) as a sub-record, the MLP / codec / SSIM / rate-variant legs at
1M, the coding stage (octree tokens and rANS, encode and decode) on the
formation's final state, and the FP64 oracle on the host on a bounded sample
of this workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X published peaks
HBM_PEAK_GBS = 8000.0
FP32_VECTOR_PEAK_TFLOPS = 157.3
# VALU issue ceiling of the per-evaluation operation counts below (one lane
# operation per op, packed FP32 not used): 256 CUs x 4 SIMDs x 16 lanes x
# 2.4 GHz
VALU_ISSUE_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
BF16_MFMA_PEAK_TFLOPS = 2500.0

NCH = 59
SH_EVERY = 16      # higher-SH coefficients updated every 16th iteration (Sec. 4.1)
# FP32 work per evaluation (counted as VALU operations, the exponential as 4):
# forward 22 + 4 (support 4, offsets 2, quadratic 6, alpha 2, thresholds 2,
# T test 2, colour 3, T 1); backward 70 + 4 (recompute, T recovery, dalpha,
# ten gradient terms, back colour, wave sums)
FLOP_PER_EVAL_FWD = 26
FLOP_PER_EVAL_BWD = 74
MLP_FLOP_PER_ROW = 2 * (64 * 128 + 128 * 128 + 128)
METRIC = "RD-step ms/iter & Gaussian-pixel evals/s (fwd+bwd), learned vs plain rate"
PERIOD = 16
CHECK = 100     # iterations between two checks of the learned rate against the coder


def _decided(decisions, use0, i):
    """Whether iteration i runs on the learned rate gradient."""
    cur = use0
    for k in sorted(decisions):
        if k > i:
            break
        cur = decisions[k]
    return cur


def group_work(g: str, n: int, V: int, P: int, E: int, W: int, H: int, items: int = 0,
               tiles: int = 0, st: int = 1, kept: int | None = None, sh_every: int = 1):
    """(bound, algorithmic amount per launch, unit) of one kernel group; E is
    the count of evaluations the blend performs (after its reach test),
    items the (splat, super-tile) items of the binning's first level, tiles
    and st the tile and super-tile counts, kept the Gaussians the mask keeps
    (the others have zero parameter gradients, which the sparse Adam
    skips), sh_every the period of the higher-SH updates (their 45 gradient
    rows are written and read only in those iterations)."""
    rows = (NCH - 45) + 45 / sh_every
    pix = V * W * H
    if g == "fakequant":          # statistics and mask (the projection quantizes)
        return "hbm", n * (NCH * 4 + 1 + 1 + 4), "B"
    if g == "preprocess":         # splat record 48 B, depth key / value / count 12 B,
        # packed tile rectangle 4 B per splat
        return "hbm", n * (NCH * 4 + 1) + V * n * (48 + 12 + 4), "B"
    if g == "depth_sort":         # four 8-bit passes, each one read + one write of key,
        # value and the packed tile rectangle carried along
        return "hbm", V * n * 4 * 24, "B"
    if g == "scan":               # sorted key, index and rectangle read (4 + 4 + 4), item
        # count written (4), item offsets scanned (4 + 4 read, 4 written); the few records
        # gathered instead of rebuilt are not counted
        return "hbm", V * n * 28, "B"
    if g == "duplicate":          # every pair written once (4 B); per item its key and
        # Gaussian index read (8 B)
        return "hbm", P * 4 + items * 8, "B"
    if g == "tile_sort":          # items emitted (sorted key, index, rectangle and item
        # offset read per splat, 8 B written per item), sorted by the super-tile in the view
        # (one 8-bit pass per 8 bits of it: 4 B histogram read, 16 B moved), keys read for
        # the tile counts (4)
        passes = max(1, -(-max(st // V - 1, 1).bit_length() // 8))
        return "hbm", V * n * 16 + items * (8 + 20 * passes + 4), "B"
    if g == "ranges":             # tile counts read, offsets and ranges written
        return "hbm", tiles * 16, "B"
    if g == "blend_fwd":
        return "alu", E * FLOP_PER_EVAL_FWD, "FLOP"
    if g == "l1":
        return "hbm", pix * 3 * 12, "B"
    if g == "grad_clear":         # records cleared, tile counts read for the large-splat slots
        return "hbm", V * n * (80 + 4), "B"
    if g == "blend_bwd":
        return "alu", E * FLOP_PER_EVAL_BWD, "FLOP"
    if g == "preprocess_bwd":     # parameters read, gradient rows written, mask and score
        # gradients written; per view the 80-byte splat gradient record and the tile count
        # (whether the splat was kept) read
        return "hbm", int(n * (NCH * 4 + rows * 4 + 4 + 4) + V * n * (80 + 4)), "B"
    if g == "fakequant_bwd":
        return "hbm", NCH * 8 * -(-n // 128), "B"
    if g == "adam":               # per iteration of the higher-SH period: the rows
        # updated (14, and the 45 higher-SH rows every sh_every-th) read as gradients for
        # every Gaussian, and y, m, v read + written for the kept ones; scores (4 B x 7)
        upd = n if kept is None else kept
        return "hbm", int(n * rows * 4 + upd * rows * 24 + n * 4 * 7), "B"
    if g in ("mlp_fwd", "mlp_bwd"):
        return "mfma", n * MLP_FLOP_PER_ROW * (1 if g == "mlp_fwd" else 2), "FLOP"
    return "hbm", 0, "B"


def roofline(g, ms, n, V, P, E, W, H, traffic_key=None, items=0, tiles=0, st=1, kept=None,
             sh_every=1):
    bound, amount, unit = group_work(g, n, V, P, E, W, H, items, tiles, st, kept, sh_every)
    dur = ms * 1e-3
    if unit == "B":
        achieved, peak, ru = amount / dur / 1e9, HBM_PEAK_GBS, "GB/s"
    elif bound == "mfma":
        achieved, peak, ru = amount / dur / 1e12, BF16_MFMA_PEAK_TFLOPS, "TFLOP/s"
    else:
        achieved, peak, ru = amount / dur / 1e12, FP32_VECTOR_PEAK_TFLOPS, "TFLOP/s"
    r = {"bound": bound, "kernel": g, "achieved": round(achieved, 3), "peak": peak,
         "unit": ru, "frac": round(achieved / peak, 5), "traffic": None,
         "algorithmic_per_launch": amount, "avg_launch_ms": round(ms, 4)}
    if bound == "alu":
        # the same count against the issue rate of single (unpacked) lane ops
        r["issue_peak_tops"] = round(VALU_ISSUE_PEAK_TOPS, 2)
        r["issue_frac"] = round(achieved / VALU_ISSUE_PEAK_TOPS, 5)
    if traffic_key:
        t = traffic_for(traffic_key)
        if t:
            r["traffic"], r["traffic_source"] = t
    return r


def traffic_for(key):
    """HBM bytes per launch measured with rocprofv3 counters for this kernel
    group, workload, tile shape and blend schedule (key "c5:group@16x16/tile"),
    valid while its sources are unchanged."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    ent = json.load(open(path)).get(key)
    if not ent:
        return None
    h = hashlib.sha256()
    for f in ent.get("kernel_files", [ent.get("kernel_file")]):
        h.update(open(os.path.join(ROOT, f), "rb").read())
    if h.hexdigest()[:16] != ent["kernel_sha256_16"]:
        return None
    return ent["bytes_per_launch"], ent["source"] + " (profiles/hbm_traffic_*.md)"


def geometry(sc, tile):
    """Tile and super-tile (8x8 tiles) counts of the scene's views."""
    gw, gh = -(-sc.width // tile[0]), -(-sc.height // tile[1])
    return {"tiles": sc.views * gw * gh, "st": sc.views * (-(-gw // 8)) * (-(-gh // 8))}


def host_info():
    model = platform.processor() or ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"cpu_model": model, "nproc": os.cpu_count(), "usable_cpus": usable}


# ---------------------------------------------------------------------------
# CPU baseline: the FP64 oracle on a bounded sample of the workload
# ---------------------------------------------------------------------------

def cpu_baseline_c5(sc, tiles_per_view=16, seed=9):
    """The oracle's render forward + backward over tiles_per_view random 16x16
    tiles per view (each tile's whole list; dL/dC a +-1/(3VHW) pattern, the
    L1 gradient's form), serial and with OpenMP over the tiles, plus the
    quantizer, mask, range proxy and the learned estimator on a
    proportional sample of Gaussians; extrapolated to the whole step."""
    import numpy as np

    import oracle
    from oracle import mlp as omlp

    n, V, W, H = sc.n, sc.views, sc.width, sc.height
    GW, GH = -(-W // 16), -(-H // 16)
    total_tiles = V * GW * GH
    rng = np.random.default_rng(seed)
    tiles = np.concatenate([v * GW * GH + np.sort(rng.choice(GW * GH, tiles_per_view,
                                                              replace=False))
                            for v in range(V)])
    frac = tiles.size / total_tiles
    t0 = time.perf_counter()
    yh, _ = oracle.fakequant(sc.params, sc.qstep, n)
    mh, ms = oracle.mask(n, 1, None, sc.score, 5, 0, 1.0)
    rp = oracle.rate_proxy(sc.params, sc.qstep, mh, n, sc.n_hat, 2.5e-5)
    t_quant = time.perf_counter() - t0
    lite = oracle.decide(yh, n, sc.cams, W, H, 16, 16, bin_pairs=False)
    t_decide = time.perf_counter() - t0 - t_quant
    p64, m64 = yh.astype(np.float64), mh.astype(np.float64)
    d = np.where(rng.random((V, 3, H, W), dtype=np.float32) < 0.5, -1.0, 1.0)
    d *= 1.0 / (3 * V * W * H)
    legs = {}
    for name, par in (("serial", False), ("openmp", True)):
        t1 = time.perf_counter()
        E, _, _ = oracle.step_tiles_sampled(p64, m64, n, sc.cams, W, H, lite, tiles, d,
                                            parallel=par)
        legs[name] = (E, time.perf_counter() - t1)
    del p64
    # learned estimator (FP64, no BF16 mirroring) on a proportional row sample
    rows = max(256, int(round(n * frac)))
    w = omlp.init_weights(3)
    idx = rng.choice(n, rows, replace=False)
    t2 = time.perf_counter()
    mmin = omlp.channel_min(sc.params, n)
    sub = np.ascontiguousarray(sc.params[:, idx])
    X = omlp.features(sub, sc.qstep, mmin, rows, mirror=False)
    f = omlp.forward(X, w, mirror=False)
    omlp.backward(X, w, np.full(rows, 1.0 / sc.n_hat), mirror=False, want_dx=True)
    t_mlp = time.perf_counter() - t2
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or host_info()["usable_cpus"]
    out = {}
    for name, (E, t) in legs.items():
        # whole step: render over every tile, estimator over every Gaussian,
        # decision layer and quantizer once
        t_step = t / frac + t_mlp * (n / rows) + t_quant + t_decide
        out[name] = {"evals_sample": E, "seconds_sample": round(t, 2),
                     "evals_per_s_sample": round(E / t, 1),
                     "step_seconds_extrapolated": round(t_step, 1),
                     "evals_per_s_step": round(E / frac / t_step, 1)}
    best = out["openmp"]
    info = host_info()
    return {"value": best["evals_per_s_step"], "unit": "Gaussian-pixel evals/s",
            "cores": threads, "kind": "oracle",
            "sample": f"FP64 oracle, render forward + backward over {tiles.size} random 16x16 "
                      f"tiles ({tiles_per_view} per view, {frac:.2%} of the pixels, whole tile "
                      f"lists), OpenMP over tiles with {threads} threads; quantizer, mask, "
                      f"range proxy and decision layer over all {n} Gaussians; learned "
                      f"estimator on {rows} Gaussians; extrapolated to one whole iteration "
                      f"(Adam not included)",
            "serial": out["serial"], "openmp": best, "cpu_model": info["cpu_model"],
            "nproc": info["nproc"], "usable_cpus": info["usable_cpus"],
            "quant_rate_s": round(t_quant, 2), "decision_layer_s": round(t_decide, 2),
            "mlp_sample_s": round(t_mlp, 3), "rate_R": rp["R"], "f_mean": float(f.mean())}


def cpu_baseline_c2(sc, lam):
    """The FP64 oracle, as it stands, on the same workload: one full step
    (forward + backward) of the 1M-Gaussian scene, single-threaded."""
    import oracle
    t0 = time.perf_counter()
    r = oracle.rd_step(sc.params, sc.qstep, sc.score, sc.given_mask, sc.cams, sc.width,
                       sc.height, sc.target, sc.n, sc.n_hat, lam)
    dt = time.perf_counter() - t0
    E = r["fw"]["evals"]
    info = host_info()
    return {"value": E / dt, "unit": "Gaussian-pixel evals/s", "cores": 1, "kind": "oracle",
            "sample": f"one full RD step (fwd+bwd) of the measured workload, "
                      f"{E} evals in {dt:.1f} s, single thread",
            "s_per_step": round(dt, 3), "cpu_model": info["cpu_model"], "nproc": info["nproc"]}


# ---------------------------------------------------------------------------
# c5: the formation iteration, learned vs plain rate
# ---------------------------------------------------------------------------

def bench_formation(args, sc, ctx, stream, dev, t):
    import numpy as np
    import torch

    from paper_2607_12656_amd import autotune
    from paper_2607_12656_amd.formation import Formation
    from paper_2607_12656_amd.rate_train import RateTrainer
    from paper_2607_12656_amd.rd import RDStep

    lam = 2.5e-5
    K, W = args.steps, args.warmup
    p0, q0, s0, target = t(sc.params), t(sc.qstep), t(sc.score), t(sc.target)
    mask = t(sc.given_mask)
    say(f"c5: scene {sc.n} x {sc.views} views {sc.width}x{sc.height} resident")

    # tile shape and blend schedule: the library's tuner on the plain step
    # (or fixed by --tile / --schedule, e.g. for counter runs, whose overhead
    # would steer the tuner)
    ctx.set_scene(sc.n, sc.npad, sc.n_hat, sc.cams, sc.width, sc.height)
    if args.tile and args.tile != "auto":
        tile = tuple(int(v) for v in args.tile.split("x"))
        schedule = args.schedule or "tile"
        tune = {"tile": tile, "schedule": schedule, "ms": None}
    else:
        tune = autotune.tune_native(ctx, p0, q0, mask, target, sc.n, sc.views, sc.width,
                                    sc.height, reps=2)
        tile, schedule = tune["tile"], tune["schedule"]
    say(f"c5: tuned {tile} {schedule}")
    rd = RDStep(ctx, sc.n, sc.npad, sc.n_hat, sc.cams, sc.width, sc.height, tile=tile,
                schedule=schedule, fused=True)

    # the estimator, trained on this scene's own coder bits (GPU only)
    t0 = time.perf_counter()
    trainer = RateTrainer(ctx, rd, p0, s0, sc.given_mask, seed=3, scenes=64)
    theta, packed, losses = trainer.train(steps=400)
    err_l, err_p = trainer.held_out_errors(theta, packed)
    train_s = time.perf_counter() - t0
    del trainer
    say(f"c5: estimator trained in {train_s:.1f} s")
    rd.forward(p0, q0, s0, target, lam, 1, None, 5, 0, count_evals=False)
    P0, _ = ctx.query()
    ctx.reserve_pairs(P0 + P0 // 2 + 4096)     # the scene moves; the count is checked after

    runs = {}
    for name, mlp in (("learned", (packed, theta)), ("plain", None)):
        p, q, s = p0.clone(), q0.clone(), s0.clone()
        f = Formation(rd, p, q, s, target, lam, mask_mode=1, seed=5, mlp=mlp,
                      sh_every=SH_EVERY)
        e_first = f.check_rate()                # the fallback rule's check before the run
        for _ in range(W):
            f.iterate()
        torch.cuda.synchronize()
        start = f.snapshot()
        use0 = f.use_learned
        # one graph per iteration of the 16-iteration period, for each rate
        # gradient the fallback rule can select (learned, plain)
        graphs = {}
        for v in ((True, False) if mlp is not None else (False,)):
            f.use_learned = v
            for j in range(PERIOD):
                ctx.graph_begin()
                f.iterate()
                graphs[(v, j)] = ctx.graph_end()
            f.restore(start)
        f.use_learned = use0
        for j in range(2):                      # first launches outside the timed region
            graphs[(use0, j)].launch(stream)
        torch.cuda.synchronize()
        f.restore(start)
        torch.cuda.synchronize()
        # the fallback rule: every CHECK iterations both estimates against the
        # coder's exact bits (one synchronization each, inside the timed
        # region); the graphs of the rate gradient it selects run next
        decisions = {}
        t0 = time.perf_counter()
        for i in range(K):
            if mlp is not None and (start[1] + i) % CHECK == 0:
                f.k = start[1] + i % PERIOD     # the noise step of the next graph
                f.check_rate()
                decisions[i] = f.use_learned
            graphs[(f.use_learned, i % PERIOD)].launch(stream)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        ctx.query()                             # raises if the reserved capacity overflowed
        learned_iters = sum(1 for i in range(K) if _decided(decisions, use0, i))

        def rerun(count_evals=False, check=False):
            """The same K iterations from the start, eagerly, with the timed
            run's fallback decisions (checks issued too when check)."""
            f.restore(start)
            f.use_learned = use0
            for i in range(K):
                if i in decisions:
                    if check:
                        f.check_rate()
                    f.use_learned = decisions[i]
                f.iterate(count_evals=count_evals)

        # the same iterations enqueued eagerly (no profiling)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rerun(check=True)
        torch.cuda.synchronize()
        dt_eager = time.perf_counter() - t0
        if name == "learned":     # the state the coding stage takes over
            coding_in = (f.params.clone(), f.q.clone(), rd.hard.clone())
        # re-runs from the same state: the method's evaluations, the blend's
        # evaluations after its reach test, per-kernel times
        counts = {}
        for mode in (0, 1):
            ctx.set_eval_count_mode(mode)
            rd.evals.zero_()
            rerun(count_evals=True)
            torch.cuda.synchronize()
            counts[mode] = int(rd.evals.item())
        ctx.set_eval_count_mode(0)
        ctx.profile_enable(True)
        rerun()
        prof = ctx.profile_read()
        ctx.profile_enable(False)
        pairs, _ = ctx.query()
        items = ctx.query_items()
        bits, kept, e_plain, e_learn = f.rate_errors()
        for g in graphs.values():
            g.close()
        kernels = {g: round(tot / cnt, 4) for g, (tot, cnt) in prof.items() if cnt}
        E, Er = counts[0], counts[1]
        runs[name] = {"ms_per_step": round(dt * 1e3 / K, 4), "value": round(E / dt, 1),
                      "eager_ms_per_step": round(dt_eager * 1e3 / K, 4),
                      "evals": E, "evals_after_reach_test": Er, "pairs_last": pairs,
                      "items_last": items,
                      "kept_last": kept, "coder_bits_last": bits,
                      "plain_proxy_error": round(e_plain, 4),
                      "learned_error": None if e_learn is None else round(e_learn, 4),
                      "rate_check_before_run": {"plain_error": round(e_first[0], 4),
                                                "learned_error": None if e_first[1] is None
                                                else round(e_first[1], 4),
                                                "learned_used": use0},
                      "fallback_rule": None if mlp is None else {
                          "check_every": CHECK, "checks": len(decisions),
                          "iterations_on_learned_gradient": learned_iters,
                          "iterations_on_plain_gradient": K - learned_iters,
                          "checks_detail": [[int(k), round(a, 4), None if b is None
                                             else round(b, 4), bool(u)]
                                            for k, a, b, u in f.checks[1:1 + len(decisions)]]},
                      "kernel_ms": kernels}
        say(f"c5 {name}: {runs[name]['ms_per_step']} ms/iter (graph), "
            f"{runs[name]['eager_ms_per_step']} eager")
        del f, start

    # the RD step alone (forward + backward, no optimizer), graph-replayed
    rd_only = {}
    R = torch.zeros(1, dtype=torch.float32, device=dev)
    for name in ("learned", "plain"):
        c = ctx

        def rd_step():
            c.quant_render_fwd(p0, q0, s0, 1, None, 5, 0, rd.hard, rd.soft, rd.stats, rd.image,
                               rd.final_T, rd.last, None)
            if name == "learned":
                c.rate_proxy(rd.stats, q0, 0.0, rd.rate3, None)
                c.rate_mlp_fwd(packed, theta, p0, q0, rd.stats, rd.hard, R, None)
            else:
                c.rate_proxy(rd.stats, q0, lam, rd.rate3, rd.rate_grad)
            c.l1_loss(rd.image, target, rd.loss, rd.dimage)
            learned = name == "learned"
            c.quant_render_bwd(p0, q0, rd.soft, 1, None if learned else rd.rate_grad,
                               None if learned else rd.stats, rd.final_T, rd.last, rd.dimage,
                               rd.grad_qparams, rd.grad_q, rd.grad_score, rd.grad_mask)
            if learned:
                c.rate_mlp_bwd(packed, theta, p0, q0, rd.stats, rd.hard, rd.soft, 1, lam,
                               rd.grad_qparams, rd.grad_q, rd.grad_score, None)
        ctx.graph_begin()
        rd_step()
        g = ctx.graph_end()
        for _ in range(2):
            g.launch(stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(K):
            g.launch(stream)
        torch.cuda.synchronize()
        rd_only[name] = round((time.perf_counter() - t0) * 1e3 / K, 4)
        g.close()
    ctx.query()

    coding = None
    if not args.no_coding:
        coding = bench_coding(ctx, dev, *coding_in, sc.n, sc.npad)
    del coding_in

    L = runs["learned"]
    geo = geometry(sc, tile)
    dom = max(L["kernel_ms"], key=L["kernel_ms"].get)
    roof = roofline(dom, L["kernel_ms"][dom], sc.n, sc.views, L["pairs_last"],
                    L["evals_after_reach_test"] // K, sc.width, sc.height,
                    traffic_key=f"c5:{dom}@{tile[0]}x{tile[1]}/{schedule}",
                    items=L["items_last"], sh_every=SH_EVERY, **geo)
    groups = {g: roofline(g, ms, sc.n, sc.views, L["pairs_last"],
                          L["evals_after_reach_test"] // K, sc.width, sc.height,
                          items=L["items_last"], kept=L["kept_last"], sh_every=SH_EVERY,
                          **geo)
              for g, ms in L["kernel_ms"].items()}
    line = {
        "metric": METRIC, "value": L["value"], "unit": "Gaussian-pixel evals/s", "n_gpus": 1,
        "steps": K, "warmup": W, "ms_per_step": L["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"c5: full formation iteration, {sc.n} Gaussians (clustered), "
                               f"{sc.views} views {sc.width}x{sc.height}, Gumbel-sigmoid mask, "
                               f"learned rate in the loop (forward + backward), fallback rule every {CHECK} iterations, "
                               f"Adam on parameters / steps / scores (higher SH every 16th, "
                               f"sparse), lambda {lam}, tile {tile[0]}x{tile[1]} "
                               f"({schedule} schedule, " + ("autotuned)" if tune["ms"] else "fixed)"),
                   "gaussians": sc.n, "views": sc.views, "width": sc.width,
                   "height": sc.height, "tile": f"{tile[0]}x{tile[1]}", "schedule": schedule,
                   "mlp_weights": "trained on the GPU on this scene's fixed-length coder "
                                  "bits (64 step vectors 2^U[-9,-3], 400 steps of 65,536 "
                                  "rows)"},
        "timing": "K iterations replayed from HIP graphs (one per iteration of the 16-"
                  "iteration higher-SH period, launched in turn), host clock around the "
                  "replays between two synchronizations; in the learned run the fallback "
                  "rule checks both rate estimates against the coder's exact bits every "
                  f"{CHECK} iterations (inside the timed region) and the graphs of the "
                  "gradient it selects run next; evaluation counts and kernel times from "
                  "re-runs of the same K iterations from the same state with the same "
                  "decisions",
        "roofline": roof,
        "group_roofline": {g: {k: r[k] for k in ("bound", "achieved", "unit", "frac")}
                           for g, r in groups.items()},
        "learned": L, "plain": runs["plain"],
        "learned_over_plain_time": round(L["ms_per_step"] / runs["plain"]["ms_per_step"], 4),
        "rd_step_graph_ms": rd_only,
        "autotune_ms": tune["ms"],
        "coding": coding,
        "mlp_training": {"seconds": round(train_s, 2), "loss": [round(v, 2) for v in losses],
                         "held_out_error_learned": round(err_l, 4),
                         "held_out_error_plain": round(err_p, 4)},
    }
    del rd
    return line


# ---------------------------------------------------------------------------
# c2 / c3: the plain RD step (forward + backward, no optimizer)
# ---------------------------------------------------------------------------

def bench_rd(args, sc, ctx, stream, dev, t, extras: bool, tile, schedule, tune=None):
    import numpy as np
    import torch

    from paper_2607_12656_amd.rd import RDStep

    lam = 2.5e-5
    steps = args.steps
    params, q, score = t(sc.params), t(sc.qstep), t(sc.score)
    mask, target = t(sc.given_mask), t(sc.target)
    rd = RDStep(ctx, sc.n, sc.npad, sc.n_hat, sc.cams, sc.width, sc.height, tile=tile,
                schedule=schedule, fused=True)

    def plain_step(count=False):
        rd.forward(params, q, score, target, lam, 0, mask, 0, 0, count_evals=count)
        rd.backward(params, q, 0)

    counts = {}
    for mode in (0, 1):
        ctx.set_eval_count_mode(mode)
        rd.evals.zero_()
        plain_step(count=True)
        torch.cuda.synchronize()
        counts[mode] = int(rd.evals.item())
    ctx.set_eval_count_mode(0)
    E, Er = counts[0], counts[1]
    P, _ = ctx.query()
    ctx.reserve_pairs(P + P // 8 + 4096)      # no host synchronization inside a step
    for _ in range(args.warmup):
        plain_step()
    ctx.query()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        plain_step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    ctx.profile_enable(True)
    for _ in range(steps):
        plain_step()
    prof = ctx.profile_read()
    ctx.profile_enable(False)
    kernels = {g: round(tot / cnt, 4) for g, (tot, cnt) in prof.items() if cnt}
    ctx.graph_begin()
    plain_step()
    graph = ctx.graph_end()
    for _ in range(max(args.warmup, 2)):
        graph.launch(stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        graph.launch(stream)
    torch.cuda.synchronize()
    gms = (time.perf_counter() - t0) * 1e3 / steps
    ctx.query()
    graph.close()
    items = ctx.query_items()
    geo = geometry(sc, tile)
    dom = max(kernels, key=kernels.get)
    roof = roofline(dom, kernels[dom], sc.n, sc.views, P, Er, sc.width, sc.height,
                    traffic_key=f"{args.workload if args.workload != 'c5' else 'c2'}:{dom}"
                                f"@{tile[0]}x{tile[1]}/{schedule}",
                    items=items, **geo)
    groups = {g: roofline(g, ms, sc.n, sc.views, P, Er, sc.width, sc.height, items=items, **geo)
              for g, ms in kernels.items()}
    line = {
        "metric": METRIC, "value": round(E / (gms * 1e-3), 1), "unit": "Gaussian-pixel evals/s",
        "ms_per_step": round(gms, 4),
        "config": {"workload": f"plain RD step, {sc.n} Gaussians (clustered), {sc.views} "
                               f"view(s) {sc.width}x{sc.height}, 20% pruned, lambda 2.5e-5, "
                               f"tile {tile[0]}x{tile[1]}",
                   "gaussians": sc.n, "views": sc.views, "width": sc.width,
                   "height": sc.height, "tile": f"{tile[0]}x{tile[1]}", "schedule": schedule,
                   "pairs": P, "items": items, "evals_per_step": E,
                   "evals_after_reach_test": Er},
        "roofline": roof,
        "group_roofline": {g: {k: r[k] for k in ("bound", "achieved", "unit", "frac")}
                           for g, r in groups.items()},
        "kernel_ms": kernels,
        "timing": "HIP-graph replays of the whole step; eager_ms_per_step: the same calls "
                  "enqueued by the host each step (no profiling); kernel_ms: HIP events on "
                  "the library's stream in a separate run",
        "eager_ms_per_step": round(ms, 4),
    }
    if tune is not None:
        line["autotune_ms"] = tune["ms"]
    if extras:
        line.update(extra_legs(args, sc, ctx, rd, stream, dev, params, q, score, mask, target,
                               E, ms))
    del rd
    return line


def extra_legs(args, sc, ctx, rd, stream, dev, params, q, score, mask, target, E, plain_ms):
    import torch
    lam = 2.5e-5
    out = {}
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
    t0 = time.perf_counter()
    for _ in range(args.steps):
        learned_step()
    torch.cuda.synchronize()
    lms = (time.perf_counter() - t0) * 1e3 / args.steps
    ctx.profile_enable(True)
    for _ in range(args.steps):
        learned_step()
    lprof = ctx.profile_read()
    ctx.profile_enable(False)
    ctx.query()
    lk = {g: round(tot / cnt, 4) for g, (tot, cnt) in lprof.items() if cnt}
    mf = lk.get("mlp_fwd", 0.0)
    out["learned_rate"] = {
        "ms_per_step": round(lms, 4), "value": round(E / (lms * 1e-3), 1),
        "mlp_fwd_ms": mf, "mlp_bwd_ms": lk.get("mlp_bwd", 0.0),
        "mlp_fwd_tflops": round(sc.n * MLP_FLOP_PER_ROW / (mf * 1e-3) / 1e12, 2) if mf else None,
        "plain_ms_per_step": round(plain_ms, 4), "timing": "eager, both"}

    # MLP alone: one training step on 65,536 rows, inference over 3M rows
    B = 65536
    Xtr = torch.randint(0, 1 << 14, (B, 64), dtype=torch.int16, device=dev)
    ttr = torch.rand(B, device=dev) * 100 + 200
    m_, v_, g_ = torch.zeros_like(theta), torch.zeros_like(theta), torch.empty_like(theta)
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
    out["mlp"] = {
        "train_step_ms_65536_rows": round(tms, 4),
        "train_tflops": round(3 * B * MLP_FLOP_PER_ROW / (tms * 1e-3) / 1e12, 2),
        "infer_ms_3M_rows": round(ims, 4),
        "infer_tflops": round(Ni * MLP_FLOP_PER_ROW / (ims * 1e-3) / 1e12, 2),
        "infer_mfma_frac": round(Ni * MLP_FLOP_PER_ROW / (ims * 1e-3) / 1e12
                                 / BF16_MFMA_PEAK_TFLOPS, 4)}
    del Xin, fo, Xtr, scratch

    # fixed-length coding of the kept Gaussians (the pruned step's mask)
    rd.forward(params, q, score, target, lam, 0, mask, 0, 0, count_evals=False)
    words = sc.n * NCH + 64
    hdr = torch.empty((NCH, 3), dtype=torch.int32, device=dev)
    payload = torch.empty(words, dtype=torch.int32, device=dev)
    info = torch.empty(3, dtype=torch.int64, device=dev)
    ctx.fl_encode(params, q, rd.hard, hdr, payload, words, info)
    torch.cuda.synchronize()
    bits, kept, flags = (int(v) for v in info.cpu())
    pad = (kept + 63) // 64 * 64
    outp = torch.empty((NCH, max(pad, 64)), dtype=torch.float32, device=dev)
    pw = (bits + 31) // 32 + 1
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    for _ in range(3):
        ctx.fl_encode(params, q, rd.hard, hdr, payload, words, info)
        ctx.fl_decode(hdr, payload, pw, kept, max(pad, 64), outp)
    ev[0].record(stream)
    for _ in range(args.steps):
        ctx.fl_encode(params, q, rd.hard, hdr, payload, words, info)
    ev[1].record(stream)
    for _ in range(args.steps):
        ctx.fl_decode(hdr, payload, pw, kept, max(pad, 64), outp)
    ev[2].record(stream)
    torch.cuda.synchronize()
    ems = ev[0].elapsed_time(ev[1]) / args.steps
    dms = ev[1].elapsed_time(ev[2]) / args.steps
    enc_bytes = sc.n * NCH * 4 + sc.n + bits / 8
    dec_bytes = bits / 8 + kept * NCH * 4
    out["codec"] = {
        "kept": kept, "payload_bits": bits, "header_bits": NCH * 72, "flags": flags,
        "bits_per_kept_gaussian": round(bits / max(kept, 1), 2),
        "encode_ms": round(ems, 4), "decode_ms": round(dms, 4),
        "encode_gbs": round(enc_bytes / (ems * 1e-3) / 1e9, 1),
        "decode_gbs": round(dec_bytes / (dms * 1e-3) / 1e9, 1),
        "encode_hbm_frac": round(enc_bytes / (ems * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "decode_hbm_frac": round(dec_bytes / (dms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    del payload, outp

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
    out["ssim"] = {"ms": round(sms, 4), "pixels": npx,
                   "gpix_per_s": round(npx / (sms * 1e-3) / 1e9, 2)}

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
    out["rate_variants"] = {"range_ms": round(time_rate("range"), 4),
                            "laplace_fwd_bwd_ms": round(time_rate("laplace"), 4)}
    return out


def say(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def bench_coding(ctx, dev, params, q, hard, n, npad, reps=10, lane_len=256):
    """Learned-coding stage, lossless parts, on the formation's final state:
    octree tokens of the kept positions, their order-1 count model and rANS
    stream (encode), then the decode back to tokens, voxels and positions.
    Two position steps: the formation's own, and 2^-12 (a deep tree).  Timed
    eagerly (host clock around reps calls between synchronizations; the
    coder allocates its scratch on first use, outside the timed calls);
    per-group times from the library's event profile."""
    import numpy as np
    import torch

    S = lane_len
    res = {}
    cap = (21 * n + 3) // 4 * 4
    tokens = torch.empty(cap, dtype=torch.uint8, device=dev)
    codes = torch.empty(n, dtype=torch.int64, device=dev)
    di = torch.empty(n, dtype=torch.int32, device=dev)
    dc = torch.empty(n, dtype=torch.int32, device=dev)
    hdr = torch.empty(30, dtype=torch.int64, device=dev)
    freq = torch.empty(257 * 256, dtype=torch.int16, device=dev)
    bits = torch.empty(1, dtype=torch.float64, device=dev)
    info = torch.empty(2, dtype=torch.int64, device=dev)
    dinfo = torch.empty(1, dtype=torch.int64, device=dev)
    oinfo = torch.empty(1, dtype=torch.int64, device=dev)
    for label, qpos in (("formation_steps", None), ("position_step_2^-12", 2.0 ** -12)):
        qq = q.clone()
        if qpos is not None:
            qq[:3] = qpos
        ctx.octree_encode(params, npad, n, qq, hard, tokens, codes, di, dc, hdr)
        h = hdr.cpu().numpy()
        T, m, kept = int(h[6]), int(h[5]), int(h[4])
        assert h[8] == 0, f"octree flags {h[8]}"
        tok = tokens[:T]
        nb = (T + 64 * S - 1) // (64 * S)
        wcap = ctx.ans_max_words(T, S)
        words = torch.empty(wcap, dtype=torch.int16, device=dev)
        off = torch.empty(nb + 1, dtype=torch.int64, device=dev)

        def encode():
            ctx.octree_encode(params, npad, n, qq, hard, tokens, codes, di, dc, hdr)
            ctx.ans_model(tok, T, 1, S, freq, bits)
            ctx.ans_encode(tok, T, 1, S, freq, words, off, info)

        encode()
        torch.cuda.synchronize()
        W = int(info[0].item())
        assert int(info[1].item()) == 0
        header = ctx.octree_header(h)
        out_tok = torch.empty(T, dtype=torch.uint8, device=dev)
        codes2 = torch.empty(max(m, 1), dtype=torch.int64, device=dev)
        xyz = torch.empty((3, max(kept, 1)), dtype=torch.float32, device=dev)

        def decode():
            ctx.ans_decode(words, W, off, T, 1, S, freq, out_tok, dinfo)
            ctx.octree_decode(header, out_tok, di, dc, qq, codes2, xyz, max(kept, 1), oinfo)

        decode()
        torch.cuda.synchronize()
        assert int(dinfo.item()) == 0 and int(oinfo.item()) == 0
        assert torch.equal(out_tok, tok) and torch.equal(codes2[:m], codes[:m])
        timed = {}
        for name, fn in (("encode", encode), ("decode", decode)):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                fn()
            torch.cuda.synchronize()
            timed[name] = (time.perf_counter() - t0) * 1e3 / reps
            ctx.profile_enable(True)
            for _ in range(reps):
                fn()
            prof = ctx.profile_read()
            ctx.profile_enable(False)
            timed[name + "_groups"] = {g: round(prof[g][0] / reps, 4) for g in ("octree", "ans")}
        nz = int(torch.count_nonzero(freq).item())
        res[label] = {
            "kept": kept, "voxels": m, "depth": int(h[0]), "tokens": T, "dups": int(h[7]),
            "lane_len": S, "blocks": nb, "words": W,
            "bits_per_kept_gaussian": round(16.0 * W / max(kept, 1), 4),
            "ideal_bits_R_geo": round(float(bits.item()), 1),
            "model_entries": nz,
            "encode_ms": round(timed["encode"], 4), "decode_ms": round(timed["decode"], 4),
            "encode_group_ms": timed["encode_groups"], "decode_group_ms": timed["decode_groups"],
            "decode_tokens_per_s": round(T / (timed["decode"] * 1e-3), 1),
        }
        say(f"coding {label}: {T} tokens, {W} words, decode {timed['decode']:.3f} ms")
        if qpos is None:
            res[label]["attributes"] = bench_attributes(ctx, dev, params, q, hard, n, npad, header,
                                                        codes, m, kept, xyz, reps, S)
            res[label]["attributes"]["geometry_and_attributes_decode_ms"] = round(
                timed["decode"] + res[label]["attributes"]["decode_ms"], 4)
            res[label]["container"] = bench_container(ctx, dev, params, q, hard, n, npad, kept,
                                                      S)
    return res


def bench_container(ctx, dev, params, q, hard, n, npad, kept, S):
    """The whole coding-stage stream as bytes (headers, model tables, rANS
    words): its size against the fixed-length coder's, and the wall time of
    encoding into a host byte string and decoding from one (host-device
    transfers included, unlike the device-resident decode times above)."""
    import numpy as np
    import torch

    from paper_2607_12656_amd.coding import decode_scene, encode_scene

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    data, sizes = encode_scene(ctx, params, npad, n, q, hard, S)
    t_enc = time.perf_counter() - t0
    decode_scene(ctx, data, dev)           # first call allocates the decoder's scratch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    scene = decode_scene(ctx, data, dev)
    torch.cuda.synchronize()
    t_dec = time.perf_counter() - t0
    fh = torch.empty((59, 3), dtype=torch.int32, device=dev)
    payload = torch.empty(59 * n + 64, dtype=torch.int32, device=dev)
    info = torch.empty(3, dtype=torch.int64, device=dev)
    ctx.fl_encode(params, q, hard, fh, payload, payload.numel(), info)
    fl_bits = int(info[0].item()) + 59 * 72
    assert scene.shape[1] == kept
    say(f"coding container: {len(data)} bytes, decode from host {t_dec * 1e3:.2f} ms")
    return {"bytes": len(data), "parts": sizes,
            "bits_per_kept_gaussian": round(8.0 * len(data) / max(kept, 1), 3),
            "fixed_length_coder_bits": fl_bits,
            "size_vs_fixed_length": round(8.0 * len(data) / fl_bits, 4),
            "encode_to_host_s": round(t_enc, 3), "decode_from_host_ms": round(t_dec * 1e3, 3)}


def bench_attributes(ctx, dev, params, q, hard, n, npad, oheader, codes, m, kept, xyz, reps, S):
    """Attribute half of the coding stage on the same state: Morton order,
    the per-channel predictor choice (previous token or none, by ideal bits),
    byte planes per channel, an order-0 rANS stream per plane (encode);
    all planes decoded in one launch, the scene rows rebuilt, and the
    positional embedding of the decoded positions (L = 12 bands, d = 32, seeded
    weights; decode).  Also the planes' ideal bits in Gaussian index order,
    against which the Morton order's gain shows."""
    import numpy as np
    import torch

    from paper_2607_12656_amd.coding import choose_predictors

    fh = torch.empty((59, 3), dtype=torch.int32, device=dev)
    payload = torch.empty(59 * n + 64, dtype=torch.int32, device=dev)
    finfo = torch.empty(3, dtype=torch.int64, device=dev)
    ctx.fl_encode(params, q, hard, fh, payload, payload.numel(), finfo)
    fl = ctx.fl_header_host(fh.cpu().numpy())
    fl_bits = int(finfo[0].item()) + 59 * 72
    perm = torch.empty(max(kept, 1), dtype=torch.int32, device=dev)
    ctx.morton_order(params, npad, n, q, hard, oheader, codes, perm)
    pred, bits_chosen, bits_all_prev = choose_predictors(ctx, params, npad, perm, kept, fl, S)
    rows = ctx.attr_plane_rows(fl, pred)
    planes = torch.empty((max(rows, 1), max(kept, 1)), dtype=torch.uint8, device=dev)
    nb = (kept + 64 * S - 1) // (64 * S)
    cap = ctx.ans_max_words(kept, S)
    freqs = torch.empty((max(rows, 1), 257 * 256), dtype=torch.int16, device=dev)
    words = torch.empty((max(rows, 1), cap), dtype=torch.int16, device=dev)
    offs = torch.empty((max(rows, 1), nb + 1), dtype=torch.int64, device=dev)
    infos = torch.empty((max(rows, 1), 2), dtype=torch.int64, device=dev)
    bits = torch.empty(max(rows, 1), dtype=torch.float64, device=dev)

    def encode(order_perm=None):
        if order_perm is None:
            ctx.morton_order(params, npad, n, q, hard, oheader, codes, perm)
            p = perm
            choose_predictors(ctx, params, npad, p, kept, fl, S)   # (the same choice)
        else:
            p = order_perm
        ctx.attr_planes(params, npad, p, kept, fl, S, planes, pred)
        for t in range(rows):
            ctx.ans_model(planes[t], kept, 0, S, freqs[t], bits[t:t + 1])
            ctx.ans_encode(planes[t], kept, 0, S, freqs[t], words[t], offs[t], infos[t])

    encode()
    torch.cuda.synchronize()
    inf = infos.cpu().numpy()[:rows]
    assert np.all(inf[:, 1] == 0)
    nwords = inf[:, 0].astype(np.int64)
    ideal_morton = float(bits[:rows].sum().item())
    out = torch.empty((59, max(kept, 1)), dtype=torch.float32, device=dev)
    dplanes = torch.empty_like(planes)
    dinfo = torch.empty(max(rows, 1), dtype=torch.int64, device=dev)
    streams = [dict(words=words[t], n_words=int(nwords[t]), block_off=offs[t], n=kept,
                    freq=freqs[t], sym=dplanes[t], order=0, lane_len=S) for t in range(rows)]
    g = torch.Generator().manual_seed(12)
    Wpe = (torch.randn((32, 75), generator=g) * 0.1).to(dev)
    bpe = (torch.randn(32, generator=g) * 0.1).to(dev)
    pe = torch.empty((max(kept, 1), 32), dtype=torch.float32, device=dev)

    def decode():
        ctx.ans_decode_multi(streams, dinfo)
        ctx.attr_reconstruct(dplanes, kept, fl, S, out, max(kept, 1), pred)
        ctx.positional_embedding(xyz, max(kept, 1), kept, 12, 32, Wpe, bpe, pe)

    decode()
    torch.cuda.synchronize()
    assert int(dinfo[:rows].abs().sum().item()) == 0
    assert torch.equal(dplanes[:rows], planes[:rows])
    timed = {}
    for name, fn in (("encode", encode), ("decode", decode)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        timed[name] = (time.perf_counter() - t0) * 1e3 / reps
    # decode pieces, from the library's event profile
    ctx.profile_enable(True)
    for _ in range(reps):
        decode()
    prof = ctx.profile_read()
    ctx.profile_enable(False)
    # the same planes in Gaussian index order
    idx = torch.nonzero(hard[:n]).reshape(-1).to(torch.int32)
    encode(idx)
    torch.cuda.synchronize()
    ideal_index = float(bits[:rows].sum().item())
    words_total = int(nwords.sum())
    res = {
        "channels": 56, "plane_rows": rows, "lane_len_W": S, "groups_G": (kept + S - 1) // S,
        "words": words_total,
        "bits_per_kept_gaussian": round(16.0 * words_total / max(kept, 1), 3),
        "ideal_bits_R_attr_morton_order": round(ideal_morton, 1),
        "channels_with_prediction": int(pred[3:].sum()),
        "ideal_bits_prediction_everywhere": round(bits_all_prev, 1),
        "ideal_bits_index_order": round(ideal_index, 1),
        "morton_over_index_bits": round(ideal_morton / max(ideal_index, 1.0), 4),
        "fixed_length_coder_bits_all_channels": fl_bits,
        "encode_ms": round(timed["encode"], 4), "decode_ms": round(timed["decode"], 4),
        "decode_group_ms": {"ans_planes_and_reconstruction_and_pe":
                            round(prof["ans"][0] / reps, 4)},
        "pe": "L = 12 power-of-two bands, d = 32, seeded weights (no trained model here)",
    }
    say(f"coding attributes: {rows} planes, {words_total} words, decode {timed['decode']:.3f} ms")
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default: 1000 iterations for c5, 20 otherwise)")
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="c5", choices=("c5", "c2", "c3"),
                    help="c5: the formation iteration at 3M Gaussians x 8 views of 1600x1060, "
                         "learned vs plain rate (default); c2: the plain RD step at 1M, one "
                         "1297x840 view; c3: the plain RD step at 3M x 8 views")
    ap.add_argument("--tile", default=None,
                    help="16x16 | 8x8 | 32x8 | auto (default: auto for c3 / c5, 16x16 for c2)")
    ap.add_argument("--schedule", default=None, choices=("tile", "stride", "queue", "block"))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the 1M sub-record's MLP / codec / SSIM / rate-variant legs")
    ap.add_argument("--no-c2", action="store_true", help="c5 only: skip the 1M sub-record")
    ap.add_argument("--no-coding", action="store_true",
                    help="c5 only: skip the coding-stage leg (octree tokens, rANS)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run one plain 256 MiB device copy first (scale for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the step runs on one GPU; --gpus must be 1 (sharding "
                                   "over GPUs is not implemented)"}))
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    from paper_2607_12656_amd import Context

    if args.steps is None:
        args.steps = 1000 if args.workload == "c5" else 20
    dev = torch.device("cuda", 0)
    stream = torch.cuda.Stream(dev)
    torch.cuda.set_stream(stream)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    ctx = Context(0, stream=stream)
    if args.calibrate_copy:
        src = torch.ones(64 << 20, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    if args.workload == "c5":
        sc = synth.make_scene("c3")
        line = bench_formation(args, sc, ctx, stream, dev, t)
        torch.cuda.synchronize()
        if not args.no_c2:
            sc2 = synth.make_scene("c2")
            sub = argparse.Namespace(**vars(args))
            sub.steps = min(args.steps, 20)
            line["c2"] = bench_rd(sub, sc2, ctx, stream, dev, t, not args.no_extras, (16, 16),
                                  "block")
            say("c2 sub-record done")
            del sc2
        if not args.no_cpu_baseline:
            line["cpu_baseline"] = cpu_baseline_c5(sc)
            say("cpu baseline done")
    else:
        sc = synth.make_scene(args.workload)
        tune = None
        choice = args.tile or ("16x16" if args.workload == "c2" else "auto")
        if choice == "auto":
            from paper_2607_12656_amd import autotune
            ctx.set_scene(sc.n, sc.npad, sc.n_hat, sc.cams, sc.width, sc.height)
            tune = autotune.tune_native(ctx, t(sc.params), t(sc.qstep), t(sc.given_mask),
                                        t(sc.target), sc.n, sc.views, sc.width, sc.height,
                                        reps=2)
            tile, schedule = tune["tile"], tune["schedule"]
        else:
            tile = tuple(int(v) for v in choice.split("x"))
            schedule = args.schedule or ("block" if args.workload == "c2" else "tile")
        line = bench_rd(args, sc, ctx, stream, dev, t, not args.no_extras, tile, schedule, tune)
        line.update({"n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
                     "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
                     "dtype": "f32", "data": "synthetic"})
        line["config"]["workload"] = f"{args.workload}: " + line["config"]["workload"]
        if not args.no_cpu_baseline and args.workload == "c2":
            line["cpu_baseline"] = cpu_baseline_c2(sc, 2.5e-5)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
