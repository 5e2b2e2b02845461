"""Autotuner for the RD step: tile shape, then blend schedule.

``tune_native`` calls the library's own tuner (``sgs_autotune``: the whole
step timed per candidate inside the library, the context left bound with the
choice); ``tune`` times any caller-supplied step function the same way.

The support rule is pixel-exact, so every candidate tile shape renders the
same image and gradients, and the blend schedule (one workgroup per 8x8
sub-tile, or resident workgroups over the sub-tiles of the tiles ordered by
list length, striding or taking them from an atomic queue, or resident
workgroups of one whole tile each striding over that order) only changes
which wave blends which sub-tile: the tuner may pick on speed alone.  The tile shapes are timed with the
per-tile schedule, then the schedules with the best shape.  Each candidate is
timed over whole forward + backward steps with HIP events on the step's
stream; results are cached per (device, N, views, width, height) in a JSON
file.
"""
from __future__ import annotations

import json
import os

CANDIDATES = ((16, 16), (8, 8), (32, 8), (32, 16), (32, 32))
SCHEDULES = ("tile", "stride", "queue", "block")


def _key(dev_name, n, V, W, H):
    return f"{dev_name}|n{n}|v{V}|{W}x{H}"


def tune(ctx, n, npad, n_hat, cams, width, height, step_fn, reps: int = 3,
         cache_path: str | None = None, candidates=CANDIDATES, schedules=SCHEDULES) -> dict:
    """step_fn(rd) runs one full step on an RDStep bound to ctx.  Returns
    {"tile": (tw, th), "schedule": name, "ms": {"16x16/tile": ..., ...},
    "cached": bool}."""
    import torch

    from .rd import RDStep
    dev_name = torch.cuda.get_device_name(ctx.device)
    key = _key(dev_name, n, cams.shape[0], width, height)
    if cache_path and os.path.exists(cache_path):
        try:
            cache = json.load(open(cache_path))
        except (OSError, ValueError):
            cache = {}
        if key in cache and "schedule" in cache[key]:
            e = cache[key]
            return {"tile": tuple(e["tile"]), "schedule": e["schedule"], "ms": e["ms"],
                    "cached": True}
    timings = {}
    stream = torch.cuda.current_stream(ctx.device)

    def run(tile, schedule):
        rd = RDStep(ctx, n, npad, n_hat, cams, width, height, tile=tile, schedule=schedule)
        step_fn(rd)                      # warm-up (allocates the pair buffers)
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(reps):
            step_fn(rd)
        b.record(stream)
        b.synchronize()
        timings[f"{tile[0]}x{tile[1]}/{schedule}"] = a.elapsed_time(b) / reps
        del rd

    for tile in candidates:
        run(tile, schedules[0])
    best = min(timings, key=timings.get)
    tile = tuple(int(v) for v in best.split("/")[0].split("x"))
    for schedule in schedules[1:]:
        run(tile, schedule)
    best = min(timings, key=timings.get)
    tile = tuple(int(v) for v in best.split("/")[0].split("x"))
    schedule = best.split("/")[1]
    if cache_path:
        cache = {}
        if os.path.exists(cache_path):
            try:
                cache = json.load(open(cache_path))
            except (OSError, ValueError):
                cache = {}
        cache[key] = {"tile": list(tile), "schedule": schedule, "ms": timings}
        tmp = cache_path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1)
        os.replace(tmp, cache_path)
    return {"tile": tile, "schedule": schedule, "ms": timings, "cached": False}


def tune_native(ctx, params, qstep, given_mask, target, n, views, width, height,
                reps: int = 3, cache_path: str | None = None) -> dict:
    """sgs_autotune on the bound scene (tile shapes with the per-sub-tile
    schedule, then the schedules with the fastest shape); the result is cached
    per (device, N, views, width, height) like ``tune``'s.  The context is left
    bound with the chosen options."""
    import torch
    dev_name = torch.cuda.get_device_name(ctx.device)
    key = "native|" + _key(dev_name, n, views, width, height)
    cache = {}
    if cache_path and os.path.exists(cache_path):
        try:
            cache = json.load(open(cache_path))
        except (OSError, ValueError):
            cache = {}
    if key in cache:
        e = cache[key]
        return {"tile": tuple(e["tile"]), "schedule": e["schedule"], "ms": e["ms"],
                "cached": True}
    tile, schedule, ms = ctx.autotune(params, qstep, given_mask, target, reps)
    order = [f"{tw}x{th}/tile" for tw, th in CANDIDATES] + \
        [f"{tile[0]}x{tile[1]}/{name}" for name in SCHEDULES[1:]]
    timings = {k: v for k, v in zip(order, ms)}
    if cache_path:
        cache[key] = {"tile": list(tile), "schedule": schedule, "ms": timings}
        tmp = cache_path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1)
        os.replace(tmp, cache_path)
    return {"tile": tuple(tile), "schedule": schedule, "ms": timings, "cached": False}
