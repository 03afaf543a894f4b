"""Autotuner of the watershed's launch parameters.

The paper fixes the result and leaves block size and the reduction rate RR to
time alone (Section 3.4, last paragraph; Section 5, parameters paragraph:
16x16 / 8x8x8 blocks and RR = 6 there). Here the free parameters are the
library's context options

* "tile2d" / "tile3d"  the watershed tile shape (shape ids of include/ws.h),
* "step3" / "rr"       Step III as a per-pixel Find (APRUF, Section 3.2) or as
                       RR pointer jumps per synchronisation (PRUF),
* "sweep_batch"        Step II sweeps launched per convergence read-back,

none of which changes a label. `tune_*` times candidate settings on the
caller's own input with HIP events (coordinate descent: tile shape first,
then the Step III form, then the sweep batch), checks that every candidate's
labels equal the default setting's bit for bit, and keeps the fastest. The
choice is cached in a JSON file keyed by (dimensionality, grey type,
connectivity, size class = floor(log2 pixels), single image or batch), so a
later call with a matching key applies it without timing anything.
"""
from __future__ import annotations

import json
import math
import os
import time

DEFAULTS = {"tile2d": 2, "tile3d": 3, "step3": 0, "rr": 6, "sweep_batch": 4}
SHAPES = {2: [2, 12, 22, 32], 3: [3, 13, 23, 33]}
STEP3 = [(0, 6), (1, 6), (1, 2)]          # (step3, rr)
SWEEP_BATCH = [4, 2, 8]


def cache_path() -> str:
    p = os.environ.get("WS_AUTOTUNE_CACHE")
    if p:
        return p
    return os.path.join(os.path.expanduser("~"), ".cache", "paper_2410_08946_amd", "autotune.json")


def key_for(ndim: int, dtype: str, conn: int, pixels: int, batch: bool = False) -> str:
    cls = int(math.floor(math.log2(max(1, int(pixels)))))
    return "%dd/%s/conn%d/2^%d/%s" % (ndim, dtype, int(conn), cls, "batch" if batch else "single")


def load_cache(path: str | None = None) -> dict:
    path = path or cache_path()
    try:
        with open(path) as f:
            d = json.load(f)
        return d if isinstance(d, dict) else {}
    except (OSError, ValueError):
        return {}


def save_cache(entries: dict, path: str | None = None) -> None:
    path = path or cache_path()
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    d = load_cache(path)
    d.update(entries)
    tmp = path + ".tmp%d" % os.getpid()
    with open(tmp, "w") as f:
        json.dump(d, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def apply(ctx, options: dict) -> None:
    """Sets every option of `options` (tuned or defaults) on the context."""
    for k in ("tile2d", "tile3d", "step3", "rr", "sweep_batch"):
        if k in options:
            ctx.set_option(k, int(options[k]))


def _grey(t) -> str:
    import torch
    return "u16" if t.dtype == torch.uint16 else "u8"


def _time(run, reps: int) -> float:
    """Smallest of `reps` timings (ms) of run() after one untimed call."""
    import torch
    run()
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        z = torch.cuda.Event(enable_timing=True)
        a.record()
        run()
        z.record()
        torch.cuda.synchronize()
        best = min(best, a.elapsed_time(z))
    return best


def _descend(ctx, run, result, ndim: int, reps: int, log: list) -> dict:
    """Coordinate descent over the option groups; every candidate's output
    (result()) must equal the default setting's."""
    import torch
    best = dict(DEFAULTS)
    apply(ctx, best)
    run()
    torch.cuda.synchronize()
    ref = [t.clone() for t in result()]
    best_ms = _time(run, reps)
    log.append({"options": dict(best), "ms": round(best_ms, 4)})
    tile_key = "tile3d" if ndim == 3 else "tile2d"
    groups = [[{tile_key: s} for s in SHAPES[ndim]],
              [{"step3": s3, "rr": rr} for s3, rr in STEP3],
              [{"sweep_batch": b} for b in SWEEP_BATCH]]
    for cands in groups:
        for cand in cands:
            opt = dict(best)
            opt.update(cand)
            if opt == best:
                continue
            apply(ctx, opt)
            run()
            torch.cuda.synchronize()
            got = result()
            if not all(torch.equal(a, b) for a, b in zip(got, ref)):
                apply(ctx, DEFAULTS)
                raise RuntimeError("autotune: labels under %s differ from the default setting's" % opt)
            ms = _time(run, reps)
            log.append({"options": dict(opt), "ms": round(ms, 4)})
            if ms < best_ms:
                best, best_ms = opt, ms
    apply(ctx, best)
    return {"options": best, "ms": round(best_ms, 4)}


def tune_watershed(ctx, grad, conn: int, reps: int = 3, cache: str | None = None, force: bool = False) -> dict:
    """Tunes ws_watershed of `grad` (uint8/uint16 device tensor) and leaves
    the chosen options set on `ctx`. Returns {"key", "options", "ms",
    "cached", "candidates", "tuning_s"}."""
    import torch
    ndim = 3 if grad.dim() == 3 else 2
    key = key_for(ndim, _grey(grad), conn, grad.numel())
    if not force:
        hit = load_cache(cache).get(key)
        if hit and "options" in hit:
            apply(ctx, hit["options"])
            return {"key": key, "options": hit["options"], "ms": hit.get("ms"), "cached": True, "candidates": [],
                    "tuning_s": 0.0}
    lab = torch.empty(grad.shape, dtype=torch.int32, device=grad.device)
    log = []
    t0 = time.perf_counter()
    res = _descend(ctx, lambda: ctx.watershed(grad, conn, out=lab), lambda: [lab], ndim, reps, log)
    dt = time.perf_counter() - t0
    save_cache({key: {"options": res["options"], "ms": res["ms"]}}, cache)
    return {"key": key, "options": res["options"], "ms": res["ms"], "cached": False, "candidates": log,
            "tuning_s": round(dt, 3)}


def tune_batch(ctx, grads, conns, NL: int, reps: int = 2, cache: str | None = None, force: bool = False) -> dict:
    """Tunes ws_batch over the images `grads` (one connectivity per image, or
    one for all) and leaves the chosen options set on `ctx`. The key uses the
    dimensionality of the first image, the connectivity of the first image
    and the batch's total pixel count."""
    import torch
    conns = [int(conns)] * len(grads) if isinstance(conns, int) else [int(c) for c in conns]
    ndim = 3 if grads[0].dim() == 3 else 2
    total = sum(int(g.numel()) for g in grads)
    key = key_for(ndim, _grey(grads[0]), conns[0], total, batch=True)
    if not force:
        hit = load_cache(cache).get(key)
        if hit and "options" in hit:
            apply(ctx, hit["options"])
            return {"key": key, "options": hit["options"], "ms": hit.get("ms"), "cached": True, "candidates": [],
                    "tuning_s": 0.0}
    dev = grads[0].device
    outs = [torch.empty((int(NL),) + tuple(g.shape), dtype=torch.int32, device=dev) for g in grads]
    nreg = [torch.zeros(int(NL), dtype=torch.int64, device=dev) for _ in grads]
    log = []
    t0 = time.perf_counter()
    res = _descend(ctx, lambda: ctx.batch(grads, conns, NL, outs=outs, nregions=nreg), lambda: outs + nreg, ndim,
                   reps, log)
    dt = time.perf_counter() - t0
    save_cache({key: {"options": res["options"], "ms": res["ms"]}}, cache)
    return {"key": key, "options": res["options"], "ms": res["ms"], "cached": False, "candidates": log,
            "tuning_s": round(dt, 3)}
