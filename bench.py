#!/usr/bin/env python3
"""Throughput of the watershed + waterfall hot path on one MI355X.

One step = the whole hot path over one volume already resident in HBM:
float32 volume -> gradient (3D Sobel magnitude quantised to uint8) ->
watershed (Alg. 1, 6-connectivity, int32 labels) -> waterfall, NL = 6 layers
(layer 0 = the watershed). Default workload: the 928 x 928 x 928 (799 Mvoxel)
synthetic volume (5000 seeded Gaussian blobs, sigma 4-32 voxels, plus
Gaussian noise of std 2), the largest single-volume configuration, evaluated
on the device. `--workload ellipses4096` runs the 4096 x 4096 uint16 image instead
(blur sigma 1 + Sobel, 8-connectivity, NL = 6); by default its figures are
also reported under "extra".

Prints ONE JSON line. `value` is Mvoxel/s over the timed steps (a HIP event
pair around every step on the stream the library launches on; p50 / p99 /
min per step are reported). `roofline` is for the priced kernel with the
largest share of device time, from a second pass of the same steps with a
HIP event pair around every launch; its `traffic` comes from the committed
rocprofv3 counter summary of the workload. `hbm_path` is the whole step
against the HBM roofline. `cpu_baseline` is the CPU oracle, pinned to one
host core, on a same-recipe sample of the workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

TRAFFIC_FILES = {
    "ellipses4096": "ellipses2d_4096x4096_u16_conn8_nl6_traffic.md",
    "blobs928": "blobs3d_928x928x928_u8_conn6_nl6_traffic.md",
}

WORKLOAD_NAMES = {
    "ellipses4096": ("2D 4096x4096 uint16 gradient (f32 ellipses+noise, blur sigma=1, Sobel), 8-connectivity, "
           "watershed + NL=6 waterfall"),
    "blobs928": ("3D 928x928x928 uint8 gradient (f32 5000 blobs + N(0,2^2), 3D Sobel), 6-connectivity, int32 labels, "
           "watershed + NL=6 waterfall"),
}


# Algorithmic bytes per pixel each kernel must move: the compulsory reads and
# writes of the method's own inputs and outputs at that step (b = bytes per
# grey value, NL = layers). Region- and edge-level kernels (ws_merge,
# wf_union, wf_compress, wf_level) touch a small, data-dependent share of the
# pixels' worth of bytes, and wf_ids names three launches of different kinds:
# none of them is priced.
def kernel_bytes_per_pixel(b, NL):
    return {
        "grad_fused": 8.0,         # read f32 image, write f32 magnitude
        "grad_blur": 8.0,          # read f32, write f32
        "grad_sobel": 8.0,         # read f32, write f32 magnitude
        "grad_quant": 4.0 + b,     # read f32, write grey
        "ws_init": b + 4.0,        # read grey, write distance
        "ws_label": b + 8.0,       # read grey + distance, write label
        "ws_find": 8.0,            # read label, write label
        "wf_pix": 4.0 + b,         # Step V: read layer-0 label + grey
        "wf_out": 4.0 * NL,        # read layer 0, write layers 1 .. NL-1
    }


def path_roofline(b, NL, N, ms_step, counter_bytes):
    """Whole-step HBM roofline: each step of the method streaming its arrays
    once -- the gradient 4 + b (read the float image, write the grey values),
    Step I b + 8, Step II b + 12, Step III 8, Step IV 12 and the canonical
    relabel 12 bytes per pixel, and b + 12 per waterfall level -- so
    B_step = 4 + 3b + 52 + (NL - 1)(b + 12) bytes per pixel; the bytes counted
    are the smaller of B_step N and the measured HBM traffic of a step (fused
    kernels cannot claim more than the method's bytes, extra sweeps count).
    `ws_wf` gives the same figure for the watershed and waterfall alone
    (2b + 52 + (NL - 1)(b + 12) bytes per pixel, without the gradient)."""
    per = 4 + 3 * b + 52 + (NL - 1) * (b + 12)
    alg = per * N
    used = min(alg, counter_bytes) if counter_bytes else alg
    sec = ms_step / 1e3
    achieved = used / sec / 1e9
    io = b + 4 * NL  # compulsory floor: read the grey values once, write the NL layers
    r = {"bound": "hbm", "bytes_per_pixel": per, "algorithmic_bytes": alg,
         "counter_bytes": counter_bytes, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
         "frac": round(achieved / HBM_PEAK_GBS, 4),
         "floor_io": {"bytes_per_pixel": io, "frac": round(io * N / sec / 1e9 / HBM_PEAK_GBS, 4)}}
    if counter_bytes:
        # the kernels' measured traffic as a rate (streaming efficiency) and
        # against the method's bytes (traffic amplification)
        r["counter_frac"] = round(counter_bytes / sec / 1e9 / HBM_PEAK_GBS, 4)
        r["amplification"] = round(counter_bytes / alg, 3)
    return r


def recorded_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` (or, for kernel "step", of all the
    library's kernels over one step; "step_ws_wf" without the gradient's) from
    the committed rocprofv3 FETCH_SIZE / WRITE_SIZE summary of the workload, or
    None when there is none or when the kernel sources changed since the
    counters were taken (the summary records the sha256 of the sources it
    measured)."""
    import hashlib
    if workload not in TRAFFIC_FILES:
        return None
    path = os.path.join(ROOT, "profiles", TRAFFIC_FILES[workload])
    if not os.path.exists(path):
        return None
    vals, sha, srcs = {}, None, []
    for line in open(path):
        f = line.split()
        if len(f) == 3 and f[0] == "traffic":
            vals[f[1]] = int(f[2])
        elif len(f) == 2 and f[0] == "sources_sha256":
            sha = f[1]
        elif len(f) > 1 and f[0] == "sources":
            srcs = f[1:]
    if kernel not in vals or not sha or not srcs:
        return None
    h = hashlib.sha256()
    for s_ in srcs:
        p_ = os.path.join(ROOT, s_)
        if not os.path.exists(p_):
            return None
        h.update(open(p_, "rb").read())
    return vals[kernel] if h.hexdigest() == sha else None


def host_info():
    """CPU model, logical CPUs (all, and usable by this process) and RAM of the host."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    ram = None
    try:
        for line in open("/proc/meminfo"):
            if line.startswith("MemTotal:"):
                ram = round(int(line.split()[1]) / 2 ** 20, 1)
                break
    except OSError:
        pass
    usable = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    return {"cpu": model, "nproc": os.cpu_count(), "usable_cpus": usable, "ram_gib": ram}


def percentiles(xs):
    import numpy as np
    a = np.asarray(xs, dtype=np.float64)
    return {"p50": round(float(np.percentile(a, 50)), 4), "p99": round(float(np.percentile(a, 99)), 4),
            "min": round(float(a.min()), 4), "max": round(float(a.max()), 4)}


def copy_bandwidth(dev):
    """Measured plain device-to-device copy rate (read + write bytes), GB/s."""
    import torch
    a = torch.empty(64 << 20, dtype=torch.int32, device=dev)
    b = torch.empty_like(a)
    a.fill_(1)
    b.copy_(a)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    reps = 10
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    gbs = 2 * a.numel() * 4 / (ms / 1e3) / 1e9
    del a, b
    return round(gbs, 1)


def pinned(fn):
    """Runs fn() with this thread pinned to one host core (the last usable
    one); returns (result, core)."""
    if not hasattr(os, "sched_setaffinity"):
        return fn(), None
    old = os.sched_getaffinity(0)
    core = max(old)
    os.sched_setaffinity(0, {core})
    try:
        return fn(), core
    finally:
        os.sched_setaffinity(0, old)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-kernel-timing", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="skip the 4096^2 figures reported under 'extra'")
    ap.add_argument("--no-structure", action="store_true",
                    help="skip the input-structure figures (one extra watershed_stages call; counter runs skip it)")
    ap.add_argument("--workload", choices=("blobs928", "ellipses4096", "batch", "serve", "recon", "schedules"),
                    default="blobs928",
                    help="blobs928: the 928^3 uint8 volume (default); ellipses4096: the 4096x4096 uint16 image; "
                         "batch: 512 uneven 2D images, one batched call vs one call per image; serve: Poisson "
                         "arrivals of mixed 2D/3D jobs through the continuous-batching server; recon: the "
                         "reconstruction waterfall "
                         "against the graph waterfall on the three single-image workloads (differing pixels per "
                         "layer, time per layer); schedules: the watershed alone under the tile schedule and the "
                         "per-pixel synchronous schedule (APRUF / PRUF / PRW forms) on the same workloads")
    ap.add_argument("--rates", default="50,100,200,500,1000,2000", help="serve workload: request rates (req/s)")
    ap.add_argument("--requests", type=int, default=200, help="serve workload: requests per rate")
    ap.add_argument("--slots", type=int, default=4, help="serve workload: execution slots")
    ap.add_argument("--burst", type=int, default=64,
                    help="serve workload: jobs of the served-against-direct comparison (0 skips it)")
    ap.add_argument("--images", type=int, default=512, help="batch workload: number of images")
    ap.add_argument("--graph", type=int, default=0, choices=(0, 1),
                    help="1: the library replays launch graphs of the gradient and waterfall calls")
    ap.add_argument("--graph-batch", type=int, default=1, choices=(0, 1),
                    help="batch workload: 1 (default) replays the batched call as one launch graph per step")
    ap.add_argument("--autotune", type=int, default=1, choices=(0, 1),
                    help="1 (default): tune tile shape and Step II / III schedule before timing (cached per input "
                         "class)")
    ap.add_argument("--autotune-cache", default=None, help="autotune JSON cache (default: the user's cache dir)")
    ap.add_argument("--retune", action="store_true", help="ignore cached autotune choices")
    ap.add_argument("--volume-cache", default=None,
                    help="blobs928: float32 file of the generated 928^3 volume (read if present, else written)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="run one plain 256 MiB device-to-device copy first (counter calibration)")
    return ap.parse_args()


def bench_batch(args):
    """512 seeded uneven 2D u8 gradient images (sides log-uniform in [128, 2048],
    content of the 256x256 blob recipe), 8-connectivity, watershed + NL = 4:
    one ws_batch call per step vs one ws_watershed + ws_waterfall per image."""
    import numpy as np
    import torch

    import gen
    import paper_2410_08946_amd as ws

    dev = torch.device("cuda:0")
    conn, NL = 8, 4
    ctx = ws.Context(0)
    print("bench: generating %d images" % args.images, file=sys.stderr, flush=True)
    import concurrent.futures as cf
    grads = []
    workers = max(1, min(16, os.cpu_count() or 1))
    with cf.ProcessPoolExecutor(max_workers=workers) as pool:
        for i, arr in enumerate(pool.map(gen.synth.batch_image, range(args.images), chunksize=8)):
            img = torch.from_numpy(arr).to(dev)
            grads.append(ctx.gradient(img, 0.0, "u8"))
            del img
            if (i + 1) % 128 == 0:
                print("bench: %d images ready" % (i + 1), file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    N = sum(int(g.numel()) for g in grads)
    outs_b = [torch.empty((NL,) + tuple(g.shape), dtype=torch.int32, device=dev) for g in grads]
    nreg_b = [torch.zeros(NL, dtype=torch.int64, device=dev) for _ in grads]
    outs_s = [torch.empty((NL,) + tuple(g.shape), dtype=torch.int32, device=dev) for g in grads]
    nreg_s = [torch.zeros(NL, dtype=torch.int64, device=dev) for _ in grads]

    # the batched call replays one launch graph per step (captured on its
    # second use); the per-image calls run directly on a context of their own
    bctx = ws.Context(0)
    tuned = None
    if args.autotune:
        from paper_2410_08946_amd import autotune
        tuned = autotune.tune_batch(bctx, grads, conn, NL, reps=2, cache=args.autotune_cache, force=args.retune)
        print("bench: batch autotune %s -> %s (%.1f s)" % (tuned["key"], tuned["options"], tuned["tuning_s"]),
              file=sys.stderr, flush=True)
    bctx.set_option("graph", args.graph_batch)

    def step_batch():
        bctx.batch(grads, conn, NL, outs=outs_b, nregions=nreg_b)

    def step_single():
        for g, o, n in zip(grads, outs_s, nreg_s):
            ctx.watershed(g, conn, out=o[0])
            ctx.waterfall(o[0], g, conn, NL, out=o, nregions=n)

    def timed(fn, steps):
        stream = torch.cuda.current_stream(dev)
        a = torch.cuda.Event(enable_timing=True)
        z = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        a.record(stream)
        for _ in range(steps):
            fn()
        z.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(z) / steps

    for _ in range(args.warmup):
        step_batch()
        step_single()
    torch.cuda.synchronize()
    print("bench: timing", file=sys.stderr, flush=True)
    r0 = bctx.stats()["graph_replays"]
    ms_b = timed(step_batch, args.steps)
    graph_launches = (bctx.stats()["graph_replays"] - r0) / args.steps
    ms_s = timed(step_single, max(1, args.steps // 4))
    same = all(torch.equal(a, b) for a, b in zip(outs_b, outs_s)) and \
        all(torch.equal(a, b) for a, b in zip(nreg_b, nreg_s))
    line = {
        "metric": "Mvoxel/s watershed+NL waterfall (batched)",
        "value": round(N / (ms_b / 1e3) / 1e6, 2),
        "unit": "Mvoxel/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_b, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": "%d uneven 2D uint8 gradient images (sides log-uniform in [128,2048], blob recipe), "
                               "8-connectivity, watershed + NL=4" % args.images, "pixels": N, "NL": NL, "conn": conn,
                   "parallelism": "single GPU"},
        "per_image_calls": {"value": round(N / (ms_s / 1e3) / 1e6, 2), "unit": "Mvoxel/s", "ms_per_step": round(ms_s, 3)},
        "batched_over_per_image": round(ms_s / ms_b, 3),
        "batched_graph_launches_per_step": graph_launches,
        "autotune": tuned,
        "identical_outputs": bool(same),
        "cpu_baseline": None if args.no_cpu_baseline else cpu_baseline_batch(args.images),
        "host": host_info(),
    }
    print(json.dumps(line), flush=True)


def _oracle_batch_job(i):
    """One image of the uneven batch through the oracle (gradient, watershed,
    NL = 4 waterfall, 8-connectivity): (voxels, seconds)."""
    import gen
    import oracle
    img = gen.synth.batch_image(i)
    t = time.perf_counter()
    g = oracle.gradient(img, 0.0, "u8")
    lab = oracle.watershed(g, 8)
    oracle.waterfall_g1(lab, g, 8, 4)
    return img.size, time.perf_counter() - t


def cpu_baseline_batch(n_images):
    """The oracle over a process pool of all usable host cores (at most 16),
    one image per task, on the first images of the batch until about 20 s of
    wall time have passed."""
    import concurrent.futures as cf
    import oracle
    oracle.build()
    workers = max(1, min(16, len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else 1))
    print("bench: timing the CPU oracle over %d processes" % workers, file=sys.stderr, flush=True)
    vox, done, busy = 0, 0, 0.0
    t0 = time.perf_counter()
    with cf.ProcessPoolExecutor(max_workers=workers) as pool:
        nxt = 0
        futs = set()
        while nxt < n_images and len(futs) < workers:
            futs.add(pool.submit(_oracle_batch_job, nxt))
            nxt += 1
        while futs:
            fin, futs = cf.wait(futs, return_when=cf.FIRST_COMPLETED)
            for f in fin:
                v, t = f.result()
                vox += v
                busy += t
                done += 1
            while nxt < n_images and len(futs) < workers and time.perf_counter() - t0 < 20.0:
                futs.add(pool.submit(_oracle_batch_job, nxt))
                nxt += 1
    dt = time.perf_counter() - t0
    # the oracle's own time (image generation excluded), all processes busy
    return {"value": round(vox / (busy / workers) / 1e6, 3), "unit": "Mvoxel/s", "cores": workers, "kind": "oracle",
            "sample": "images 0..%d of the uneven batch (%d voxels), gradient + watershed + NL=4 waterfall each, "
                      "one image per task over %d processes; rate = voxels / (summed oracle seconds / processes) "
                      "= %.1f s, %.1f s wall with image generation" % (done - 1, vox, workers, busy / workers, dt)}


def bench_serve(args):
    """Poisson arrivals (rates swept) of mixed jobs: 70 % square 2D u8 images
    (sides 512-4096, 8-connectivity), 30 % cubic 3D u8 volumes (sides 128-512,
    6-connectivity), NL = 4, through the continuous-batching server with
    device-memory admission. Latency = arrival -> labels ready on the device;
    the client then releases each result (a consumer that hands labels on)."""
    import numpy as np
    import torch

    import gen
    import paper_2410_08946_amd as ws
    from paper_2410_08946_amd import serve

    dev = torch.device("cuda:0")
    NL = 4
    ctx = ws.Context(0)
    pool2, pool3 = [], []
    for spec in gen.synth.serving_pool_specs():
        f = gen.synth.blobs_device(spec["shape"], spec["seed"], spec["n_blobs"], spec["sigma"], scale=spec["scale"],
                                   noise=spec["noise"], salt=spec["salt"], device=dev)
        g = ctx.gradient(f, 0.0, "u8")
        (pool2 if len(spec["shape"]) == 2 else pool3).append((g, spec["conn"]))
        del f
    torch.cuda.synchronize()
    print("bench: pool ready (%d 2D, %d 3D)" % (len(pool2), len(pool3)), file=sys.stderr, flush=True)
    def release(j):
        # the client hands each result on once its labels are ready
        j.out = j.nregions = None

    results = []
    for rate in [float(r) for r in args.rates.split(",")]:
        rng = np.random.default_rng(4)
        gaps = rng.exponential(1.0 / rate, size=args.requests)
        picks = rng.random(args.requests)
        idx = rng.integers(0, 1 << 30, size=args.requests)
        srv = serve.Server(slots=args.slots, max_job_pixels=max(int(g.numel()) for g, _ in pool2 + pool3))
        jobs = []
        t0 = time.perf_counter()
        t_next = t0
        for k in range(args.requests):
            t_next += gaps[k]
            while time.perf_counter() < t_next:
                time.sleep(max(0.0, min(0.001, t_next - time.perf_counter())))
            g, conn = (pool2[idx[k] % len(pool2)] if picks[k] < 0.7 else pool3[idx[k] % len(pool3)])
            jobs.append(srv.submit(serve.Job(grad=g, conn=conn, NL=NL, jid=k, on_done=release)))
        srv.drain()
        t_end = max(j.t_done for j in jobs)
        lat = [1e3 * (j.t_done - j.t_arrival) for j in jobs if j.error is None]
        vox = sum(int(j.grad.numel()) for j in jobs if j.error is None)
        results.append({"rate": rate, "requests": args.requests, "completed": len(lat),
                        "p50_ms": round(serve.percentile(lat, 50), 3), "p99_ms": round(serve.percentile(lat, 99), 3),
                        "throughput_mvox_s": round(vox / (t_end - t0) / 1e6, 2),
                        "micro_batches": srv.batches, "max_concurrent_slots": srv.max_concurrent})
        print("bench: rate %g done: %s" % (rate, results[-1]), file=sys.stderr, flush=True)
        srv.close()
        del srv, jobs
        torch.cuda.empty_cache()
    best = max(r["throughput_mvox_s"] for r in results)
    direct = serve_vs_direct(args, ctx, pool2, pool3, NL) if args.burst > 0 else None
    line = {
        "metric": "Mvoxel/s watershed+NL waterfall (served), p50/p99 latency",
        "value": best,
        "unit": "Mvoxel/s",
        "n_gpus": 1,
        "steps": args.requests,
        "warmup": 0,
        "ms_per_step": None,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": "Poisson serving: 70%% 2D u8 512^2-4096^2 (8-conn), 30%% 3D u8 128^3-512^3 (6-conn), "
                               "NL=4, %d slots, device-memory admission" % args.slots,
                   "parallelism": "single GPU"},
        "rates": results,
        "served_vs_direct": direct,
    }
    print(json.dumps(line), flush=True)


def serve_vs_direct(args, ctx, pool2, pool3, NL):
    """The same job sequence (the serving mix, args.burst jobs) run once as one
    ws_watershed + ws_waterfall call per job on one stream and once through the
    server with every job submitted at once; both timed from the first call to
    the last result on the device, outputs compared job by job."""
    import numpy as np
    import torch

    from paper_2410_08946_amd import serve

    rng = np.random.default_rng(5)
    picks, idx = rng.random(args.burst), rng.integers(0, 1 << 30, size=args.burst)
    seq = [pool2[idx[k] % len(pool2)] if picks[k] < 0.7 else pool3[idx[k] % len(pool3)] for k in range(args.burst)]
    vox = sum(int(g.numel()) for g, _ in seq)

    def run_direct():
        res = []
        for g, conn in seq:
            lab = ctx.watershed(g, conn)
            res.append(ctx.waterfall(lab, g, conn, NL))
        return res

    run_direct()  # grows the context's buffers to the largest job
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    direct = run_direct()
    torch.cuda.synchronize()
    t_direct = time.perf_counter() - t0
    srv = serve.Server(slots=args.slots, max_job_pixels=max(int(g.numel()) for g, _ in pool2 + pool3))
    t0 = time.perf_counter()
    jobs = [srv.submit(serve.Job(grad=g, conn=conn, NL=NL, jid=k)) for k, (g, conn) in enumerate(seq)]
    srv.drain()
    t_served = max(j.t_done for j in jobs) - t0
    torch.cuda.synchronize()  # every slot's stream, before comparing on the default one
    same = all(j.error is None and torch.equal(j.out, o) and torch.equal(j.nregions, n)
               for j, (o, n) in zip(jobs, direct))
    srv.close()
    r = {"jobs": args.burst, "voxels": vox, "direct_ms": round(1e3 * t_direct, 2),
         "served_ms": round(1e3 * t_served, 2), "direct_mvox_s": round(vox / t_direct / 1e6, 1),
         "served_mvox_s": round(vox / t_served / 1e6, 1), "served_over_direct": round(t_direct / t_served, 3),
         "identical_outputs": bool(same)}
    print("bench: served vs direct: %s" % r, file=sys.stderr, flush=True)
    del jobs, direct
    torch.cuda.empty_cache()
    return r


def bench_recon(args):
    """Reconstruction waterfall (Alg. 4 Steps V-VI, re-watershed per layer)
    against the graph waterfall on the 256^2, 4096^2 and 928^3 workloads, from
    the same watershed: region counts and differing pixels per layer, and the
    time each added layer costs (cumulative runs with NL = 2 .. N; the paper
    reports later reconstruction layers to be slower)."""
    import numpy as np
    import torch

    import gen
    import paper_2410_08946_amd as ws

    dev = torch.device("cuda:0")
    ctx = ws.Context(0)
    reps = max(1, min(args.steps, 5))

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        z = torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            fn()
        z.record()
        torch.cuda.synchronize()
        return a.elapsed_time(z) / reps

    results = {}
    for name in ("blobs256", "ellipses4096", "blobs928"):
        cfg = gen.CONFIGS[name]
        shape = tuple(cfg["shape"])
        print("bench: recon %s %s" % (name, shape), file=sys.stderr, flush=True)
        if name == "blobs928":
            img = gen.synth.blobs3d_device(shape, seed=cfg["seed"], device=dev)
        else:
            img = torch.from_numpy(gen.config_image(name)).to(dev)
        grad = ctx.gradient(img, cfg["sigma"], cfg["dtype"])
        del img
        conn, NL = cfg["conn"], cfg["NL"]
        lab = ctx.watershed(grad, conn)
        g1, n1 = ctx.waterfall(lab, grad, conn, NL)
        rc, nr = ctx.waterfall_recon(lab, grad, conn, NL)
        torch.cuda.synchronize()
        diff = [int((g1[k] != rc[k]).sum()) for k in range(NL)]
        t_g1 = timed(lambda: ctx.waterfall(lab, grad, conn, NL, out=g1, nregions=n1))
        cum = [timed(lambda k=k: ctx.waterfall_recon(lab, grad, conn, k, out=rc[:k], nregions=nr[:k]))
               for k in range(1, NL + 1)]
        N = int(np.prod(shape))
        results[name] = {
            "pixels": N, "NL": NL, "conn": conn,
            "regions_g1": n1.cpu().tolist(), "regions_recon": nr.cpu().tolist(),
            "differing_pixels": diff, "differing_fraction": [round(d / N, 6) for d in diff],
            "ms_g1_all_layers": round(t_g1, 3),
            "ms_recon_all_layers": round(cum[-1], 3),
            "ms_recon_per_layer": [round(cum[0], 3)] + [round(cum[k] - cum[k - 1], 3) for k in range(1, NL)],
        }
        del g1, rc, lab, grad
        torch.cuda.empty_cache()
    line = {
        "metric": "reconstruction vs graph waterfall: differing pixels per layer",
        "value": results["ellipses4096"]["differing_pixels"][-1],
        "unit": "pixels",
        "n_gpus": 1,
        "steps": reps,
        "warmup": 1,
        "ms_per_step": results["ellipses4096"]["ms_recon_all_layers"],
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u16",
        "data": "synthetic",
        "config": {"workload": "256^2 u8 NL=3, 4096^2 u16 NL=6, 928^3 u8 NL=6: reconstruction waterfall vs graph "
                               "waterfall from the same watershed", "parallelism": "single GPU"},
        "per_workload": results,
    }
    print(json.dumps(line), flush=True)


def bench_schedules(args):
    """The watershed alone (Alg. 1 Steps I-IV and canonical labels) under each
    schedule on the 256^2, 4096^2 and 928^3 workloads: the tile schedule with
    APRUF / PRUF Step III, and the per-pixel synchronous schedule of Section 3.3
    with APRUF, PRUF and PRW (Alg. 2) forms. Every variant's labels must equal
    the default's; reports time, Mvoxel/s and the sweep / synchronisation /
    pass counts."""
    import numpy as np
    import torch

    import gen
    import paper_2410_08946_amd as ws

    dev = torch.device("cuda:0")
    ctx = ws.Context(0)
    reps = max(1, min(args.steps, 5))
    variants = [("tile_apruf", 0, 0, 0), ("tile_pruf", 0, 1, 0), ("pixel_apruf_sync", 1, 0, 0),
                ("pixel_pruf_sync", 1, 1, 0), ("pixel_prw_sync", 1, 1, 1)]

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        z = torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            fn()
        z.record()
        torch.cuda.synchronize()
        return a.elapsed_time(z) / reps

    results = {}
    for name in ("blobs256", "ellipses4096", "blobs928"):
        cfg = gen.CONFIGS[name]
        shape = tuple(cfg["shape"])
        if name == "blobs928":
            img = gen.synth.blobs3d_device(shape, seed=cfg["seed"], device=dev)
        else:
            img = torch.from_numpy(gen.config_image(name)).to(dev)
        grad = ctx.gradient(img, cfg["sigma"], cfg["dtype"])
        del img
        conn = cfg["conn"]
        N = int(np.prod(shape))
        ref = ctx.watershed(grad, conn)
        lab = torch.empty_like(ref)
        per = {}
        for vname, sched, step3, step4 in variants:
            print("bench: schedules %s %s" % (name, vname), file=sys.stderr, flush=True)
            ctx.set_option("schedule", sched)
            ctx.set_option("step3", step3)
            ctx.set_option("step4", step4)
            ctx.watershed(grad, conn, out=lab)
            torch.cuda.synchronize()
            same = bool(torch.equal(lab, ref))
            st = ctx.stats()
            ms = timed(lambda: ctx.watershed(grad, conn, out=lab))
            per[vname] = {"ms": round(ms, 3), "mvoxel_s": round(N / ms / 1e3, 1), "identical": same,
                          "step2_sweeps": st["sweeps_launched"], "step2_sweeps_changing": st["sweeps_changing"],
                          "step3_syncs": st["step3_syncs"], "step4_passes": st["step4_passes"]}
            print("bench: schedules %s %s %s" % (name, vname, per[vname]), file=sys.stderr, flush=True)
        ctx.set_option("schedule", 0)
        ctx.set_option("step3", 0)
        ctx.set_option("step4", 0)
        results[name] = {"pixels": N, "conn": conn, "variants": per}
        del grad, ref, lab
        torch.cuda.empty_cache()
    e2d = results["ellipses4096"]["variants"]
    line = {
        "metric": "watershed Mvoxel/s by schedule",
        "value": e2d["tile_apruf"]["mvoxel_s"],
        "unit": "Mvoxel/s",
        "n_gpus": 1,
        "steps": reps,
        "warmup": 1,
        "ms_per_step": e2d["tile_apruf"]["ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u16",
        "data": "synthetic",
        "config": {"workload": "watershed only (Steps I-IV + canonical labels) of the 256^2 u8, 4096^2 u16 and "
                               "928^3 u8 gradients, tile vs per-pixel synchronous schedules",
                   "parallelism": "single GPU"},
        "all_identical": all(v["identical"] for r in results.values() for v in r["variants"].values()),
        "per_workload": results,
    }
    print(json.dumps(line), flush=True)


def measure_single(args, name, steps, warmup, kernel_timing, cpu_baseline):
    """Times `steps` whole steps of workload `name` (ellipses4096 / blobs928) with the input
    resident in HBM and returns the fields of its JSON line."""
    import numpy as np
    import torch

    import gen
    import paper_2410_08946_amd as ws

    cfg = gen.CONFIGS[name]
    shape = tuple(cfg["shape"])
    sigma, conn, NL, gdt = cfg["sigma"], cfg["conn"], cfg["NL"], cfg["dtype"]
    N = int(np.prod(shape))
    b = 2 if gdt == "u16" else 1
    dev = torch.device("cuda:0")
    img = None
    if name == "blobs928":
        # too large for the host generator: the same recipe evaluated on the
        # device (or read back from a file an earlier run of this recipe wrote)
        img_d = None
        cache = args.volume_cache
        if cache and os.path.exists(cache) and os.path.getsize(cache) == 4 * N:
            print("bench: reading the 928^3 volume from %s" % cache, file=sys.stderr, flush=True)
            import numpy as np
            host = np.fromfile(cache, dtype=np.float32).reshape(shape)
            img_d = torch.from_numpy(host).to(dev)
            del host
        if img_d is None:
            print("bench: generating the 928^3 volume on the device", file=sys.stderr, flush=True)
            img_d = gen.synth.blobs3d_device(shape, seed=cfg["seed"], device=dev)
            if cache:
                img_d.cpu().numpy().tofile(cache)
                print("bench: wrote the volume to %s" % cache, file=sys.stderr, flush=True)
    else:
        print("bench: generating the 4096x4096 image", file=sys.stderr, flush=True)
        img = gen.config_image(name)
        img_d = torch.from_numpy(img).to(dev)
    grad_d = torch.empty(shape, dtype=torch.uint16 if gdt == "u16" else torch.uint8, device=dev)
    out_d = torch.empty((NL,) + shape, dtype=torch.int32, device=dev)
    nreg_d = torch.zeros(NL, dtype=torch.int64, device=dev)
    ctx = ws.Context(0)
    tuned = None
    if args.autotune:
        # tile shape and Step II / III schedule for this input class (labels
        # checked equal for every candidate); reported, not timed
        from paper_2410_08946_amd import autotune
        key = autotune.key_for(len(shape), gdt, conn, N)
        hit = None if args.retune else autotune.load_cache(args.autotune_cache).get(key)
        if hit and "options" in hit:
            autotune.apply(ctx, hit["options"])
            tuned = {"key": key, "options": hit["options"], "ms": hit.get("ms"), "cached": True, "candidates": [],
                     "tuning_s": 0.0}
        else:
            ctx.gradient(img_d, sigma, gdt, out=grad_d)
            tuned = autotune.tune_watershed(ctx, grad_d, conn, reps=3, cache=args.autotune_cache, force=True)
        print("bench: %s autotune %s -> %s (%.1f s)" % (name, tuned["key"], tuned["options"], tuned["tuning_s"]),
              file=sys.stderr, flush=True)
    ctx.set_option("graph", args.graph)

    def step():
        ctx.gradient(img_d, sigma, gdt, out=grad_d)
        ctx.watershed(grad_d, conn, out=out_d[0])
        ctx.waterfall(out_d[0], grad_d, conn, NL, out=out_d, nregions=nreg_d)

    print("bench: %s warmup %d" % (name, warmup), file=sys.stderr, flush=True)
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()

    # one event pair per step on the stream the library launches on
    stream = torch.cuda.current_stream(dev)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev[0].record(stream)
    for i in range(steps):
        step()
        ev[i + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per_step = [ev[i].elapsed_time(ev[i + 1]) for i in range(steps)]
    ms_total = ev[0].elapsed_time(ev[steps])
    ms_step = ms_total / steps
    value = N * steps / (ms_total / 1e3) / 1e6
    print("bench: %s timed %d steps, %.3f ms/step (wall %.3f ms/step)" %
          (name, steps, ms_step, wall * 1e3 / steps), file=sys.stderr, flush=True)
    stats = ctx.stats()
    nregions = nreg_d.cpu().tolist()

    # Stage split (host-synchronised, separate pass).
    stages = {}
    for stage, fn in (("gradient", lambda: ctx.gradient(img_d, sigma, gdt, out=grad_d)),
                      ("watershed", lambda: ctx.watershed(grad_d, conn, out=out_d[0])),
                      ("waterfall", lambda: ctx.waterfall(out_d[0], grad_d, conn, NL, out=out_d, nregions=nreg_d))):
        a = torch.cuda.Event(enable_timing=True)
        z = torch.cuda.Event(enable_timing=True)
        reps = max(1, steps // 2)
        torch.cuda.synchronize()
        a.record(stream)
        for _ in range(reps):
            fn()
        z.record(stream)
        torch.cuda.synchronize()
        stages[stage] = round(a.elapsed_time(z) / reps, 4)

    # Input structure that drives the time (outside the timed region): basins,
    # plateau pixels resolved by Step II and their largest geodesic distance,
    # minimal-plateau pixels, Step II sweeps.
    structure = None
    if not args.no_structure:
        bal, arrow = ctx.watershed_stages(grad_d, conn)
        neg = bal < 0
        structure = {"basins": nregions[0], "plateau_pixels": int(neg.sum()),
                     "max_geodesic_distance": int(-bal.min()) if bool(neg.any()) else 0,
                     "minimal_plateau_pixels": int(((bal == 2) | (bal == 3)).sum()),
                     "step2_sweeps": stats.get("sweeps_launched"),
                     "step2_sweeps_changing": stats.get("sweeps_changing")}
        del bal, arrow, neg
        torch.cuda.empty_cache()

    roofline = None
    kernels = {}
    if kernel_timing:
        ctx.set_option("timing", 1)
        ctx.timing_reset()
        for _ in range(steps):
            step()
        torch.cuda.synchronize()
        kt = ctx.timing_read()
        ctx.set_option("timing", 0)
        per = kernel_bytes_per_pixel(b, NL)
        for kname, (ms, cnt) in kt.items():
            kernels[kname] = {"launches_per_step": cnt / steps, "avg_us": round(ms * 1e3 / cnt, 2),
                              "ms_per_step": round(ms / steps, 4)}
        priced = {k: v for k, v in kt.items() if k in per}
        if priced:
            dom = max(priced, key=lambda k: priced[k][0])
            ms, cnt = priced[dom]
            avg_s = ms / cnt / 1e3
            bytes_per_launch = per[dom] * N
            achieved = bytes_per_launch / avg_s / 1e9
            roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                        "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                        "traffic": recorded_traffic(dom, name),
                        "bytes_per_pixel": per[dom], "bytes_per_launch": bytes_per_launch,
                        "avg_launch_us": round(avg_s * 1e6, 2)}

    cpu = None
    if cpu_baseline:
        cpu = cpu_baseline_single(name, cfg, img, img_d)
    ws_wf_ms = stages["watershed"] + stages["waterfall"]
    bws = 2 * b + 52 + (NL - 1) * (b + 12)
    cb = recorded_traffic("step_ws_wf", name)
    used = min(bws * N, cb) if cb else bws * N
    res = {
        "value": round(value, 2),
        "ms_per_step": round(ms_step, 4),
        "step_ms": percentiles(per_step),
        "config": {"workload": WORKLOAD_NAMES[name], "shape": list(shape), "pixels": N, "NL": NL, "conn": conn,
                   "grey": gdt, "parallelism": "single GPU"},
        "dtype": gdt,
        "stages_ms": stages,
        "step2_sweeps": stats.get("sweeps_launched"),
        "nregions": nregions,
        "input_structure": structure,
        "kernels": kernels,
        "roofline": roofline,
        "hbm_path": path_roofline(b, NL, N, ms_step, recorded_traffic("step", name)),
        "hbm_path_ws_wf": {"bytes_per_pixel": bws, "algorithmic_bytes": bws * N, "counter_bytes": cb,
                           "ms": round(ws_wf_ms, 4), "achieved": round(used / (ws_wf_ms / 1e3) / 1e9, 1),
                           "frac": round(used / (ws_wf_ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4)},
        "cpu_baseline": cpu,
        "autotune": tuned,
    }
    del img_d, grad_d, out_d
    ctx.close()
    torch.cuda.empty_cache()
    return res


def cpu_baseline_single(name, cfg, img, img_d):
    """The CPU oracle, pinned to one host core, on whole steps (gradient +
    watershed + NL-layer waterfall) of a same-recipe sample: the full
    4096x4096 image, or a 24-plane slab of the 928^3 volume (the device's
    float planes copied to the host; about 20 s of CPU work)."""
    import oracle
    sigma, conn, NL, gdt = cfg["sigma"], cfg["conn"], cfg["NL"], cfg["dtype"]
    if name == "blobs928":
        z0, z1 = 452, 476
        sample = img_d[z0:z1].cpu().numpy()
        what = "planes %d..%d of the 928^3 volume (928x928x%d = %d voxels)" % (z0, z1 - 1, z1 - z0, sample.size)
    else:
        sample = img
        what = "the 4096x4096 image"
    print("bench: timing the CPU oracle on %s" % what, file=sys.stderr, flush=True)

    def run():
        reps, dt = 0, 0.0
        while reps < 4 and (reps == 0 or dt < 10.0):
            t = time.perf_counter()
            g = oracle.gradient(sample, sigma, gdt)
            lab = oracle.watershed(g, conn)
            oracle.waterfall_g1(lab, g, conn, NL)
            dt += time.perf_counter() - t
            reps += 1
        return reps, dt

    (reps, dt), core = pinned(run)
    return {"value": round(sample.size * reps / dt / 1e6, 3), "unit": "Mvoxel/s", "cores": 1, "kind": "oracle",
            "sample": "%d full step(s) (gradient + watershed + NL=%d waterfall) of %s, single-threaded C oracle "
                      "(gcc -O2) pinned to host core %s, %.1f s" % (reps, NL, what, core, dt),
            "host": host_info()}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: the library runs on one GPU only; --gpus %d is not supported" % args.gpus,
              file=sys.stderr, flush=True)
        sys.exit(2)
    if args.workload == "batch":
        bench_batch(args)
        return
    if args.workload == "serve":
        bench_serve(args)
        return
    if args.workload == "recon":
        bench_recon(args)
        return
    if args.workload == "schedules":
        bench_schedules(args)
        return
    import torch

    dev = torch.device("cuda:0")
    if args.calib_copy:
        a = torch.empty(64 << 20, dtype=torch.int32, device=dev)
        bb = torch.empty_like(a)
        a.fill_(1)
        torch.cuda.synchronize()
        bb.copy_(a)
        torch.cuda.synchronize()
        del a, bb
    name = args.workload
    r = measure_single(args, name, args.steps, args.warmup, not args.no_kernel_timing, not args.no_cpu_baseline)
    line = {
        "metric": "Mvoxel/s watershed+NL waterfall",
        "value": r["value"],
        "unit": "Mvoxel/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": r["dtype"],
        "data": "synthetic",
    }
    line.update({k: v for k, v in r.items() if k not in ("value", "ms_per_step", "dtype")})
    line["copy_bandwidth_gbs"] = copy_bandwidth(dev)
    line["host"] = host_info()
    if name == "blobs928" and not args.no_extra:
        # the 4096^2 image: a smaller, partly cache-resident workload
        e = measure_single(args, "ellipses4096", max(1, args.steps // 2), 2, False, False)
        line["extra"] = {"ellipses4096": {k: e[k] for k in ("value", "ms_per_step", "step_ms", "config", "stages_ms",
                                                  "nregions", "input_structure", "hbm_path", "hbm_path_ws_wf",
                                                  "autotune")}}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
