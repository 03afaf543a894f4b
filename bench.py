#!/usr/bin/env python3
"""Throughput of the watershed + waterfall hot path on one MI355X.

One step = the whole hot path over one image already resident in HBM:
float32 image -> gradient (blur sigma 1 + Sobel, quantised to uint16) ->
watershed (Alg. 1, 8-connectivity) -> waterfall, NL = 6 layers (layer 0 =
the watershed). Workload: 4096 x 4096 synthetic image (2000 seeded ellipses
with intensities U[0, 65535] plus Gaussian noise of std 500), the 16.8-Mpixel
configuration the Mvoxel/s metric is quoted on.

Prints ONE JSON line. `value` is Mvoxel/s over the timed steps (hipEvents on
the stream the library launches on). `roofline` is for the kernel with the
largest share of device time, from a second pass of the same steps with a
HIP event pair around every launch. `cpu_baseline` is the CPU oracle timed on
the host on one full step of the same workload.
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

# Algorithmic bytes per pixel each kernel must move (compulsory reads and
# writes of its inputs/outputs; b = bytes per grey value). Region-level
# kernels (wf_union, wf_compress, wf_compact, ws_merge) touch a vanishing
# share of the pixels and are not priced.
def kernel_bytes_per_pixel(b):
    return {
        "grad_blur": 8.0,          # read f32, write f32
        "grad_sobel": 8.0,         # read f32, write f32 magnitude
        "grad_quant": 4.0 + b,     # read f32, write grey
        "ws_init": b + 4.0,        # read grey, write distance
        "ws_label": b + 8.0,       # read grey + distance, write label
        "ws_find": 8.0,            # read label, write label
        "wf_init": 4.0,            # read label
        "wf_edge": 4.0 + b,        # read label + grey
        "wf_relabel": 8.0,         # read label, write label
    }


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-kernel-timing", action="store_true")
    ap.add_argument("--calib-copy", action="store_true",
                    help="run one plain 256 MiB device-to-device copy first (counter calibration)")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only; --gpus %d is not supported" % args.gpus,
              file=sys.stderr, flush=True)
        sys.exit(2)
    import numpy as np
    import torch

    import gen
    import paper_2410_08946_amd as ws

    cfg = gen.CONFIGS["c1"]
    ny, nx = cfg["shape"]
    sigma, conn, NL = cfg["sigma"], cfg["conn"], cfg["NL"]
    N = nx * ny
    b = 2
    dev = torch.device("cuda:0")
    print("bench: generating the 4096x4096 image", file=sys.stderr, flush=True)
    img = gen.config_image("c1")
    img_d = torch.from_numpy(img).to(dev)
    grad_d = torch.empty((ny, nx), dtype=torch.uint16, device=dev)
    out_d = torch.empty((NL, ny, nx), dtype=torch.int32, device=dev)
    nreg_d = torch.zeros(NL, dtype=torch.int64, device=dev)
    ctx = ws.Context(0)
    if args.calib_copy:
        a = torch.empty(64 << 20, dtype=torch.int32, device=dev)
        bb = torch.empty_like(a)
        a.fill_(1)
        torch.cuda.synchronize()
        bb.copy_(a)
        torch.cuda.synchronize()
        del a, bb

    def step():
        ctx.gradient(img_d, sigma, "u16", out=grad_d)
        ctx.watershed(grad_d, conn, out=out_d[0])
        ctx.waterfall(out_d[0], grad_d, conn, NL, out=out_d, nregions=nreg_d)

    print("bench: warmup %d" % args.warmup, file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    stream = torch.cuda.current_stream(dev)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(args.steps):
        step()
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_total = e0.elapsed_time(e1)
    ms_step = ms_total / args.steps
    value = N * args.steps / (ms_total / 1e3) / 1e6
    print("bench: timed %d steps, %.3f ms/step (wall %.3f ms/step)" % (args.steps, ms_step, wall * 1e3 / args.steps),
          file=sys.stderr, flush=True)
    stats = ctx.stats()
    nregions = nreg_d.cpu().tolist()

    # Stage split (host-synchronised, separate pass).
    stages = {}
    for name, fn in (("gradient", lambda: ctx.gradient(img_d, sigma, "u16", out=grad_d)),
                     ("watershed", lambda: ctx.watershed(grad_d, conn, out=out_d[0])),
                     ("waterfall", lambda: ctx.waterfall(out_d[0], grad_d, conn, NL, out=out_d, nregions=nreg_d))):
        a = torch.cuda.Event(enable_timing=True)
        z = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        a.record(stream)
        for _ in range(max(1, args.steps // 2)):
            fn()
        z.record(stream)
        torch.cuda.synchronize()
        stages[name] = round(a.elapsed_time(z) / max(1, args.steps // 2), 4)

    roofline = None
    kernels = {}
    if not args.no_kernel_timing:
        ctx.set_option("timing", 1)
        ctx.timing_reset()
        for _ in range(args.steps):
            step()
        torch.cuda.synchronize()
        kt = ctx.timing_read()
        ctx.set_option("timing", 0)
        per = kernel_bytes_per_pixel(b)
        for name, (ms, cnt) in kt.items():
            kernels[name] = {"launches_per_step": cnt / args.steps, "avg_us": round(ms * 1e3 / cnt, 2),
                             "ms_per_step": round(ms / args.steps, 4)}
        priced = {k: v for k, v in kt.items() if k in per}
        if priced:
            dom = max(priced, key=lambda k: priced[k][0])
            ms, cnt = priced[dom]
            avg_s = ms / cnt / 1e3
            bytes_per_launch = per[dom] * N
            achieved = bytes_per_launch / avg_s / 1e9
            roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                        "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                        "bytes_per_launch": bytes_per_launch, "avg_launch_us": round(avg_s * 1e6, 2)}

    cpu = None
    if not args.no_cpu_baseline:
        print("bench: timing the CPU oracle on one step", file=sys.stderr, flush=True)
        import oracle
        t = time.perf_counter()
        g = oracle.gradient(img, sigma, "u16")
        lab = oracle.watershed(g, conn)
        oracle.waterfall_g1(lab, g, conn, NL)
        dt = time.perf_counter() - t
        cpu = {"value": round(N / dt / 1e6, 3), "unit": "Mvoxel/s", "cores": 1, "kind": "oracle",
               "sample": "one full step (gradient + watershed + NL=6 waterfall) of the 4096x4096 image, "
                         "single-threaded C oracle, %.1f s" % dt}

    line = {
        "metric": "Mvoxel/s watershed+NL waterfall",
        "value": round(value, 2),
        "unit": "Mvoxel/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u16",
        "data": "synthetic",
        "config": {"workload": "2D 4096x4096 uint16 gradient (f32 ellipses+noise, blur sigma=1, Sobel), "
                               "8-connectivity, watershed + NL=6 waterfall", "pixels": N, "NL": NL, "conn": conn,
                   "parallelism": "single GPU"},
        "stages_ms": stages,
        "step2_sweeps": stats.get("sweeps_launched"),
        "nregions": nregions,
        "kernels": kernels,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
