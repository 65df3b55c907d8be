"""Benchmark: 1080p virtual views/s of the view-interpolation forward pass on
one MI355X.

A step is one call of the library over the dense-view batch: an 8-camera arc
of synthetic 1080p images (7 adjacent pairs) with 16 phases per pair
(t = k/17, k = 1..16), i.e. 112 views, BF16 convolutions with fp32
accumulation, inputs resident in HBM. Reported beside it:

* the plain FP32 path on one 1080p pair, batch 1, t in {1/4, 1/2, 3/4};
* PSNR of one BF16 view against the FP64 CPU oracle, and the oracle's own
  time for that view on the host cores (the CPU baseline);
* per-step latency p50/p99;
* the roofline of the dominant kernel class (the 3x3 256->256 convs) from
  HIP events recorded on the library's stream over the timed steps.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import tempfile
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "1080p virtual views/s, BF16 vs FP32 at PSNR≥45dB vs FP64 oracle; p99 latency"
PEAK_BF16_TFLOPS = 2500.0
PEAK_FP32_TFLOPS = 157.3
PEAK_HBM_GBS = 8000.0


def percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return float("nan")
    k = (len(xs) - 1) * q
    lo, hi = math.floor(k), math.ceil(k)
    return xs[lo] + (xs[hi] - xs[lo]) * (k - lo)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-oracle", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--no-fp32", action="store_true", help="skip the plain FP32 leg")
    ap.add_argument("--height", type=int, default=1080)
    ap.add_argument("--width", type=int, default=1920)
    ap.add_argument("--phases", type=int, default=16)
    ap.add_argument("--cams", type=int, default=8)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): each view is independent, "
              "so more GPUs would each take a contiguous camera range; that path is not built.",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2112_10603_amd import Net
    from synth import scenes
    from synth.weights import write_weights_file

    dev = torch.device("cuda:0")
    H, W = args.height, args.width
    td = tempfile.mkdtemp()
    wpath = write_weights_file(os.path.join(td, "w.ffvw"), seed=0)
    arc = scenes.camera_arc(3, H, W, args.cams, 1024, (8.0, 64.0), 48.0, 0.01, device=dev)
    torch.cuda.synchronize()
    pairs = [(arc[i], arc[i + 1]) for i in range(args.cams - 1)]
    ts = [k / (args.phases + 1) for k in range(1, args.phases + 1)]
    n_views = len(pairs) * len(ts)
    print(f"[bench] {n_views} views of {H}x{W} per step, BF16", file=sys.stderr, flush=True)

    net = Net(wpath, "bf16", 0, workspace_bytes=128 << 30)
    out = torch.empty((len(pairs), len(ts), 3, H, W), dtype=torch.float32, device=dev)
    for _ in range(args.warmup):
        net.interpolate(pairs, ts, out)
    torch.cuda.synchronize()
    net.set_profiling(True)
    step_ms = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record(net.stream)
        net.interpolate(pairs, ts, out)
        ev1.record(net.stream)
        ev1.synchronize()
        step_ms.append(ev0.elapsed_time(ev1))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    stats = {k: net.kernel_stats(k) for k in ("conv256", "conv", "convT", "pixel", "head")}
    net.set_profiling(False)
    ms_per_step = 1000.0 * wall / args.steps
    value = n_views / (wall / args.steps)
    print(f"[bench] bf16 {ms_per_step:.2f} ms/step, {value:.1f} views/s", file=sys.stderr, flush=True)

    dom = stats["conv256"]
    roof = None
    if dom["launches"] > 0:
        avg_ms = dom["ms"] / dom["launches"]
        flops_per_launch = dom["work"] / dom["launches"]
        achieved = flops_per_launch / (avg_ms * 1e-3) / 1e12
        roof = {"bound": "mfma", "achieved": round(achieved, 2), "peak": PEAK_BF16_TFLOPS,
                "unit": "TFLOP/s", "frac": round(achieved / PEAK_BF16_TFLOPS, 4), "traffic": None,
                "kernel": "conv_igemm bf16, 3x3 256->256 (VIBlock conv3-8)",
                "avg_launch_ms": round(avg_ms, 4), "flops_per_launch": flops_per_launch}
    conv_ms = sum(stats[k]["ms"] for k in ("conv256", "conv", "convT"))
    conv_flops = sum(stats[k]["work"] for k in ("conv256", "conv", "convT"))
    breakdown = {k: {"launches": v["launches"], "ms_per_step": round(v["ms"] / args.steps, 3)}
                 for k, v in stats.items()}

    # one BF16 view kept for the PSNR check: pair 0, t = 8/17
    j_ref = len(ts) // 2 - 1
    bf16_view = out[0, j_ref].cpu().numpy()
    net.close()
    del out

    fp32 = None
    if not args.no_fp32:
        net32 = Net(wpath, "fp32", 0, workspace_bytes=64 << 30)
        l, r = pairs[0]
        o1 = torch.empty((1, 1, 3, H, W), dtype=torch.float32, device=dev)
        for t in (0.25, 0.5, 0.75):
            net32.interpolate([(l, r)], [t], o1)
        torch.cuda.synchronize()
        lat = []
        reps = 2
        t1 = time.perf_counter()
        for _ in range(reps):
            for t in (0.25, 0.5, 0.75):
                a = time.perf_counter()
                net32.interpolate([(l, r)], [t], o1)
                lat.append(1000.0 * (time.perf_counter() - a))
        w32 = time.perf_counter() - t1
        v32 = 3 * reps / w32
        fp32 = {"views_per_s": round(v32, 2), "ms_per_view_p50": round(percentile(lat, 0.5), 2),
                "workload": "one 1080p pair, batch 1, t in {0.25, 0.5, 0.75}, FP32 convs"}
        net32.close()
        print(f"[bench] fp32 plain {v32:.2f} views/s", file=sys.stderr, flush=True)

    cpu = None
    psnr = None
    if not args.no_oracle:
        from oracle import vinet as oracle
        try:
            from threadpoolctl import threadpool_info
            cores = max([p.get("num_threads", 1) for p in threadpool_info()] + [1])
        except Exception:
            cores = os.cpu_count()
        Wo = oracle.load_weights(wpath)
        xl = arc[0].cpu().numpy()
        xr = arc[1].cpu().numpy()
        a = time.perf_counter()
        ref = oracle.vinet_forward(xl, xr, ts[j_ref], Wo)
        dt = time.perf_counter() - a
        mse = float(np.mean((bf16_view.astype(np.float64) - ref) ** 2))
        psnr = 10 * math.log10(1.0 / mse) if mse > 0 else float("inf")
        cpu = {"value": round(1.0 / dt, 5), "unit": "views/s", "cores": cores, "kind": "oracle",
               "sample": f"one {H}x{W} view (pair 0, t=8/17) through the FP64 numpy oracle, "
                         f"{dt:.1f} s"}
        print(f"[bench] oracle {dt:.1f} s/view, PSNR {psnr:.2f} dB", file=sys.stderr, flush=True)

    line = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "views/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16",
        "data": "synthetic",
        "config": {"workload": f"dense views: {args.cams}-camera synthetic arc at {H}x{W}, "
                               f"{len(pairs)} adjacent pairs x {len(ts)} phases t=k/{len(ts) + 1} "
                               f"= {n_views} views per call, BF16 convs, fp32 accumulation",
                   "views_per_step": n_views, "height": H, "width": W},
        "roofline": roof,
        "cpu_baseline": cpu,
        "psnr_db_vs_oracle": None if psnr is None else round(psnr, 2),
        "latency_ms": {"p50": round(percentile(step_ms, 0.5), 3),
                       "p99": round(percentile(step_ms, 0.99), 3), "per": "step"},
        "fp32_plain": fp32,
        "bf16_vs_fp32": None if fp32 is None else round(value / fp32["views_per_s"], 2),
        "conv_mfma_util": round(conv_flops / (conv_ms * 1e-3) / 1e12 / PEAK_BF16_TFLOPS, 4)
        if conv_ms > 0 else None,
        "kernel_ms_per_step": breakdown,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
