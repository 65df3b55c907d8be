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
# FP8 accuracy bound against the BF16 path on the same input: e4m3 keeps 3
# mantissa bits (unit roundoff 2^-4), bf16 7 (2^-8); to first order the
# output error grows with the unit roundoff, so the MSE may grow by at most
# (2^-4 / 2^-8)^2 = 256 (24.08 dB), plus a factor 2 (3.01 dB) for values
# beyond the calibrated range that saturate
FP8_PSNR_DROP_DB = 27.09


COUNTERS_FILE = os.path.join(ROOT, "profiles", "conv_igemm_dense1080p_bf16_hbm_counters.md")
MFMA_FILE = os.path.join(ROOT, "profiles", "conv_igemm_dense1080p_bf16_mfma_util.md")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2112_10603_amd", "csrc", f)
                  for f in ("conv_kernel.h", "conv_halo.h", "conv_resident.h", "conv_resident_s2.h", "conv.hip",
                            "pixel.hip")]


def _counters_text(path=COUNTERS_FILE):
    """A committed counter summary, or None when the kernel sources no
    longer hash to the value its counters were taken with."""
    import hashlib
    import re
    try:
        text = open(path).read()
    except OSError:
        return None
    h = re.search(r"kernel-source-sha256: ([0-9a-f]{64})", text)
    if not h:
        return None
    cur = hashlib.sha256()
    for f in KERNEL_SOURCES:
        cur.update(open(f, "rb").read())
    return text if cur.hexdigest() == h.group(1) else None


def measured_traffic():
    """HBM bytes per launch of the 256->256 conv class from the committed
    counter summary (two rocprofv3 --pmc passes, FETCH_SIZE and WRITE_SIZE,
    scaled by a plain copy), or None when it is stale."""
    import re
    text = _counters_text()
    t = re.search(r"conv256-traffic-bytes-per-launch: (\d+)", text) if text else None
    return int(t.group(1)) if t else None


def measured_pixel_hbm():
    """HBM GB/s of the per-pixel passes (warps, blend, resampling) over one
    step, from the same committed counters: their FETCH + WRITE bytes over
    their summed kernel-trace durations; None when stale."""
    text = _counters_text()
    if not text:
        return None
    gb = ms = 0.0
    for line in text.splitlines():
        f = [c.strip() for c in line.split("|")]
        if len(f) >= 9 and f[5] == "pixel":
            try:
                ms += float(f[4])
                gb += float(f[6]) + float(f[7])
            except ValueError:
                continue
    return round(gb / (ms * 1e-3), 1) if ms > 0 else None


def measured_mfma_busy():
    """MFMA-busy fraction of the convolutions from the committed rocprofv3
    --pmc summary (MfmaUtil: SQ_VALU_MFMA_BUSY_CYCLES over GRBM_GUI_ACTIVE
    times the SIMD count, each launch weighted by its trace duration), or
    None when it is stale."""
    import re
    text = _counters_text(MFMA_FILE)
    if not text:
        return None
    out = {}
    for key in ("conv256", "conv", "convT", "all-convs"):
        m = re.search(rf"^mfma-busy-{key}: ([0-9.]+)$", text, re.M)
        if m:
            out[key.replace("-", "_")] = float(m.group(1))
    if not out:
        return None
    out["counter"] = "MfmaUtil = SQ_VALU_MFMA_BUSY_CYCLES / (GRBM_GUI_ACTIVE x SIMDs), duration-weighted"
    return out


def conv256_ideal_bytes(n_views, Hp, Wp, width=256):
    """Algorithmic HBM bytes per launch of the 256->256 conv class, averaged
    over its launches in one step: each launch reads its BF16 input once,
    writes its BF16 output once and reads its weights once. The class is the
    six 3x3 256->256 convs of each VIBlock (at 1/16, 1/8, 1/4 of the padded
    pixels) and the deepest U-Net encoder conv (1/16)."""
    w_bytes = width * width * 9 * 2
    sizes = []
    for s in range(3):
        px = (Hp * (1 << s) // 16) * (Wp * (1 << s) // 16)
        sizes += [px] * 6
    sizes.append((Hp // 16) * (Wp // 16))
    per = [2 * n_views * px * width * 2 + w_bytes for px in sizes]
    return sum(per) / len(per)


def pixel_bytes_min(n_cams, n_views, H, W, e=2, base=32):
    """Algorithmic HBM bytes of one call's per-pixel passes: every source a
    pass needs read once and every product written once, at the real
    channel counts (images and flow/mask fp32, activations e bytes). Per
    camera: ingest + pad to the 16-multiple grid and the bilinear 1/4 and
    1/2 copies. Per view: the stage-0 input; the two stage transitions of
    Eq. 2 (previous flow and mask at half size, the stage's two images in,
    the 18-channel input and the upsampled flow and mask out); the final
    warp and Eq. 1 blend (flow and mask, both views in; the blend and the
    17-channel refinement input out); the halved flow pyramid and the
    context-feature warps (both views' features in, both warped copies out).
    Returns (pixel-class bytes, output-head bytes)."""
    Hp, Wp = (H + 15) // 16 * 16, (W + 15) // 16 * 16
    P = Hp * Wp
    cam = 12 * H * W + 12 * P + (12 * P + 12 * P / 16) + (12 * P + 12 * P / 4)
    view = 24 * P / 16 + 7 * e * P / 16
    for Pp, Ps in ((P / 16, P / 4), (P / 4, P)):
        view += 20 * Pp + 24 * Ps + 18 * e * Ps + 20 * Ps
    view += 20 * P + 24 * P + 12 * P + 17 * e * P
    cw = (base // 2, base, 2 * base, 4 * base)
    for k in range(1, 5):
        Pk = P / 4 ** k
        view += 16 * P / 4 ** (k - 1) + 16 * Pk          # flow pyramid level k
        view += 16 * Pk + 2 * cw[k - 1] * e * Pk * 2      # context warps of level k
    head = (base // 2) * e * P + 12 * P + 12 * H * W
    return n_cams * cam + n_views * view, n_views * head


def clamped_frac(img):
    """Fraction of output values the final clamp to [0, 1] decided (exactly
    0 or 1)."""
    import numpy as np
    a = np.asarray(img)
    return round(float(np.mean((a <= 0.0) | (a >= 1.0))), 6)


def error_stats(got, ref):
    """Max-abs error, PSNR (peak 1, FP64) and clamped fraction of one output
    against the oracle's."""
    import numpy as np
    d = np.asarray(got, np.float64) - np.asarray(ref, np.float64)
    mse = float(np.mean(d * d))
    return {"max_abs": float(f"{float(np.abs(d).max()):.3e}"),
            "psnr_db": round(10 * math.log10(1.0 / mse), 2) if mse > 0 else float("inf"),
            "clamped_frac": clamped_frac(got)}


def percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return float("nan")
    k = (len(xs) - 1) * q
    lo, hi = math.floor(k), math.ceil(k)
    return xs[lo] + (xs[hi] - xs[lo]) * (k - lo)


def serve_leg(wpath, dev, seconds, rate_fraction=None, capacity=None, users=64, per_user_rps=30.0,
              max_batch=32, budget=64 << 30, tick_ms=5.0, pool=256):
    """Multi-user serving: two 8-camera arcs (1280x720 and 1920x1080), each
    request a random adjacent pair, t ~ U(0, 1), resolution 50/50; Poisson
    arrivals (users x per_user_rps, or rate_fraction x capacity). Requests
    that find no free output buffer are shed. Returns counts and latency
    percentiles of completed requests (submit -> written)."""
    import numpy as np
    import torch

    from paper_2112_10603_amd import Net
    from synth import scenes

    net = Net(wpath, "bf16", 0, hbm_budget_bytes=budget, tick_ms=tick_ms, max_batch_views=max_batch)
    arcs = {720: scenes.camera_arc(50, 720, 1280, 8, 1024, (8.0, 64.0), 48.0, 0.01, device=dev),
            1080: scenes.camera_arc(51, 1080, 1920, 8, 1024, (8.0, 64.0), 48.0, 0.01, device=dev)}
    for res, arc in arcs.items():
        for j in range(8):
            net.register_camera(res * 100 + j, arc[j].contiguous())
    bufs = {res: [torch.empty((3,) + tuple(arcs[res].shape[2:]), device=dev) for _ in range(pool)]
            for res in arcs}
    free = {res: list(range(pool)) for res in arcs}
    rate = users * per_user_rps if rate_fraction is None else rate_fraction * capacity
    rng = np.random.default_rng(52)
    n_max = int(rate * seconds * 1.5) + 10
    arrivals = np.cumsum(rng.exponential(1.0 / rate, n_max))
    arrivals = arrivals[arrivals < seconds]
    res_pick = rng.random(len(arrivals)) < 0.5
    pair_pick = rng.integers(0, 7, len(arrivals))
    t_pick = rng.uniform(0.0, 1.0, len(arrivals))
    pending = {}
    lat = []
    shed = 0
    i = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    while True:
        now = time.perf_counter() - t0
        while i < len(arrivals) and arrivals[i] <= now:
            res = 720 if res_pick[i] else 1080
            if free[res]:
                b = free[res].pop()
                cam = res * 100 + int(pair_pick[i])
                tk = net.submit(cam, cam + 1, float(t_pick[i]), bufs[res][b])
                pending[tk] = (res, b)
            else:
                shed += 1
            i += 1
        for tk in list(pending):
            tm = net.poll(tk)
            if tm is not None:
                res, b = pending.pop(tk)
                free[res].append(b)
                if now <= seconds:
                    lat.append(1000.0 * (tm["t_done"] - tm["t_submit"]))
        if now > seconds:
            break
        time.sleep(0.0005)
    window = time.perf_counter() - t0
    st = net.serving_stats()
    in_flight = len(pending)
    # drain what was admitted before closing (outputs must stay alive)
    while pending:
        for tk in list(pending):
            if net.poll(tk) is not None:
                pending.pop(tk)
        time.sleep(0.001)
    net.close()
    return {"offered_rps": round(len(arrivals) / seconds, 1),
            "completed_views_per_s": round(len(lat) / window, 2),
            "p50_ms": round(percentile(lat, 0.5), 2), "p99_ms": round(percentile(lat, 0.99), 2),
            "completed": len(lat), "client_shed_no_output_buffer": shed,
            "client_pool_buffers_per_resolution": pool,
            "client_waiting_at_end": in_flight, "server_queued_at_end": st["queued"],
            "admitted": st["admitted"], "window_s": round(window, 2), "max_batch_views": max_batch,
            "budget_gib": budget >> 30, "tick_ms": tick_ms}


PEAK_FP8_TFLOPS = 5000.0


def fp8_calibrated_net(wpath, dev, workspace_bytes):
    """An FP8 net calibrated on a 256x256 crop of a separately seeded 4K
    scene (seed 99), t = 1/2."""
    from paper_2112_10603_amd import Net
    from synth import scenes
    cal = scenes.uhd_arc(2, seed=99, device=dev)
    net = Net(wpath, "fp8", 0, workspace_bytes=workspace_bytes)
    net.calibrate(cal[0, :, 1000:1256, 1800:2056].contiguous(),
                  cal[1, :, 1000:1256, 1800:2056].contiguous(), 0.5)
    return net


def conv_roofline(stats, steps):
    """conv256 class and all-conv TFLOP/s from the library's per-class HIP
    event timing, against the FP8 dense peak."""
    out = {}
    c = stats["conv256"]
    if c["ms"] > 0:
        tf = c["work"] / (c["ms"] * 1e-3) / 1e12
        out["conv256"] = {"avg_launch_ms": round(c["ms"] / c["launches"], 4), "tflops": round(tf, 1),
                          "frac_of_fp8_peak": round(tf / PEAK_FP8_TFLOPS, 4)}
    ms = sum(stats[k]["ms"] for k in ("conv256", "conv", "convT"))
    work = sum(stats[k]["work"] for k in ("conv256", "conv", "convT"))
    if ms > 0:
        out["all_convs"] = {"ms_per_step": round(ms / steps, 3), "tflops": round(work / (ms * 1e-3) / 1e12, 1)}
    return out


def fp8_dense_leg(wpath, dev, pairs, ts, steps=5, warmup=2):
    """FP8 on the dense 1080p batch (the same 112 views as the headline
    step): calibrated as the 4K leg, conv tiles autotuned in FP8, views/s and
    the conv classes' TFLOP/s against the FP8 peak. Returns the result and
    pair 0's view at the oracle check's phase."""
    import torch
    net = fp8_calibrated_net(wpath, dev, 128 << 30)
    H, W = pairs[0][0].shape[1:]
    out = torch.empty((len(pairs), len(ts), 3, H, W), dtype=torch.float32, device=dev)
    net.autotune(pairs, ts, out)
    net.set_profiling(True)
    for _ in range(warmup):
        net.interpolate(pairs, ts, out)
    torch.cuda.synchronize()
    net.set_profiling(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        net.interpolate(pairs, ts, out)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    stats = {k: net.kernel_stats(k) for k in ("conv256", "conv", "convT")}
    net.set_profiling(False)
    view = out[0, len(ts) // 2 - 1].cpu().numpy()
    n = len(pairs) * len(ts)
    res = {"views_per_s": round(n / dt, 2), "ms_per_step": round(1000 * dt, 2), "views_per_step": n,
           "workload": f"the dense batch ({n} views of {H}x{W}); VIBlock 128/256-ch convs fp8 e4m3, "
                       "other convs bf16; tiles autotuned in fp8",
           "conv_roofline": conv_roofline(stats, steps)}
    net.close()
    return res, view


def fp8_4k_leg(wpath, dev, reps=3, with_oracle=True, crops_per_pair=4, tune_file=None):
    """FP8 at 4K: 4 independent pairs of 3x2160x3840 (disparity 0..96 px),
    t = 0.5, one call for all four; FP8 e4m3 VIBlock convs calibrated on a
    256x256 crop of a separately seeded 4K scene. Error against the FP64
    oracle on seeded 256x256 input crops (4 per pair; the library and the
    oracle both run on the crop, since a crop of the 4K output is not the
    network applied to a crop)."""
    import numpy as np
    import torch

    from paper_2112_10603_amd import Net
    from synth import scenes

    pairs = [scenes.uhd_arc(2, seed=40 + i, device=dev) for i in range(4)]
    net = fp8_calibrated_net(wpath, dev, 64 << 30)
    pv = [(p[0], p[1]) for p in pairs]
    out = torch.empty((4, 1, 3, 2160, 3840), dtype=torch.float32, device=dev)
    if tune_file and os.path.exists(tune_file):
        net.load_tuning(tune_file)
    else:
        net.autotune(pv, [0.5], out)
        if tune_file:
            net.save_tuning(tune_file)
    net.set_profiling(True)
    net.interpolate(pv, [0.5], out)
    torch.cuda.synchronize()
    net.set_profiling(True)
    t0 = time.perf_counter()
    for _ in range(reps):
        net.interpolate(pv, [0.5], out)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    stats = {k: net.kernel_stats(k) for k in ("conv256", "conv", "convT")}
    net.set_profiling(False)
    res = {"views_per_s": round(4 / dt, 2), "ms_per_call": round(1000 * dt, 2),
           "workload": "4 pairs 2160x3840, t=0.5, one call; VIBlock 128/256-ch convs fp8 e4m3 "
                       "(per-channel scales), other convs bf16; tiles autotuned in fp8",
           "conv_roofline": conv_roofline(stats, reps)}
    if with_oracle:
        from oracle import vinet as oracle
        Wo = oracle.load_weights(wpath)
        net16 = Net(wpath, "bf16", 0, workspace_bytes=8 << 30)
        rng = np.random.default_rng(7)
        s8, s16, slack = [], [], []
        t_or = time.perf_counter()
        for p in pairs:
            for _ in range(crops_per_pair):
                y0 = int(rng.integers(0, 2160 - 256))
                x0 = int(rng.integers(0, 3840 - 256))
                l = p[0, :, y0:y0 + 256, x0:x0 + 256].contiguous()
                r = p[1, :, y0:y0 + 256, x0:x0 + 256].contiguous()
                got = net.interpolate([(l, r)], [0.5])[0, 0].cpu().numpy()
                g16 = net16.interpolate([(l, r)], [0.5])[0, 0].cpu().numpy()
                ref = oracle.vinet_forward(l.cpu().numpy(), r.cpu().numpy(), 0.5, Wo)
                s8.append(error_stats(got, ref))
                s16.append(error_stats(g16, ref))
                slack.append(s8[-1]["psnr_db"] - (s16[-1]["psnr_db"] - FP8_PSNR_DROP_DB))
        net16.close()
        p8 = [x["psnr_db"] for x in s8]
        p16 = [x["psnr_db"] for x in s16]
        res["psnr_db_vs_oracle_256_crops"] = {"min": round(min(p8), 2), "mean": round(sum(p8) / len(p8), 2),
                                               "n": len(p8)}
        res["max_abs_vs_oracle_256_crops"] = max(x["max_abs"] for x in s8)
        res["clamped_frac_256_crops"] = round(sum(x["clamped_frac"] for x in s8) / len(s8), 6)
        res["bf16_same_crops"] = {"psnr_db_min": round(min(p16), 2), "psnr_db_mean": round(sum(p16) / len(p16), 2),
                                  "max_abs": max(x["max_abs"] for x in s16)}
        res["bound"] = {"rule": f"PSNR_fp8 >= PSNR_bf16 - {FP8_PSNR_DROP_DB} dB on the same crop",
                        "min_slack_db": round(min(slack), 2), "met": min(slack) >= 0.0}
        res["oracle_s_per_256_crop"] = round((time.perf_counter() - t_or) / len(p8), 2)
    net.close()
    return res


def lap_loss_leg(views, gt, reps=10):
    """The Eq. 3 Laplacian-pyramid loss (training side) on a batch of
    synthesised views against a reference image: forward only, and forward
    with the gradient; milliseconds per view and GB/s against the algorithmic
    bytes (read both images once; write the gradient once)."""
    import torch

    from paper_2112_10603_amd import lap_loss

    n, _, H, W = views.shape
    res = {"views": n, "size": f"{H}x{W}"}
    for grad in (False, True):
        lap_loss(views, gt, grad=grad)
        s = torch.cuda.current_stream(views.device)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        for _ in range(reps):
            lap_loss(views, gt, grad=grad)
        e1.record(s)
        e1.synchronize()
        ms = e0.elapsed_time(e1) / reps
        nbytes = n * 3 * H * W * 4 * (3 if grad else 2)
        key = "loss_and_grad" if grad else "loss"
        res[key] = {"ms_per_view": round(ms / n, 4), "gbs_algorithmic": round(nbytes / (ms * 1e-3) / 1e9, 1),
                    "note": "includes the call's workspace allocation and stream synchronisation"}
    return res


def next_leg(wpath, dev, reps=5):
    """The paper's two other inference modes, timed on the GPU beside the
    direct t-plane path (BF16, batch of one pair, inputs resident):
    * w/o Refine (the Eq. 1 blend alone; Table 1) against the full network,
      one 1280x720 pair at t = 1/2;
    * recursive midpoints (section 4) against direct phases for the dyadic
      t in {1/4, 1/2, 3/4}, one 1080p pair: two dependent levels (1 + 2
      syntheses) versus one call with three phases, and how far the two
      results lie apart (PSNR of one against the other; both are valid
      views of different methods)."""
    import numpy as np
    import torch

    from paper_2112_10603_amd import Net
    from synth import scenes

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        a = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return 1000.0 * (time.perf_counter() - a) / reps

    net = Net(wpath, "bf16", 0, workspace_bytes=32 << 30)
    hd = scenes.camera_arc(50, 720, 1280, 2, 1024, (8.0, 64.0), 48.0, 0.01, device=dev)
    p720 = [(hd[0], hd[1])]
    o1 = torch.empty((1, 1, 3, 720, 1280), device=dev)
    full_ms = timed(lambda: net.interpolate(p720, [0.5], o1))
    blend_ms = timed(lambda: net.interpolate_blend(p720, [0.5], o1))
    fhd = scenes.camera_arc(2, 1080, 1920, 2, 1024, (8.0, 64.0), 48.0, 0.01, device=dev)
    p1080 = [(fhd[0], fhd[1])]
    od = torch.empty((1, 3, 3, 1080, 1920), device=dev)
    orc = torch.empty((1, 3, 3, 1080, 1920), device=dev)
    direct_ms = timed(lambda: net.interpolate(p1080, [0.25, 0.5, 0.75], od))
    rec_ms = timed(lambda: net.interpolate_recursive(p1080, 2, orc))
    mse = torch.mean((od.double() - orc.double()) ** 2).item()
    net.close()
    return {"w/o_refine_720p": {"full_ms": round(full_ms, 3), "blend_only_ms": round(blend_ms, 3),
                                "paper_table1_ms_rtx_a6000": {"full": 12.85, "w/o_refine": 6.27}},
            "recursive_vs_direct_1080p_dyadic": {
                "direct_3_phases_ms": round(direct_ms, 3), "recursive_2_levels_ms": round(rec_ms, 3),
                "psnr_db_between_methods": round(10 * math.log10(1.0 / mse), 2) if mse > 0 else None}}


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
    ap.add_argument("--no-serve", action="store_true", help="skip the serving leg")
    ap.add_argument("--serve-seconds", type=float, default=4.0)
    ap.add_argument("--no-fp8", action="store_true", help="skip the FP8 4K leg")
    ap.add_argument("--no-tune", action="store_true", help="skip conv tile autotuning")
    ap.add_argument("--no-next", action="store_true", help="skip the w/o-refine and recursive leg")
    ap.add_argument("--fp8-only", action="store_true",
                    help="run only the FP8 4K leg (its own JSON line, no oracle; for profiling); "
                         "--tune-file then names the FP8 tuning table")
    ap.add_argument("--tune-file", default=None,
                    help="load the conv tuning table from this file if it exists, else tune and "
                         "save it there")
    ap.add_argument("--copy-calib", action="store_true",
                    help="first run a plain 1 GiB device-to-device copy (counter calibration)")
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
    if args.fp8_only:
        td = tempfile.mkdtemp()
        wpath = write_weights_file(os.path.join(td, "w.ffvw"), seed=0)
        print(json.dumps(fp8_4k_leg(wpath, dev, with_oracle=False, tune_file=args.tune_file)), flush=True)
        return
    if args.copy_calib:
        src = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print("[bench] copy calibration: 1 GiB read + 1 GiB written", file=sys.stderr, flush=True)
        del src, dst
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
    tune = None
    if args.tune_file and os.path.exists(args.tune_file):
        tune = {"launch_shapes": net.load_tuning(args.tune_file), "loaded_from": args.tune_file}
        print(f"[bench] loaded {tune['launch_shapes']} conv tile choices", file=sys.stderr, flush=True)
    elif not args.no_tune:
        a = time.perf_counter()
        n_tuned = net.autotune(pairs, ts, out)
        tune = {"launch_shapes": n_tuned, "seconds": round(time.perf_counter() - a, 2)}
        print(f"[bench] autotuned {n_tuned} conv launch shapes in {tune['seconds']} s",
              file=sys.stderr, flush=True)
        if args.tune_file:
            net.save_tuning(args.tune_file)
    # profiling on before the warm-up, so the warm-up captures the graph the
    # timed steps replay; switching it on again clears the warm-up's stats
    net.set_profiling(True)
    for _ in range(max(1, args.warmup)):
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
    # the committed counters were taken on this workload only
    default_workload = (H, W, args.cams, args.phases) == (1080, 1920, 8, 16)
    roof = None
    if dom["launches"] > 0:
        avg_ms = dom["ms"] / dom["launches"]
        flops_per_launch = dom["work"] / dom["launches"]
        achieved = flops_per_launch / (avg_ms * 1e-3) / 1e12
        traffic = measured_traffic() if default_workload else None
        Hp, Wp = (H + 15) // 16 * 16, (W + 15) // 16 * 16
        roof = {"bound": "mfma", "achieved": round(achieved, 2), "peak": PEAK_BF16_TFLOPS,
                "unit": "TFLOP/s", "frac": round(achieved / PEAK_BF16_TFLOPS, 4), "traffic": traffic,
                "traffic_unit": "HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, copy-scaled)",
                "algorithmic_bytes_per_launch": round(conv256_ideal_bytes(n_views, Hp, Wp)),
                "kernel": "conv_igemm bf16, 3x3 256->256 (VIBlock conv3-8)",
                "avg_launch_ms": round(avg_ms, 4), "flops_per_launch": flops_per_launch}
    # per-pixel passes: algorithmic bytes (every source read once, every
    # product written once, real channel counts) over their measured time,
    # against the 8 TB/s HBM peak; the library's own byte model (4-tap
    # gathers, padded channel layouts) is reported beside it
    px = stats["pixel"]
    hd = stats["head"]
    pixel_passes = None
    if px["ms"] > 0:
        px_bytes, head_bytes = pixel_bytes_min(args.cams, n_views, H, W)
        px_s = px["ms"] / args.steps * 1e-3
        gbs = px_bytes / px_s / 1e9
        pixel_passes = {"ms_per_step": round(px["ms"] / args.steps, 3),
                        "algorithmic_gb_per_step": round(px_bytes / 1e9, 2),
                        "achieved_gbs_algorithmic": round(gbs, 1),
                        "frac_of_hbm_peak": round(gbs / PEAK_HBM_GBS, 3),
                        "library_model_gb_per_step": round(px["work"] / args.steps / 1e9, 2),
                        "achieved_gbs_library_model": round(px["work"] / (px["ms"] * 1e-3) / 1e9, 1),
                        "hbm_gbs_measured": measured_pixel_hbm() if default_workload else None,
                        "kernels": "ingest, pyramid, stage transitions (warps), final warp + blend, "
                                   "flow pyramid, context warps"}
        if hd["ms"] > 0:
            hg = head_bytes / (hd["ms"] / args.steps * 1e-3) / 1e9
            pixel_passes["head"] = {"ms_per_step": round(hd["ms"] / args.steps, 3),
                                    "algorithmic_gb_per_step": round(head_bytes / 1e9, 2),
                                    "achieved_gbs_algorithmic": round(hg, 1),
                                    "frac_of_hbm_peak": round(hg / PEAK_HBM_GBS, 3)}
    conv_ms = sum(stats[k]["ms"] for k in ("conv256", "conv", "convT"))
    conv_flops = sum(stats[k]["work"] for k in ("conv256", "conv", "convT"))
    breakdown = {k: {"launches": v["launches"], "ms_per_step": round(v["ms"] / args.steps, 3)}
                 for k, v in stats.items()}

    # cluster frame of the middle camera from this step's outputs (the
    # Multiview Organizer): its real view between 16 views on either side
    stitch = None
    if len(pairs) >= 2 and len(ts) == 16 and H % 4 == 0 and W % 4 == 0:
        from paper_2112_10603_amd import stitch_cluster
        c = len(pairs) // 2 + 1 if len(pairs) > 2 else 1
        left = [out[c - 1, k] for k in range(16)]    # far (t ~ 0) to near the camera
        right = [out[c, k] for k in range(16)]       # near the camera outwards
        frame = torch.empty((3, H, 3 * W), device=dev)
        cs = torch.cuda.current_stream(dev)
        stitch_cluster(arc[c], left, right, frame)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = 20
        e0.record(cs)
        for _ in range(reps):
            stitch_cluster(arc[c], left, right, frame)
        e1.record(cs)
        e1.synchronize()
        ms = e0.elapsed_time(e1) / reps
        nbytes = 33 * 3 * H * W * 4 + 3 * H * 3 * W * 4
        stitch = {"ms_per_cluster_frame": round(ms, 4), "frame": f"3x{H}x{3 * W} fp32, 33 views",
                  "hbm_gbs_algorithmic": round(nbytes / (ms * 1e-3) / 1e9, 1),
                  "paper_table2_adaptive_stitch_ms": 1.27}
        del frame

    # one BF16 view kept for the PSNR check: pair 0, t = 8/17
    j_ref = len(ts) // 2 - 1
    bf16_view = out[0, j_ref].cpu().numpy()
    # the training-side loss of Eq. 3 over pair 0's views against camera 1
    lap = None
    if H >= 33 and W >= 33:
        lap = lap_loss_leg(out[0].contiguous(), arc[1].expand(len(ts), -1, -1, -1).contiguous())
    net.close()
    del out

    fp32 = None
    fp32_view = None
    if not args.no_fp32:
        # the plain FP32 path: one 1080p pair, batch 1, one call per phase;
        # 3 warm-up calls, then the median of 21 calls timed with HIP events
        # on the library's stream
        net32 = Net(wpath, "fp32", 0, workspace_bytes=64 << 30)
        l, r = pairs[0]
        o1 = torch.empty((1, 1, 3, H, W), dtype=torch.float32, device=dev)
        for t in (0.25, 0.5, 0.75):
            net32.interpolate([(l, r)], [t], o1)
        torch.cuda.synchronize()
        lat = []
        for _ in range(7):
            for t in (0.25, 0.5, 0.75):
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(net32.stream)
                net32.interpolate([(l, r)], [t], o1)
                e1.record(net32.stream)
                e1.synchronize()
                lat.append(e0.elapsed_time(e1))
        med = percentile(lat, 0.5)
        v32 = 1000.0 / med
        fp32 = {"views_per_s": round(v32, 2), "ms_per_view_p50": round(med, 3),
                "ms_per_view_p99": round(percentile(lat, 0.99), 3), "timed_calls": len(lat),
                "warmup_calls": 3,
                "workload": "one 1080p pair, batch 1, t in {0.25, 0.5, 0.75}, FP32 convs; "
                            "views/s = 1000 / median ms per call"}
        # the same view the oracle computes below (pair 0, t = 8/17)
        net32.interpolate([(l, r)], [ts[j_ref]], o1)
        fp32_view = o1[0, 0].cpu().numpy()
        net32.close()
        print(f"[bench] fp32 plain {v32:.2f} views/s", file=sys.stderr, flush=True)

    serving = None
    if not args.no_serve:
        sat = serve_leg(wpath, dev, args.serve_seconds)
        print(f"[bench] serving at offered {sat['offered_rps']} req/s: "
              f"{sat['completed_views_per_s']} views/s, p99 {sat['p99_ms']} ms",
              file=sys.stderr, flush=True)
        sub = serve_leg(wpath, dev, args.serve_seconds, rate_fraction=0.7,
                        capacity=max(1.0, sat["completed_views_per_s"]))
        print(f"[bench] serving at 70% capacity: p50 {sub['p50_ms']} ms, p99 {sub['p99_ms']} ms",
              file=sys.stderr, flush=True)
        serving = {"workload": "two 8-camera arcs (1280x720, 1920x1080), 64 users x 30 req/s "
                               "Poisson, random adjacent pair, t~U(0,1), 50/50 resolution, "
                               "5 ms tick, 64 GiB budget, BF16",
                   "saturation": sat, "at_70pct_capacity": sub}

    fp8 = None
    if not args.no_fp8:
        fp8 = fp8_4k_leg(wpath, dev, with_oracle=not args.no_oracle)
        print(f"[bench] fp8 4K: {fp8['views_per_s']} views/s", file=sys.stderr, flush=True)

    fp8_dense = None
    fp8_dense_view = None
    if not args.no_fp8:
        fp8_dense, fp8_dense_view = fp8_dense_leg(wpath, dev, pairs, ts)
        print(f"[bench] fp8 dense: {fp8_dense['views_per_s']} views/s", file=sys.stderr, flush=True)

    modes = None
    if not args.no_next:
        modes = next_leg(wpath, dev)
        print(f"[bench] modes: {modes}", file=sys.stderr, flush=True)

    cpu = None
    psnr = None
    accuracy = None
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
        accuracy = {"view": f"pair 0, t=8/17, full {H}x{W} output against the FP64 oracle",
                    "oracle_clamped_frac": clamped_frac(ref),
                    "bf16": error_stats(bf16_view, ref)}
        if fp32_view is not None:
            accuracy["fp32"] = error_stats(fp32_view, ref)
            accuracy["fp32"]["target_max_abs"] = 1e-4
            accuracy["fp32"]["target_met"] = accuracy["fp32"]["max_abs"] <= 1e-4
        if fp8_dense_view is not None:
            accuracy["fp8"] = error_stats(fp8_dense_view, ref)
        accuracy["bf16"]["target_psnr_db"] = 45.0
        accuracy["bf16"]["target_met"] = accuracy["bf16"]["psnr_db"] >= 45.0
        psnr = accuracy["bf16"]["psnr_db"]
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
        "accuracy_vs_oracle": accuracy,
        "latency_ms": {"p50": round(percentile(step_ms, 0.5), 3),
                       "p99": round(percentile(step_ms, 0.99), 3),
                       "per": "step of the dense-view batch (serving request latency in 'serving')"},
        "fp32_plain": fp32,
        "serving": serving,
        "fp8_4k": fp8,
        "fp8_dense_1080p": fp8_dense,
        "inference_modes": modes,
        "pixel_passes": pixel_passes,
        "cluster_stitch": stitch,
        "lap_loss_eq3": lap,
        "bf16_vs_fp32": None if fp32 is None else round(value / fp32["views_per_s"], 2),
        "conv_mfma_util": round(conv_flops / (conv_ms * 1e-3) / 1e12 / PEAK_BF16_TFLOPS, 4)
        if conv_ms > 0 else None,
        "conv_mfma_util_target": {"target": 0.60,
                                  "met": bool(conv_ms > 0 and conv_flops / (conv_ms * 1e-3) / 1e12
                                              / PEAK_BF16_TFLOPS >= 0.60)},
        "mfma_busy_rocprof": measured_mfma_busy() if default_workload else None,
        "kernel_ms_per_step": breakdown,
        "autotune": tune,
        "timed_as": "one hipGraph replay per step (captured on the first warm-up call), "
                    "event-record nodes around each kernel class",
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
