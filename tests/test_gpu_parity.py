"""Whole-network parity: the HIP path (through the C ABI) against the FP64
oracle on the same seeded inputs and weights.

Bars: FP32 max-abs <= 1e-4 on [0, 1] pixels; BF16 PSNR >= 45 dB; the
closed-form structured-weight cases exact up to fp32 rounding."""
import math
import os

import numpy as np
import pytest
import torch

from oracle import vinet as O
from synth import scenes
from synth.weights import write_weights_file

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")


def psnr(a, b):
    mse = float(np.mean((np.asarray(a, np.float64) - np.asarray(b, np.float64)) ** 2))
    return float("inf") if mse == 0 else 10 * math.log10(1.0 / mse)


@pytest.fixture(scope="module")
def wfile(tmp_path_factory):
    return write_weights_file(str(tmp_path_factory.mktemp("w") / "w0.ffvw"), seed=0)


@pytest.fixture(scope="module")
def oracle_w(wfile):
    return O.load_weights(wfile)


def _net(path, precision="fp32", **kw):
    from paper_2112_10603_amd import Net
    return Net(path, precision, 0, **kw)


def test_small_fp32_parity_with_taps(wfile, oracle_w):
    """128x128, right = left shifted 4 px, t = 0.5 (the small workload)."""
    print("case small fp32 128x128", flush=True)
    xl, xr = scenes.small_pair()
    net = _net(wfile)
    net.set_debug(True)
    out = net.interpolate([(xl.to(DEV), xr.to(DEV))], [0.5])[0, 0].cpu().numpy()
    taps = {}
    ref = O.vinet_forward(xl.numpy(), xr.numpy(), 0.5, oracle_w, taps)
    for s in range(3):
        g = net.debug_tap(f"F{s}").cpu().numpy()
        want = np.concatenate([taps[f"F{s}"], taps[f"M{s}"]])
        e = np.abs(g - want).max()
        print(f"  stage {s} flow/mask max-abs {e:.3e} (|F| max {np.abs(want).max():.2f})")
        assert e < 1e-3, (s, e)
    i2 = net.debug_tap("I2").cpu().numpy()
    e = np.abs(i2 - taps["I2"]).max()
    print(f"  I2 max-abs {e:.3e}")
    assert e < 1e-4
    err = np.abs(out - ref).max()
    print(f"  output max-abs {err:.3e}")
    assert err <= 1e-4
    net.close()


@pytest.mark.parametrize("H,W", [(128, 128), (72, 136)])
def test_refinement_stages_fp32(wfile, oracle_w, H, W):
    """Stage by stage through the refinement path (section 3.1, "Refinement
    Network"): the U-Net input, the context features of both views and their
    warped copies at each level, every encoder and decoder output, against
    the oracle's intermediates, relative to each tensor's magnitude."""
    print(f"case refinement taps fp32 {H}x{W}", flush=True)
    xl, xr = scenes.random_pair(23, H, W, d_max=6.0)
    net = _net(wfile)
    net.set_debug(True)
    net.interpolate([(xl.to(DEV), xr.to(DEV))], [0.4])
    taps = {}
    O.vinet_forward(xl.numpy(), xr.numpy(), 0.4, oracle_w, taps)
    want = {"x0": taps["x0"]}
    for k in range(1, 5):
        want[f"d{k}"] = taps[f"d{k}"]
        want[f"u{k}"] = taps[f"u{k}"]
        want[f"cl{k}"] = taps["ctx_l"][k - 1]
        want[f"cr{k}"] = taps["ctx_r"][k - 1]
        want[f"wcl{k}"] = taps["wc"][k - 1][0]
        want[f"wcr{k}"] = taps["wc"][k - 1][1]
    for name, ref in want.items():
        got = net.debug_tap(name).cpu().numpy()
        assert got.shape == ref.shape, (name, got.shape, ref.shape)
        scale = max(1.0, float(np.abs(ref).max()))
        e = float(np.abs(got - ref).max()) / scale
        print(f"  {name:5s} {str(ref.shape):18s} rel max-abs {e:.2e}")
        assert e <= 1e-4, (name, e)
    net.close()


@pytest.mark.parametrize("H,W,t", [(72, 136, 0.3), (48, 50, 1.0), (33, 17, 0.0)])
def test_ragged_fp32_parity(wfile, oracle_w, H, W, t):
    """Sizes that are not multiples of 16 (replicate pad + crop), several
    tiles and a ragged tail in every conv."""
    print(f"case ragged fp32 {H}x{W} t={t}", flush=True)
    xl, xr = scenes.random_pair(21, H, W, d_max=5.0)
    net = _net(wfile)
    out = net.interpolate([(xl.to(DEV), xr.to(DEV))], [t])[0, 0].cpu().numpy()
    ref = O.vinet_forward(xl.numpy(), xr.numpy(), t, oracle_w)
    err = np.abs(out - ref).max()
    print(f"  max-abs {err:.3e}")
    assert err <= 1e-4
    net.close()


def test_zero_heads_closed_form(tmp_path):
    print("case zero heads", flush=True)
    p = write_weights_file(str(tmp_path / "z.ffvw"), seed=3, kind="zero_heads")
    xl, xr = scenes.random_pair(7, 40, 72)
    for prec in ("fp32", "bf16"):
        net = _net(p, prec)
        out = net.interpolate([(xl.to(DEV), xr.to(DEV))], [0.3])[0, 0].cpu().numpy()
        want = 0.5 * (xl.numpy().astype(np.float64) + xr.numpy().astype(np.float64))
        err = np.abs(out - want).max()
        print(f"  {prec} max-abs {err:.3e}")
        assert err <= 1e-6
        net.close()


def test_constant_flow_closed_form(tmp_path):
    """Flow (2, 0, -2, 0), mask 1/2, zero residual: the exact middle view of
    a pair 4 px apart (except the 2 clamped columns on each side)."""
    print("case constant flow", flush=True)
    p = write_weights_file(str(tmp_path / "c.ffvw"), seed=0, kind="const_flow")
    xl, xr = scenes.small_pair()
    for prec in ("fp32", "bf16"):
        net = _net(p, prec)
        out = net.interpolate([(xl.to(DEV), xr.to(DEV))], [0.5])[0, 0].cpu().numpy()
        W = xl.shape[2]
        err = np.abs(out[:, :, 2:W - 2] - xl.numpy()[:, :, 4:]).max()
        print(f"  {prec} max-abs {err:.3e}")
        assert err <= 1e-6
        assert np.isfinite(out).all()
        net.close()


def test_batched_pairs_and_phases_match_single(wfile, oracle_w):
    """3 pairs (sharing cameras) x 3 phases in one call: every view equals
    the same view computed alone, bit for bit (the kernels' arithmetic per
    output does not depend on the batch), and matches the oracle."""
    print("case batch invariance", flush=True)
    arc = scenes.camera_arc(31, 64, 96, 4, 96, (3.0, 10.0), 6.0, 0.01).to(DEV)
    pairs = [(arc[i], arc[i + 1]) for i in range(3)]
    ts = [0.25, 0.5, 0.75]
    for prec in ("fp32", "bf16"):
        net = _net(wfile, prec)
        batch = net.interpolate(pairs, ts).cpu()
        for i in range(3):
            for j, t in enumerate(ts):
                alone = net.interpolate([pairs[i]], [t])[0, 0].cpu()
                assert torch.equal(alone, batch[i, j]), (prec, i, j)
        if prec == "fp32":
            ref = O.vinet_forward(arc[1].cpu().numpy(), arc[2].cpu().numpy(), 0.75, oracle_w)
            assert np.abs(batch[1, 2].numpy() - ref).max() <= 1e-4
        net.close()


def test_chunked_workspace_matches(wfile):
    """A workspace cap that forces one view per chunk gives identical views."""
    print("case chunking", flush=True)
    arc = scenes.camera_arc(32, 48, 64, 3, 64, (3.0, 8.0), 4.0, 0.01).to(DEV)
    pairs = [(arc[0], arc[1]), (arc[1], arc[2])]
    a = _net(wfile, "bf16")
    full = a.interpolate(pairs, [0.1, 0.9]).cpu()
    a.close()
    b = _net(wfile, "bf16", workspace_bytes=1)
    small = b.interpolate(pairs, [0.1, 0.9]).cpu()
    b.close()
    assert torch.equal(full, small)


@pytest.mark.slow
@pytest.mark.parametrize("t", [0.25, 8 / 17])
def test_fp32_full_1080p_parity(wfile, oracle_w, t):
    """The plain FP32 path on the full 1080x1920 pair (disparity 0-48 px,
    padded to 1088 rows inside) against the FP64 oracle: max-abs <= 1e-4 on
    every output value."""
    print(f"case fp32 1080p t={t:.4f}", flush=True)
    arc = scenes.hd_arc(2)
    net = _net(wfile, workspace_bytes=16 << 30)
    out = net.interpolate([(arc[0].to(DEV), arc[1].to(DEV))], [t])[0, 0].cpu().numpy()
    net.close()
    ref = O.vinet_forward(arc[0].numpy(), arc[1].numpy(), t, oracle_w)
    e = float(np.abs(out.astype(np.float64) - ref).max())
    print(f"  max-abs {e:.3e}, PSNR {psnr(out, ref):.2f} dB", flush=True)
    assert e <= 1e-4


def test_bf16_psnr_small(wfile, oracle_w):
    print("case bf16 psnr 128", flush=True)
    xl, xr = scenes.small_pair()
    net = _net(wfile, "bf16")
    out = net.interpolate([(xl.to(DEV), xr.to(DEV))], [0.5])[0, 0].cpu().numpy()
    ref = O.vinet_forward(xl.numpy(), xr.numpy(), 0.5, oracle_w)
    p = psnr(out, ref)
    print(f"  PSNR {p:.2f} dB, max-abs {np.abs(out - ref).max():.3e}")
    assert p >= 45.0
    net.close()


def test_bf16_psnr_hd_crop(wfile, oracle_w):
    """A 256x384 crop of the 1080p arc (blob sizes and disparities of the
    1080p workload)."""
    print("case bf16 psnr hd crop", flush=True)
    arc = scenes.hd_arc(2)
    xl = arc[0, :, 400:656, 700:1084].contiguous()
    xr = arc[1, :, 400:656, 700:1084].contiguous()
    net = _net(wfile, "bf16")
    out = net.interpolate([(xl.to(DEV), xr.to(DEV))], [0.5])[0, 0].cpu().numpy()
    ref = O.vinet_forward(xl.numpy(), xr.numpy(), 0.5, oracle_w)
    p = psnr(out, ref)
    print(f"  PSNR {p:.2f} dB")
    assert p >= 45.0
    net.close()


@pytest.mark.parametrize("H,W,t", [(72, 136, 0.3), (33, 17, 0.0)])
def test_ragged_bf16_psnr(wfile, oracle_w, H, W, t):
    """BF16 at sizes whose pixel count is not a multiple of the output
    head's 32-pixel groups or of its blocks: every pass's ragged tail, the
    head's partly filled last pair of groups included."""
    print(f"case ragged bf16 {H}x{W} t={t}", flush=True)
    xl, xr = scenes.random_pair(23, H, W, d_max=5.0)
    net = _net(wfile, "bf16")
    out = net.interpolate([(xl.to(DEV), xr.to(DEV))], [t])[0, 0].cpu().numpy()
    ref = O.vinet_forward(xl.numpy(), xr.numpy(), t, oracle_w)
    p = psnr(out, ref)
    print(f"  PSNR {p:.2f} dB, max-abs {np.abs(out - ref).max():.3e}")
    assert np.isfinite(out).all()
    assert p >= 45.0
    net.close()


def test_argument_errors(wfile):
    from paper_2112_10603_amd import FfvError
    net = _net(wfile)
    x = torch.rand(3, 32, 32, device=DEV)
    with pytest.raises(FfvError) as e:
        net.interpolate([(x, x)], [1.5])
    assert e.value.code == -1
    with pytest.raises(FfvError):
        net.interpolate([(x, x)], [float("nan")])
    y = torch.rand(3, 32, 48, device=DEV)
    with pytest.raises(FfvError):
        net.interpolate([(x, x), (y, y)], [0.5])
    net.close()


@pytest.mark.parametrize("H,W", [(2, 2), (2, 37), (19, 2), (16, 16)])
def test_smallest_sizes_parity(wfile, oracle_w, H, W):
    """The smallest images the boundary accepts (H, W >= 2; one 16 x 16
    padded tile, the whole network at 4 x 4 pixels and below in its first
    stage): FP32 within 1e-4 of the oracle, BF16 at >= 45 dB."""
    print(f"case smallest size {H}x{W}", flush=True)
    xl, xr = scenes.random_pair(31 + H + W, H, W, d_max=1.0)
    ref = O.vinet_forward(xl.numpy(), xr.numpy(), 0.4, oracle_w)
    for prec in ("fp32", "bf16"):
        net = _net(wfile, prec)
        out = net.interpolate([(xl.to(DEV), xr.to(DEV))], [0.4])[0, 0].cpu().numpy()
        net.close()
        assert out.shape == (3, H, W)
        err = float(np.abs(out.astype(np.float64) - ref).max())
        print(f"  {prec} max-abs {err:.3e}, PSNR {psnr(out, ref):.2f} dB", flush=True)
        if prec == "fp32":
            assert err <= 1e-4
        else:
            assert psnr(out, ref) >= 45.0


def test_empty_and_degenerate_calls_through_abi(wfile):
    """Empty batches, sizes below 2 or above the pixel limit, null pointers
    and phases outside [0, 1] are refused with FFV_ERR_ARG before any
    launch, and the net still works afterwards."""
    import ctypes

    from paper_2112_10603_amd import ffv
    print("case empty and degenerate calls", flush=True)
    net = _net(wfile)
    L = ffv.lib()
    x = torch.rand(3, 8, 8, device=DEV)
    out = torch.empty(3, 8, 8, device=DEV)
    ok = (ffv.ffv_pair * 1)(ffv.ffv_pair(x.data_ptr(), x.data_ptr(), 8, 8))
    t = (ctypes.c_float * 1)(0.5)
    h = net._h
    assert L.ffv_interpolate(h, ok, 0, t, 1, out.data_ptr()) == -1
    assert L.ffv_interpolate(h, ok, 1, t, 0, out.data_ptr()) == -1
    assert L.ffv_interpolate(h, None, 1, t, 1, out.data_ptr()) == -1
    assert L.ffv_interpolate(h, ok, 1, None, 1, out.data_ptr()) == -1
    assert L.ffv_interpolate(h, ok, 1, t, 1, None) == -1
    # sizes below 2, and one above the 2^28-pixel limit (refused before any allocation)
    for hh, ww in ((1, 8), (8, 1), (0, 0), (-4, 8), (16385, 16385)):
        bad = (ffv.ffv_pair * 1)(ffv.ffv_pair(x.data_ptr(), x.data_ptr(), hh, ww))
        assert L.ffv_interpolate(h, bad, 1, t, 1, out.data_ptr()) == -1, (hh, ww)
    for tv in (-0.01, 1.01, float("inf")):
        tb = (ctypes.c_float * 1)(tv)
        assert L.ffv_interpolate(h, ok, 1, tb, 1, out.data_ptr()) == -1, tv
    got = net.interpolate([(x, x)], [0.5])[0, 0]
    assert bool(torch.isfinite(got).all())
    net.close()
