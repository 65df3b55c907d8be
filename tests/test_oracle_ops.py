"""Pins for the oracle's operators: brute-force definitions on tiny tensors,
closed forms, and independent library routines (torch CPU float64)."""
import numpy as np
import pytest
import torch
import torch.nn.functional as Fn

from oracle import vinet as O

rng = np.random.default_rng(1234)


def brute_conv(x, w, b, stride):
    C, H, W = x.shape
    Co = w.shape[0]
    Ho, Wo = (H - 1) // stride + 1, (W - 1) // stride + 1
    out = np.zeros((Co, Ho, Wo))
    for o in range(Co):
        for i in range(Ho):
            for j in range(Wo):
                acc = b[o]
                for c in range(C):
                    for dy in range(3):
                        for dx in range(3):
                            yy, xx = stride * i + dy - 1, stride * j + dx - 1
                            if 0 <= yy < H and 0 <= xx < W:
                                acc += w[o, c, dy, dx] * x[c, yy, xx]
                out[o, i, j] = acc
    return out


def brute_convT(x, w, b):
    Ci, H, W = x.shape
    Co = w.shape[1]
    out = np.tile(b[:, None, None], (1, 2 * H, 2 * W)).astype(np.float64)
    for c in range(Ci):
        for iy in range(H):
            for ix in range(W):
                for ky in range(4):
                    for kx in range(4):
                        y, xx = 2 * iy - 1 + ky, 2 * ix - 1 + kx
                        if 0 <= y < 2 * H and 0 <= xx < 2 * W:
                            out[:, y, xx] += w[c, :, ky, kx] * x[c, iy, ix]
    return out


@pytest.mark.parametrize("stride", [1, 2])
@pytest.mark.parametrize("shape", [(3, 5, 7), (2, 6, 4), (4, 1, 3)])
def test_conv2d_bruteforce(stride, shape):
    C, H, W = shape
    x = rng.standard_normal(shape)
    w = rng.standard_normal((5, C, 3, 3))
    b = rng.standard_normal(5)
    np.testing.assert_allclose(O.conv2d(x, w, b, stride), brute_conv(x, w, b, stride),
                               rtol=0, atol=1e-12)


@pytest.mark.parametrize("stride", [1, 2])
def test_conv2d_torch(stride):
    x = rng.standard_normal((6, 18, 22))
    w = rng.standard_normal((9, 6, 3, 3))
    b = rng.standard_normal(9)
    ref = Fn.conv2d(torch.from_numpy(x)[None], torch.from_numpy(w), torch.from_numpy(b),
                    stride=stride, padding=1)[0].numpy()
    np.testing.assert_allclose(O.conv2d(x, w, b, stride), ref, rtol=0, atol=1e-12)


def test_conv2d_delta_kernels():
    x = rng.standard_normal((3, 8, 10))
    # centre tap identity
    w = np.zeros((3, 3, 3, 3))
    for c in range(3):
        w[c, c, 1, 1] = 1.0
    np.testing.assert_array_equal(O.conv2d(x, w, np.zeros(3), 1), x)
    # top-left tap: out(i, j) = x(i-1, j-1), zero on the first row/column
    w = np.zeros((3, 3, 3, 3))
    for c in range(3):
        w[c, c, 0, 0] = 1.0
    y = O.conv2d(x, w, np.zeros(3), 1)
    np.testing.assert_array_equal(y[:, 1:, 1:], x[:, :-1, :-1])
    assert np.all(y[:, 0, :] == 0) and np.all(y[:, :, 0] == 0)
    # stride 2 centre tap = subsampling at even positions
    w = np.zeros((3, 3, 3, 3))
    for c in range(3):
        w[c, c, 1, 1] = 1.0
    np.testing.assert_array_equal(O.conv2d(x, w, np.zeros(3), 2), x[:, ::2, ::2])


@pytest.mark.parametrize("shape", [(3, 4, 5), (2, 1, 1), (5, 3, 2)])
def test_convT_bruteforce(shape):
    Ci, H, W = shape
    x = rng.standard_normal(shape)
    w = rng.standard_normal((Ci, 4, 4, 4))
    b = rng.standard_normal(4)
    np.testing.assert_allclose(O.conv_transpose2d(x, w, b), brute_convT(x, w, b),
                               rtol=0, atol=1e-12)


def test_convT_torch():
    x = rng.standard_normal((7, 9, 13))
    w = rng.standard_normal((7, 5, 4, 4))
    b = rng.standard_normal(5)
    ref = Fn.conv_transpose2d(torch.from_numpy(x)[None], torch.from_numpy(w),
                              torch.from_numpy(b), stride=2, padding=1)[0].numpy()
    np.testing.assert_allclose(O.conv_transpose2d(x, w, b), ref, rtol=0, atol=1e-12)


def test_convT_equals_zero_insert_then_flipped_conv():
    """A stride-2 transposed conv is a conv (flipped, channel-swapped kernel,
    padding 2) over the zero-inserted input; checked with a plain loop conv."""
    x = rng.standard_normal((3, 4, 6))
    w = rng.standard_normal((3, 2, 4, 4))
    b = np.zeros(2)
    C, H, W = x.shape
    z = np.zeros((C, 2 * H - 1, 2 * W - 1))
    z[:, ::2, ::2] = x
    zp = np.pad(z, ((0, 0), (2, 2), (2, 2)))
    wf = w[:, :, ::-1, ::-1]
    out = np.zeros((2, 2 * H, 2 * W))
    for o in range(2):
        for yy in range(2 * H):
            for xx in range(2 * W):
                out[o, yy, xx] = np.sum(wf[:, o] * zp[:, yy:yy + 4, xx:xx + 4])
    np.testing.assert_allclose(O.conv_transpose2d(x, w, b), out, rtol=0, atol=1e-12)


@pytest.mark.parametrize("hw_in,hw_out", [((16, 24), (4, 6)), ((16, 24), (8, 12)),
                                          ((8, 12), (16, 24)), ((7, 9), (5, 13)),
                                          ((3, 5), (11, 4))])
def test_resample_torch(hw_in, hw_out):
    x = rng.standard_normal((3,) + hw_in)
    ref = Fn.interpolate(torch.from_numpy(x)[None], size=hw_out, mode="bilinear",
                         align_corners=False)[0].numpy()
    np.testing.assert_allclose(O.resample(x, *hw_out), ref, rtol=0, atol=1e-12)


def test_resample_closed_forms():
    x = np.full((2, 12, 20), 0.37)
    np.testing.assert_allclose(O.resample(x, 3, 5), 0.37, rtol=0, atol=1e-15)
    np.testing.assert_allclose(O.resample(x, 24, 40), 0.37, rtol=0, atol=1e-15)
    # down by 2 with half-pixel centres is exactly the 2x2 box mean
    y = rng.standard_normal((3, 10, 14))
    box = 0.25 * (y[:, 0::2, 0::2] + y[:, 1::2, 0::2] + y[:, 0::2, 1::2] + y[:, 1::2, 1::2])
    np.testing.assert_allclose(O.resample(y, 5, 7), box, rtol=0, atol=1e-14)
    # down by 4 averages rows/cols 4i+1 and 4i+2
    d4 = 0.25 * (y[:, 1::4, 1::4][:, :2, :3] + y[:, 2::4, 1::4][:, :2, :3]
                 + y[:, 1::4, 2::4][:, :2, :3] + y[:, 2::4, 2::4][:, :2, :3])
    np.testing.assert_allclose(O.resample(y[:, :8, :12], 2, 3), d4, rtol=0, atol=1e-14)
    # up by 2 of a linear ramp stays linear away from the clamped border
    ramp = np.broadcast_to(np.arange(8.0)[None, None, :], (1, 4, 8)).copy()
    up = O.resample(ramp, 8, 16)
    xs = (np.arange(16) + 0.5) / 2 - 0.5
    np.testing.assert_allclose(up[0, 0, 1:15], xs[1:15], rtol=0, atol=1e-14)


def test_warp_zero_flow_identity():
    x = rng.standard_normal((3, 9, 11))
    np.testing.assert_array_equal(O.warp(x, np.zeros((2, 9, 11))), x)


@pytest.mark.parametrize("dx,dy", [(2, 0), (-3, 1), (0, -2), (20, 5)])
def test_warp_integer_shift(dx, dy):
    H, W = 7, 10
    x = rng.standard_normal((2, H, W))
    f = np.zeros((2, H, W))
    f[0], f[1] = dx, dy
    out = O.warp(x, f)
    for i in range(H):
        for j in range(W):
            yy = min(max(i + dy, 0), H - 1)
            xx = min(max(j + dx, 0), W - 1)
            assert np.array_equal(out[:, i, j], x[:, yy, xx])


def test_warp_affine_exact():
    """Bilinear sampling reproduces a bilinear function exactly for sample
    points inside the image."""
    H, W = 12, 16
    gy, gx = np.mgrid[0:H, 0:W].astype(np.float64)
    img = np.stack([0.3 + 0.02 * gx - 0.01 * gy + 0.001 * gx * gy, 0.5 - 0.03 * gx])
    fx = 0.37 + 0.05 * gx - 0.1 * gy * 0.2
    fy = -0.61 + 0.02 * gy
    px, py = gx + fx, gy + fy
    inside = (px >= 0) & (px <= W - 1) & (py >= 0) & (py <= H - 1)
    want = np.stack([0.3 + 0.02 * px - 0.01 * py + 0.001 * px * py, 0.5 - 0.03 * px])
    out = O.warp(img, np.stack([fx, fy]))
    np.testing.assert_allclose(out[:, inside], want[:, inside], rtol=0, atol=1e-12)
    assert inside.sum() > 0.5 * H * W


def test_warp_grid_sample():
    H, W = 13, 17
    x = rng.standard_normal((4, H, W))
    f = rng.standard_normal((2, H, W)) * 6.0
    gy, gx = np.mgrid[0:H, 0:W].astype(np.float64)
    grid = np.stack([2 * (gx + f[0]) / (W - 1) - 1, 2 * (gy + f[1]) / (H - 1) - 1], -1)
    ref = Fn.grid_sample(torch.from_numpy(x)[None], torch.from_numpy(grid)[None],
                         mode="bilinear", padding_mode="border", align_corners=True)[0].numpy()
    np.testing.assert_allclose(O.warp(x, f), ref, rtol=0, atol=1e-12)


def test_blend_limits_and_symmetry():
    wl = rng.uniform(size=(3, 4, 5))
    wr = rng.uniform(size=(3, 4, 5))
    m = rng.standard_normal((1, 4, 5)) * 3
    np.testing.assert_allclose(O.blend(wl, wr, np.full((1, 4, 5), 800.0)), wl, atol=1e-15)
    np.testing.assert_allclose(O.blend(wl, wr, np.full((1, 4, 5), -800.0)), wr, atol=1e-15)
    np.testing.assert_allclose(O.blend(wl, wr, np.zeros((1, 4, 5))), 0.5 * (wl + wr), atol=1e-15)
    np.testing.assert_allclose(O.blend(wl, wr, m), O.blend(wr, wl, -m), atol=1e-14)


def test_sigmoid_values():
    assert O.sigmoid(0.0) == 0.5
    np.testing.assert_allclose(O.sigmoid(np.log(3.0)), 0.75, atol=1e-15)


def test_pad_replicate():
    x = rng.standard_normal((3, 5, 6))
    p = O.pad_replicate(x, 16, 16)
    assert p.shape == (3, 16, 16)
    np.testing.assert_array_equal(p[:, :5, :6], x)
    np.testing.assert_array_equal(p[:, 10, :6], x[:, 4, :])
    np.testing.assert_array_equal(p[:, :5, 12], x[:, :, 5])
    np.testing.assert_array_equal(p[:, 15, 15], x[:, 4, 5])
