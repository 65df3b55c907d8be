"""Pins for the cluster-frame oracle (oracle/stitch.py): brute-force box
means, closed forms on constant and linear images, the tile placement."""
import numpy as np
import pytest

from oracle import stitch as S


def test_box_down_brute_force():
    rng = np.random.default_rng(4)
    x = rng.random((3, 12, 20))
    got = S.box_down(x, 4)
    want = np.zeros((3, 3, 5))
    for c in range(3):
        for i in range(3):
            for j in range(5):
                acc = 0.0
                for a in range(4):
                    for b in range(4):
                        acc += x[c, 4 * i + a, 4 * j + b]
                want[c, i, j] = acc / 16
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-15)


def test_box_down_of_linear_image_is_block_centre():
    """A box mean of a linear function equals its value at the box centre."""
    H, W, g = 16, 24, 4
    y, x = np.mgrid[0:H, 0:W].astype(np.float64)
    img = np.stack([0.5 + 0.01 * x - 0.02 * y, 0.03 * x, 0.25 - 0.01 * y])
    got = S.box_down(img, g)
    yc, xc = np.mgrid[0:H // g, 0:W // g].astype(np.float64)
    yc, xc = g * yc + (g - 1) / 2, g * xc + (g - 1) / 2
    want = np.stack([0.5 + 0.01 * xc - 0.02 * yc, 0.03 * xc, 0.25 - 0.01 * yc])
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-14)


def test_cluster_layout_constant_views():
    """View k of the left side filled with k, of the right side with 100 + k:
    every tile is that constant, in raster order; the middle is the real view."""
    H, W = 8, 12
    rng = np.random.default_rng(1)
    hr = rng.random((3, H, W))
    left = [np.full((3, H, W), float(k)) for k in range(16)]
    right = [np.full((3, H, W), 100.0 + k) for k in range(16)]
    out = S.stitch_cluster(hr, left, right)
    assert out.shape == (3, H, 3 * W)
    np.testing.assert_array_equal(out[:, :, W:2 * W], hr)
    for k in range(16):
        r, q = divmod(k, 4)
        ys, xs = slice(2 * r, 2 * r + 2), slice(3 * q, 3 * q + 3)
        np.testing.assert_array_equal(out[:, ys, xs], k)
        np.testing.assert_array_equal(out[:, ys, 2 * W + 3 * q:2 * W + 3 * q + 3], 100.0 + k)


def test_cluster_bad_arguments():
    v = np.zeros((3, 8, 8))
    with pytest.raises(ValueError):
        S.stitch_cluster(v, [v] * 3, [v] * 3)  # not a square
    with pytest.raises(ValueError):
        S.stitch_cluster(v, [v] * 4, [v] * 9)
    with pytest.raises(ValueError):
        S.box_down(np.zeros((3, 10, 8)), 4)
