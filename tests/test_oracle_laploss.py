"""Pins of the oracle's Laplacian-pyramid loss (paper section 3.1, Eq. 3)
and of its gradient: a library filter, closed forms of the pyramid on
constants, ramps and the Nyquist checkerboard, a dense-matrix brute force on
tiny images and central finite differences."""
import numpy as np
import pytest
from scipy import ndimage

from oracle import laploss as LL


def test_blur_is_mirror_mode_binomial_filter():
    """The blur equals scipy's separable correlation with [1,4,6,4,1]/16 in
    'mirror' mode (reflection about the edge sample), at gain 1 and 2."""
    rng = np.random.default_rng(0)
    x = rng.standard_normal((2, 9, 13))
    for gain in (1.0, 2.0):
        k = gain * np.array([1, 4, 6, 4, 1]) / 16.0
        ref = ndimage.correlate1d(ndimage.correlate1d(x, k, axis=1, mode="mirror"), k, axis=2, mode="mirror")
        assert np.allclose(LL.blur(x, gain), ref, atol=1e-14)


@pytest.mark.parametrize("h,w", [(33, 33), (40, 57), (64, 64)])
def test_constant_image_has_zero_bands(h, w):
    """blur, reduce and expand keep a constant exactly (mirror padding keeps
    the zero-insertion parity at both edges), so every band is zero and the
    loss ignores a constant offset."""
    c = np.full((3, h, w), 0.37)
    assert np.allclose(LL.reduce(c), 0.37, atol=1e-15)
    assert np.allclose(LL.expand(c[:, ::2, ::2], h, w), 0.37, atol=1e-15)
    for band in LL.laplacian_pyramid(c):
        assert np.abs(band).max() < 1e-14
    rng = np.random.default_rng(1)
    x, y = rng.random((3, h, w)), rng.random((3, h, w))
    assert abs(LL.lap_loss(x + 0.5, y + 0.5) - LL.lap_loss(x, y)) < 1e-12


def test_linear_ramp_bands_vanish_inside():
    """The symmetric filter reproduces linear functions and the
    zero-insertion expand (gain 2 per axis) interpolates them exactly, so
    every band of a linear ramp is zero away from the borders (mirror
    padding bends the ramp within the filter's reach of an edge, and the
    coarser levels carry that a few samples in: 5 samples per level)."""
    h = w = 192
    yy, xx = np.mgrid[0:h, 0:w].astype(np.float64)
    ramp = np.stack([0.01 * xx + 0.02 * yy, -0.03 * xx + 0.005 * yy, 0.004 * xx])
    bands = LL.laplacian_pyramid(ramp)
    for i, band in enumerate(bands):
        m = 5
        inner = band[:, m:band.shape[1] - m, m:band.shape[2] - m]
        assert inner.size > 0 and np.abs(inner).max() < 1e-12, i
        assert np.abs(band).max() > 1e-6, i  # the borders do differ


@pytest.mark.parametrize("a", [0.25, 1.0])
def test_checkerboard_is_pure_first_band(a):
    """(-1)^(x+y) is annihilated by the binomial filter ((1-4+6-4+1)/16 = 0
    per axis, also at mirrored edges), so L^1 is the image itself, the other
    bands are zero, the loss is a * 2^0 * mean|+-1| = a, and away from the
    borders (where the adjoint of the mirrored filter no longer annihilates
    it) the gradient is sign(d) / N exactly."""
    h, w = 36, 50
    yy, xx = np.mgrid[0:h, 0:w]
    d = a * np.stack([(-1.0) ** (xx + yy)] * 3)
    bands = LL.laplacian_pyramid(d)
    assert np.allclose(bands[0], d, atol=1e-14)
    for band in bands[1:]:
        assert np.abs(band).max() < 1e-14
    gt = np.zeros_like(d)
    assert abs(LL.lap_loss(d, gt) - a) < 1e-14
    g = LL.lap_loss_grad(d, gt)
    m = 6
    assert np.allclose(g[:, m:h - m, m:w - m], (np.sign(d) / d.size)[:, m:h - m, m:w - m], atol=1e-18, rtol=0)
    assert abs(g.sum() - (np.sign(d) / d.size).sum()) < 1e-3  # and it stays a signed 1/N field


def _operator_matrices(h, w):
    """Dense matrices of every band level of a 1-channel h x w image, built
    by brute force from index formulas: B (blur, mirror taps), D (keep even
    samples), U (zero insertion), per axis, composed as Kronecker products."""
    k = np.array([1, 4, 6, 4, 1]) / 16.0

    def blur1(n, gain):
        m = np.zeros((n, n))
        for j in range(n):
            for t in range(5):
                i = j + t - 2
                i = -i if i < 0 else i
                i = 2 * (n - 1) - i if i > n - 1 else i
                m[j, i] += gain * k[t]
        return m

    def down1(n):
        m = np.zeros(((n + 1) // 2, n))
        for j in range(0, n, 2):
            m[j // 2, j] = 1.0
        return m

    mats = []
    g_h, g_w = np.eye(h), np.eye(w)  # image -> G^i, per axis
    nh, nw = h, w
    for _ in range(5):
        rh = down1(nh) @ blur1(nh, 1.0)
        rw = down1(nw) @ blur1(nw, 1.0)
        eh = blur1(nh, 2.0) @ down1(nh).T
        ew = blur1(nw, 2.0) @ down1(nw).T
        band = np.kron(g_h, g_w) - np.kron(eh @ rh @ g_h, ew @ rw @ g_w)
        mats.append(band)
        g_h, g_w = rh @ g_h, rw @ g_w
        nh, nw = (nh + 1) // 2, (nw + 1) // 2
    return mats


def test_brute_force_matrices_loss_and_gradient():
    """On a 1-channel 35 x 37 image every band equals its dense matrix
    applied to the image, and loss and gradient follow from the matrices:
    sum_i 2^(i-1) mean|M_i d| and sum_i 2^(i-1) M_i^T sign(M_i d) / N_i."""
    h, w = 35, 37
    mats = _operator_matrices(h, w)
    rng = np.random.default_rng(3)
    x, gt = rng.random((1, h, w)), rng.random((1, h, w))
    d = (x - gt).reshape(-1)
    bands = LL.laplacian_pyramid(x - gt)
    want_loss, want_grad = 0.0, np.zeros(h * w)
    for i, m in enumerate(mats):
        b = m @ d
        assert np.allclose(bands[i].reshape(-1), b, atol=1e-13), i
        want_loss += 2.0 ** i * np.mean(np.abs(b))
        want_grad += 2.0 ** i * (m.T @ np.sign(b)) / b.size
    assert abs(LL.lap_loss(x, gt) - want_loss) < 1e-12
    assert np.allclose(LL.lap_loss_grad(x, gt).reshape(-1), want_grad, atol=1e-15)


def test_gradient_matches_central_differences():
    """Away from kinks (no band value near zero) the loss is linear in each
    pixel locally: central differences with step 1e-7 give the gradient."""
    h, w = 33, 34
    rng = np.random.default_rng(4)
    x, gt = rng.random((3, h, w)), rng.random((3, h, w))
    g = LL.lap_loss_grad(x, gt)
    bands = LL.laplacian_pyramid(x - gt)
    eps = 1e-7
    checked = 0
    for (c, yy, xx) in [(0, 0, 0), (1, 16, 17), (2, 32, 33), (0, 5, 30), (2, 20, 1)]:
        xp, xm = x.copy(), x.copy()
        xp[c, yy, xx] += eps
        xm[c, yy, xx] -= eps
        # skip a pixel whose perturbation could flip a band's sign
        if min(np.abs(b).min() for b in bands) < 10 * eps:
            continue
        fd = (LL.lap_loss(xp, gt) - LL.lap_loss(xm, gt)) / (2 * eps)
        assert abs(fd - g[c, yy, xx]) < 1e-6 * max(1.0, abs(g[c, yy, xx])) + 1e-9, (c, yy, xx)
        checked += 1
    assert checked >= 3


def test_small_images_rejected():
    with pytest.raises(ValueError):
        LL.laplacian_pyramid(np.zeros((3, 32, 64)))
