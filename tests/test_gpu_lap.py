"""The Eq. 3 Laplacian-pyramid loss kernels (through the C ABI) against the
FP64 oracle (oracle/laploss.py): loss per image and gradient, on random
images of several (ragged) sizes, closed forms, and the full 1080p size."""
import numpy as np
import pytest
import torch

from oracle import laploss as LL
from synth import scenes

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")


def _gpu(x, gt, grad=True):
    from paper_2112_10603_amd import lap_loss
    xd = torch.from_numpy(np.ascontiguousarray(x, np.float32)).to(DEV)
    gd = torch.from_numpy(np.ascontiguousarray(gt, np.float32)).to(DEV)
    out = lap_loss(xd, gd, grad=grad)
    if grad:
        return out[0].cpu().numpy(), out[1].cpu().numpy()
    return out.cpu().numpy()


def _sign_safe_mask(d, tol=1e-5):
    """Level-0 samples whose gradient cannot depend on a sign the FP32 and
    FP64 evaluations may decide differently: a box around every band value
    with |L| < tol (radius 8 * 2^i + 8 at level i, mapped to level 0)."""
    bands = LL.laplacian_pyramid(d)
    mask = np.ones(d.shape, bool)
    for i, b in enumerate(bands):
        c, ys, xs = np.nonzero(np.abs(b) < tol)
        r = 8 * 2 ** i + 8
        for ch, y, x in zip(c, ys, xs):
            mask[ch, max(0, y * 2 ** i - r):y * 2 ** i + r + 1, max(0, x * 2 ** i - r):x * 2 ** i + r + 1] = False
    return mask


@pytest.mark.parametrize("n,h,w", [(2, 64, 64), (1, 33, 47), (3, 100, 75), (1, 181, 240)])
def test_lap_loss_and_gradient_vs_oracle(n, h, w):
    print(f"case lap loss n={n} {h}x{w}", flush=True)
    rng = np.random.default_rng(h * 1000 + w)
    x = rng.random((n, 3, h, w)).astype(np.float32)
    gt = rng.random((n, 3, h, w)).astype(np.float32)
    loss, g = _gpu(x, gt)
    for i in range(n):
        xi, gi = x[i].astype(np.float64), gt[i].astype(np.float64)
        ref = LL.lap_loss(xi, gi)
        assert abs(loss[i] - ref) <= 2e-6 * ref, (i, loss[i], ref)
        gref = LL.lap_loss_grad(xi, gi)
        m = _sign_safe_mask(xi - gi)
        assert m.mean() > 0.5
        scale = np.abs(gref).max()
        err = np.abs(g[i].astype(np.float64) - gref)[m].max()
        assert err <= 1e-5 * scale, (i, err, scale)


def test_lap_loss_closed_forms():
    """x == gt: loss 0 and gradient 0; a constant offset: loss 0; the Nyquist
    checkerboard of amplitude a: loss a exactly up to fp32 rounding."""
    print("case lap loss closed forms", flush=True)
    rng = np.random.default_rng(5)
    x = rng.random((2, 3, 48, 80)).astype(np.float32)
    loss, g = _gpu(x, x)
    assert np.all(loss == 0.0) and np.all(g == 0.0)
    loss = _gpu(x + np.float32(0.25), x, grad=False)
    assert np.all(np.abs(loss) < 1e-6)
    yy, xx = np.mgrid[0:36, 0:50]
    a = 0.375
    d = (a * np.stack([(-1.0) ** (xx + yy)] * 3)).astype(np.float32)[None]
    loss = _gpu(d, np.zeros_like(d), grad=False)
    assert abs(loss[0] - a) < 1e-6


def test_lap_loss_repeatable_and_errors():
    from paper_2112_10603_amd import lap_loss
    from paper_2112_10603_amd.ffv import FfvError
    print("case lap loss repeat/errors", flush=True)
    rng = np.random.default_rng(6)
    x = torch.from_numpy(rng.random((4, 3, 70, 90)).astype(np.float32)).to(DEV)
    gt = torch.from_numpy(rng.random((4, 3, 70, 90)).astype(np.float32)).to(DEV)
    l1, g1 = lap_loss(x, gt, grad=True)
    l2, g2 = lap_loss(x, gt, grad=True)
    assert torch.equal(l1, l2) and torch.equal(g1, g2)
    assert torch.equal(lap_loss(x, gt), l1)
    small = torch.zeros((1, 3, 32, 64), device=DEV)
    with pytest.raises(FfvError) as e:
        lap_loss(small, small)
    assert e.value.code == -1


@pytest.mark.slow
def test_lap_loss_full_1080p():
    """Two cameras of the 1080p synthetic arc as (x, gt): loss and gradient
    against the oracle at the full size."""
    print("case lap loss 1080p", flush=True)
    arc = scenes.hd_arc(2).numpy()
    loss, g = _gpu(arc[0:1], arc[1:2])
    xi, gi = arc[0].astype(np.float64), arc[1].astype(np.float64)
    ref = LL.lap_loss(xi, gi)
    assert abs(loss[0] - ref) <= 2e-6 * ref, (loss[0], ref)
    gref = LL.lap_loss_grad(xi, gi)
    m = _sign_safe_mask(xi - gi)
    scale = np.abs(gref).max()
    assert np.abs(g[0].astype(np.float64) - gref)[m].max() <= 1e-5 * scale
