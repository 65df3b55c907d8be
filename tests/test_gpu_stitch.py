"""Multi-view cluster frames through the C ABI against oracle/stitch.py."""
import numpy as np
import pytest
import torch

from oracle import stitch as S

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")


@pytest.mark.parametrize("n,H,W", [(16, 64, 96), (4, 30, 44), (1, 7, 9), (64, 64, 96), (16, 1080 // 4 * 4, 480)])
def test_stitch_vs_oracle(n, H, W):
    from paper_2112_10603_amd import stitch_cluster
    print(f"case stitch n={n} {H}x{W}", flush=True)
    g = {1: 1, 4: 2, 16: 4, 64: 8}[n]
    H, W = H // g * g, W // g * g
    rng = np.random.default_rng(n + H)
    hr = rng.random((3, H, W)).astype(np.float32)
    left = [rng.random((3, H, W)).astype(np.float32) for _ in range(n)]
    right = [rng.random((3, H, W)).astype(np.float32) for _ in range(n)]
    got = stitch_cluster(torch.from_numpy(hr).to(DEV), [torch.from_numpy(v).to(DEV) for v in left],
                         [torch.from_numpy(v).to(DEV) for v in right])
    torch.cuda.synchronize()
    ref = S.stitch_cluster(hr, left, right)
    assert got.shape == (3, H, 3 * W)
    err = np.abs(got.cpu().numpy().astype(np.float64) - ref).max()
    print(f"  max-abs {err:.3e}")
    assert err <= 1e-6
    np.testing.assert_array_equal(got[:, :, W:2 * W].cpu().numpy(), hr)


def test_stitch_errors():
    from paper_2112_10603_amd import stitch_cluster
    from paper_2112_10603_amd.ffv import FfvError
    print("case stitch errors", flush=True)
    v = torch.zeros((3, 16, 16), device=DEV)
    with pytest.raises(FfvError):
        stitch_cluster(v, [v] * 3, [v] * 3)  # not a square count
    w = torch.zeros((3, 18, 16), device=DEV)
    with pytest.raises(FfvError):
        stitch_cluster(w, [w] * 16, [w] * 16)  # height not a multiple of 4
    with pytest.raises(ValueError):
        stitch_cluster(v, [v] * 4, [torch.zeros((3, 8, 8), device=DEV)] * 4)
