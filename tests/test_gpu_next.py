"""The blend-only output (the paper's "w/o Refine" variant, Table 1) and
dense views by recursive midpoints (section 4), through the C ABI, against
the oracle's vinet_forward(refine=False) and vinet_recursive."""
import numpy as np
import pytest
import torch

from oracle import vinet as O
from synth import scenes
from synth.weights import write_weights_file

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")


@pytest.fixture(scope="module")
def wfile(tmp_path_factory):
    return write_weights_file(str(tmp_path_factory.mktemp("wn") / "w.ffvw"), seed=0)


@pytest.fixture(scope="module")
def zfile(tmp_path_factory):
    return write_weights_file(str(tmp_path_factory.mktemp("wz") / "z.ffvw"), seed=3, kind="zero_heads")


@pytest.mark.parametrize("H,W,t", [(40, 88, 0.3), (64, 64, 0.5), (33, 17, 1.0)])
def test_blend_fp32_parity(wfile, H, W, t):
    from paper_2112_10603_amd import Net
    print(f"case blend fp32 {H}x{W} t={t}", flush=True)
    Wo = O.load_weights(wfile)
    xl, xr = scenes.random_pair(23, H, W, d_max=5.0)
    net = Net(wfile, "fp32", 0)
    got = net.interpolate_blend([(xl.to(DEV), xr.to(DEV))], [t])[0, 0].cpu().numpy()
    net.close()
    ref = O.vinet_forward(xl.numpy(), xr.numpy(), t, Wo, refine=False)
    err = np.abs(got.astype(np.float64) - ref).max()
    print(f"  max-abs {err:.3e}")
    assert err <= 1e-4


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_blend_zero_heads_is_average(zfile, precision):
    from paper_2112_10603_amd import Net
    print(f"case blend zero heads {precision}", flush=True)
    xl, xr = scenes.random_pair(7, 40, 72)
    net = Net(zfile, precision, 0)
    got = net.interpolate_blend([(xl.to(DEV), xr.to(DEV))], [0.7])[0, 0].cpu().numpy()
    net.close()
    want = 0.5 * (xl.numpy().astype(np.float64) + xr.numpy().astype(np.float64))
    assert np.abs(got - want).max() <= 1e-7


def test_blend_bf16_psnr(wfile):
    from paper_2112_10603_amd import Net
    print("case blend bf16 psnr 128", flush=True)
    xl, xr = scenes.small_pair()
    net = Net(wfile, "bf16", 0)
    got = net.interpolate_blend([(xl.to(DEV), xr.to(DEV))], [0.5])[0, 0].cpu().numpy()
    net.close()
    ref = O.vinet_forward(xl.numpy(), xr.numpy(), 0.5, O.load_weights(wfile), refine=False)
    psnr = 10 * np.log10(1.0 / np.mean((got.astype(np.float64) - ref) ** 2))
    print(f"  PSNR {psnr:.2f} dB")
    assert psnr >= 45.0


def test_recursive_fp32_parity(wfile):
    from paper_2112_10603_amd import Net
    print("case recursive fp32 levels 2", flush=True)
    Wo = O.load_weights(wfile)
    xl, xr = scenes.random_pair(29, 48, 64, d_max=6.0)
    net = Net(wfile, "fp32", 0)
    got = net.interpolate_recursive([(xl.to(DEV), xr.to(DEV))], 2)[0].cpu().numpy()
    net.close()
    ref = O.vinet_recursive(xl.numpy(), xr.numpy(), 2, Wo)
    assert got.shape == (3, 3, 48, 64)
    for k in range(3):
        err = np.abs(got[k].astype(np.float64) - ref[k]).max()
        print(f"  view t={(k + 1) / 4}: max-abs {err:.3e}")
        assert err <= 1e-4


def test_recursive_zero_heads_linear(zfile):
    from paper_2112_10603_amd import Net
    print("case recursive zero heads levels 3", flush=True)
    xl, xr = scenes.random_pair(9, 32, 48)
    net = Net(zfile, "bf16", 0)
    got = net.interpolate_recursive([(xl.to(DEV), xr.to(DEV))], 3)[0].cpu().numpy()
    net.close()
    a, b = xl.numpy().astype(np.float64), xr.numpy().astype(np.float64)
    for k in range(1, 8):
        t = k / 8
        assert np.abs(got[k - 1] - ((1 - t) * a + t * b)).max() <= 1e-6


@pytest.mark.parametrize("precision", ["bf16", "fp32"])
def test_recursive_equals_composed_midpoints(wfile, precision):
    """Two pairs, three levels: every view equals the t = 1/2 synthesis of
    its two neighbours computed by separate interpolate calls (the per-view
    arithmetic does not depend on the batch), bit for bit."""
    from paper_2112_10603_amd import Net
    print(f"case recursive composed {precision}", flush=True)
    arc = scenes.camera_arc(31, 40, 56, 3, 64, (3.0, 8.0), 4.0, 0.01).to(DEV)
    pairs = [(arc[0].contiguous(), arc[1].contiguous()), (arc[1].contiguous(), arc[2].contiguous())]
    net = Net(wfile, precision, 0)
    got = net.interpolate_recursive(pairs, 3)
    for i, (l, r) in enumerate(pairs):
        views = {0: l, 8: r}
        for level in (1, 2, 3):
            step = 8 >> level
            for k in range(step, 8, 2 * step):
                views[k] = net.interpolate([(views[k - step], views[k + step])], [0.5])[0, 0]
        for k in range(1, 8):
            assert torch.equal(got[i, k - 1], views[k]), (i, k)
    net.close()


def test_recursive_argument_errors(wfile):
    from paper_2112_10603_amd import Net
    from paper_2112_10603_amd.ffv import FfvError
    print("case recursive errors", flush=True)
    xl, xr = scenes.random_pair(3, 32, 32)
    net = Net(wfile, "bf16", 0)
    for levels in (0, 11):
        with pytest.raises((FfvError, ValueError)):
            net.interpolate_recursive([(xl.to(DEV), xr.to(DEV))], levels,
                                      out=torch.empty((1, 1, 3, 32, 32), device=DEV))
    net.close()
