"""Kernel-unit parity: the library's implicit-GEMM conv kernel against the
oracle's conv2d / conv_transpose2d on odd and adversarial shapes (channel
counts that are not tile multiples, ragged spatial sizes, stride 2, the
transposed phases, every tile shape)."""
import numpy as np
import pytest
import torch

from oracle import vinet as O

pytestmark = pytest.mark.gpu

CASES = [
    # (cin, cout, h, w, stride, transposed)
    (3, 16, 17, 23, 2, False),
    (7, 128, 9, 13, 2, False),
    (18, 128, 12, 20, 2, False),
    (17, 32, 10, 6, 2, False),
    (16, 16, 5, 7, 1, False),
    (64, 64, 11, 9, 1, False),
    (256, 256, 8, 12, 1, False),
    (128, 256, 6, 10, 2, False),
    (40, 33, 7, 7, 1, False),
    (256, 128, 5, 6, 0, True),
    (128, 5, 7, 9, 0, True),
    (512, 128, 3, 4, 0, True),
    (64, 16, 6, 5, 0, True),
    (24, 7, 4, 3, 0, True),
]


def _ref(x, w, b, stride, transposed, relu):
    out = []
    for i in range(x.shape[0]):
        y = O.conv_transpose2d(x[i], w, b) if transposed else O.conv2d(x[i], w, b, stride)
        out.append(np.maximum(y, 0) if relu else y)
    return np.stack(out)


@pytest.mark.parametrize("cin,cout,h,w,stride,transposed", CASES)
@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_conv_kernel_vs_oracle(cin, cout, h, w, stride, transposed, precision):
    from paper_2112_10603_amd import op_conv
    print(f"case cin={cin} cout={cout} h={h} w={w} s={stride} T={transposed} {precision}", flush=True)
    rng = np.random.default_rng(cin * 1000 + cout)
    n = 2
    x = rng.standard_normal((n, cin, h, w)).astype(np.float32)
    if transposed:
        wt = (rng.standard_normal((cin, cout, 4, 4)) / np.sqrt(4 * cin)).astype(np.float32)
    else:
        wt = (rng.standard_normal((cout, cin, 3, 3)) / np.sqrt(9 * cin)).astype(np.float32)
    b = rng.standard_normal(cout).astype(np.float32)
    relu = cout % 2 == 0
    if precision == "bf16":
        # the kernel rounds inputs and weights to bf16 (nearest even)
        xr = torch.from_numpy(x).bfloat16().float().numpy()
        wr = torch.from_numpy(wt).bfloat16().float().numpy()
    else:
        xr, wr = x, wt
    ref = _ref(xr.astype(np.float64), wr.astype(np.float64), b.astype(np.float64), stride,
               transposed, relu)
    absref = _ref(np.abs(xr).astype(np.float64), np.abs(wr).astype(np.float64),
                  np.abs(b).astype(np.float64), stride, transposed, False)
    got = op_conv(torch.from_numpy(x).cuda(), wt, b, stride=max(stride, 1),
                  transposed=transposed, relu=relu, precision=precision).cpu().numpy()
    assert got.shape == ref.shape
    err = np.abs(got.astype(np.float64) - ref)
    # fp32 accumulation over K terms: bounded by a small multiple of the sum
    # of |terms|
    bound = 2e-5 * absref + 1e-6
    assert np.all(err <= bound), (err.max(), (err / (absref + 1e-12)).max())


VARIANT_CASES = [
    # (cin, cout, h, w, stride, transposed): shapes that span several M tiles
    (64, 256, 40, 52, 1, False),
    (128, 128, 37, 45, 2, False),
    (256, 128, 19, 23, 0, True),
    (64, 16, 21, 27, 0, True),
]


@pytest.mark.parametrize("cin,cout,h,w,stride,transposed", VARIANT_CASES)
def test_conv_tile_variants_agree(cin, cout, h, w, stride, transposed):
    """Every (N tile, pixel-block width) the autotuner may choose computes
    the same output: each element is one fp32 MFMA chain over the same K
    order, whatever the tiling, so the results agree bit for bit and match
    the oracle."""
    from paper_2112_10603_amd import op_conv
    print(f"case tile variants cin={cin} cout={cout} h={h} w={w} s={stride} T={transposed}", flush=True)
    rng = np.random.default_rng(cin + 7 * cout)
    x = rng.standard_normal((2, cin, h, w)).astype(np.float32)
    if transposed:
        wt = (rng.standard_normal((cin, cout, 4, 4)) / np.sqrt(4 * cin)).astype(np.float32)
    else:
        wt = (rng.standard_normal((cout, cin, 3, 3)) / np.sqrt(9 * cin)).astype(np.float32)
    b = rng.standard_normal(cout).astype(np.float32)
    xd = torch.from_numpy(x).cuda()
    base = op_conv(xd, wt, b, stride=max(stride, 1), transposed=transposed, relu=True,
                   precision="bf16").cpu()
    xr = torch.from_numpy(x).bfloat16().double().numpy()
    wr = torch.from_numpy(wt).bfloat16().double().numpy()
    ref = _ref(xr, wr, b.astype(np.float64), stride, transposed, True)
    absref = _ref(np.abs(xr), np.abs(wr), np.abs(b).astype(np.float64), stride, transposed, False)
    assert np.all(np.abs(base.numpy() - ref) <= 2e-5 * absref + 1e-6)
    rows = 4 * cout if (transposed and cout <= 16) else cout
    for n_tile in (256, 128, 64, 32):
        if n_tile >= 2 * ((rows + 31) // 32 * 32):
            continue
        for tile_w in (8, 16, 32, 64):
            got = op_conv(xd, wt, b, stride=max(stride, 1), transposed=transposed, relu=True,
                          precision="bf16", n_tile=n_tile, tile_w=tile_w).cpu()
            assert torch.equal(got, base), (n_tile, tile_w, (got - base).abs().max().item())
    halo = ((not transposed and stride == 1) or (transposed and cout <= 16)) and cin % 64 == 0
    if halo:
        got = op_conv(xd, wt, b, stride=max(stride, 1), transposed=transposed, relu=True,
                      precision="bf16", n_tile=1).cpu()
        assert torch.equal(got, base), ("halo", (got - base).abs().max().item())


HALO_CASES = [
    # (cin, cout, h, w, transposed): stride-1 3x3 convs and phase-merged
    # transposed convs, ragged against the 16x16 block, several N tiles
    (64, 16, 37, 45, False),
    (128, 64, 20, 33, False),
    (64, 40, 16, 16, False),
    (128, 5, 23, 19, True),
    (64, 16, 17, 31, True),
    (192, 8, 9, 40, True),
]


@pytest.mark.parametrize("cin,cout,h,w,transposed", HALO_CASES)
@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_conv_halo_kernel_vs_oracle(cin, cout, h, w, transposed, precision):
    """The halo-reuse kernel (one input halo per channel slice, nine taps read
    from LDS) against the oracle, on shapes where blocks straddle the image
    border and the output grid is not a multiple of 16."""
    from paper_2112_10603_amd import op_conv
    print(f"case halo cin={cin} cout={cout} h={h} w={w} T={transposed} {precision}", flush=True)
    rng = np.random.default_rng(cin * 31 + cout)
    n = 3
    x = rng.standard_normal((n, cin, h, w)).astype(np.float32)
    if transposed:
        wt = (rng.standard_normal((cin, cout, 4, 4)) / np.sqrt(4 * cin)).astype(np.float32)
    else:
        wt = (rng.standard_normal((cout, cin, 3, 3)) / np.sqrt(9 * cin)).astype(np.float32)
    b = rng.standard_normal(cout).astype(np.float32)
    if precision == "bf16":
        xr = torch.from_numpy(x).bfloat16().double().numpy()
        wr = torch.from_numpy(wt).bfloat16().double().numpy()
    else:
        xr, wr = x.astype(np.float64), wt.astype(np.float64)
    ref = _ref(xr, wr, b.astype(np.float64), 1, transposed, True)
    absref = _ref(np.abs(xr), np.abs(wr), np.abs(b).astype(np.float64), 1, transposed, False)
    xd = torch.from_numpy(x).cuda()
    got = op_conv(xd, wt, b, stride=1, transposed=transposed, relu=True, precision=precision,
                  n_tile=1).cpu().numpy()
    err = np.abs(got.astype(np.float64) - ref)
    assert np.all(err <= 2e-5 * absref + 1e-6), (err.max(), (err / (absref + 1e-12)).max())
