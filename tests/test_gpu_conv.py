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


def _resident_fits(cin, cout, bn, transposed, stride, elem):
    """Whether the resident-weight kernel runs the layer: a stride-1 3x3
    conv, a phase-merged transposed conv (at most 16 outputs) or one phase
    of a transposed conv, whole K steps of channels, at most bn GEMM columns
    and weights that fit its LDS buffer."""
    if not transposed and stride != 1:
        return False
    merged = transposed and cout <= 16
    rows = 4 * cout if merged else cout
    taps = 4 if (transposed and not merged) else 9
    cin_pad = (cin + 7) // 8 * 8
    if cin_pad % (128 // elem) or rows > bn:
        return False
    return bn * (taps * cin_pad * elem // 16 + 1) <= 4800


VARIANT_CASES = [
    # (cin, cout, h, w, stride, transposed): shapes that span several M tiles
    (64, 256, 40, 52, 1, False),
    (128, 128, 37, 45, 2, False),
    (256, 128, 19, 23, 0, True),
    (64, 16, 21, 27, 0, True),
    (64, 40, 33, 29, 1, False),
    (128, 5, 18, 35, 0, True),
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
    for code, bn in ((4, 32), (5, 64)):  # resident-weight kernels, where they apply
        if _resident_fits(cin, cout, bn, transposed, stride, 2):
            got = op_conv(xd, wt, b, stride=max(stride, 1), transposed=transposed, relu=True,
                          precision="bf16", n_tile=code).cpu()
            assert torch.equal(got, base), ("resident", bn, (got - base).abs().max().item())
    if (transposed or stride == 1) and cin % 64 == 0:
        per_phase = transposed and cout > 16
        codes = (2, 3, 10) + ((9,) if not per_phase or cout <= 64 else ())
        if per_phase and cout > 128:
            codes = (2,)
        for code in codes:  # 128- and 256-channel halo tiles, 2 x 4-wave layout
            for tile_w in (8, 16, 32):
                got = op_conv(xd, wt, b, stride=max(stride, 1), transposed=transposed, relu=True,
                              precision="bf16", n_tile=code, tile_w=tile_w).cpu()
                assert torch.equal(got, base), ("halo tile", code, tile_w, (got - base).abs().max().item())


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


HALO_TILE_CASES = [
    # (cin, cout, h, w, transposed): the 128/256-channel halo tiles on
    # stride-1 convs, per-phase transposed convs (cout > 16) and
    # phase-merged ones (cout <= 16), ragged against every block shape
    (256, 256, 19, 37, False),
    (64, 128, 33, 21, False),
    (128, 200, 9, 70, False),
    (256, 128, 13, 22, True),
    (128, 5, 23, 19, True),
    (128, 40, 11, 19, True),
    (256, 64, 13, 17, True),
]


@pytest.mark.parametrize("cin,cout,h,w,transposed", HALO_TILE_CASES)
@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_conv_halo_tiles_vs_oracle(cin, cout, h, w, transposed, precision):
    """The conv kernel's halo variant (one (TH+2) x (TW+2) input halo per
    channel slice, every tap read from LDS) against the oracle, for both N
    tiles and the three block widths it accepts; on per-phase transposed
    convs the 256-column tile computes two output phases at once."""
    from paper_2112_10603_amd import op_conv
    rng = np.random.default_rng(cin * 13 + cout + h)
    n = 2
    per_phase = transposed and cout > 16
    codes = (2, 3, 10) + ((9,) if not per_phase or cout <= 64 else ())
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
    for code in codes:
        for tile_w in (8, 16, 32):
            print(f"case halo tile {code} tw={tile_w} cin={cin} cout={cout} h={h} w={w} T={transposed} "
                  f"{precision}", flush=True)
            got = op_conv(xd, wt, b, stride=1, transposed=transposed, relu=True, precision=precision,
                          n_tile=code, tile_w=tile_w).cpu().numpy()
            err = np.abs(got.astype(np.float64) - ref)
            assert np.all(err <= 2e-5 * absref + 1e-6), (code, tile_w, err.max())


def test_conv_halo_tile_rejects_other_layers():
    """A stride-2 conv, or a block width whose halo would not fit, is
    refused with an error (nothing is launched)."""
    from paper_2112_10603_amd import op_conv
    from paper_2112_10603_amd.ffv import FfvError
    print("case halo tile rejects", flush=True)
    rng = np.random.default_rng(5)
    x = torch.from_numpy(rng.standard_normal((1, 64, 12, 12)).astype(np.float32)).cuda()
    wt = rng.standard_normal((64, 64, 3, 3)).astype(np.float32)
    b = np.zeros(64, np.float32)
    with pytest.raises(FfvError):
        op_conv(x, wt, b, stride=2, precision="bf16", n_tile=3, tile_w=16)
    with pytest.raises(FfvError):
        op_conv(x, wt, b, stride=1, precision="bf16", n_tile=3, tile_w=64)
    with pytest.raises(FfvError):
        op_conv(x, wt, b, stride=2, precision="bf16", n_tile=10, tile_w=16)
    with pytest.raises(FfvError):
        op_conv(x, wt, b, stride=1, precision="bf16", n_tile=10, tile_w=64)


RESIDENT_CASES = [
    # (n, cin, cout, h, w, transposed): the resident-weight kernels on
    # stride-1 convs and phase-merged transposed convs; the last two have
    # more 16x16 blocks than workgroups, so each workgroup walks several
    (2, 64, 16, 37, 45, False),
    (2, 64, 40, 16, 16, False),
    (3, 128, 5, 23, 19, True),
    (2, 64, 16, 17, 31, True),
    (8, 64, 16, 128, 160, False),
    (6, 128, 5, 100, 90, True),
    (2, 128, 32, 13, 22, True),
    (2, 64, 64, 15, 17, True),
    (2, 64, 24, 19, 21, True),
    (6, 128, 32, 70, 90, True),
]


@pytest.mark.parametrize("n,cin,cout,h,w,transposed", RESIDENT_CASES)
@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_conv_resident_vs_oracle(n, cin, cout, h, w, transposed, precision):
    """The persistent resident-weight kernel against the oracle, for every
    N tile whose weights fit; bf16 results also equal the default tiling's
    bit for bit."""
    from paper_2112_10603_amd import op_conv
    elem = 2 if precision == "bf16" else 4
    codes = [code for code, bn in ((4, 32), (5, 64)) if _resident_fits(cin, cout, bn, transposed, 1, elem)]
    if not codes:
        pytest.skip("weights do not fit the resident buffer at this precision")
    rng = np.random.default_rng(n * 101 + cin + cout + h)
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
    base = op_conv(xd, wt, b, stride=1, transposed=transposed, relu=True, precision=precision).cpu()
    for code in codes:
        print(f"case resident {code} n={n} cin={cin} cout={cout} h={h} w={w} T={transposed} {precision}",
              flush=True)
        got = op_conv(xd, wt, b, stride=1, transposed=transposed, relu=True, precision=precision,
                      n_tile=code).cpu()
        err = np.abs(got.numpy().astype(np.float64) - ref)
        assert np.all(err <= 2e-5 * absref + 1e-6), (code, err.max())
        if precision == "bf16":
            assert torch.equal(got, base), (code, (got - base).abs().max().item())


def test_conv_resident_rejects_large_weights():
    """Weights that do not fit the resident buffer (256 input channels at 32
    columns), or a stride-2 conv, are refused with an error."""
    from paper_2112_10603_amd import op_conv
    from paper_2112_10603_amd.ffv import FfvError
    print("case resident rejects", flush=True)
    rng = np.random.default_rng(9)
    x = torch.from_numpy(rng.standard_normal((1, 256, 16, 16)).astype(np.float32)).cuda()
    wt = rng.standard_normal((16, 256, 3, 3)).astype(np.float32)
    b = np.zeros(16, np.float32)
    with pytest.raises(FfvError):
        op_conv(x, wt, b, stride=1, precision="bf16", n_tile=4)
    x2 = torch.from_numpy(rng.standard_normal((1, 64, 16, 16)).astype(np.float32)).cuda()
    w2 = rng.standard_normal((16, 64, 3, 3)).astype(np.float32)
    with pytest.raises(FfvError):
        op_conv(x2, w2, b, stride=2, precision="bf16", n_tile=4)


STAGED_CASES = [
    # (n, cin, cout, h, w, stride, transposed, n_tile, tile_w): layers whose
    # bf16 output the kernels stage through LDS for 16-byte stores
    (2, 64, 256, 21, 35, 1, False, 256, 16),
    (2, 128, 128, 19, 23, 2, False, 128, 32),
    (2, 256, 128, 9, 13, 0, True, 128, 16),
    (2, 256, 256, 19, 37, 1, False, 3, 32),
    (2, 256, 128, 13, 22, 0, True, 2, 16),
    (2, 64, 16, 37, 45, 1, False, 4, 16),
    (2, 64, 64, 30, 50, 1, False, 5, 16),
    (2, 64, 16, 17, 31, 0, True, 5, 16),
    (8, 64, 16, 128, 160, 1, False, 5, 16),
    (6, 64, 8, 60, 70, 0, True, 4, 16),
    (2, 128, 32, 19, 23, 0, True, 4, 16),
    (2, 64, 64, 21, 18, 0, True, 5, 16),
    (2, 256, 128, 13, 22, 0, True, 3, 32),
    (2, 128, 40, 11, 19, 0, True, 3, 8),
    (2, 256, 64, 13, 17, 0, True, 9, 16),
    (2, 64, 256, 21, 35, 1, False, 9, 32),
    (2, 256, 256, 19, 37, 1, False, 10, 16),
    (2, 128, 128, 13, 22, 0, True, 10, 8),
    (2, 64, 40, 11, 19, 0, True, 10, 32),
]


@pytest.mark.parametrize("n,cin,cout,h,w,stride,transposed,n_tile,tile_w", STAGED_CASES)
def test_conv_bf16_output_epilogues(n, cin, cout, h, w, stride, transposed, n_tile, tile_w):
    """bf16 outputs as the network's layers write them (the LDS-staged
    16-byte-store epilogues): equal to the float32 output of the same
    variant rounded to bf16, for every layer kind and tile."""
    from paper_2112_10603_amd import op_conv
    print(f"case bf16 out n={n} cin={cin} cout={cout} h={h} w={w} s={stride} T={transposed} "
          f"tile={n_tile}/{tile_w}", flush=True)
    rng = np.random.default_rng(cin * 7 + cout + h * 3 + n_tile)
    x = rng.standard_normal((n, cin, h, w)).astype(np.float32)
    if transposed:
        wt = (rng.standard_normal((cin, cout, 4, 4)) / np.sqrt(4 * cin)).astype(np.float32)
    else:
        wt = (rng.standard_normal((cout, cin, 3, 3)) / np.sqrt(9 * cin)).astype(np.float32)
    b = rng.standard_normal(cout).astype(np.float32)
    xd = torch.from_numpy(x).cuda()
    kw = dict(stride=max(stride, 1), transposed=transposed, relu=True, precision="bf16",
              n_tile=n_tile, tile_w=tile_w)
    f32 = op_conv(xd, wt, b, **kw).cpu()
    got = op_conv(xd, wt, b, act_out=True, **kw).cpu()
    assert torch.equal(got, f32.bfloat16().float()), (got - f32.bfloat16().float()).abs().max().item()


S2_CASES = [
    # (n, cin, cout, h, w, stride, n_tile): convs with 8 to 32 input channels
    # (the first conv of a VIBlock, the U-Net and context levels) through the
    # persistent few-channel kernel; odd sizes, and some with more output
    # blocks than workgroups
    (2, 24, 128, 35, 70, 2, 8),
    (2, 8, 128, 17, 33, 2, 8),
    (2, 7, 128, 20, 30, 2, 8),
    (2, 17, 32, 33, 66, 2, 6),
    (2, 32, 64, 30, 44, 2, 7),
    (2, 16, 32, 40, 40, 2, 6),
    (2, 3, 16, 25, 31, 2, 6),
    (2, 24, 64, 21, 37, 2, 7),
    (4, 24, 128, 130, 250, 2, 8),
    (8, 17, 32, 140, 200, 2, 6),
    (2, 32, 32, 37, 45, 1, 6),
    (2, 16, 16, 20, 33, 1, 6),
    (2, 24, 128, 19, 23, 1, 8),
    (2, 32, 64, 17, 40, 1, 7),
    (6, 32, 32, 70, 100, 1, 6),
]


@pytest.mark.parametrize("n,cin,cout,h,w,stride,n_tile", S2_CASES)
def test_conv_few_channel_resident_equals_generic(n, cin, cout, h, w, stride, n_tile):
    """The persistent few-channel kernel walks K in the generic kernel's
    chunk order, so its bf16 output equals the default tiling's bit for bit;
    the default tiling's float output (oracle-checked above) rounds to it."""
    from paper_2112_10603_amd import op_conv
    print(f"case few-channel resident n={n} cin={cin} cout={cout} h={h} w={w} s={stride} tile={n_tile}",
          flush=True)
    rng = np.random.default_rng(n * 13 + cin * 7 + cout + h)
    x = rng.standard_normal((n, cin, h, w)).astype(np.float32)
    wt = (rng.standard_normal((cout, cin, 3, 3)) / np.sqrt(9 * cin)).astype(np.float32)
    b = rng.standard_normal(cout).astype(np.float32)
    xd = torch.from_numpy(x).cuda()
    base = op_conv(xd, wt, b, stride=stride, relu=True, precision="bf16", n_tile=128 if cout > 64 else 32,
                   tile_w=16, act_out=True).cpu()
    got = op_conv(xd, wt, b, stride=stride, relu=True, precision="bf16", n_tile=n_tile, tile_w=16,
                  act_out=True).cpu()
    assert torch.equal(got, base), (got - base).abs().max().item()
    if n == 2:
        xr = torch.from_numpy(x).bfloat16().double().numpy()
        wr = torch.from_numpy(wt).bfloat16().double().numpy()
        ref = _ref(xr, wr, b.astype(np.float64), stride, False, True)
        absref = _ref(np.abs(xr), np.abs(wr), np.abs(b).astype(np.float64), stride, False, False)
        # bf16 output: half an ulp of the value on top of the accumulation bound
        assert np.all(np.abs(got.numpy() - ref) <= 2e-5 * absref + np.abs(ref) * 2.0 ** -8 + 1e-6)


def test_conv_stride2_resident_rejects():
    """Float outputs or 64 input channels are refused."""
    from paper_2112_10603_amd import op_conv
    from paper_2112_10603_amd.ffv import FfvError
    print("case stride-2 resident rejects", flush=True)
    rng = np.random.default_rng(11)
    x = torch.from_numpy(rng.standard_normal((1, 24, 20, 20)).astype(np.float32)).cuda()
    wt = rng.standard_normal((128, 24, 3, 3)).astype(np.float32)
    b = np.zeros(128, np.float32)
    with pytest.raises(FfvError):
        op_conv(x, wt, b, stride=2, precision="bf16", n_tile=8, tile_w=16)  # float output
    x2 = torch.from_numpy(rng.standard_normal((1, 64, 20, 20)).astype(np.float32)).cuda()
    w2 = rng.standard_normal((128, 64, 3, 3)).astype(np.float32)
    with pytest.raises(FfvError):
        op_conv(x2, w2, b, stride=2, precision="bf16", n_tile=8, tile_w=16, act_out=True)
