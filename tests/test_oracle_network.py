"""Pins for the oracle's whole-network evaluation: the layer table's shapes,
closed forms under structured weights, and an independent float64
re-implementation from torch library routines."""
import os
import re

import numpy as np
import pytest

from oracle import vinet as O
from synth import scenes
from synth.weights import make_weights, write_weights_file

from .torch_reference import forward as torch_forward

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table3_layers.txt")


def _ratio(expr, i):
    expr = expr.replace("2^i", str(2 ** i))
    num, _, den = expr.partition("/")
    return float(num) / float(den or 1)


def test_layer_table_shapes(random_weights_file):
    """Every layer's output width and resolution match the supplementary layer
    table; ReLU layers are non-negative, the heads are not clipped."""
    W = O.load_weights(random_weights_file)
    H, Wd = 128, 256
    xl, xr = scenes.random_pair(5, H, Wd)
    taps = {}
    O.vinet_forward(xl.numpy(), xr.numpy(), 0.5, W, taps)
    layers = taps["layers"]
    rows = [ln.split() for ln in open(GOLDEN) if ln.strip() and not ln.startswith("#")]
    n = 0
    for name, ratio, cout, relu in rows:
        for i in (range(3) if "{i}" in name else [None]):
            nm = name.replace("{i}", str(i)) if i is not None else name
            r = _ratio(ratio, i or 0)
            y = layers[nm]
            assert y.shape == (int(cout), int(H * r), int(Wd * r)), (nm, y.shape)
            if relu == "1":
                assert y.min() >= 0.0, nm
            else:
                assert y.min() < 0.0 or nm == "unet.head", nm
            n += 1
    assert n == 3 * 10 + 8 + 13


def test_param_count_matches_layer_table():
    from synth.weights import param_count
    # widths from the layer table at base width 32, with the t plane input
    assert param_count(32, True) == 16411042


def test_zero_heads_gives_average(weights_dir):
    """All flow/mask heads and the refine head zero: F = 0, M = 0 so both
    warps are identities, the mask is 1/2 and the residual 2*sigma(0)-1 = 0:
    the output is the plain average of the two views (ragged size, so the
    replicate padding and the crop are exercised)."""
    p = write_weights_file(str(weights_dir / "zero.ffvw"), seed=3, kind="zero_heads")
    W = O.load_weights(p)
    xl, xr = scenes.random_pair(7, 40, 72)
    out = O.vinet_forward(xl.numpy(), xr.numpy(), 0.3, W)
    want = 0.5 * (xl.numpy().astype(np.float64) + xr.numpy().astype(np.float64))
    np.testing.assert_allclose(out, want, rtol=0, atol=1e-15)


def test_constant_flow_heads_give_true_middle_view(weights_dir):
    """Stage-0 head bias (1/2, 0, -1/2, 0, 0) at quarter resolution doubles
    twice to a full-resolution flow of (2, 0, -2, 0); with the right view the
    left shifted by 4 px, both warps land on T(x + 2): the exact middle view
    (Eq. 1 with M = 1/2) wherever neither sample is clamped."""
    p = write_weights_file(str(weights_dir / "cflow.ffvw"), seed=0, kind="const_flow")
    W = O.load_weights(p)
    xl, xr = scenes.small_pair()
    taps = {}
    out = O.vinet_forward(xl.numpy(), xr.numpy(), 0.5, W, taps)
    np.testing.assert_array_equal(taps["F2"][0], 2.0)
    np.testing.assert_array_equal(taps["F2"][2], -2.0)
    np.testing.assert_array_equal(taps["F2"][1], 0.0)
    np.testing.assert_array_equal(taps["M2"], 0.0)
    W_ = xl.shape[2]
    np.testing.assert_array_equal(out[:, :, 2:W_ - 2], xl.numpy()[:, :, 4:].astype(np.float64))


@pytest.mark.parametrize("H,W_,t,tp", [(64, 64, 0.5, True), (40, 88, 0.25, True),
                                       (48, 32, 0.5, False)])
def test_cross_implementation(weights_dir, H, W_, t, tp):
    """Random weights: no output value is fixed by the paper, so the numpy
    oracle is checked against a second float64 evaluation built from torch
    library routines (grid_sample, interpolate, conv2d, conv_transpose2d,
    avg_pool2d for the flow pyramid)."""
    seed = 11
    Wd = make_weights(seed, 32, tp)
    p = write_weights_file(str(weights_dir / f"x{tp}.ffvw"), seed=seed, t_plane=tp)
    W = O.load_weights(p)
    xl, xr = scenes.random_pair(13, H, W_, d_max=6.0)
    a = O.vinet_forward(xl.numpy(), xr.numpy(), t, W)
    b = torch_forward(xl.numpy(), xr.numpy(), t, Wd, t_plane=tp)
    assert a.shape == (3, H, W_)
    np.testing.assert_allclose(a, b, rtol=0, atol=1e-10)
    assert 0.01 < np.mean((a > 0) & (a < 1))


def test_t_changes_output(random_weights_file):
    W = O.load_weights(random_weights_file)
    xl, xr = scenes.random_pair(3, 32, 32)
    a = O.vinet_forward(xl.numpy(), xr.numpy(), 0.2, W)
    b = O.vinet_forward(xl.numpy(), xr.numpy(), 0.8, W)
    assert np.abs(a - b).max() > 1e-6


def test_bad_arguments(random_weights_file):
    W = O.load_weights(random_weights_file)
    x = np.zeros((3, 16, 16))
    with pytest.raises(ValueError):
        O.vinet_forward(x, x, 1.5, W)
    with pytest.raises(ValueError):
        O.vinet_forward(x, np.zeros((3, 16, 32)), 0.5, W)


def test_weights_roundtrip(random_weights_file):
    W = O.load_weights(random_weights_file)
    ref = make_weights(0, 32, True)
    assert set(W["layers"]) == set(ref)
    for name, (w, b) in ref.items():
        np.testing.assert_array_equal(W["layers"][name][2], w.astype(np.float64))
        np.testing.assert_array_equal(W["layers"][name][3], b.astype(np.float64))
    head = open(random_weights_file, "rb").read(4096)
    assert re.search(rb"sha256 [0-9a-f]{64}", head)


def test_blend_only_closed_forms(weights_dir):
    """The "w/o Refine" output (the Eq. 1 blend alone): zero heads give the
    plain average; constant-flow heads give the true middle view T(x + 2)."""
    pz = write_weights_file(str(weights_dir / "zero_b.ffvw"), seed=3, kind="zero_heads")
    xl, xr = scenes.random_pair(7, 40, 72)
    out = O.vinet_forward(xl.numpy(), xr.numpy(), 0.7, O.load_weights(pz), refine=False)
    want = 0.5 * (xl.numpy().astype(np.float64) + xr.numpy().astype(np.float64))
    np.testing.assert_allclose(out, want, rtol=0, atol=1e-15)
    pc = write_weights_file(str(weights_dir / "cflow_b.ffvw"), seed=0, kind="const_flow")
    xl, xr = scenes.small_pair()
    out = O.vinet_forward(xl.numpy(), xr.numpy(), 0.5, O.load_weights(pc), refine=False)
    W_ = xl.shape[2]
    np.testing.assert_array_equal(out[:, :, 2:W_ - 2], xl.numpy()[:, :, 4:].astype(np.float64))


def test_blend_only_equals_full_net_without_residual(weights_dir):
    """Random flow/mask weights with a zero output head: the residual
    2*sigma(0) - 1 is exactly 0 and the blend lies in [0, 1], so the full
    network's output equals the blend-only output up to the rounding of
    (I2 + 1) - 1, i.e. within one ulp of 1.0."""
    p = write_weights_file(str(weights_dir / "zref.ffvw"), seed=5, kind="zero_refine")
    W = O.load_weights(p)
    xl, xr = scenes.random_pair(17, 36, 52, d_max=5.0)
    full = O.vinet_forward(xl.numpy(), xr.numpy(), 0.4, W)
    blend = O.vinet_forward(xl.numpy(), xr.numpy(), 0.4, W, refine=False)
    assert blend.shape == (3, 36, 52)
    np.testing.assert_allclose(full, blend, rtol=0, atol=2.3e-16)
    # and a random output head does change it
    W2 = O.load_weights(write_weights_file(str(weights_dir / "rref.ffvw"), seed=5))
    assert np.abs(O.vinet_forward(xl.numpy(), xr.numpy(), 0.4, W2) - blend).max() > 1e-3


@pytest.mark.parametrize("levels", [1, 2, 3])
def test_recursive_midpoints_zero_heads_are_linear(weights_dir, levels):
    """Dense views by recursive midpoints: 2^n - 1 views (paper, section 4:
    n levels give 2^n - 1 virtual views). With zero heads every synthesis is
    the average of its two inputs, so the view at t = k/2^n is exactly the
    linear blend (1 - t) X_l + t X_r."""
    p = write_weights_file(str(weights_dir / "zero_r.ffvw"), seed=3, kind="zero_heads")
    W = O.load_weights(p)
    xl, xr = scenes.random_pair(9, 32, 48)
    a, b = xl.numpy().astype(np.float64), xr.numpy().astype(np.float64)
    views = O.vinet_recursive(xl.numpy(), xr.numpy(), levels, W)
    n = 1 << levels
    assert len(views) == n - 1
    for k, v in enumerate(views, start=1):
        t = k / n
        np.testing.assert_allclose(v, (1 - t) * a + t * b, rtol=0, atol=1e-14)


def test_recursive_wiring(random_weights_file):
    """Level 1 is the t = 1/2 synthesis; level 2 synthesises the middles of
    (X_l, V_1/2) and (V_1/2, X_r)."""
    W = O.load_weights(random_weights_file)
    xl, xr = scenes.random_pair(19, 32, 32, d_max=4.0)
    a, b = xl.numpy(), xr.numpy()
    v = O.vinet_recursive(a, b, 2, W)
    mid = O.vinet_forward(a, b, 0.5, W)
    np.testing.assert_array_equal(v[1], mid)
    np.testing.assert_array_equal(v[0], O.vinet_forward(a, mid, 0.5, W))
    np.testing.assert_array_equal(v[2], O.vinet_forward(mid, b, 0.5, W))
    with pytest.raises(ValueError):
        O.vinet_recursive(a, b, 0, W)
