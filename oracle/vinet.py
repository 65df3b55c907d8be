"""FP64 CPU oracle of the view-interpolation network (VINet) forward pass.

TEST INFRASTRUCTURE ONLY. This module is the plain, slow reference that the
GPU library is checked against. It may be imported only by the tests, by the
smoke check and by the benchmark's CPU-baseline leg; the product path never
calls it, and it shares no code with the GPU library (it reads the same
weights file with its own parser).

Everything is numpy float64, one (pair, t) at a time, planar [C, H, W].

What it computes (paper section 3.1 and the supplementary layer table), with
the readings taken where the paper is silent:

* Eq. 1: the virtual view is the mask-weighted blend of the left view warped
  by F_m->l and the right view warped by F_m->r.
* Eq. 2: three VIBlocks estimate flow and mask coarse to fine; stages 1 and 2
  add a residual to the x2-upscaled previous estimate. The mask is carried as
  a logit and squashed by a sigmoid where it blends. The per-stage blends of
  Eq. 2 are a training device and are not on the inference path.
* Layer table (supplementary): VIBlock_i = conv s2 -> 4B, conv s2 -> 8B,
  6 x conv -> 8B, convT s2 -> 4B, convT s2 -> 5 (ReLU after all but the
  last); ContextNet = 4 x (conv s2, conv) at widths B/2, B, 2B, 4B; the
  RefineNet U-Net = 4 x (conv s2, conv) at B, 2B, 4B, 8B, then 4 convT s2 to
  4B, 2B, B, B/2, then a conv to 3 channels with a sigmoid. B = 32 gives the
  table's widths.
* Refinement (section 3.1, "Refinement Network"): context features of both
  views are warped to the middle view and concatenated into the U-Net
  encoder; the U-Net output r in (0, 1) becomes the residual 2r - 1 added to
  the blended view, clamped to [0, 1].

Readings (where the paper is silent or ambiguous):

* convolutions are 3x3 with padding 1; transposed convs are 4x4, stride 2,
  padding 1 (exact x2);
* stage s runs on the views resampled to 2^s/4 of the (padded) size with
  bilinear, half-pixel-centre sampling and no antialiasing;
* flows are in pixels of the stage's grid and are doubled when upscaled;
* warps are backward bilinear with the sample position clamped to the image
  (border mode);
* input sizes are replicate-padded at the bottom/right to a multiple of 16
  and the output is cropped back;
* an optional constant phase plane t is the last input channel of every
  VIBlock, so that views at any t in [0, 1] can be synthesised;
* VIBlock input channels: stage 0 [L, R, (t)], stages 1-2
  [L, R, W_l, W_r, M~, F~, (t)]; U-Net input [X_l, X_r, W_l, W_r, M, F];
  flow channel order (F_l.x, F_l.y, F_r.x, F_r.y), then the mask logit.
"""
from __future__ import annotations

import struct

import numpy as np

# --------------------------------------------------------------------------
# weights file (own reader; see the file layout documented with the writer)
# --------------------------------------------------------------------------


def load_weights(path: str) -> dict:
    """Read a ``.ffvw`` file into ``{"base_width", "t_plane", "layers"}``.

    ``layers[name] = (kind, stride, w float64, b float64)`` with conv weights
    ``[cout, cin, 3, 3]`` and transposed-conv weights ``[cin, cout, 4, 4]``.
    """
    with open(path, "rb") as fh:
        raw = fh.read()
    if raw[:4] != b"FFVW":
        raise ValueError("not a weights file")
    version, hlen, _ = struct.unpack("<III", raw[4:16])
    if version != 1:
        raise ValueError("unsupported weights version")
    text = raw[16:16 + hlen].decode("ascii")
    start = (16 + hlen + 63) // 64 * 64
    meta: dict = {"layers": {}}
    rows = []
    for line in text.splitlines():
        f = line.split()
        if not f:
            continue
        if f[0] == "layer":
            rows.append(f[1:])
        elif f[0] in ("base_width", "t_plane", "seed", "n_floats", "layers"):
            meta[f[0] if f[0] != "layers" else "n_layers"] = int(f[1])
        elif f[0] == "sha256":
            meta["sha256"] = f[1]
    payload = np.frombuffer(raw, dtype="<f4", count=meta["n_floats"], offset=start)
    for name, kind, cin, cout, stride, wo, wc, bo, bc in rows:
        cin, cout, stride = int(cin), int(cout), int(stride)
        w = payload[int(wo):int(wo) + int(wc)].astype(np.float64)
        b = payload[int(bo):int(bo) + int(bc)].astype(np.float64)
        shape = (cout, cin, 3, 3) if kind == "conv" else (cin, cout, 4, 4)
        meta["layers"][name] = (kind, stride, w.reshape(shape), b)
    meta["t_plane"] = bool(meta["t_plane"])
    return meta


# --------------------------------------------------------------------------
# operators
# --------------------------------------------------------------------------


def relu(x):
    return np.maximum(x, 0.0)


def sigmoid(x):
    return 1.0 / (1.0 + np.exp(-x))


def pad_replicate(x, Hp, Wp):
    """Replicate the last row/column of ``x`` [C, H, W] out to Hp x Wp."""
    C, H, W = x.shape
    return np.pad(x, ((0, 0), (0, Hp - H), (0, Wp - W)), mode="edge")


def conv2d(x, w, b, stride):
    """3x3 convolution, zero padding 1, given stride (section 3.1 layer table).

    out[o, i, j] = b[o] + sum_{c, dy, dx} w[o, c, dy, dx]
                   * x[c, stride*i + dy - 1, stride*j + dx - 1]
    with x = 0 outside the image. Evaluated as im2col + matmul in row bands.
    """
    C, H, W = x.shape
    Co = w.shape[0]
    Ho = (H - 1) // stride + 1
    Wo = (W - 1) // stride + 1
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1)))
    wmat = w.reshape(Co, C * 9)
    out = np.empty((Co, Ho, Wo))
    band = max(1, int(2.0e7 // (C * 9 * Wo)))
    for r0 in range(0, Ho, band):
        r1 = min(Ho, r0 + band)
        cols = np.empty((C, 3, 3, r1 - r0, Wo))
        for dy in range(3):
            for dx in range(3):
                cols[:, dy, dx] = xp[:, stride * r0 + dy: stride * (r1 - 1) + dy + 1: stride,
                                     dx: dx + stride * (Wo - 1) + 1: stride]
        out[:, r0:r1] = (wmat @ cols.reshape(C * 9, -1)).reshape(Co, r1 - r0, Wo)
    out += b[:, None, None]
    return out


def conv_transpose2d(x, w, b):
    """4x4 transposed convolution, stride 2, padding 1 (output 2H x 2W).

    out[o, y, x] = b[o] + sum over (c, iy, ix, ky, kx) with
    y = 2*iy - 1 + ky and x = 2*ix - 1 + kx of w[c, o, ky, kx] * x[c, iy, ix].
    Evaluated as one matmul per tap, scatter-added into the output.
    """
    Ci, H, W = x.shape
    Co = w.shape[1]
    full = np.zeros((Co, 2 * H + 2, 2 * W + 2))
    xm = x.reshape(Ci, H * W)
    for ky in range(4):
        for kx in range(4):
            wt = np.ascontiguousarray(w[:, :, ky, kx].T)
            contrib = (wt @ xm).reshape(Co, H, W)
            full[:, ky: ky + 2 * H: 2, kx: kx + 2 * W: 2] += contrib
    return full[:, 1: 1 + 2 * H, 1: 1 + 2 * W] + b[:, None, None]


def _half_pixel_taps(n_out, n_in):
    i = np.arange(n_out, dtype=np.float64)
    s = np.maximum(0.0, (i + 0.5) * (n_in / n_out) - 0.5)
    i0 = np.minimum(np.floor(s).astype(np.int64), n_in - 1)
    i1 = np.minimum(i0 + 1, n_in - 1)
    return i0, i1, s - i0


def resample(x, h, w):
    """Bilinear resampling of ``x`` [C, H, W] to h x w, half-pixel centres,
    no antialiasing (used for the image pyramid, flow/mask upscaling and the
    flow pyramid)."""
    C, H, W = x.shape
    y0, y1, by = _half_pixel_taps(h, H)
    x0, x1, ax = _half_pixel_taps(w, W)
    r0 = x[:, y0, :]
    r1 = x[:, y1, :]
    top = r0[:, :, x0] * (1.0 - ax) + r0[:, :, x1] * ax
    bot = r1[:, :, x0] * (1.0 - ax) + r1[:, :, x1] * ax
    return top * (1.0 - by)[:, None] + bot * by[:, None]


def warp(x, f):
    """Backward bilinear warp of ``x`` [C, H, W] by flow ``f`` [2, H, W]
    (f[0] along width, f[1] along height, in pixels): out(u) = x(u + f(u))
    with the sample position clamped to [0, W-1] x [0, H-1] (Eq. 1)."""
    C, H, W = x.shape
    gy, gx = np.mgrid[0:H, 0:W].astype(np.float64)
    px = np.clip(gx + f[0], 0.0, W - 1.0)
    py = np.clip(gy + f[1], 0.0, H - 1.0)
    x0 = np.floor(px).astype(np.int64)
    y0 = np.floor(py).astype(np.int64)
    x1 = np.minimum(x0 + 1, W - 1)
    y1 = np.minimum(y0 + 1, H - 1)
    a = px - x0
    b = py - y0
    return ((1 - a) * (1 - b) * x[:, y0, x0] + a * (1 - b) * x[:, y0, x1]
            + (1 - a) * b * x[:, y1, x0] + a * b * x[:, y1, x1])


def blend(wl, wr, m_logit):
    """Eq. 1 with the mask as a logit: sigma(M) * W_l + (1 - sigma(M)) * W_r."""
    m = sigmoid(m_logit)
    return m * wl + (1.0 - m) * wr


# --------------------------------------------------------------------------
# network
# --------------------------------------------------------------------------


def _layer(W, name, kind):
    k, stride, w, b = W["layers"][name]
    assert k == kind, (name, k, kind)
    return stride, w, b


def _record(taps, name, y):
    if taps is not None:
        taps.setdefault("layers", {})[name] = y


def conv_layer(W, name, x, act=True, taps=None):
    stride, w, b = _layer(W, name, "conv")
    assert w.shape[1] == x.shape[0], (name, w.shape, x.shape)
    y = conv2d(x, w, b, stride)
    y = relu(y) if act else y
    _record(taps, name, y)
    return y


def convT_layer(W, name, x, act=True, taps=None):
    _, w, b = _layer(W, name, "convT")
    assert w.shape[0] == x.shape[0], (name, w.shape, x.shape)
    y = conv_transpose2d(x, w, b)
    y = relu(y) if act else y
    _record(taps, name, y)
    return y


def vib_block(W, s, x, taps=None):
    """VIBlock_s (layer table): 8 convs (first two stride 2) and 2 convT;
    returns the 5-channel residual (flow l, flow r, mask logit)."""
    a = conv_layer(W, f"vib{s}.conv1", x, taps=taps)
    a = conv_layer(W, f"vib{s}.conv2", a, taps=taps)
    for i in range(3, 9):
        a = conv_layer(W, f"vib{s}.conv{i}", a, taps=taps)
    a = convT_layer(W, f"vib{s}.convT1", a, taps=taps)
    res = convT_layer(W, f"vib{s}.convT2", a, act=False, taps=taps)
    if taps is not None:
        taps[f"vib{s}.res"] = res
    return res


def context_net(W, x, taps=None):
    """ContextNet (layer table): 4 levels of (conv s2, conv), all ReLU;
    returns the features at 1/2, 1/4, 1/8, 1/16."""
    feats = []
    c = x
    for k in range(4):
        c = conv_layer(W, f"ctx.conv{2 * k + 1}", c, taps=taps)
        c = conv_layer(W, f"ctx.conv{2 * k + 2}", c, taps=taps)
        feats.append(c)
    return feats


def _enc(W, k, z, taps=None):
    z = conv_layer(W, f"unet.enc{2 * k + 1}", z, taps=taps)
    return conv_layer(W, f"unet.enc{2 * k + 2}", z, taps=taps)


def vinet_forward(xl, xr, t, W, taps: dict | None = None, refine: bool = True):
    """Synthesise the view at phase ``t`` between ``xl`` and ``xr``.

    ``xl``, ``xr``: [3, H, W] in [0, 1] (any float type; computed in float64).
    ``W``: the dict from ``load_weights``. Returns [3, H, W] float64.
    If ``taps`` is a dict, intermediate tensors are stored in it.
    ``refine=False`` returns the flow-and-mask blend of Eq. 1 alone (the
    paper's "w/o Refine" variant of its ablation, Table 1), cropped: no
    context features, no U-Net, no residual.
    """
    xl = np.asarray(xl, dtype=np.float64)
    xr = np.asarray(xr, dtype=np.float64)
    if xl.shape != xr.shape or xl.ndim != 3 or xl.shape[0] != 3:
        raise ValueError("views must both be [3, H, W]")
    if not (0.0 <= t <= 1.0):
        raise ValueError("t must lie in [0, 1]")
    _, H, Wd = xl.shape
    Hp = -(-H // 16) * 16
    Wp = -(-Wd // 16) * 16
    Xl = pad_replicate(xl, Hp, Wp)
    Xr = pad_replicate(xr, Hp, Wp)
    tp = W["t_plane"]

    # coarse-to-fine flow and mask (Eq. 2)
    F = M = None
    for s in range(3):
        h, w = Hp * 2 ** s // 4, Wp * 2 ** s // 4
        Ls = Xl if s == 2 else resample(Xl, h, w)
        Rs = Xr if s == 2 else resample(Xr, h, w)
        tplane = [np.full((1, h, w), float(t))] if tp else []
        if s == 0:
            x = np.concatenate([Ls, Rs] + tplane)
            if taps is not None:
                taps["x0_vib"] = x
            res = vib_block(W, 0, x, taps)
            F, M = res[0:4], res[4:5]
        else:
            Ft = 2.0 * resample(F, h, w)
            Mt = resample(M, h, w)
            Wl = warp(Ls, Ft[0:2])
            Wr = warp(Rs, Ft[2:4])
            x = np.concatenate([Ls, Rs, Wl, Wr, Mt, Ft] + tplane)
            if taps is not None:
                taps[f"x{s}_vib"] = x
            res = vib_block(W, s, x, taps)
            F, M = Ft + res[0:4], Mt + res[4:5]
        if taps is not None:
            taps[f"F{s}"] = F
            taps[f"M{s}"] = M

    # final blend (Eq. 1)
    Wl = warp(Xl, F[0:2])
    Wr = warp(Xr, F[2:4])
    I2 = blend(Wl, Wr, M)
    if taps is not None:
        taps["I2"] = I2
    if not refine:
        return I2[:, :H, :Wd]

    # context features, warped to the middle view by the flow pyramid
    cl = context_net(W, Xl, taps)
    cr = context_net(W, Xr)
    wc = []
    Fk = F
    for k in range(4):
        Fk = 0.5 * resample(Fk, Fk.shape[1] // 2, Fk.shape[2] // 2)
        wc.append((warp(cl[k], Fk[0:2]), warp(cr[k], Fk[2:4])))

    # context-aware U-Net
    x0 = np.concatenate([Xl, Xr, Wl, Wr, M, F])
    d1 = _enc(W, 0, x0, taps)
    d2 = _enc(W, 1, np.concatenate([d1, wc[0][0], wc[0][1]]), taps)
    d3 = _enc(W, 2, np.concatenate([d2, wc[1][0], wc[1][1]]), taps)
    d4 = _enc(W, 3, np.concatenate([d3, wc[2][0], wc[2][1]]), taps)
    u1 = convT_layer(W, "unet.dec1", np.concatenate([d4, wc[3][0], wc[3][1]]), taps=taps)
    u2 = convT_layer(W, "unet.dec2", np.concatenate([u1, d3]), taps=taps)
    u3 = convT_layer(W, "unet.dec3", np.concatenate([u2, d2]), taps=taps)
    u4 = convT_layer(W, "unet.dec4", np.concatenate([u3, d1]), taps=taps)
    r = sigmoid(conv_layer(W, "unet.head", u4, act=False, taps=taps))
    out = np.clip(I2 + 2.0 * r - 1.0, 0.0, 1.0)
    if taps is not None:
        taps.update({"d1": d1, "d2": d2, "d3": d3, "d4": d4,
                     "u1": u1, "u2": u2, "u3": u3, "u4": u4, "r": r,
                     "ctx_l": cl, "ctx_r": cr, "wc": wc, "x0": x0})
    return out[:, :H, :Wd]


def vinet_recursive(xl, xr, levels, W, refine: bool = True):
    """Dense views by recursive midpoints (the paper's dense-view scheme,
    section 4, Fig. 6): level 1 synthesises the middle view of (xl, xr);
    each further level synthesises the middle view of every adjacent pair
    of the views so far. ``levels`` = n gives the 2^n - 1 views at
    t = k / 2^n, k = 1 .. 2^n - 1, returned in order of k as a list of
    [3, H, W] float64 arrays. Every synthesis is ``vinet_forward`` at t = 1/2.
    """
    if levels < 1:
        raise ValueError("levels must be >= 1")
    n = 1 << levels
    views = {0: np.asarray(xl, dtype=np.float64), n: np.asarray(xr, dtype=np.float64)}
    for level in range(1, levels + 1):
        step = n >> level
        for k in range(step, n, 2 * step):
            views[k] = vinet_forward(views[k - step], views[k + step], 0.5, W, refine=refine)
    return [views[k] for k in range(1, n)]
