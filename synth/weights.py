"""Seeded synthetic weights for the view-interpolation network, and the
``.ffvw`` file that carries them.

This module draws random numbers and writes/reads a container file. It holds
none of the network's arithmetic: the layer list below is only the set of
tensor shapes to draw (names, kinds, channel counts, strides), taken from the
layer table of the paper's supplementary material (per-layer output widths of
VIBlock_i, ContextNet and RefineNet). The oracle and the GPU library each
define the network on their own and check the shapes they find here.

Layer naming (canonical draw order: VIBlock 0..2, ContextNet, U-Net encoder,
U-Net decoder, output head; weights then bias for each layer):

* ``vib{s}.conv1`` .. ``vib{s}.conv8``  3x3 convs (conv1, conv2 stride 2)
* ``vib{s}.convT1``, ``vib{s}.convT2``  4x4 stride-2 transposed convs
* ``ctx.conv1`` .. ``ctx.conv8``       3x3 convs (odd ones stride 2)
* ``unet.enc1`` .. ``unet.enc8``       3x3 convs (odd ones stride 2)
* ``unet.dec1`` .. ``unet.dec4``       4x4 stride-2 transposed convs
* ``unet.head``                         3x3 conv to 3 channels

Weight layouts: conv ``[cout, cin, 3, 3]``; transposed conv
``[cin, cout, 4, 4]``. Values are stored as little-endian float32.

Draws (``numpy.random.default_rng(seed)``, PCG64): weights He-normal with
std = sqrt(2 / fan_in), fan_in = cin*9 (conv) or cin*4 (transposed conv, the
taps that reach one output pixel); biases N(0, 0.05^2). The output head's
weights are additionally scaled by 0.1 and its bias is zero (not drawn), so
that the refinement stays a residual under random weights.

File layout (``.ffvw``, version 1)::

    bytes 0..3   b"FFVW"
    bytes 4..7   uint32 version (1)
    bytes 8..11  uint32 header_len
    bytes 12..15 uint32 0
    header_len bytes of ASCII text, lines of whitespace-separated fields:
        base_width <B>
        t_plane <0|1>
        seed <seed>
        n_floats <N>
        sha256 <64 hex digits of the payload>
        layers <L>
        layer <name> <conv|convT> <cin> <cout> <stride> <w_off> <w_cnt> <b_off> <b_cnt>
        ...
        end
    payload at offset round_up(16 + header_len, 64): N float32 values.

Offsets and counts are in floats from the start of the payload. The checksum
is SHA-256 (FIPS 180-4) over the payload bytes.
"""
from __future__ import annotations

import hashlib
import struct
from dataclasses import dataclass

import numpy as np

MAGIC = b"FFVW"
VERSION = 1


@dataclass(frozen=True)
class LayerShape:
    name: str
    kind: str  # "conv" or "convT"
    cin: int
    cout: int
    stride: int


def layer_shapes(base_width: int = 32, t_plane: bool = True) -> list[LayerShape]:
    """Tensor shapes to draw, in canonical order (see module docstring)."""
    B = base_width
    if B % 2 != 0 or B < 2:
        raise ValueError("base width must be even and >= 2")
    tp = 1 if t_plane else 0
    out: list[LayerShape] = []
    for s in range(3):
        cin1 = (6 if s == 0 else 17) + tp
        out.append(LayerShape(f"vib{s}.conv1", "conv", cin1, 4 * B, 2))
        out.append(LayerShape(f"vib{s}.conv2", "conv", 4 * B, 8 * B, 2))
        for i in range(3, 9):
            out.append(LayerShape(f"vib{s}.conv{i}", "conv", 8 * B, 8 * B, 1))
        out.append(LayerShape(f"vib{s}.convT1", "convT", 8 * B, 4 * B, 2))
        out.append(LayerShape(f"vib{s}.convT2", "convT", 4 * B, 5, 2))
    ctx_w = [B // 2, B, 2 * B, 4 * B]
    cin = 3
    for k, w in enumerate(ctx_w):
        out.append(LayerShape(f"ctx.conv{2 * k + 1}", "conv", cin, w, 2))
        out.append(LayerShape(f"ctx.conv{2 * k + 2}", "conv", w, w, 1))
        cin = w
    enc_w = [B, 2 * B, 4 * B, 8 * B]
    enc_in = [17, 2 * B, 4 * B, 8 * B]
    for k in range(4):
        out.append(LayerShape(f"unet.enc{2 * k + 1}", "conv", enc_in[k], enc_w[k], 2))
        out.append(LayerShape(f"unet.enc{2 * k + 2}", "conv", enc_w[k], enc_w[k], 1))
    dec = [(16 * B, 4 * B), (8 * B, 2 * B), (4 * B, B), (2 * B, B // 2)]
    for k, (ci, co) in enumerate(dec):
        out.append(LayerShape(f"unet.dec{k + 1}", "convT", ci, co, 2))
    out.append(LayerShape("unet.head", "conv", B // 2, 3, 1))
    return out


def weight_shape(L: LayerShape) -> tuple[int, int, int, int]:
    if L.kind == "conv":
        return (L.cout, L.cin, 3, 3)
    return (L.cin, L.cout, 4, 4)


def make_weights(
    seed: int = 0,
    base_width: int = 32,
    t_plane: bool = True,
) -> dict[str, tuple[np.ndarray, np.ndarray]]:
    """Draw every layer's (weight, bias) as float32 arrays, canonical order."""
    rng = np.random.default_rng(seed)
    out: dict[str, tuple[np.ndarray, np.ndarray]] = {}
    for L in layer_shapes(base_width, t_plane):
        shp = weight_shape(L)
        fan_in = L.cin * (9 if L.kind == "conv" else 4)
        w = rng.standard_normal(shp) * np.sqrt(2.0 / fan_in)
        if L.name == "unet.head":
            w = w * 0.1
            b = np.zeros(L.cout)
        else:
            b = rng.standard_normal(L.cout) * 0.05
        out[L.name] = (w.astype(np.float32), b.astype(np.float32))
    return out


def structured_weights(
    kind: str,
    seed: int = 0,
    base_width: int = 32,
    t_plane: bool = True,
) -> dict[str, tuple[np.ndarray, np.ndarray]]:
    """Random weights with the output heads replaced by fixed values.

    ``kind="zero_heads"``: every VIBlock's last transposed conv and the
    output head have zero weights and zero bias.

    ``kind="const_flow"``: as ``zero_heads``, but VIBlock 0's last bias is
    (0.5, 0, -0.5, 0, 0).

    ``kind="zero_refine"``: only the output head is zero (random flow and
    mask), so the refinement residual is exactly 0.
    """
    W = make_weights(seed, base_width, t_plane)
    if kind not in ("zero_heads", "const_flow", "zero_refine"):
        raise ValueError(kind)
    if kind == "zero_refine":
        w, b = W["unet.head"]
        W["unet.head"] = (np.zeros_like(w), np.zeros_like(b))
        return W
    for name in ["vib0.convT2", "vib1.convT2", "vib2.convT2", "unet.head"]:
        w, b = W[name]
        W[name] = (np.zeros_like(w), np.zeros_like(b))
    if kind == "const_flow":
        w, b = W["vib0.convT2"]
        W["vib0.convT2"] = (w, np.array([0.5, 0.0, -0.5, 0.0, 0.0], np.float32))
    return W


def save_ffvw(
    path: str,
    weights: dict[str, tuple[np.ndarray, np.ndarray]],
    base_width: int,
    t_plane: bool,
    seed: int,
) -> None:
    shapes = layer_shapes(base_width, t_plane)
    chunks: list[np.ndarray] = []
    rows: list[str] = []
    off = 0
    for L in shapes:
        w, b = weights[L.name]
        if tuple(w.shape) != weight_shape(L) or tuple(b.shape) != (L.cout,):
            raise ValueError(f"bad shape for {L.name}")
        wf = np.ascontiguousarray(w, dtype="<f4").ravel()
        bf = np.ascontiguousarray(b, dtype="<f4").ravel()
        rows.append(
            f"layer {L.name} {L.kind} {L.cin} {L.cout} {L.stride} "
            f"{off} {wf.size} {off + wf.size} {bf.size}"
        )
        chunks += [wf, bf]
        off += wf.size + bf.size
    payload = np.concatenate(chunks).astype("<f4").tobytes()
    digest = hashlib.sha256(payload).hexdigest()
    head = [
        f"base_width {base_width}",
        f"t_plane {1 if t_plane else 0}",
        f"seed {seed}",
        f"n_floats {off}",
        f"sha256 {digest}",
        f"layers {len(shapes)}",
        *rows,
        "end",
    ]
    text = ("\n".join(head) + "\n").encode("ascii")
    start = (16 + len(text) + 63) // 64 * 64
    with open(path, "wb") as fh:
        fh.write(MAGIC + struct.pack("<III", VERSION, len(text), 0))
        fh.write(text)
        fh.write(b"\0" * (start - 16 - len(text)))
        fh.write(payload)


def write_weights_file(
    path: str,
    seed: int = 0,
    base_width: int = 32,
    t_plane: bool = True,
    kind: str | None = None,
) -> str:
    """Draw weights (random, or ``structured_weights(kind)``) and save them."""
    if kind is None:
        W = make_weights(seed, base_width, t_plane)
    else:
        W = structured_weights(kind, seed, base_width, t_plane)
    save_ffvw(path, W, base_width, t_plane, seed)
    return path


def param_count(base_width: int = 32, t_plane: bool = True) -> int:
    n = 0
    for L in layer_shapes(base_width, t_plane):
        s = weight_shape(L)
        n += s[0] * s[1] * s[2] * s[3] + L.cout
    return n
