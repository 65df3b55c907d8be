"""FP64 CPU oracle of the multi-view cluster frame (the paper's Multiview
Organizer, section 3.2 "Streaming Strategy" and the supplement's dense-view
paragraph: a camera's high-resolution real view stitched with its
neighbouring interpolated views, downscaled, 16 per side for 33 views).

TEST INFRASTRUCTURE ONLY: imported by the tests and the benchmark's
CPU-baseline leg, never by the product path.

Readings (the paper gives no tile geometry):

* each side holds g*g views (g = 4 for 16 per side), each downscaled by g in
  both directions with a g x g box mean (area average), so a side's tiles
  fill exactly one H x W block, placed in raster order (view 0 top-left);
* the frame is [left block | real view | right block], 3 x H x 3W;
* left-side views are ordered from the far neighbour to the camera,
  right-side views from the camera outwards (as they lie along the arc).
"""
from __future__ import annotations

import numpy as np


def box_down(x, g):
    """g x g box mean of a [C, H, W] image (H, W multiples of g)."""
    x = np.asarray(x, dtype=np.float64)
    c, h, w = x.shape
    if h % g or w % g:
        raise ValueError("size must be a multiple of the downscale factor")
    return x.reshape(c, h // g, g, w // g, g).mean(axis=(2, 4))


def stitch_cluster(hr, left, right):
    """``hr``: [3, H, W]; ``left``, ``right``: lists of g*g views [3, H, W].

    Returns the cluster frame [3, H, 3W] float64."""
    hr = np.asarray(hr, dtype=np.float64)
    n = len(left)
    g = int(round(n ** 0.5))
    if g * g != n or len(right) != n or n == 0:
        raise ValueError("each side needs the same perfect-square number of views")
    c, H, W = hr.shape
    th, tw = H // g, W // g
    out = np.zeros((c, H, 3 * W))
    out[:, :, W:2 * W] = hr
    for side, views in ((0, left), (2, right)):
        for k, v in enumerate(views):
            r, q = divmod(k, g)
            out[:, r * th:(r + 1) * th, side * W + q * tw:side * W + (q + 1) * tw] = box_down(v, g)
    return out
