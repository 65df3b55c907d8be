"""Seeded synthetic multi-view scenes.

Stand-ins for the paper's captured data (a 12-camera 1080p rig and Vimeo90K
triplets, neither of which is available here). Each camera image is a smooth
analytic colour texture seen through a smooth horizontal disparity field:

* texture ``T(x, y)``: ``S = sum_b a_b * c_b * exp(-((x-mx_b)^2 + (y-my_b)^2)
  / (2 s_b^2))`` per colour channel, ``T = 1 - exp(-S)`` in [0, 1). Each blob
  is evaluated where ``|x - mx_b| <= 5 s_b`` and ``|y - my_b| <= 5 s_b`` (a
  condition on the sample coordinate, so shifted copies stay exact);
* disparity ``D(x, y)``: a sum of 16 Gaussians, rescaled to span exactly
  ``[0, d_max]`` over the pixel grid;
* camera ``j``: ``C_j(x, y) = clip(T(x + j*D(x, y), y) + N(0, noise^2), 0, 1)``,
  the noise drawn by a torch generator on the target device, seeded from
  the scene seed (so it is made where it is used, with no host copy).

The small case uses a constant shift instead: the right view is the left
view moved by exactly 4 px (``X_r(x, y) = T(x + 4, y)``), no noise.

Images are returned planar ``[3, H, W]`` float32 (RGB in [0, 1]). Random
parameters come from ``numpy.random.default_rng(seed)``; the rendering runs in
float64 with torch on the requested device (CPU or GPU) and is the same
function of the drawn parameters on either.
"""
from __future__ import annotations

import numpy as np
import torch


def _texture_params(rng, n_blobs, sigma_range, H, W, margin):
    s = rng.uniform(sigma_range[0], sigma_range[1], n_blobs)
    mx = rng.uniform(-margin, W + margin, n_blobs)
    my = rng.uniform(-margin, H + margin, n_blobs)
    a = rng.uniform(0.5, 1.0, n_blobs)
    c = rng.uniform(0.0, 1.0, (n_blobs, 3))
    return {"s": s, "mx": mx, "my": my, "a": a, "c": c}


def _render_texture(p, xs, ys, x_lo_shift, device):
    """Evaluate T at sample coordinates ``(xs, ys)`` (float64 tensors [H, W]).

    ``x_lo_shift`` bounds ``xs - x_pixel`` from below and above as
    ``(lo, hi)`` so that each blob touches only a pixel window.
    """
    H, W = xs.shape
    S = torch.zeros((3, H, W), dtype=torch.float64, device=device)
    lo, hi = x_lo_shift
    for b in range(len(p["s"])):
        s = float(p["s"][b])
        mx = float(p["mx"][b])
        my = float(p["my"][b])
        r = 5.0 * s
        y0 = max(0, int(np.floor(my - r)))
        y1 = min(H, int(np.ceil(my + r)) + 1)
        # sample x = pixel x + shift, shift in [lo, hi]
        x0 = max(0, int(np.floor(mx - r - hi)))
        x1 = min(W, int(np.ceil(mx + r - lo)) + 1)
        if y0 >= y1 or x0 >= x1:
            continue
        sx = xs[y0:y1, x0:x1]
        sy = ys[y0:y1, x0:x1]
        dx = sx - mx
        dy = sy - my
        inside = (dx.abs() <= r) & (dy.abs() <= r)
        g = torch.exp(-(dx * dx + dy * dy) / (2.0 * s * s)) * inside
        amp = float(p["a"][b])
        for ch in range(3):
            S[ch, y0:y1, x0:x1] += (amp * float(p["c"][b, ch])) * g
    return 1.0 - torch.exp(-S)


def disparity_field(rng, H, W, d_max, device="cpu"):
    """Smooth disparity in [0, d_max] (float64 [H, W])."""
    k = 16
    a = rng.uniform(0.5, 1.0, k)
    mx = rng.uniform(0, W, k)
    my = rng.uniform(0, H, k)
    s = rng.uniform(0.1, 0.3, k) * min(H, W)
    ys = torch.arange(H, dtype=torch.float64, device=device)[:, None]
    xs = torch.arange(W, dtype=torch.float64, device=device)[None, :]
    G = torch.zeros((H, W), dtype=torch.float64, device=device)
    for i in range(k):
        G += float(a[i]) * torch.exp(
            -((xs - float(mx[i])) ** 2 + (ys - float(my[i])) ** 2) / (2.0 * float(s[i]) ** 2)
        )
    g0, g1 = G.min(), G.max()
    return d_max * (G - g0) / (g1 - g0)


def shifted_pair(seed: int = 1, H: int = 128, W: int = 128, n_blobs: int = 64,
                 sigma_range=(4.0, 16.0), shift: int = 4, device="cpu"):
    """Left/right views where ``right(x, y) = T(x + shift, y)`` exactly."""
    rng = np.random.default_rng(seed)
    margin = shift + 4.0 * sigma_range[1]
    p = _texture_params(rng, n_blobs, sigma_range, H, W, margin)
    ys = torch.arange(H, dtype=torch.float64, device=device)[:, None].expand(H, W)
    xs = torch.arange(W, dtype=torch.float64, device=device)[None, :].expand(H, W)
    left = _render_texture(p, xs, ys, (0.0, 0.0), device)
    right = _render_texture(p, xs + shift, ys, (float(shift), float(shift)), device)
    return left.float().contiguous(), right.float().contiguous()


def texture_at(seed: int, H: int, W: int, xs, ys, n_blobs: int = 64,
               sigma_range=(4.0, 16.0), shift: int = 4, device="cpu"):
    """T of ``shifted_pair(seed, ...)`` at arbitrary sample coordinates."""
    rng = np.random.default_rng(seed)
    margin = shift + 4.0 * sigma_range[1]
    p = _texture_params(rng, n_blobs, sigma_range, H, W, margin)
    xs = torch.as_tensor(xs, dtype=torch.float64, device=device)
    ys = torch.as_tensor(ys, dtype=torch.float64, device=device)
    lo = float((xs - torch.arange(xs.shape[1], dtype=torch.float64, device=device)[None]).min())
    hi = float((xs - torch.arange(xs.shape[1], dtype=torch.float64, device=device)[None]).max())
    return _render_texture(p, xs, ys, (lo, hi), device)


def camera_arc(seed: int, H: int, W: int, n_cams: int, n_blobs: int,
               sigma_range, d_max: float, noise: float = 0.01, device="cpu"):
    """``n_cams`` views of one scene, camera j at disparity ``j * D``.

    Returns float32 ``[n_cams, 3, H, W]`` on ``device``.
    """
    rng = np.random.default_rng(seed)
    margin = (n_cams - 1) * d_max + 4.0 * sigma_range[1]
    p = _texture_params(rng, n_blobs, sigma_range, H, W, margin)
    D = disparity_field(rng, H, W, d_max, device)
    ys = torch.arange(H, dtype=torch.float64, device=device)[:, None].expand(H, W)
    xs = torch.arange(W, dtype=torch.float64, device=device)[None, :].expand(H, W)
    out = torch.empty((n_cams, 3, H, W), dtype=torch.float32, device=device)
    gen = torch.Generator(device=device)
    gen.manual_seed(int(rng.integers(0, 2**62)))
    for j in range(n_cams):
        T = _render_texture(p, xs + j * D, ys, (0.0, j * d_max), device)
        if noise > 0:
            T = T + noise * torch.randn((3, H, W), generator=gen, dtype=torch.float64,
                                        device=device)
        out[j] = T.clamp(0.0, 1.0).float()
    return out


# Workload recipes (shapes and distributions of the paper's workloads; see
# the module docstring for why these stand in for its datasets).
def small_pair(device="cpu"):
    """3x128x128, 64 blobs (sigma 4..16 px), right = left shifted by 4 px."""
    return shifted_pair(seed=1, H=128, W=128, n_blobs=64, sigma_range=(4.0, 16.0),
                        shift=4, device=device)


def hd_arc(n_cams: int = 2, seed: int = 2, H: int = 1080, W: int = 1920, device="cpu"):
    """1080p arc: 1024 blobs (sigma 8..64 px), disparity 0..48 px, 1 % noise."""
    return camera_arc(seed, H, W, n_cams, 1024, (8.0, 64.0), 48.0, 0.01, device)


def uhd_arc(n_cams: int = 2, seed: int = 40, H: int = 2160, W: int = 3840, device="cpu"):
    """4K pairs: 4096 blobs (sigma 16..128 px), disparity 0..96 px, 1 % noise."""
    return camera_arc(seed, H, W, n_cams, 4096, (16.0, 128.0), 96.0, 0.01, device)


def random_pair(seed: int, H: int, W: int, d_max: float = 8.0, n_blobs: int | None = None,
                device="cpu"):
    """A generic two-camera pair at any size (used for ragged test sizes)."""
    if n_blobs is None:
        n_blobs = max(16, (H * W) // 256)
    smin = max(2.0, min(H, W) / 32)
    arc = camera_arc(seed, H, W, 2, n_blobs, (smin, 4 * smin), d_max, 0.01, device)
    return arc[0].contiguous(), arc[1].contiguous()
