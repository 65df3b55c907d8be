"""FP64 CPU oracle of the Laplacian-pyramid colour loss of the paper's
training objective (section 3.1, "Loss functions", Eq. 3) and of its
gradient with respect to the synthesised image.

TEST INFRASTRUCTURE ONLY: imported by the tests, never by the library, and
sharing no code with it.

Eq. 3 weighs the L1 distance between the i-th Laplacian-pyramid levels of
the synthesised view and of the ground truth by 2^(i-1), for i = 1..5. The
paper does not define the pyramid; the readings taken here:

* blur: the separable binomial filter [1, 4, 6, 4, 1] / 16 with mirror
  padding (the edge sample is not repeated), applied per channel;
* reduce: G^1 is the image, G^(i+1) the even-indexed samples of blur(G^i)
  (sizes ceil(n / 2));
* expand: zeros between the samples of G^(i+1) up to the size of G^i, then
  blur with 4x the filter (2x per axis), so a constant survives exactly;
* level i (1..5) is the band G^i - expand(G^(i+1)); the low-pass residual
  G^6 is not a term;
* ||.||_1 of a level is the mean absolute value over its elements (all
  channels), so every level counts as one average, weighted by 2^(i-1).

Mirror padding needs at least 3 samples per axis at level 5, hence
height and width >= 33.

Every level is linear in the image, so the loss of (x, y) is the loss of
(x - y, 0), and its gradient with respect to x is the adjoint pyramid applied
to the weighted signs of the levels.
"""
from __future__ import annotations

import numpy as np

KERNEL = np.array([1.0, 4.0, 6.0, 4.0, 1.0]) / 16.0
LEVELS = 5
MIN_SIZE = 33


def _mirror(i: int, n: int) -> int:
    """Index i reflected into [0, n) about the edge samples (no repeat)."""
    if i < 0:
        i = -i
    if i > n - 1:
        i = 2 * (n - 1) - i
    return i


def _blur_axis(x: np.ndarray, axis: int, gain: float = 1.0) -> np.ndarray:
    """Filter [1, 4, 6, 4, 1] / 16 (times gain) along one axis, mirror padded."""
    n = x.shape[axis]
    out = np.zeros_like(x)
    for j in range(n):
        acc = 0.0
        for k, c in enumerate(KERNEL):
            acc = acc + c * np.take(x, _mirror(j + k - 2, n), axis=axis)
        idx = [slice(None)] * x.ndim
        idx[axis] = j
        out[tuple(idx)] = gain * acc
    return out


def blur(x: np.ndarray, gain: float = 1.0) -> np.ndarray:
    """Separable binomial blur of a [C, H, W] image (gain per axis)."""
    return _blur_axis(_blur_axis(x, 1, gain), 2, gain)


def reduce(x: np.ndarray) -> np.ndarray:
    """G^(i+1) from G^i: blur, then keep the even rows and columns."""
    return blur(x)[:, ::2, ::2]


def expand(x: np.ndarray, h: int, w: int) -> np.ndarray:
    """Zeros inserted between samples up to h x w, then blur with gain 2 per
    axis (4 in all)."""
    up = np.zeros((x.shape[0], h, w))
    up[:, ::2, ::2] = x
    return blur(up, 2.0)


def laplacian_pyramid(x: np.ndarray, levels: int = LEVELS) -> list[np.ndarray]:
    """Band levels L^1..L^levels of a [C, H, W] image (G^i - expand(G^(i+1)))."""
    g = np.asarray(x, np.float64)
    if min(g.shape[1:]) < MIN_SIZE:
        raise ValueError(f"height and width must be >= {MIN_SIZE}")
    bands = []
    for _ in range(levels):
        nxt = reduce(g)
        bands.append(g - expand(nxt, g.shape[1], g.shape[2]))
        g = nxt
    return bands


def lap_loss(x: np.ndarray, gt: np.ndarray) -> float:
    """Eq. 3: sum over i = 1..5 of 2^(i-1) * mean |L^i(x) - L^i(gt)|."""
    lx = laplacian_pyramid(x)
    lg = laplacian_pyramid(gt)
    return float(sum(2.0 ** i * np.mean(np.abs(a - b)) for i, (a, b) in enumerate(zip(lx, lg))))


# ------------------------------------------------------------- adjoints
def _blur_axis_t(y: np.ndarray, axis: int, gain: float = 1.0) -> np.ndarray:
    """Adjoint of _blur_axis: every output sample's weighted inputs receive
    its value back (mirror-padded taps fold onto the samples they read)."""
    n = y.shape[axis]
    out = np.zeros_like(y)
    for j in range(n):
        yj = np.take(y, j, axis=axis)
        for k, c in enumerate(KERNEL):
            src = _mirror(j + k - 2, n)
            idx = [slice(None)] * y.ndim
            idx[axis] = src
            out[tuple(idx)] += gain * c * yj
    return out


def blur_t(y: np.ndarray, gain: float = 1.0) -> np.ndarray:
    return _blur_axis_t(_blur_axis_t(y, 2, gain), 1, gain)


def reduce_t(y: np.ndarray, h: int, w: int) -> np.ndarray:
    """Adjoint of reduce: zeros between samples up to h x w, then blur^T."""
    up = np.zeros((y.shape[0], h, w))
    up[:, ::2, ::2] = y
    return blur_t(up)


def expand_t(y: np.ndarray) -> np.ndarray:
    """Adjoint of expand: blur^T (gain 2 per axis), then the even samples."""
    return blur_t(y, 2.0)[:, ::2, ::2]


def lap_loss_grad(x: np.ndarray, gt: np.ndarray) -> np.ndarray:
    """d lap_loss / d x (sign(0) taken as 0): level i contributes
    2^(i-1) / N_i * sign(L^i(x) - L^i(gt)) through the adjoint of the map
    from the image to L^i."""
    d = np.asarray(x, np.float64) - np.asarray(gt, np.float64)
    bands = laplacian_pyramid(d)
    # sizes of G^1..G^6
    sizes = [d.shape[1:]]
    for _ in range(LEVELS):
        h, w = sizes[-1]
        sizes.append(((h + 1) // 2, (w + 1) // 2))
    # backward through the chain G^1 -> G^2 -> ... : the seed of level i
    # is s_i = w_i sign(L^i); L^i = G^i - expand(G^(i+1)) and
    # G^(i+1) = reduce(G^i), so the gradient reaching G^i is
    # s_i + reduce^T(grad of G^(i+1)) - reduce^T(expand^T(s_i)) ...
    # accumulated from the coarsest level down.
    grad_next = np.zeros((d.shape[0],) + sizes[LEVELS])  # d loss / d G^6
    for i in range(LEVELS - 1, -1, -1):
        h, w = sizes[i]
        s = (2.0 ** i / bands[i].size) * np.sign(bands[i])
        # d loss / d G^(i+1) gathers grad_next and -expand^T(s)
        g_next = grad_next - expand_t(s)
        grad_next = s + reduce_t(g_next, h, w)
    return grad_next
