"""Seeded synthetic grayscale images for the KAZE scale-space workloads.

The paper evaluates on natural photographs (8 sizes from 240x400 to 1920x1200,
6 images each, Sec. IV) that are not available.  These images stand in for
them: smooth structure at many scales (Gaussian blobs), hard edges that a
nonlinear diffusion should preserve (filled ellipses and rectangles), and a
small amount of sensor-like noise, clipped to [0, 1].

This module holds no arithmetic of the method itself.  Both the FP64 oracle
and the GPU harness draw their inputs from here, and nothing else is shared
between them.

Recipe (one ``numpy.random.default_rng(seed)`` PCG64 stream, drawn in this
order):

1. I = 0.5 everywhere.
2. ``n_blobs`` Gaussian blobs: centre ~ U[0,W) x U[0,H), width
   s ~ U[2, max(3, 0.04 min(W,H))], amplitude ~ U[-0.4, 0.4]; each adds
   amp * exp(-r^2 / (2 s^2)) inside a +-4s box.
3. ``n_shapes`` filled shapes painted in order: ellipse or rectangle with
   probability 1/2, centre uniform, half-extents ~ U[0.01, 0.08] min(W,H),
   angle ~ U[0, pi), grey value ~ U[0, 1]; pixels whose centre lies inside
   take that value.
4. Additive noise N(0, noise^2) on every pixel.
5. Clip to [0, 1]; return row-major float32 [H][W].
"""
from __future__ import annotations

import math

import numpy as np

__all__ = ["shape_counts", "kaze_image", "batch_sizes", "surrogate_params", "WORKLOADS"]

# (width, height, n_blobs, n_shapes) of the two reference workloads; other
# sizes scale the counts with the pixel count (never below the small case).
_SMALL = (320, 240, 40, 20)
_LARGE = (1920, 1200, 80, 60)


def shape_counts(W: int, H: int) -> tuple[int, int]:
    """Blob and shape counts for a W x H image of this generator."""
    if (W, H) == _SMALL[:2]:
        return _SMALL[2], _SMALL[3]
    if (W, H) == _LARGE[:2]:
        return _LARGE[2], _LARGE[3]
    scale = (W * H) / float(_LARGE[0] * _LARGE[1])
    return (max(_SMALL[2], int(round(_LARGE[2] * scale))),
            max(_SMALL[3], int(round(_LARGE[3] * scale))))


def kaze_image(W: int, H: int, seed: int, n_blobs: int | None = None,
               n_shapes: int | None = None, noise: float = 0.01) -> np.ndarray:
    """One synthetic image, float32 [H][W] in [0, 1] (recipe in the module doc)."""
    if W < 1 or H < 1:
        raise ValueError("image must be at least 1x1")
    nb_def, ns_def = shape_counts(W, H)
    n_blobs = nb_def if n_blobs is None else int(n_blobs)
    n_shapes = ns_def if n_shapes is None else int(n_shapes)
    rng = np.random.default_rng(seed)
    img = np.full((H, W), 0.5, dtype=np.float64)
    mn = float(min(W, H))

    for _ in range(n_blobs):
        cx = rng.uniform(0.0, W)
        cy = rng.uniform(0.0, H)
        s = rng.uniform(2.0, max(3.0, 0.04 * mn))
        amp = rng.uniform(-0.4, 0.4)
        x0, x1 = max(0, int(cx - 4 * s)), min(W, int(cx + 4 * s) + 1)
        y0, y1 = max(0, int(cy - 4 * s)), min(H, int(cy + 4 * s) + 1)
        if x0 >= x1 or y0 >= y1:
            continue
        xs = np.arange(x0, x1, dtype=np.float64) - cx
        ys = np.arange(y0, y1, dtype=np.float64) - cy
        r2 = ys[:, None] ** 2 + xs[None, :] ** 2
        img[y0:y1, x0:x1] += amp * np.exp(-r2 / (2.0 * s * s))

    for _ in range(n_shapes):
        ellipse = rng.random() < 0.5
        cx = rng.uniform(0.0, W)
        cy = rng.uniform(0.0, H)
        a = rng.uniform(0.01, 0.08) * mn
        b = rng.uniform(0.01, 0.08) * mn
        ang = rng.uniform(0.0, math.pi)
        val = rng.uniform(0.0, 1.0)
        rad = math.hypot(a, b)
        x0, x1 = max(0, int(cx - rad)), min(W, int(cx + rad) + 2)
        y0, y1 = max(0, int(cy - rad)), min(H, int(cy + rad) + 2)
        if x0 >= x1 or y0 >= y1:
            continue
        xs = np.arange(x0, x1, dtype=np.float64) - cx
        ys = np.arange(y0, y1, dtype=np.float64) - cy
        ca, sa = math.cos(ang), math.sin(ang)
        u = ca * xs[None, :] + sa * ys[:, None]
        v = -sa * xs[None, :] + ca * ys[:, None]
        if ellipse:
            inside = (u / a) ** 2 + (v / b) ** 2 <= 1.0
        else:
            inside = (np.abs(u) <= a) & (np.abs(v) <= b)
        img[y0:y1, x0:x1][inside] = val

    img += rng.normal(0.0, noise, size=img.shape)
    np.clip(img, 0.0, 1.0, out=img)
    return img.astype(np.float32)


def batch_sizes(n: int, seed: int, wmin: int, wmax: int, hmin: int, hmax: int
                ) -> list[tuple[int, int]]:
    """``n`` uneven (W, H) pairs, W ~ U{wmin..wmax}, H ~ U{hmin..hmax}."""
    rng = np.random.default_rng(seed)
    ws = rng.integers(wmin, wmax + 1, size=n)
    hs = rng.integers(hmin, hmax + 1, size=n)
    return [(int(w), int(h)) for w, h in zip(ws, hs)]


# Named workloads: (description, list of (W, H, seed)).
def _uneven_batch():
    return [(w, h, 3000 + j) for j, (w, h) in
            enumerate(batch_sizes(64, 3, 640, 1920, 480, 1200))]


WORKLOADS = {
    "kaze_320x240": lambda: [(320, 240, 1)],
    "kaze_1920x1200": lambda: [(1920, 1200, 2)],
    "kaze_batch64_uneven": _uneven_batch,
    "kaze_4k32_720p32": lambda: ([(3840, 2160, 5000 + j) for j in range(32)]
                                 + [(1280, 720, 5100 + j) for j in range(32)]),
    # eight images of the single-image size: a working set (levels and
    # responses, 2.4 GB) well above the 256 MB last-level cache
    "kaze_8x1920x1200": lambda: [(1920, 1200, 8000 + j) for j in range(8)],
}


def surrogate_params(seed: int, channels=(3, 32, 32, 32, 32, 32, 1),
                     last_scale: float = 0.1) -> np.ndarray:
    """Seeded initial parameters of a stack of 3x3 convolutions, flat float32:
    per layer the weights [co][ci][3][3] (He-normal, std sqrt(2 / (9 ci)))
    then the biases [co] (zero).  The last layer's weights are scaled by
    ``last_scale``."""
    rng = np.random.default_rng(seed)
    parts = []
    nl = len(channels) - 1
    for li, (ci, co) in enumerate(zip(channels[:-1], channels[1:])):
        W = rng.normal(0.0, math.sqrt(2.0 / (9 * ci)), size=(co, ci, 3, 3))
        if li == nl - 1:
            W *= last_scale
        parts += [W.ravel(), np.zeros(co)]
    return np.concatenate(parts).astype(np.float32)
