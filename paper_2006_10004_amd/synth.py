"""Seeded synthetic shape images: the inputs of the benchmarks and tests.

This module only draws inputs.  It holds none of the decomposition's
arithmetic, so both the HIP path and the CPU oracle can be fed from it.

Recipe (one numpy ``Generator(PCG64(seed))`` per image, draws in this order):
  1. for each shape, in order: kind, centre (cy, cx) ~ U[0,H) x U[0,W)
     (shapes may cross the border), size parameters, one contrast per channel;
  2. Gaussian noise N(0, sigma^2), i.i.d. per pixel and channel;
  3. clip to [0, 1], cast to float32.
Shapes are painted in draw order on a constant background: a pixel takes
background + the contrast of the last shape covering it (painter's order).
Membership is tested at integer pixel coordinates (i = row, j = column):
  disk       (i-cy)^2 + (j-cx)^2 <= r^2,             r ~ U[lo, hi]
  rectangle  |i-cy| <= hy and |j-cx| <= hx,          hy, hx ~ U[lo, hi]
  ellipse    rotated by theta ~ U[0, pi), semi-axes a, b ~ U[lo, hi]
These stand in for the natural-image datasets the paper measures on, which
are not available here: the shapes are the eigenfunction-like structures
(disks, ellipses) the paper itself tests on.
"""
from __future__ import annotations

import dataclasses

import numpy as np

DISK, RECT, ELLIPSE = 0, 1, 2


@dataclasses.dataclass(frozen=True)
class ShapeSpec:
    H: int
    W: int
    C: int = 1
    n_shapes: int = 5
    kinds: tuple = (DISK, RECT)
    size_lo: float = 4.0
    size_hi: float = 16.0
    contrast: float = 0.5
    sigma: float = 0.02
    background: float = 0.2


# Workload shapes (sizes, counts and distributions of the decomposition
# workloads; dt/K/iterations live with the callers).
SMALL_64 = ShapeSpec(64, 64, 1, 5, (DISK, RECT), 4, 16, 0.5, 0.02, 0.2)
IMAGE_512 = ShapeSpec(512, 512, 1, 40, (DISK, RECT, ELLIPSE), 3, 120, 0.6, 0.03, 0.5)


def serving_spec(side: int) -> ShapeSpec:
    """3-channel image for the mixed-size serving workload (side in 128..1024)."""
    hi = 120.0 * side / 512.0
    return ShapeSpec(side, side, 3, 40, (DISK, RECT, ELLIPSE), 3, max(hi, 8.0), 0.6, 0.03, 0.5)


def megapixel_spec(side: int) -> ShapeSpec:
    """3-channel megapixel image (1024 or 2048 side), 300 shapes."""
    return ShapeSpec(side, side, 3, 300, (DISK, RECT, ELLIPSE), 3, 400, 0.6, 0.02, 0.5)


def shapes_image(spec: ShapeSpec, seed: int) -> np.ndarray:
    """Draw one C x H x W float32 image in [0, 1] following the recipe above."""
    rng = np.random.Generator(np.random.PCG64(seed))
    H, W, C = spec.H, spec.W, spec.C
    img = np.full((C, H, W), spec.background, dtype=np.float64)
    for _ in range(spec.n_shapes):
        kind = spec.kinds[int(rng.integers(len(spec.kinds)))]
        cy = rng.uniform(0, H)
        cx = rng.uniform(0, W)
        if kind == DISK:
            r = rng.uniform(spec.size_lo, spec.size_hi)
            ext = (r, r)
        elif kind == RECT:
            hy = rng.uniform(spec.size_lo, spec.size_hi)
            hx = rng.uniform(spec.size_lo, spec.size_hi)
            ext = (hy, hx)
        else:
            a = rng.uniform(spec.size_lo, spec.size_hi)
            b = rng.uniform(spec.size_lo, spec.size_hi)
            th = rng.uniform(0, np.pi)
            ext = (max(a, b), max(a, b))
        # the shape lies within its half-extents of the centre: evaluate its
        # mask on that box (with a 2-pixel margin) only
        i0, i1 = max(0, int(np.floor(cy - ext[0])) - 2), min(H, int(np.ceil(cy + ext[0])) + 3)
        j0, j1 = max(0, int(np.floor(cx - ext[1])) - 2), min(W, int(np.ceil(cx + ext[1])) + 3)
        ii = np.arange(i0, i1, dtype=np.float64)[:, None]
        jj = np.arange(j0, j1, dtype=np.float64)[None, :]
        if kind == DISK:
            mask = (ii - cy) ** 2 + (jj - cx) ** 2 <= r * r
        elif kind == RECT:
            mask = (np.abs(ii - cy) <= hy) & (np.abs(jj - cx) <= hx)
        else:
            ct, st = np.cos(th), np.sin(th)
            y = ii - cy
            x = jj - cx
            xr = ct * x + st * y
            yr = -st * x + ct * y
            mask = (xr / a) ** 2 + (yr / b) ** 2 <= 1.0
        contrasts = rng.uniform(-spec.contrast, spec.contrast, size=C)
        for c in range(C):
            img[c, i0:i1, j0:j1][mask] = spec.background + contrasts[c]
    if spec.sigma > 0:
        img += rng.normal(0.0, spec.sigma, size=img.shape)
    np.clip(img, 0.0, 1.0, out=img)
    return img.astype(np.float32)


def disk_image(H: int, W: int, cy: float, cx: float, r: float, contrast: float,
               background: float = 0.0) -> np.ndarray:
    """Noise-free H x W float32 indicator of one disk (an eigenfunction shape)."""
    ii = np.arange(H, dtype=np.float64)[:, None]
    jj = np.arange(W, dtype=np.float64)[None, :]
    img = np.full((H, W), background, dtype=np.float64)
    img[(ii - cy) ** 2 + (jj - cx) ** 2 <= r * r] += contrast
    return img.astype(np.float32)


def step_image(H: int, a: int, b: int, c: float) -> np.ndarray:
    """H x (a+b) float32 image: the left a columns at c, the right b at 0."""
    img = np.zeros((H, a + b), dtype=np.float32)
    img[:, :a] = c
    return img


def plateau_image(H: int, levels, lengths) -> np.ndarray:
    """H x sum(lengths) float32 image constant along columns: a 1-D signal of
    plateaus (levels[m] repeated lengths[m] times) copied to every row."""
    row = np.concatenate([np.full(n, v, dtype=np.float64) for v, n in zip(levels, lengths)])
    return np.repeat(row[None, :], H, axis=0).astype(np.float32)
