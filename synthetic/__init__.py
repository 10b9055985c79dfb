"""Seeded synthetic inputs for the blob-detection filter bank.

Shared by the tests, the smoke check and the benchmark.  This module holds no
filter arithmetic at all (no design, blur, high-pass or detection code): it
only draws images and lists workload parameters, so that the oracle and the
HIP path can be fed identical inputs without sharing any of the method.

The paper's aerial imagery is not available; these frames stand in for it:
smooth backgrounds, shot noise and bright/dark blobs of many sizes.  All
generators use numpy's PCG64 (``default_rng(seed)``).
"""

from __future__ import annotations

import math

import numpy as np


def geometric_scales(sigma_min: float, sigma_max: float, count: int) -> list:
    """sigma_i = sigma_min (sigma_max / sigma_min)^(i / (count - 1)), endpoints
    included."""
    if count == 1:
        return [float(sigma_min)]
    return [float(sigma_min * (sigma_max / sigma_min) ** (i / (count - 1))) for i in range(count)]


def _gaussian_blob(img: np.ndarray, cy: float, cx: float, r: float, amp: float, reach: float = 4.0):
    H, W = img.shape
    y0, y1 = max(0, int(cy - reach * r)), min(H, int(cy + reach * r) + 2)
    x0, x1 = max(0, int(cx - reach * r)), min(W, int(cx + reach * r) + 2)
    if y0 >= y1 or x0 >= x1:
        return
    yy = np.arange(y0, y1)[:, None] - cy
    xx = np.arange(x0, x1)[None, :] - cx
    img[y0:y1, x0:x1] += amp * np.exp(-(yy * yy + xx * xx) / (2.0 * r * r))


def _disk_blob(img: np.ndarray, cy: float, cx: float, r: float, amp: float):
    H, W = img.shape
    y0, y1 = max(0, int(cy - r) - 1), min(H, int(cy + r) + 2)
    x0, x1 = max(0, int(cx - r) - 1), min(W, int(cx + r) + 2)
    if y0 >= y1 or x0 >= x1:
        return
    yy = np.arange(y0, y1)[:, None] - cy
    xx = np.arange(x0, x1)[None, :] - cx
    img[y0:y1, x0:x1] += amp * ((yy * yy + xx * xx) <= r * r)


def tiny_frame(seed: int = 0, size: int = 256, nblobs: int = 5, noise: bool = True) -> np.ndarray:
    """256 x 256 float32 test image: uniform [0, 1) noise plus `nblobs`
    Gaussian blobs A exp(-d^2 / 2 r^2), r ~ U[3, 12], A ~ U[0.5, 2], centres
    ~ U[r, size - r].  With noise=False the noise is replaced by
    0.5 + a gentle quadratic ramp (the blob draws are unchanged)."""
    rng = np.random.default_rng(seed)
    noise_field = rng.random((size, size))
    if noise:
        img = noise_field.astype(np.float64)
    else:
        v = np.linspace(-1.0, 1.0, size)[:, None]
        u = np.linspace(-1.0, 1.0, size)[None, :]
        img = 0.5 + 0.05 * (u * u + 0.5 * u * v - 0.3 * v * v) + 0.0 * noise_field
    for _ in range(nblobs):
        r = rng.uniform(3.0, 12.0)
        amp = rng.uniform(0.5, 2.0)
        cy = rng.uniform(r, size - r)
        cx = rng.uniform(r, size - r)
        _gaussian_blob(img, cy, cx, r, amp)
    return img.astype(np.float32)


def aerial_frame(H: int, W: int, seed: int, nblobs: int | None = None,
                 max_value: int = 4095) -> np.ndarray:
    """Aerial-like uint16 frame with 12-bit values.

    Background 1200 + 400 (a1 u + a2 v) + 300 (a3 u^2 + a4 u v + a5 v^2),
    u, v in [-1, 1] along x, y and a_i ~ U[-1, 1]; `nblobs` blobs (default
    200 per 2048^2 pixels), each a disk or a Gaussian (p = 1/2), bright or
    dark (p = 1/2), radius log-uniform on [2, 64], |A| ~ U[200, 1500] DN,
    centre uniform over the frame; lambda = clip(background + blobs, 0, 4095)
    and the stored value is clip(Poisson(lambda), 0, 4095)."""
    rng = np.random.default_rng(seed)
    if nblobs is None:
        nblobs = max(1, int(round(200 * H * W / (2048 * 2048))))
    a = rng.uniform(-1.0, 1.0, 5)
    u = np.linspace(-1.0, 1.0, W)[None, :]
    v = np.linspace(-1.0, 1.0, H)[:, None]
    img = 1200.0 + 400.0 * (a[0] * u + a[1] * v) + 300.0 * (a[2] * u * u + a[3] * u * v + a[4] * v * v)
    img = np.broadcast_to(img, (H, W)).copy()
    for _ in range(nblobs):
        disk = rng.random() < 0.5
        sign = 1.0 if rng.random() < 0.5 else -1.0
        r = math.exp(rng.uniform(math.log(2.0), math.log(64.0)))
        amp = sign * rng.uniform(200.0, 1500.0)
        cy = rng.uniform(0.0, H)
        cx = rng.uniform(0.0, W)
        if disk:
            _disk_blob(img, cy, cx, r, amp)
        else:
            _gaussian_blob(img, cy, cx, r, amp)
    lam = np.clip(img, 0.0, float(max_value))
    counts = rng.poisson(lam)
    return np.clip(counts, 0, max_value).astype(np.uint16)


# --------------------------------------------------------------------------
# Workloads
# --------------------------------------------------------------------------

TINY = dict(name="tiny-256-f32-iir2", H=256, W=256, sigmas=[4.0], iir_order=2,
            tau=0.5, border=1, seed=0)

FULL_FRAME = dict(name="frame-2048-u16-8scales", H=2048, W=2048,
                  sigmas=geometric_scales(2.0, 64.0, 8), iir_order=3, fir_rule="3sigma",
                  tau=40.0, border=1, seed=1)

BATCH_SIZES = [(512, 512), (1080, 1920), (3072, 4096), (2048, 2048)]
BATCH = dict(name="batch-64-frames-12scales", sigmas=geometric_scales(1.5, 96.0, 12),
             iir_order=3, tau=40.0, border=1)

PRECISION = dict(name="frame-8192-f16-bf16", H=8192, W=8192, seed=3, nblobs=3200,
                 fir_lengths=[33, 65, 129, 257], iir_order=3)

DIFFERENTIATION = dict(name="batch-16x1024-f32-4scales", H=1024, W=1024, frames=16,
                       sigmas=[3.0, 6.0, 12.0, 24.0], nblobs=50)


def batch_frames(count: int = 64, seed: int = 2):
    """64 frames, 16 of each size in BATCH_SIZES, in the order of
    default_rng(seed).permutation; frame f uses aerial_frame(seed=1000 + f)
    with 200 blobs per 2048^2 pixels.  Returns a list of (H, W, seed)."""
    kinds = [BATCH_SIZES[i % 4] for i in range(count)]
    order = np.random.default_rng(seed).permutation(count)
    return [(kinds[o][0], kinds[o][1], 1000 + f) for f, o in enumerate(order)]


def normalised_frame(H: int, W: int, seed: int, nblobs: int | None = None) -> np.ndarray:
    """aerial_frame / 4095 as float64 in [0, 1]."""
    return aerial_frame(H, W, seed, nblobs).astype(np.float64) / 4095.0


# The test pattern of the paper's Hessian figures (Section 5, Figs 6 and 7):
# solid black ellipses on a white background, one column per semi-major axis
# (4, 8, 16, 32, 64 px, left to right) and one row per orientation of the
# major axis (0 to 45 degrees in equal steps, top to bottom).  The figures do
# not give the cell sizes, the number of orientations or the rasterisation;
# here every cell is 4 a wide and 256 px tall, there are 5 orientations, and a
# pixel's value is its uncovered area fraction from 4 x 4 sub-samples.
ELLIPSE_AXES = (4, 8, 16, 32, 64)
ELLIPSE_ANGLES = (0.0, 11.25, 22.5, 33.75, 45.0)


def ellipse_pattern(aspect: float = 2.0, axes=ELLIPSE_AXES, angles=ELLIPSE_ANGLES, row_height: int = 256,
                    supersample: int = 4):
    """Returns (image float64 [H, W] in [0, 1], list of (cy, cx, a, b, angle_deg)).
    Semi-minor axis b = a / aspect."""
    widths = [4 * a for a in axes]
    H, W = row_height * len(angles), sum(widths)
    img = np.ones((H, W))
    ss = supersample
    offs = (np.arange(ss) + 0.5) / ss - 0.5
    items = []
    for i, ang in enumerate(angles):
        cy = float(i * row_height + row_height // 2)     # centres on pixel centres
        x0 = 0
        for a, w in zip(axes, widths):
            cx = float(x0 + w // 2)
            b = a / aspect
            t = math.radians(ang)
            c, s = math.cos(t), math.sin(t)
            ry = int(math.ceil(a)) + 2
            ys = np.arange(int(cy) - ry, int(cy) + ry + 2)
            xs = np.arange(int(cx) - ry, int(cx) + ry + 2)
            cover = np.zeros((len(ys), len(xs)))
            for dy in offs:
                for dx in offs:
                    yy = ys[:, None] + dy - cy
                    xx = xs[None, :] + dx - cx
                    u = xx * c + yy * s       # along the major axis
                    v = -xx * s + yy * c
                    cover += (u * u) / (a * a) + (v * v) / (b * b) <= 1.0
            img[ys[0]:ys[-1] + 1, xs[0]:xs[-1] + 1] -= cover / (ss * ss)
            items.append((cy, cx, float(a), float(b), ang))
            x0 += w
    return img, items
