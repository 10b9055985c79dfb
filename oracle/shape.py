"""High-pass stage and blob detection -- oracle side (test infrastructure only).

* hpf: the interpolating central differences of Eq 8 / Table I, applied to a
  blur plane with clamp-to-edge extension (the paper does not state the
  high-pass boundary; replicate is the reading used throughout).
* laplacian: the scale-normalised Laplacian sigma^2 (D20 + D02) built from the
  d = 2 taps [1, -2, 1] along x and along y (Section 5 high-pass stage).
* detect_extrema: multi-scale strict local extrema of the normalised Laplacian
  (3 x 3 neighbourhood in space times the adjacent scales), thresholded; the
  list is ordered by (scale, y, x).  This detector is not the paper's (the
  paper thresholds each scale's Hessian determinant on its own); it is the
  multi-scale rule this project is specified with.
* detect_hessian: the paper's detector, Eqs 26-27 with Thresholds #1 and #2.
"""

from __future__ import annotations

import numpy as np

from .design import hpf_taps


def hpf_1d(x: np.ndarray, d: int, axis: int) -> np.ndarray:
    """y(n) = sum_m h_d(m) x(n-m) along `axis`, h_d from Eq 8 (Table I),
    clamp-to-edge extension."""
    taps = hpf_taps(d)
    xm = np.moveaxis(np.asarray(x, dtype=np.float64), axis, -1)
    N = xm.shape[-1]
    n = np.arange(N)
    y = np.zeros_like(xm)
    for m, hm in taps.items():
        y += hm * xm[..., np.clip(n - m, 0, N - 1)]
    return np.moveaxis(y, -1, axis)


def derivative(B: np.ndarray, dx: int, dy: int) -> np.ndarray:
    """D_{dx,dy}: d = dx taps along x (axis -1), then d = dy along y (axis -2)."""
    return hpf_1d(hpf_1d(B, dx, axis=-1), dy, axis=-2)


def laplacian(B: np.ndarray, sigma: float) -> np.ndarray:
    """V = sigma^2 (D20 + D02) of one blur plane [H, W]."""
    return sigma * sigma * (derivative(B, 2, 0) + derivative(B, 0, 2))


def laplacian_bank(Bs: np.ndarray, sigmas) -> np.ndarray:
    return np.stack([laplacian(Bs[s], sigmas[s]) for s in range(len(sigmas))])


BLOB_DTYPE = np.dtype([("y", np.int32), ("x", np.int32), ("scale", np.int32),
                       ("polarity", np.int32), ("value", np.float64)])


def detect_extrema(V: np.ndarray, tau: float, border: int = 1) -> np.ndarray:
    """Strict multi-scale extrema of V [S, H, W].

    A pixel (s, y, x) with border <= y < H - border and border <= x < W - border
    is reported when, over every neighbour (s + ds, y + dy, x + dx),
    ds, dy, dx in {-1, 0, 1}, not all zero, that lies inside the [S, H, W]
    volume:
      * V < every neighbour and V <= -tau: a bright blob, polarity +1;
      * V > every neighbour and V >= tau:  a dark blob,   polarity -1.
    Ties are never extrema.  Returns a structured array ordered by (s, y, x)."""
    V = np.asarray(V, dtype=np.float64)
    S, H, W = V.shape
    lo_nb = np.full(V.shape, np.inf)    # min over neighbours
    hi_nb = np.full(V.shape, -np.inf)   # max over neighbours
    for ds in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                if ds == 0 and dy == 0 and dx == 0:
                    continue
                shifted = np.full((S, H, W), np.nan)
                s0, s1 = max(0, -ds), min(S, S - ds)
                y0, y1 = max(0, -dy), min(H, H - dy)
                x0, x1 = max(0, -dx), min(W, W - dx)
                # shifted[s, y, x] = V[s + ds, y + dy, x + dx] where that exists
                shifted[s0:s1, y0:y1, x0:x1] = V[s0 + ds:s1 + ds, y0 + dy:y1 + dy, x0 + dx:x1 + dx]
                valid = ~np.isnan(shifted)
                lo_nb = np.where(valid, np.minimum(lo_nb, shifted), lo_nb)
                hi_nb = np.where(valid, np.maximum(hi_nb, shifted), hi_nb)
    inside = np.zeros(V.shape, dtype=bool)
    if H - 2 * border > 0 and W - 2 * border > 0:
        inside[:, border:H - border, border:W - border] = True
    bright = inside & (V < lo_nb) & (V <= -tau)
    dark = inside & (V > hi_nb) & (V >= tau)
    out = []
    for s in range(S):
        ys, xs = np.nonzero(bright[s] | dark[s])
        for y, x in zip(ys, xs):   # np.nonzero is row-major: ordered by (y, x)
            out.append((y, x, s, 1 if bright[s, y, x] else -1, V[s, y, x]))
    return np.array(out, dtype=BLOB_DTYPE)


def detect_hessian(B: np.ndarray, sigma: float, t1: float, t2: float | None,
                   border: int = 1):
    """The paper's blob detector on one blur plane (Section 5):
        H = [[D20, D11], [D11, D02]]                           (Eq 26)
        detect when sigma^4 |H| > T1 (Threshold #1) and, if T2 is given,
        sqrt(dx^2 + dy^2) < T2 (Threshold #2) with
        dx = (D01 D11 - D02 D10) / |H|,  dy = (D10 D11 - D20 D01) / |H|  (Eq 27).
    Returns (mask [H, W] bool, normalised determinant, dx, dy)."""
    D20 = derivative(B, 2, 0)
    D02 = derivative(B, 0, 2)
    D11 = derivative(B, 1, 1)
    D10 = derivative(B, 1, 0)
    D01 = derivative(B, 0, 1)
    det = D20 * D02 - D11 * D11
    with np.errstate(divide="ignore", invalid="ignore"):
        dx = (D01 * D11 - D02 * D10) / det
        dy = (D10 * D11 - D20 * D01) / det
    ndet = sigma ** 4 * det
    mask = ndet > t1
    if t2 is not None:
        mask &= np.sqrt(dx * dx + dy * dy) < t2
    Hh, Ww = B.shape
    inside = np.zeros_like(mask)
    inside[border:Hh - border, border:Ww - border] = True
    return mask & inside, ndet, dx, dy
