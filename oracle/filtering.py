"""Filter application -- oracle side (test infrastructure only; see package header).

All arithmetic is float64.  Images are row-major arrays [H, W]: n runs left to
right along x (axis 1) and top to bottom along y (axis 0), origin top-left
(Appendix, Eqs A7-A8).  Separable 2-D filtering applies the 1-D filter along
x first, then along y (Sections 2 and 5).

Boundary handling:
  "replicate" -- edge pixels are held constant out to +-infinity.  For the
                 recursions this is the steady-state initialisation of Eq A32
                 (the internal states equal their steady-state response to a
                 step of the edge value); for the FIR and the high-pass stage it
                 is the same clamp-to-edge extension.
  "zero"      -- zero padding, the paper's FIR start-up (Section 5) and the
                 zero-state start of a recursion.
"""

from __future__ import annotations

import numpy as np

from .design import IIRCoefficients

BOUNDARIES = ("replicate", "zero")


def iir_1d(x: np.ndarray, coef: IIRCoefficients, boundary: str = "replicate") -> np.ndarray:
    """Three-term non-causal DE along the LAST axis, vectorised over the others.

        y+(n) = sum_m bp[m] x(n-m) - sum_m ap[m] y+(n-m),  n = 0 .. N-1   (A10a)
        y-(n) = sum_m bm[m] x(n+m) - sum_m am[m] y-(n+m),  n = N-1 .. 0   (A10b)
        y(n)  = y+(n) + y-(n) + b0 x(n)                                    (A6, A10c)

    Initial conditions (Eq A32, read semantically): for "replicate" the input
    before the first sample is x(0) forever, so the forward recursion's past
    outputs sit at the steady-state value x(0) B+(1)/A+(1); symmetrically at
    the right end with x(N-1) and B-(1)/A-(1).  For "zero" all past inputs and
    outputs are 0."""
    if boundary not in BOUNDARIES:
        raise ValueError(boundary)
    x = np.asarray(x, dtype=np.float64)
    K = coef.order
    N = x.shape[-1]
    bp, ap, bm, am = coef.bp, coef.ap, coef.bm, coef.am
    y_plus = np.empty_like(x)
    y_minus = np.empty_like(x)

    # forward (causal) part, left-to-right / top-to-bottom
    if boundary == "replicate":
        g_plus = sum(bp[1:]) / sum(ap)          # B+(1)/A+(1), steady-state gain
        x_past = [x[..., 0]] * K                # x(n-1), .., x(n-K)
        y_past = [x[..., 0] * g_plus] * K       # y+(n-1), .., y+(n-K)
    else:
        x_past = [np.zeros(x.shape[:-1])] * K
        y_past = [np.zeros(x.shape[:-1])] * K
    for n in range(N):
        acc = np.zeros(x.shape[:-1])
        for m in range(1, K + 1):
            acc = acc + bp[m] * x_past[m - 1] - ap[m] * y_past[m - 1]
        y_plus[..., n] = acc
        x_past = [x[..., n]] + x_past[:-1]
        y_past = [acc] + y_past[:-1]

    # backward (anti-causal) part, right-to-left / bottom-to-top
    if boundary == "replicate":
        g_minus = sum(bm[1:]) / sum(am)
        x_next = [x[..., N - 1]] * K            # x(n+1), .., x(n+K)
        y_next = [x[..., N - 1] * g_minus] * K
    else:
        x_next = [np.zeros(x.shape[:-1])] * K
        y_next = [np.zeros(x.shape[:-1])] * K
    for n in range(N - 1, -1, -1):
        acc = np.zeros(x.shape[:-1])
        for m in range(1, K + 1):
            acc = acc + bm[m] * x_next[m - 1] - am[m] * y_next[m - 1]
        y_minus[..., n] = acc
        x_next = [x[..., n]] + x_next[:-1]
        y_next = [acc] + y_next[:-1]

    return y_plus + y_minus + coef.b0 * x


def _extend(x: np.ndarray, n_left: int, n_right: int, boundary: str) -> np.ndarray:
    """Extend the last axis by n_left / n_right samples (clamp or zeros)."""
    pad = [(0, 0)] * (x.ndim - 1) + [(n_left, n_right)]
    if boundary == "replicate":
        return np.pad(x, pad, mode="edge")
    if boundary == "zero":
        return np.pad(x, pad, mode="constant")
    raise ValueError(boundary)


def fir_1d(x: np.ndarray, taps: np.ndarray, boundary: str = "replicate") -> np.ndarray:
    """Non-recursive FIR along the LAST axis, Eq A5:
        y(n) = sum_{m=-K..K} h(m) x(n-m),   taps[K + m] = h(m)."""
    x = np.asarray(x, dtype=np.float64)
    taps = np.asarray(taps, dtype=np.float64)
    K = (len(taps) - 1) // 2
    N = x.shape[-1]
    xe = _extend(x, K, K, boundary)          # xe[..., K + j] = x_ext(j)
    y = np.zeros_like(x)
    for m in range(-K, K + 1):
        y += taps[K + m] * xe[..., K - m: K - m + N]
    return y


def fir_matrix(taps: np.ndarray, N: int, boundary: str = "replicate") -> np.ndarray:
    """The N x N matrix of the FIR of Eq A5 on a length-N signal with its
    extension folded in:  (T x)(n) = sum_{m=-K..K} h(m) x_ext(n - m), where
    x_ext(j) = x(clamp(j)) ("replicate") or 0 outside [0, N) ("zero"), so
    T[n, j] = sum of h(m) over the m with ext(n - m) = j."""
    taps = np.asarray(taps, dtype=np.float64)
    K = (len(taps) - 1) // 2
    T = np.zeros((N, N))
    n = np.arange(N)
    for m in range(-K, K + 1):
        j = n - m
        if boundary == "replicate":
            T[n, np.clip(j, 0, N - 1)] += taps[K + m]   # one entry per row n: no repeated index
        elif boundary == "zero":
            ok = (j >= 0) & (j < N)
            T[n[ok], j[ok]] += taps[K + m]
        else:
            raise ValueError(boundary)
    return T


def blur_2d_matrix(image: np.ndarray, taps: np.ndarray, boundary: str = "replicate") -> np.ndarray:
    """The separable FIR blur of blur_2d as two matrix products,
    B = T_H X T_W^T (the x filter acts on the rows of X, the y filter on the
    columns); the same linear map, summed in another order.  For full-size
    frames, where the shifted sums of fir_1d take minutes."""
    X = np.asarray(image, dtype=np.float64)
    H, W = X.shape
    return fir_matrix(taps, H, boundary) @ (X @ fir_matrix(taps, W, boundary).T)


def blur_2d_matrix_adjoint(G: np.ndarray, taps: np.ndarray, boundary: str = "replicate") -> np.ndarray:
    """The transpose of the separable FIR blur of blur_2d_matrix applied to a
    plane G:  X_bar = T_H^T G T_W, by definition of the transpose of
    B = T_H X T_W^T.  With the replicate extension the transposed matrices
    carry the folded tails (the columns of T for j = 0 and N - 1 collect every
    tap whose source position was clamped there)."""
    G = np.asarray(G, dtype=np.float64)
    H, W = G.shape
    return fir_matrix(taps, H, boundary).T @ (G @ fir_matrix(taps, W, boundary))


def apply_1d(x: np.ndarray, filt, boundary: str, axis: int) -> np.ndarray:
    """Apply an IIR (IIRCoefficients) or FIR (tap array) blur along `axis`."""
    xm = np.moveaxis(np.asarray(x, dtype=np.float64), axis, -1)
    if isinstance(filt, IIRCoefficients):
        ym = iir_1d(xm, filt, boundary)
    else:
        ym = fir_1d(xm, filt, boundary)
    return np.moveaxis(ym, -1, axis)


def blur_2d(image: np.ndarray, filt, boundary: str = "replicate") -> np.ndarray:
    """Separable 2-D blur: x (along rows, axis -1) first, then y (axis -2)
    (Sections 2 and 5).  Leading axes are batch axes."""
    rows = apply_1d(image, filt, boundary, axis=-1)
    return apply_1d(rows, filt, boundary, axis=-2)


def blur_bank(image: np.ndarray, filters, boundary: str = "replicate") -> np.ndarray:
    """One blur plane per scale: returns [S, H, W] float64."""
    return np.stack([blur_2d(image, f, boundary) for f in filters])


def brute_force_2d(image: np.ndarray, h: np.ndarray, boundary: str = "replicate") -> np.ndarray:
    """Direct 2-D convolution with the separable kernel h(a) h(b) over the 2-D
    extended image (clamp for "replicate", zeros for "zero"):

        B(i, j) = sum_{a, b = -R..R} h(a) h(b) X_ext(i - a, j - b),   h[R + a] = h(a).

    For an IIR, h is its impulse response truncated where the tail is below
    float64 resolution.  Used on tiny images only: every output pixel is a
    full (2R+1)^2 sum, no separability is used."""
    X = np.asarray(image, dtype=np.float64)
    H, W = X.shape
    h = np.asarray(h, dtype=np.float64)
    R = (len(h) - 1) // 2
    kernel = np.outer(h, h)                   # kernel[R + a, R + b] = h(a) h(b)
    out = np.empty((H, W))
    ii = np.arange(-R, R + 1)
    for i in range(H):
        rows = i - ii                          # i - a for a = -R..R
        for j in range(W):
            cols = j - ii
            if boundary == "replicate":
                patch = X[np.clip(rows, 0, H - 1)[:, None], np.clip(cols, 0, W - 1)[None, :]]
            else:
                rv = (rows >= 0) & (rows < H)
                cv = (cols >= 0) & (cols < W)
                patch = np.zeros((2 * R + 1, 2 * R + 1))
                patch[np.ix_(rv, cv)] = X[np.ix_(rows[rv], cols[cv])]
            out[i, j] = np.sum(kernel * patch)
    return out


def impulse_response_by_recursion(coef: IIRCoefficients, half_length: int) -> np.ndarray:
    """h(m), m = -R..R, obtained as the output of the DE for a unit impulse at
    the centre of a zero-initialised signal of length 2R+1 (Appendix: the IR of
    an IIR is the DE's response to an impulse, run until it has decayed)."""
    R = half_length
    x = np.zeros(2 * R + 1)
    x[R] = 1.0
    y = iir_1d(x, coef, boundary="zero")
    # y(n) = h(n - R), so h(m) = y[R + m]; the IR index runs opposite to n, but
    # the blur is symmetric so the two orientations coincide.
    return y
