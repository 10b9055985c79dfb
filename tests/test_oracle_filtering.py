"""Pins of the oracle's filtering and shape-analysis functions.  CPU only."""

import math

import numpy as np
import pytest

import synthetic as syn
from oracle import design, filtering, shape


def iir(K, sigma):
    return design.repeated_pole(K, sigma)


# ------------------------------------------------------------ boundaries

@pytest.mark.parametrize("K,sigma", [(2, 1.5), (2, 4.0), (3, 2.0), (3, 24.0), (3, 96.0)])
def test_constant_image_is_preserved(K, sigma):
    """Replicate extension + unit dc gain: a constant frame blurs to itself
    (Eq A32 steady state; Eq 11/Eq 7 with l = 0)."""
    img = np.full((19, 33), 3.25)
    out = filtering.blur_2d(img, iir(K, sigma), "replicate")
    assert np.max(np.abs(out - 3.25)) < 1e-13 * sigma ** 3 + 1e-14


@pytest.mark.parametrize("taps", [design.colored_sg_taps(4.0), design.gaussian_taps(3.0, 9)])
def test_constant_image_fir(taps):
    img = np.full((17, 40), -2.5)
    out = filtering.blur_2d(img, taps, "replicate")
    assert np.max(np.abs(out + 2.5)) < 1e-13


# ------------------------------------------------- vanishing moments

@pytest.mark.parametrize("K,sigma", [(2, 3.0), (3, 3.0), (3, 6.0)])
@pytest.mark.parametrize("degree", [0, 1, 2, 3])
def test_monomials_pass_unchanged_in_the_interior(K, sigma, degree):
    """Eq 7 with D = 3 (plus symmetry for the odd moments): filtering n^l,
    l <= 3, returns n^l wherever the truncated tails are negligible."""
    N = 1600
    n = np.arange(N, dtype=np.float64) - N / 2
    x = (n / 100.0) ** degree
    y = filtering.iir_1d(x[None, :], iir(K, sigma), "replicate")[0]
    lo, hi = 500, N - 500
    assert np.max(np.abs(y[lo:hi] - x[lo:hi])) < 1e-10 * max(1.0, np.max(np.abs(x)))


def test_quartic_is_not_passed():
    """The fourth moment does not vanish (D = 3): n^4 is altered."""
    N = 1600
    n = (np.arange(N, dtype=np.float64) - N / 2) / 100.0
    y = filtering.iir_1d((n ** 4)[None, :], iir(3, 6.0), "replicate")[0]
    assert np.max(np.abs(y[500:1100] - n[500:1100] ** 4)) > 1e-4


def test_sg_fir_passes_quadratics():
    taps = design.colored_sg_taps(5.0)
    n = (np.arange(400, dtype=np.float64) - 200) / 50.0
    for deg in (0, 1, 2, 3):
        y = filtering.fir_1d((n ** deg)[None, :], taps)[0]
        assert np.max(np.abs(y[50:350] - n[50:350] ** deg)) < 1e-11


# ------------------------------------------- separable == brute-force 2-D

def truncated_ir(K, sigma):
    dsg = design.design_repeated_pole(K, sigma)
    p = float(dsg.p)
    R = 10
    while R ** K * p ** R > 1e-18:
        R += 10
    return dsg.impulse_response(np.arange(-R, R + 1))


@pytest.mark.parametrize("K,sigma", [(2, 1.5), (3, 1.5), (2, 4.0), (3, 4.0)])
@pytest.mark.parametrize("boundary", ["replicate", "zero"])
def test_separable_equals_brute_force_iir(K, sigma, boundary):
    rng = np.random.default_rng(11)
    img = rng.random((12, 16)) * 10.0 + np.arange(16)[None, :] * 0.3
    sep = filtering.blur_2d(img, iir(K, sigma), boundary)
    bf = filtering.brute_force_2d(img, truncated_ir(K, sigma), boundary)
    assert np.max(np.abs(sep - bf)) < 1e-11 * np.max(np.abs(bf))


@pytest.mark.parametrize("boundary", ["replicate", "zero"])
def test_separable_equals_brute_force_fir(boundary):
    rng = np.random.default_rng(12)
    img = rng.random((14, 18))
    taps = design.colored_sg_taps(2.0)
    sep = filtering.blur_2d(img, taps, boundary)
    bf = filtering.brute_force_2d(img, taps, boundary)
    assert np.max(np.abs(sep - bf)) < 1e-13


@pytest.mark.parametrize("boundary", ["replicate", "zero"])
@pytest.mark.parametrize("shape_hw,sigma,K", [((14, 18), 2.0, None), ((9, 31), 4.0, 20), ((23, 6), 1.5, 11)])
def test_matrix_form_of_the_fir_equals_brute_force(boundary, shape_hw, sigma, K):
    """Eq A5 as the matrix products T_H X T_W^T (extension folded into the
    matrices), against the direct 2-D sum over the extended image, also with
    taps longer than the frame (every tap folds onto an edge sample)."""
    rng = np.random.default_rng(sum(shape_hw))
    img = rng.random(shape_hw) * 7.0 - 2.0
    taps = design.colored_sg_taps(sigma, K=K)
    got = filtering.blur_2d_matrix(img, taps, boundary)
    bf = filtering.brute_force_2d(img, taps, boundary)
    assert np.max(np.abs(got - bf)) < 1e-13 * max(1.0, np.max(np.abs(bf)))


def test_iir_equals_fir_with_its_impulse_response():
    """The DE with steady-state initialisation computes exactly the convolution
    of the replicate-extended signal with the infinite IR."""
    rng = np.random.default_rng(13)
    x = rng.random((3, 300))
    for K, sigma in [(2, 2.5), (3, 7.0)]:
        y_iir = filtering.iir_1d(x, iir(K, sigma), "replicate")
        y_fir = filtering.fir_1d(x, truncated_ir(K, sigma), "replicate")
        assert np.max(np.abs(y_iir - y_fir)) < 1e-12


def test_zero_boundary_superposition():
    rng = np.random.default_rng(14)
    a, b = rng.random((2, 8, 40))
    c = iir(3, 5.0)
    lhs = filtering.blur_2d(2.0 * a - 3.0 * b, c, "zero")
    rhs = 2.0 * filtering.blur_2d(a, c, "zero") - 3.0 * filtering.blur_2d(b, c, "zero")
    assert np.max(np.abs(lhs - rhs)) < 1e-12


def test_rows_then_columns_order():
    """x first then y; in exact arithmetic the order does not matter."""
    rng = np.random.default_rng(15)
    img = rng.random((20, 24))
    c = iir(3, 3.0)
    xy = filtering.blur_2d(img, c)
    yx = filtering.apply_1d(filtering.apply_1d(img, c, "replicate", -2), c, "replicate", -1)
    assert np.max(np.abs(xy - yx)) < 1e-12


# ----------------------------------------------------------- high pass

def test_hpf_on_polynomials():
    y, x = np.mgrid[0:30, 0:40].astype(np.float64)
    f = 0.5 * x * x - 2.0 * x * y + 3.0 * y * y + 4.0 * x - y + 7.0
    inner = (slice(2, -2), slice(2, -2))
    assert np.allclose(shape.derivative(f, 2, 0)[inner], 1.0, atol=1e-12)
    assert np.allclose(shape.derivative(f, 0, 2)[inner], 6.0, atol=1e-12)
    assert np.allclose(shape.derivative(f, 1, 1)[inner], -2.0, atol=1e-12)
    assert np.allclose(shape.derivative(f, 1, 0)[inner], (x - 2 * y + 4)[inner], atol=1e-12)
    assert np.allclose(shape.derivative(f, 0, 1)[inner], (-2 * x + 6 * y - 1)[inner], atol=1e-12)
    assert np.allclose(shape.laplacian(f, 3.0)[inner], 9.0 * 7.0, atol=1e-11)


def test_hpf_replicate_edges():
    """At the border the clamp makes the outside sample equal the edge one."""
    x = np.array([[1.0, 4.0, 9.0, 16.0]])
    d2 = shape.hpf_1d(x, 2, axis=1)
    assert d2[0].tolist() == [3.0 - 0.0, 1 - 8 + 9, 4 - 18 + 16, 9 - 32 + 16]


# ----------------------------------------------------------- detection

def detect_by_loops(V, tau, border):
    S, H, W = V.shape
    out = []
    for s in range(S):
        for y in range(border, H - border):
            for x in range(border, W - border):
                v = V[s, y, x]
                nb = [V[s2, y2, x2]
                      for s2 in range(s - 1, s + 2) for y2 in range(y - 1, y + 2)
                      for x2 in range(x - 1, x + 2)
                      if (s2, y2, x2) != (s, y, x) and 0 <= s2 < S and 0 <= y2 < H and 0 <= x2 < W]
                if all(v < u for u in nb) and v <= -tau:
                    out.append((y, x, s, 1))
                elif all(v > u for u in nb) and v >= tau:
                    out.append((y, x, s, -1))
    return out


@pytest.mark.parametrize("S,border", [(1, 1), (3, 1), (4, 0), (2, 2)])
def test_detect_extrema_matches_explicit_loops(S, border):
    rng = np.random.default_rng(20 + S)
    V = np.round(rng.standard_normal((S, 11, 13)), 1)   # rounding creates ties
    got = shape.detect_extrema(V, 0.3, border)
    exp = detect_by_loops(V, 0.3, border)
    assert [(int(b["y"]), int(b["x"]), int(b["scale"]), int(b["polarity"])) for b in got] == exp
    assert len(exp) > 0


def test_detect_ties_are_not_extrema():
    V = np.zeros((1, 5, 5))
    V[0, 2, 2] = -1.0
    V[0, 2, 3] = -1.0
    assert len(shape.detect_extrema(V, 0.5, 1)) == 0
    V[0, 2, 3] = -0.9
    got = shape.detect_extrema(V, 0.5, 1)
    assert [(int(b["y"]), int(b["x"]), int(b["polarity"])) for b in got] == [(2, 2, 1)]


def test_bright_blob_centre_found_at_its_scale():
    """A Gaussian bump centred at (40, 50) gives a bright (polarity +1)
    detection at its centre."""
    y, x = np.mgrid[0:96, 0:96].astype(np.float64)
    img = 1.0 + 2.0 * np.exp(-((y - 40) ** 2 + (x - 50) ** 2) / (2 * 6.0 ** 2))
    sig = [2.0, 4.0, 8.0]
    V = shape.laplacian_bank(filtering.blur_bank(img, [iir(3, s) for s in sig]), sig)
    got = shape.detect_extrema(V, 0.05, 1)
    bright = [(int(b["y"]), int(b["x"])) for b in got if b["polarity"] == 1]
    assert (40, 50) in bright


def test_hessian_newton_step_exact_on_quadratic():
    """Eq 27: on a quadratic surface the central differences are exact, so the
    Newton offset points exactly at the extremum."""
    y, x = np.mgrid[0:20, 0:20].astype(np.float64)
    x0, y0 = 9.3, 11.6
    B = -1.5 * (x - x0) ** 2 - 0.7 * (y - y0) ** 2 + 0.4 * (x - x0) * (y - y0)
    mask, ndet, dx, dy = shape.detect_hessian(B, 2.0, t1=0.0, t2=None)
    inner = (slice(2, -2), slice(2, -2))
    assert np.allclose(dx[inner], (x0 - x)[inner], atol=1e-10)
    assert np.allclose(dy[inner], (y0 - y)[inner], atol=1e-10)
    assert np.allclose(ndet[inner], 16.0 * (3.0 * 1.4 - 0.16), atol=1e-10)
    mask2, *_ = shape.detect_hessian(B, 2.0, t1=0.0, t2=0.75)
    ys, xs = np.nonzero(mask2)
    assert (12, 9) in list(zip(ys.tolist(), xs.tolist()))
    assert all(math.hypot(xx - x0, yy - y0) < 0.75 for yy, xx in zip(ys, xs))


def test_hessian_ellipse_pattern_scale_selection():
    """Section 5 (Figs 6 and 7): on the ellipse test pattern (aspect 2) with
    the repeated-pole blur at lambda = 2 sigma = 4 .. 64, one scale-invariant
    Threshold #1 on sigma^4 |H| keeps the centres of the ellipses whose
    semi-major axis equals lambda and none of the others; adding Threshold #2
    on the Newton offset leaves exactly one pixel, the centre, per matched
    ellipse."""
    img, items = syn.ellipse_pattern(2.0)
    for lam in syn.ELLIPSE_AXES:
        sg = lam / 2
        B = filtering.blur_2d(img, design.repeated_pole(3, sg))
        mask1, *_ = shape.detect_hessian(B, sg, 0.035, None, 1)
        for (cy, cx, a, b, ang) in items:
            iy, ix = int(cy), int(cx)
            hit = bool(mask1[iy - 2:iy + 3, ix - 2:ix + 3].any())
            assert hit == (a == lam), (lam, a, ang)
        mask2, *_ = shape.detect_hessian(B, sg, 0.035, 0.6, 1)
        got = sorted(zip(*[v.tolist() for v in np.nonzero(mask2)]))
        assert got == sorted((int(cy), int(cx)) for (cy, cx, a, b, ang) in items if a == lam), lam


@pytest.mark.parametrize("boundary", ["replicate", "zero"])
@pytest.mark.parametrize("shape_hw,sigma,K", [((13, 17), 2.0, None), ((8, 29), 4.0, 20), ((1, 9), 1.5, 6),
                                               ((21, 1), 3.0, 30)])
def test_fir_adjoint_dot_product_against_brute_force(boundary, shape_hw, sigma, K):
    """<G x, y> = <x, G^T y> with G the direct 2-D sum over the extended image
    (independent of the matrices the adjoint is built from), also with taps
    longer than the frame and single-row / single-column frames."""
    rng = np.random.default_rng(3 * shape_hw[0] + shape_hw[1])
    x = rng.standard_normal(shape_hw)
    y = rng.standard_normal(shape_hw)
    taps = design.colored_sg_taps(sigma, K=K)
    lhs = float(np.sum(filtering.brute_force_2d(x, taps, boundary) * y))
    rhs = float(np.sum(x * filtering.blur_2d_matrix_adjoint(y, taps, boundary)))
    assert abs(lhs - rhs) <= 1e-12 * max(1.0, abs(lhs))


def test_fir_adjoint_replicate_folds_tails_onto_edges():
    """With the replicate extension, the adjoint of a constant-preserving blur
    preserves the total: sum G^T y = sum y (every output draws unit weight)."""
    rng = np.random.default_rng(8)
    y = rng.standard_normal((12, 15))
    taps = design.gaussian_taps(3.0, 11)
    assert abs(filtering.blur_2d_matrix_adjoint(y, taps).sum() - y.sum()) < 1e-12
    zero = filtering.blur_2d_matrix_adjoint(y, taps, "zero")
    assert abs(zero.sum() - y.sum()) > 1e-3      # the zero extension loses the tails
