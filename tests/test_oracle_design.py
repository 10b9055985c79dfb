"""Pins of the oracle's filter design against what the paper prints and what
the mathematics fixes.  CPU only."""

import json
import math
import os

import mpmath as mp
import numpy as np
import pytest

from oracle import design, filtering

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def poly(coeffs, x):
    return sum(c * x ** i for i, c in enumerate(coeffs))


# ---------------------------------------------------------------- Table IV

def test_table_iv_sigma8_printed_values():
    g = golden("table_iv_sigma8.json")
    c = design.table_iv(g["sigma"])
    tol = 0.5 * 10 ** -g["decimals"] + 1e-12
    assert abs(c.b0 - g["b0"]) <= tol
    for m in range(4):
        assert abs(c.bp[m] - g["bp"][m]) <= tol
        assert abs(c.ap[m] - g["ap"][m]) <= tol


@pytest.mark.parametrize("sigma", [0.7, 2.0, 8.0, 23.8, 64.0, 96.0])
def test_table_iv_closed_form_matches_printed_polynomials(sigma):
    g = golden("table_iv_sigma8.json")["closed_form_poly"]
    p = math.exp(-1 / sigma)
    c = design.table_iv(sigma)
    assert c.b0 == pytest.approx(poly(g["b0"], p), rel=1e-13, abs=1e-15)
    for m in (1, 2, 3):
        assert c.bp[m] == pytest.approx(poly(g["bp%d" % m], p), rel=1e-9, abs=1e-15)


@pytest.mark.parametrize("sigma", [0.5, 1.0, 2.0, 8.0, 24.0, 64.0, 96.0])
def test_general_procedure_reproduces_table_iv(sigma):
    """Section 4.3 (Eqs 12-15, 23-24, A17) with L_D = 1, Lbar_pi = 2 must give
    Table IV exactly; compared in high precision against the printed form."""
    dsg = design.design_repeated_pole(3, sigma)
    with mp.workdps(50):
        p = dsg.p
        b0 = p ** 3 / 16 - 9 * p / 16 + mp.mpf(1) / 2
        bp = [0, 3 * p ** 4 / 32 - 3 * p ** 2 / 8 + mp.mpf(9) / 32,
              -3 * p ** 5 / 32 + 9 * p ** 3 / 16 - 15 * p / 32,
              p ** 6 / 32 - 9 * p ** 4 / 32 + 9 * p ** 2 / 32 - mp.mpf(1) / 32]
        ap = [1, -3 * p, 3 * p ** 2, -p ** 3]
        scale = max(abs(v) for v in bp[1:])
        assert abs(dsg.b0_mp - b0) < mp.mpf(10) ** -30
        for m in range(1, 4):
            assert abs(dsg.bp_mp[m] - bp[m]) < mp.mpf(10) ** -30 * max(1, 1 / scale)
            assert abs(dsg.ap_mp[m] - ap[m]) < mp.mpf(10) ** -40


# ------------------------------------------- constraints fixed by the paper

def moments_by_recursion(coef, R):
    """IR from the DE driven by an impulse (independent of the F-matrix route),
    then moments sum m^l h(m) and Nyquist sums sum (-1)^m m^l h(m)."""
    h = filtering.impulse_response_by_recursion(coef, R)
    m = np.arange(-R, R + 1, dtype=np.float64)
    mom = [float(np.sum(m ** l * h)) for l in range(5)]
    nyq = [float(np.sum((-1.0) ** np.abs(m) * m ** l * h)) for l in range(3)]
    return h, mom, nyq


@pytest.mark.parametrize("K,sigma", [(2, 1.5), (2, 4.0), (2, 12.0), (3, 2.0), (3, 8.0), (3, 16.0)])
def test_vanishing_moments_and_nyquist_nulls(K, sigma):
    """dc gain 1, second moment 0 (Eq 7 with D = 3), odd moments 0 (symmetry),
    H(pi) = 0 and, for K = 3, H''(pi) = 0 (the Lbar_pi constraints)."""
    coef = design.repeated_pole(K, sigma)
    R = int(60 * sigma) + 100
    h, mom, nyq = moments_by_recursion(coef, R)
    # float64 direct-form recursion: rounding grows roughly like sigma^3 eps
    assert mom[0] == pytest.approx(1.0, abs=1e-10)
    assert abs(mom[1]) < 1e-10
    assert abs(mom[2]) < 1e-9 * sigma ** 2
    assert abs(mom[3]) < 1e-8 * sigma ** 3
    assert abs(nyq[0]) < 1e-11
    if K == 3:
        assert abs(nyq[2]) < 1e-11
    # the fourth moment does NOT vanish (D = 3 only): guards against a design
    # that trivially zeroes every moment
    assert abs(mom[4]) > 1e-3 * sigma ** 4


@pytest.mark.parametrize("K,sigma", [(2, 4.0), (3, 8.0), (3, 1.0), (2, 30.0)])
def test_closed_form_impulse_response_equals_recursion(K, sigma):
    """h(m) = sum_k c_k |m|^k p^|m| + c_imp delta(m) (Eqs 12a, 23) must equal
    the impulse response of the DE obtained through Eq A17."""
    dsg = design.design_repeated_pole(K, sigma)
    R = int(50 * sigma) + 50
    h_rec = filtering.impulse_response_by_recursion(dsg.coefficients(), R)
    h_cf = dsg.impulse_response(np.arange(-R, R + 1))
    assert np.max(np.abs(h_rec - h_cf)) < 1e-12 * np.max(np.abs(h_cf))


@pytest.mark.parametrize("K,sigma", [(2, 3.0), (3, 5.0)])
def test_F_matrix_equals_moment_sums(K, sigma):
    """Eq 15 derivatives of F_k at dc / pi, computed in the design by
    differentiating Eq 24, must equal the moment sums
    (-1)^(l/2) sum_m m^l f_k(m) e^{-i m omega0} evaluated by brute force."""
    dsg = design.design_repeated_pole(K, sigma)
    p = float(dsg.p)
    n_k = K + 1
    R = int(80 * sigma) + 100
    m = np.arange(-R, R + 1, dtype=np.float64)
    am = np.abs(m)
    rows = [(0, 0.0), (2, 0.0)] + [(2 * lb, math.pi) for lb in range(K - 1)]
    for r, (l, w0) in enumerate(rows):
        for k in range(n_k):
            if k == n_k - 1:
                f = (m == 0).astype(np.float64)
            else:
                f = np.where(am == 0, 1.0 if k == 0 else 0.0, am ** k * p ** am)
            brute = (-1.0) ** (l // 2) * np.sum(m ** l * f * np.cos(m * w0))
            assert float(dsg.F[r, k]) == pytest.approx(brute, rel=1e-9, abs=1e-9)


def test_order2_coefficients_fixed_by_three_constraints():
    """K = 2 is not printed.  Its 3 unknowns (b0, b+_1, b+_2 at a given p) are
    fixed by dc gain 1, zero second moment and H(pi) = 0; solve those three
    linear equations independently from the IR written as the DE output and
    compare."""
    sigma = 4.0
    p = math.exp(-1 / sigma)
    ap = [1.0, -2 * p, p * p]
    R = 600

    def ir(b0, b1, b2):
        c = design.IIRCoefficients(b0=b0, bp=[0.0, b1, b2], ap=ap)
        return filtering.impulse_response_by_recursion(c, R)

    m = np.arange(-R, R + 1, dtype=np.float64)
    basis = [ir(1, 0, 0), ir(0, 1, 0), ir(0, 0, 1)]
    M = np.array([[b.sum(), (m * m * b).sum(), ((-1.0) ** np.abs(m) * b).sum()] for b in basis]).T
    sol = np.linalg.solve(M, [1.0, 0.0, 0.0])
    c = design.repeated_pole(2, sigma)
    assert c.b0 == pytest.approx(sol[0], rel=1e-10)
    assert c.bp[1] == pytest.approx(sol[1], rel=1e-10)
    assert c.bp[2] == pytest.approx(sol[2], rel=1e-10)


# --------------------------------------------------- Appendix, Example 1

@pytest.mark.parametrize("lam", [1.5, 8.0, 40.0])
def test_three_term_decomposition_reproduces_example1(lam):
    g = golden("example1_blunt_exponential.json")
    b0, bp, ap = design.blunt_exponential(3, lam)
    with mp.workdps(50):
        p = mp.exp(-1 / mp.mpf(lam))
        assert abs(b0 - poly(g["b0"], p)) < mp.mpf(10) ** -35
        for m in (1, 2, 3):
            assert abs(bp[m] - poly(g["bp%d" % m], p)) < mp.mpf(10) ** -35
            assert abs(ap[m] - poly(g["ap"][str(m)], p)) < mp.mpf(10) ** -40


def test_example1_normalising_factor():
    """Eq A22: c0 makes H(1) = 1: (z^-1 + 2 + z)^3 -> 64 and the denominator
    -> (1 - p)^6, so c0 = (1 - p)^6 / 64 -- compared with the printed
    polynomial."""
    g = golden("example1_blunt_exponential.json")
    for lam in (2.0, 8.0):
        p = math.exp(-1 / lam)
        assert poly(g["c0"], p) == pytest.approx((1 - p) ** 6 / 64, rel=1e-12)


# ------------------------------------------------- Butterworth (Sec. 4.4)

def test_filter_e_printed_values():
    g = golden("butterworth.json")["filter_e"]
    c = design.butterworth(g["L_B"], g["omega_c"])
    tol = 0.5 * 10 ** -g["decimals"] + 1e-4   # printed omega_c is itself rounded
    assert abs(c.b0 - g["b0"]) <= tol
    for m in range(3):
        assert abs(c.bp[m] - g["bp"][m]) <= tol
        assert abs(c.ap[m] - g["ap"][m]) <= tol


@pytest.mark.parametrize("wc", [0.05, 0.1472, 0.4])
def test_butterworth_example2_closed_forms(wc):
    g = golden("butterworth.json")["example2"]
    c = design.butterworth(6, wc)
    for m in (1, 2, 3):
        e = g["a%d" % m]
        assert c.ap[m] == pytest.approx(poly(e["num"], wc) / poly(e["den"], wc), rel=1e-12)
    a0 = poly(g["a0"]["base"], wc) ** g["a0"]["power"]
    assert c.b0 == pytest.approx(poly(g["b0_times_3a0"], wc) / 3 / a0, rel=1e-11)
    for m in (1, 2, 3):
        assert c.bp[m] == pytest.approx(poly(g["b%d_times_3a0" % m], wc) / 3 / a0, rel=1e-11)


def test_butterworth_unit_dc_and_nyquist_flatness():
    c = design.butterworth(4, math.sqrt(2 * math.log(2)) / 8)
    h, mom, nyq = moments_by_recursion(c, 800)
    assert mom[0] == pytest.approx(1.0, abs=1e-12)
    assert abs(mom[2]) < 1e-8       # flat to order L_B - 1 = 3 at dc
    assert abs(nyq[0]) < 1e-12
    assert abs(nyq[2]) < 1e-10


# ------------------------------------------------ Table I / II / III

def test_table_i_from_eq8():
    g = golden("table_i_hpf_taps.json")
    for d in range(5):
        taps = design.hpf_taps(d)
        got = [taps.get(m, 0.0) for m in g["m"]]
        assert got == pytest.approx(g["taps"][str(d)], abs=0)


def rho_dc(taps: dict, l: int) -> complex:
    """rho_{d,l} = d^l/domega^l sum_m h(m) e^{-i m omega} at omega = 0 (Eq 6, A2)."""
    return sum(h * (-1j * m) ** l for m, h in taps.items())


def test_table_ii_rho_values():
    g = golden("table_ii_rho.json")
    for d in range(5):
        taps = design.hpf_taps(d)
        for l in range(5):
            exp = complex(*g["rho"][str(d)][l])
            assert rho_dc(taps, l) == pytest.approx(exp, abs=1e-12)


def test_table_iii_one_and_two_stage_rho():
    g = golden("table_iii_rho.json")
    sigma, K = g["sigma"], g["K"]
    tol = 0.5 * 10 ** -g["decimals"] + 1e-12
    lpf = design.gaussian_taps(sigma, K)
    for d in range(5):
        one = design.gaussian_derivative_taps(sigma, K, d)
        one_taps = {m: one[K + m] for m in range(-K, K + 1)}
        hpf = design.hpf_taps(d)
        two_taps = {}
        for m1 in range(-K, K + 1):
            for m2, h2 in hpf.items():
                two_taps[m1 + m2] = two_taps.get(m1 + m2, 0.0) + lpf[K + m1] * h2
        for l in range(5):
            e1 = complex(*g["one_stage"][str(d)][l])
            e2 = complex(*g["two_stage"][str(d)][l])
            # Reading: the printed one-stage (d=4, l=2) entry 0.0000 is taken as
            # a misprint.  The same sampled filter reproduces the printed l=4
            # value 23.9896, and there (4,2) is 7.3e-4, the aliasing of a
            # sigma = 1 Gaussian's 4th derivative.
            if not (d == 4 and l == 2):
                assert abs(rho_dc(one_taps, l) - e1) <= tol, (d, l, rho_dc(one_taps, l))
            else:
                assert 5e-4 < abs(rho_dc(one_taps, l)) < 1e-3
            assert abs(rho_dc(two_taps, l) - e2) <= tol, (d, l, rho_dc(two_taps, l))


# ------------------------------------------------------- FIR blurs

@pytest.mark.parametrize("K", [2, 3, 7, 20])
def test_colored_sg_reduces_to_classic_sg_when_uncoloured(K):
    """With omega_c = 0, Sbar = I (Eq 22b) and Eq 20 minimises the white-noise
    gain: the quadratic Savitzky-Golay smoother, whose weights are the textbook
    [3(3K^2 + 3K - 1) - 15 m^2] / [(2K - 1)(2K + 1)(2K + 3)]."""
    h = design.colored_sg_taps(1.0, K=K, omega_c=0.0)
    m = np.arange(-K, K + 1, dtype=np.float64)
    classic = (3 * (3 * K * K + 3 * K - 1) - 15 * m * m) / ((2 * K - 1) * (2 * K + 1) * (2 * K + 3))
    assert np.max(np.abs(h - classic)) < 1e-13


def cng_quadrature(h, omega_c, n=20001):
    """CNG = (1/pi) int_{omega_c}^{pi} |H(omega)|^2 d omega (Eq 21), by the
    trapezoidal rule on a dense grid (independent of the Eq 22 closed form)."""
    K = (len(h) - 1) // 2
    m = np.arange(-K, K + 1)
    w = np.linspace(omega_c, math.pi, n)
    H = np.cos(np.outer(w, m)) @ h       # symmetric h: H is real
    return np.trapezoid(H * H, w) / math.pi


@pytest.mark.parametrize("sigma", [2.0, 5.38, 14.5])
def test_colored_sg_constraints_and_optimality(sigma):
    K = design.fir_half_length(sigma)
    wc = 3.0 / sigma
    h = design.colored_sg_taps(sigma)
    m = np.arange(-K, K + 1, dtype=np.float64)
    assert len(h) == 2 * K + 1
    assert np.allclose(h, h[::-1], atol=0)
    assert h.sum() == pytest.approx(1.0, abs=1e-12)
    assert abs((m * m * h).sum()) < 1e-10 * K * K
    base = cng_quadrature(h, wc)
    # any symmetric perturbation that keeps both constraints raises the CNG
    rng = np.random.default_rng(5)
    for _ in range(6):
        q = rng.standard_normal(K + 1)
        pert = np.array([q[abs(int(v))] for v in m])
        A = np.stack([np.ones_like(m), m * m])
        pert -= A.T @ np.linalg.lstsq(A.T, pert, rcond=None)[0]
        pert *= 1e-3 / np.max(np.abs(pert))
        assert cng_quadrature(h + pert, wc) > base
    assert base < cng_quadrature(design.gaussian_taps(sigma, K), wc) * 10


def test_gaussian_taps():
    for sigma, K in [(1.0, 5), (4.0, 12), (23.8, 72)]:
        h = design.gaussian_taps(sigma, K)
        m = np.arange(-K, K + 1)
        assert h.sum() == pytest.approx(1.0, abs=1e-14)
        assert np.allclose(h / h[K], np.exp(-m * m / (2 * sigma * sigma)), rtol=1e-13)


def test_fir_half_length_rules():
    assert design.fir_half_length(2.0) == 6
    assert design.fir_half_length(64.0) == 192
    assert design.fir_half_length(3.28) == 10
    assert design.fir_half_length(4.0, "5sigma") == 20


# ------------------------------------------------ sigma derivatives of the FIR designs

def _central(f, sigma, h):
    """Fourth-order central difference of f at sigma."""
    return (-f(sigma + 2 * h) + 8 * f(sigma + h) - 8 * f(sigma - h) + f(sigma - 2 * h)) / (12 * h)


@pytest.mark.parametrize("sigma,K", [(0.8, 3), (2.0, 6), (9.5, 29), (40.0, 120)])
def test_gaussian_taps_dsigma_is_the_derivative(sigma, K):
    got = design.gaussian_taps_dsigma(sigma, K)
    ref = _central(lambda s: design.gaussian_taps(s, K), sigma, 1e-3 * sigma)
    assert np.max(np.abs(got - ref)) <= 1e-8 * np.max(np.abs(ref))
    assert abs(got.sum()) < 1e-15            # Eq 11 holds at every sigma
    assert np.allclose(got, got[::-1], rtol=0, atol=1e-18)   # symmetric taps


@pytest.mark.parametrize("sigma,K", [(1.2, None), (2.0, 6), (5.4, None), (14.5, 44), (64.0, 192), (10.0, 50)])
def test_colored_sg_taps_dsigma_is_the_derivative(sigma, K):
    Kk = K if K is not None else design.fir_half_length(sigma)
    got = design.colored_sg_taps_dsigma(sigma, Kk)
    ref = _central(lambda s: design.colored_sg_taps(s, K=Kk), sigma, 1e-3 * sigma)
    assert np.max(np.abs(got - ref)) <= 2e-6 * np.max(np.abs(ref))
    m = np.arange(-Kk, Kk + 1, dtype=np.float64)
    scale = np.sum(np.abs(got)) * max(1.0, Kk * Kk)
    # the dc constraints rho = [1, 0] hold at every sigma: their derivatives vanish
    assert abs(got.sum()) <= 1e-12 * np.sum(np.abs(got))
    assert abs(np.sum(m * m * got)) <= 1e-10 * scale
    assert np.allclose(got, got[::-1], rtol=0, atol=1e-15 * np.max(np.abs(got)))
