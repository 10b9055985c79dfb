"""Filter design -- oracle side (test infrastructure only; see package header).

Notation follows the paper: p is the repeated pole, sigma the scale, K the
order of each one-sided recursion, b0 / bp / ap the central, forward and
(equal, by symmetry) backward difference-equation coefficients of Eq A10:

    y(n)  = y+(n) + y-(n) + b0 x(n)                                   (A6)
    y+(n) = sum_{m=1..K} bp[m] x(n-m) - sum_{m=1..K} ap[m] y+(n-m)    (A10a)
    y-(n) = sum_{m=1..K} bm[m] x(n+m) - sum_{m=1..K} am[m] y-(n+m)    (A10b)

with ap[0] = am[0] = 1, bp[0] = bm[0] = 0, bm = bp and am = ap for the
symmetric blurs used here.

The general procedures run in arbitrary precision (mpmath, ``DPS`` digits)
because the constraint matrix F becomes ill-conditioned as p -> 1
(Section 4.3 notes that the attainable order is limited by arithmetic
precision); results are handed back as float64.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field

import mpmath as mp
import numpy as np

DPS = 60


@dataclass
class IIRCoefficients:
    """Three-term DE coefficients (Eqs A6-A10)."""

    b0: float
    bp: list  # bp[0] = 0, bp[1..K]
    ap: list  # ap[0] = 1, ap[1..K]
    bm: list = field(default=None)
    am: list = field(default=None)

    def __post_init__(self):
        if self.bm is None:
            self.bm = list(self.bp)
        if self.am is None:
            self.am = list(self.ap)

    @property
    def order(self) -> int:
        return len(self.ap) - 1


# --------------------------------------------------------------------------
# Repeated-pole IIR blur (Section 4.3)
# --------------------------------------------------------------------------

def pole(sigma: float) -> float:
    """Section 4.3: the poles of the forward part are all at p = exp(-1/sigma),
    sigma being the mean of the one-sided exponential."""
    return math.exp(-1.0 / sigma)


def table_iv(sigma: float) -> IIRCoefficients:
    """Filter D, the closed form of Table IV (L_D = 1, Lbar_pi = 2, K = 3),
    evaluated in float64 at p = exp(-1/sigma).  Pinned by the sigma = 8 values
    printed under Table IV and by the general procedure below."""
    p = pole(sigma)
    b0 = p ** 3 / 16 - 9 * p / 16 + 0.5
    bp = [
        0.0,
        3 * p ** 4 / 32 - 3 * p ** 2 / 8 + 9 / 32,
        -3 * p ** 5 / 32 + 9 * p ** 3 / 16 - 15 * p / 32,
        p ** 6 / 32 - 9 * p ** 4 / 32 + 9 * p ** 2 / 32 - 1 / 32,
    ]
    ap = [1.0, -3 * p, 3 * p ** 2, -(p ** 3)]
    return IIRCoefficients(b0=b0, bp=bp, ap=ap)


# Laurent polynomials in z are dicts {exponent: coefficient}.

def _lmul(a: dict, b: dict) -> dict:
    out: dict = {}
    for ea, ca in a.items():
        for eb, cb in b.items():
            out[ea + eb] = out.get(ea + eb, 0) + ca * cb
    return out


def _ladd(*terms) -> dict:
    out: dict = {}
    for scale, poly in terms:
        for e, c in poly.items():
            out[e] = out.get(e, 0) + scale * c
    return out


def _lpow(a: dict, n: int) -> dict:
    out = {0: mp.mpf(1)}
    for _ in range(n):
        out = _lmul(out, a)
    return out


def one_sided_basis_numerator(k: int, p) -> list:
    """Eq 24 needs the one-sided Z transform of f_k^+(m) = m^k p^m (Eq 23b):

        F_k^+(z) = sum_{m>=0} m^k p^m z^{-m} = N_k(z^{-1}) / (1 - p z^{-1})^{k+1}.

    N_k has degree <= k, so multiplying the first k+1 terms of the power
    series by (1 - p w)^{k+1} and keeping degrees 0..k gives it exactly.
    Returns [N_k[0], ..., N_k[k]] (coefficients of w^0..w^k, w = z^{-1})."""
    series = [mp.mpf(1) if (m == 0 and k == 0) else mp.mpf(m) ** k * p ** m
              for m in range(k + 1)]
    binom = [mp.binomial(k + 1, j) * (-p) ** j for j in range(k + 2)]
    return [mp.fsum(binom[j] * series[i - j] for j in range(i + 1)) for i in range(k + 1)]


def _basis_fr(k: int, n_k: int, p):
    """F_k(omega) of the k-th basis function, Eq 24 with Delta_d = 0
    (symmetric blur): F_k(z) = F_k^+(z) + F_k^+(1/z) - f_k^+(0); the last
    basis function (k = N_K - 1) is the unit impulse, F(z) = 1."""
    if k == n_k - 1:
        return lambda w: mp.mpf(1)
    num = one_sided_basis_numerator(k, p)
    f0 = 1 if k == 0 else 0

    def fr(omega):
        zi = mp.expj(-omega)   # z^{-1} on the unit circle
        z = mp.expj(omega)
        fwd = mp.fsum(num[i] * zi ** i for i in range(k + 1)) / (1 - p * zi) ** (k + 1)
        bwd = mp.fsum(num[i] * z ** i for i in range(k + 1)) / (1 - p * z) ** (k + 1)
        return mp.re(fwd + bwd - f0)

    return fr


@dataclass
class RepeatedPoleDesign:
    """Everything the Section 4.3 procedure produces for one (K, sigma)."""

    K: int
    sigma: float
    p: object          # mpf
    F: object          # mp.matrix, N_K x N_K (Eq 14)
    rho: object        # mp.matrix, N_K x 1 (Eq 13)
    c: list            # basis coefficients (Eq 12), mpf
    B: dict            # numerator of H(z) = B(z)/A(z), Laurent in z
    A: dict            # denominator
    ap_mp: list        # A+(z) coefficients (Eq A19), mpf
    b0_mp: object      # central coefficient (Eq A17 solve)
    bp_mp: list        # forward numerator (Eq A17 solve)

    def coefficients(self) -> IIRCoefficients:
        return IIRCoefficients(b0=float(self.b0_mp), bp=[float(v) for v in self.bp_mp],
                               ap=[float(v) for v in self.ap_mp])

    def impulse_response(self, m):
        """h(m) = sum_k c_k f_k(m) (Eqs 12a, 23), float64 for integer array m."""
        m = np.abs(np.asarray(m, dtype=np.int64))
        n_k = len(self.c)
        p = float(self.p)
        h = np.zeros(m.shape, dtype=np.float64)
        for k in range(n_k - 1):
            fk = np.where(m == 0, 1.0 if k == 0 else 0.0,
                          m.astype(np.float64) ** k * p ** m.astype(np.float64))
            h += float(self.c[k]) * fk
        h += float(self.c[n_k - 1]) * (m == 0)
        return h


def design_repeated_pole(K: int, sigma: float, L_D: int = 1) -> RepeatedPoleDesign:
    """The general design procedure of Section 4.3 for the d = 0 blur.

    * D = 2 L_D + 1; d = 0 so Delta_d = 0 and only even l appear.
    * Lbar_dc = L_D + 1 constraints at dc (l = 0, 2, ..), rho_dc = [1, 0, ..]
      (rho^dc_{0,l} = i^0 0! delta_{0,l}, Eq 4); Lbar_pi = K - L_D constraints
      at omega = pi, all zero.  N_K = Lbar_dc + Lbar_pi = K + 1.
    * Basis (Eq 23): f_k(m) = |m|^k p^|m| for k < N_K - 1 and the unit impulse
      for k = N_K - 1.
    * F rows are the l-th omega-derivatives of F_k(omega) at dc / pi (Eq 15),
      c = F^{-1} rho (Section 4).
    * H(z) = sum_k c_k F_k(z) (Eq 12b) is put over the common denominator
      A(z) = (1 - p z^{-1})^K (1 - p z)^K, then split into forward, central and
      backward parts by the linear system of Eq A17.

    K = 3 with L_D = 1 is Table IV.  K = 2 (Lbar_pi = 1) is not printed in the
    paper; this procedure is how it is obtained here."""
    if K < L_D + 1:
        raise ValueError("need K >= L_D + 1")
    with mp.workdps(DPS):
        p = mp.exp(-1 / mp.mpf(sigma))
        lbar_dc = L_D + 1
        lbar_pi = K - L_D
        n_k = lbar_dc + lbar_pi
        frs = [_basis_fr(k, n_k, p) for k in range(n_k)]
        F = mp.matrix(n_k, n_k)
        rho = mp.matrix(n_k, 1)
        for lb in range(lbar_dc):
            for k in range(n_k):
                F[lb, k] = mp.diff(frs[k], 0, 2 * lb)
        for lb in range(lbar_pi):
            for k in range(n_k):
                F[lbar_dc + lb, k] = mp.diff(frs[k], mp.pi, 2 * lb)
        rho[0] = 1
        c_vec = mp.lu_solve(F, rho)
        c = [c_vec[k] for k in range(n_k)]

        # H(z) = B(z)/A(z) over the common denominator A = A+ A-.
        one_m_pzi = {0: mp.mpf(1), -1: -p}   # 1 - p z^{-1}
        one_m_pz = {0: mp.mpf(1), 1: -p}     # 1 - p z
        A = _lmul(_lpow(one_m_pzi, K), _lpow(one_m_pz, K))
        B: dict = {}
        for k in range(n_k - 1):
            num = one_sided_basis_numerator(k, p)
            n_fwd = {-i: num[i] for i in range(k + 1)}
            n_bwd = {i: num[i] for i in range(k + 1)}
            t_fwd = _lmul(n_fwd, _lmul(_lpow(one_m_pzi, K - k - 1), _lpow(one_m_pz, K)))
            t_bwd = _lmul(n_bwd, _lmul(_lpow(one_m_pz, K - k - 1), _lpow(one_m_pzi, K)))
            f0 = 1 if k == 0 else 0
            B = _ladd((1, B), (c[k], t_fwd), (c[k], t_bwd), (-c[k] * f0, A))
        B = _ladd((1, B), (c[n_k - 1], A))

        # A+(z) from its K roots inside the unit circle (Eq A19): all at p.
        ap = polynomial_from_roots([p] * K)
        b0, bp, _ = three_term_decomposition(B, A, ap)
    return RepeatedPoleDesign(K=K, sigma=sigma, p=p, F=F, rho=rho, c=c, B=B, A=A,
                              ap_mp=ap, b0_mp=b0, bp_mp=bp)


def repeated_pole(K: int, sigma: float) -> IIRCoefficients:
    """Float64 DE coefficients of the repeated-pole blur: Table IV for K = 3,
    the general Section 4.3 procedure otherwise."""
    if K == 3:
        return table_iv(sigma)
    return design_repeated_pole(K, sigma).coefficients()


# --------------------------------------------------------------------------
# Three-term decomposition (Eqs A11-A19)
# --------------------------------------------------------------------------

def polynomial_from_roots(roots) -> list:
    """A+(z) = z^{-K} prod_m (z - p_m) = 1 + sum_m a+_m z^{-m}  (Eq A19).
    Returns [a_0 = 1, a_1, .., a_K] (real parts; complex roots come in
    conjugate pairs)."""
    coeffs = [mp.mpf(1)]
    for r in roots:
        nxt = [mp.mpf(0)] * (len(coeffs) + 1)
        for i, cval in enumerate(coeffs):
            nxt[i] += cval
            nxt[i + 1] -= cval * r
        coeffs = nxt
    return [mp.re(v) for v in coeffs]


def three_term_decomposition(B: dict, A: dict, ap: list):
    """Solve b = A~ b~ (Eqs A15-A17) for the realisable three-term form.

    B, A: Laurent numerator / denominator of the symmetric non-realisable
    H(z) (exponents -K..K).  ap: A+(z) coefficients [1, a+_1, .., a+_K].
    The backward denominator is A-(z) = A+(1/z) (a-_m = a+_m), A(z) =
    a0 A+(z) A-(z) with a0 = a_0 / a^pm_0 (Eq A18 and the text after A19).
    The unknowns are b~ = [a0 b+_K .. a0 b+_1, b0, a0 b-_1 .. a0 b-_K]; the
    columns of A~ are z^{-m} A-(z), A+(z)A-(z) and z^{m} A+(z).

    Returns (central coefficient b0/a0 of the realisable DE (the B0/A0 term
    of Eq A13a), [0, b+_1..b+_K], [0, b-_1..b-_K])."""
    K = len(ap) - 1
    a_plus = {-m: ap[m] for m in range(K + 1)}
    a_minus = {m: ap[m] for m in range(K + 1)}
    a_pm = _lmul(a_plus, a_minus)
    a0 = A.get(0, 0) / a_pm[0]
    cols = []
    for m in range(K, 0, -1):
        cols.append(_lmul({-m: mp.mpf(1)}, a_minus))
    cols.append(a_pm)
    for m in range(1, K + 1):
        cols.append(_lmul({m: mp.mpf(1)}, a_plus))
    n = 2 * K + 1
    At = mp.matrix(n, n)
    bvec = mp.matrix(n, 1)
    for r, e in enumerate(range(-K, K + 1)):
        bvec[r] = B.get(e, 0)
        for cidx, col in enumerate(cols):
            At[r, cidx] = col.get(e, 0)
    bt = mp.lu_solve(At, bvec)
    bp = [mp.mpf(0)] + [bt[K - m] / a0 for m in range(1, K + 1)]
    bm = [mp.mpf(0)] + [bt[K + m] / a0 for m in range(1, K + 1)]
    b0 = bt[K] / a0
    return b0, bp, bm


# --------------------------------------------------------------------------
# Appendix Example 1 (Eq A21) and Example 2 / Section 4.4 Butterworth
# --------------------------------------------------------------------------

def blunt_exponential(K: int, lam: float):
    """Example 1, Eq A21: H(z) = c0 {(z^{-1} + 2 + z)/(-p z^{-1} + 1 + p^2 - p z)}^K,
    p = exp(-1/lambda), c0 for unit dc gain; decomposed with Eq A17 (A23-A25).
    Returns (b0, bp, ap) as mpf lists."""
    with mp.workdps(DPS):
        p = mp.exp(-1 / mp.mpf(lam))
        num = _lpow({-1: mp.mpf(1), 0: mp.mpf(2), 1: mp.mpf(1)}, K)
        den = _lpow({-1: -p, 0: 1 + p * p, 1: -p}, K)
        c0 = mp.fsum(den.values()) / mp.fsum(num.values())
        B = {e: c0 * v for e, v in num.items()}
        ap = polynomial_from_roots([p] * K)
        b0, bp, _ = three_term_decomposition(B, den, ap)
        return b0, bp, ap


def butterworth(L_B: int, omega_c: float) -> IIRCoefficients:
    """Section 4.4 / Eqs 25, A26: L_B-th order analogue Butterworth,
    H(s) = 1/(1 + (-s^2/omega_c^2)^{L_B/2}), discretised by the bilinear
    transform s = 2(z-1)/(z+1).  With n = L_B/2, multiplying through by
    omega_c^{2n} (z+1)^{2n} z^{-n}:
        B(z) = omega_c^{2n} (z^{-1} + 2 + z)^n
        A(z) = omega_c^{2n} (z^{-1} + 2 + z)^n + (-4)^n (z^{-1} - 2 + z)^n.
    A+ collects the n roots of A inside the unit circle (Eq A19), then Eq A17.
    K (per-direction order) = L_B/2."""
    n = L_B // 2
    with mp.workdps(DPS):
        wc = mp.mpf(omega_c)
        plus = _lpow({-1: mp.mpf(1), 0: mp.mpf(2), 1: mp.mpf(1)}, n)
        minus = _lpow({-1: mp.mpf(1), 0: mp.mpf(-2), 1: mp.mpf(1)}, n)
        B = {e: wc ** (2 * n) * v for e, v in plus.items()}
        A = _ladd((wc ** (2 * n), plus), ((-4) ** n, minus))
        # z^n A(z) as an ordinary polynomial, highest power first for polyroots
        poly = [A.get(e, 0) for e in range(n, -n - 1, -1)]
        roots = mp.polyroots(poly, maxsteps=200, extraprec=200)
        inside = [r for r in roots if abs(r) < 1]
        ap = polynomial_from_roots(inside)
        b0, bp, _ = three_term_decomposition(B, A, ap)
        return IIRCoefficients(b0=float(b0), bp=[float(v) for v in bp], ap=[float(v) for v in ap])


# --------------------------------------------------------------------------
# FIR blurs
# --------------------------------------------------------------------------

def fir_half_length(sigma: float, rule: str = "3sigma") -> int:
    """Half-length K of an FIR blur.  The paper uses K = ceil(5 sigma) for the
    coloured SG blur (Section 4.2) and K = 5 sigma for the Gaussian (Table V
    notes); the 6 sigma + 1 length rule gives K = ceil(3 sigma)."""
    if rule == "3sigma":
        return int(math.ceil(3.0 * sigma - 1e-9))
    if rule == "5sigma":
        return int(math.ceil(5.0 * sigma - 1e-9))
    raise ValueError(rule)


def gaussian_taps(sigma: float, K: int) -> np.ndarray:
    """Filter A: sampled Gaussian g_0 (Eq 9c) on m = -K..K, renormalised to unit
    dc gain (Eq 11).  Returns h[0..2K] = h(-K..K)."""
    m = np.arange(-K, K + 1, dtype=np.float64)
    g0 = np.exp(-m * m / (2.0 * sigma * sigma)) / (sigma * math.sqrt(2.0 * math.pi))
    return g0 / g0.sum()


def gaussian_derivative_taps(sigma: float, K: int, d: int) -> np.ndarray:
    """One-stage sampled Gaussian derivative filters of Eqs 9a-9b with the dc
    renormalisation constant c_g of Eq 11 (taken from d = 0).  Derivatives of
    g_0 are the probabilists' Hermite form g_d(x) = (-1/sigma)^d He_d(x/sigma) g_0(x).
    Returns h_d[0..2K] = h_d(-K..K), h_d(m) = c_g g_d(m) (Eq 9a, T_s = 1), in
    the y(n) = sum h(m) x(n-m) convention of the Appendix."""
    m = np.arange(-K, K + 1, dtype=np.float64)
    x = m / sigma
    he = [np.ones_like(x), x.copy()]
    for k in range(1, d):
        he.append(x * he[k] - k * he[k - 1])
    g0 = np.exp(-m * m / (2.0 * sigma * sigma)) / (sigma * math.sqrt(2.0 * math.pi))
    cg = 1.0 / g0.sum()
    return cg * (-1.0 / sigma) ** d * he[d] * g0


def colored_sg_taps(sigma: float, K: int | None = None, omega_c: float | None = None,
                    L_D: int = 1) -> np.ndarray:
    """Filter C: coloured Savitzky-Golay blur (Section 4.2).

    Minimises the coloured-noise gain (Eq 21) subject to the dc constraints
    rho^dc_{0,l} = delta_{0,l} for even l < D, via the Lagrange system of
    Eq 20 with S = T Sbar T^T (Eq 22).  Basis: pairs of unit impulses (Eq 16,
    Delta_d = 0): f_k(m) = mu_k (delta_{-k,m} + delta_{k,m}), mu_0 = 1/2, so
    h(0) = c_0 and h(+-k) = c_k.

    Defaults: K = ceil(3 sigma) (length 6 sigma + 1), omega_c = 3 / sigma.
    Returns h[0..2K] = h(-K..K)."""
    if K is None:
        K = fir_half_length(sigma, "3sigma")
    if omega_c is None:
        omega_c = 3.0 / sigma
    M = 2 * K + 1
    n_k = K + 1
    # Sbar (Eq 22b; read as m1 != m2 in the first branch).  sin(pi (m1 - m2))
    # vanishes for integer m1 != m2, leaving -sin(omega_c (m1 - m2)) / (m1 - m2).
    idx = np.arange(-K, K + 1)
    dm = (idx[:, None] - idx[None, :]).astype(np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        off = -np.sin(omega_c * dm) / dm
    Sbar = np.where(dm == 0, math.pi - omega_c, off) / math.pi
    # T (Eq 22c): T[k, K + m1] = delta_{k, |m1|}
    T = np.zeros((n_k, M))
    for m1 in range(-K, K + 1):
        T[abs(m1), K + m1] = 1.0
    S = T @ Sbar @ T.T
    # F^dc rows l = 0, 2, .., 2 L_D: l-th derivative at dc of
    # F_k(omega) = 2 mu_k cos(k omega) is 2 mu_k (-1)^{l/2} k^l.
    lbar = L_D + 1
    mu = np.ones(n_k)
    mu[0] = 0.5
    k = np.arange(n_k, dtype=np.float64)
    F = np.zeros((lbar, n_k))
    for lb in range(lbar):
        l = 2 * lb
        kl = np.where(k == 0, 1.0 if l == 0 else 0.0, k ** l)
        F[lb] = 2.0 * mu * (-1.0) ** lb * kl
    rho = np.zeros(lbar)
    rho[0] = 1.0
    kkt = np.zeros((n_k + lbar, n_k + lbar))
    kkt[:n_k, :n_k] = S
    kkt[:n_k, n_k:] = F.T
    kkt[n_k:, :n_k] = F
    rhs = np.concatenate([np.zeros(n_k), rho])
    sol = np.linalg.solve(kkt, rhs)
    c = sol[:n_k]
    return np.array([c[abs(m)] for m in range(-K, K + 1)])


def gaussian_taps_dsigma(sigma: float, K: int) -> np.ndarray:
    """d h / d sigma of gaussian_taps(sigma, K) at fixed K.  With
    g(m) = exp(-m^2 / (2 sigma^2)) (Eq 9c; its 1/(sigma sqrt(2 pi)) factor
    cancels in the renormalisation of Eq 11) and h = g / sum g:
        dg(m)/dsigma = g(m) m^2 / sigma^3,
        dh(m)/dsigma = h(m) (m^2 - sum_j h(j) j^2) / sigma^3.
    Returns dh[0..2K] = dh(-K..K)."""
    h = gaussian_taps(sigma, K)
    m2 = np.arange(-K, K + 1, dtype=np.float64) ** 2
    return h * (m2 - np.sum(h * m2)) / sigma ** 3


def colored_sg_taps_dsigma(sigma: float, K: int | None = None, L_D: int = 1) -> np.ndarray:
    """d h / d sigma of colored_sg_taps(sigma, K) at fixed K with
    omega_c = 3 / sigma (Section 4.2).  The taps solve the Lagrange system of
    Eq 20,  [S F^T; F 0] [c; lambda] = [0; rho],  in which only S depends on
    sigma, through omega_c in Sbar (Eq 22b):
        d Sbar(d) / d omega_c = -cos(omega_c d) / pi   (d = 0 included),
        d omega_c / d sigma   = -3 / sigma^2.
    Differentiating the system,  [S F^T; F 0] [dc; dlambda] = [-dS c; 0],
    so F dc = 0: the dc gain and second moment stay fixed.
    Returns dh[0..2K] = dh(-K..K)."""
    if K is None:
        K = fir_half_length(sigma, "3sigma")
    omega_c = 3.0 / sigma
    domega = -3.0 / (sigma * sigma)
    M = 2 * K + 1
    n_k = K + 1
    idx = np.arange(-K, K + 1)
    dm = (idx[:, None] - idx[None, :]).astype(np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        off = -np.sin(omega_c * dm) / dm
    Sbar = np.where(dm == 0, math.pi - omega_c, off) / math.pi
    dSbar = -np.cos(omega_c * dm) / math.pi * domega
    T = np.zeros((n_k, M))
    for m1 in range(-K, K + 1):
        T[abs(m1), K + m1] = 1.0
    S = T @ Sbar @ T.T
    dS = T @ dSbar @ T.T
    lbar = L_D + 1
    mu = np.ones(n_k)
    mu[0] = 0.5
    k = np.arange(n_k, dtype=np.float64)
    F = np.zeros((lbar, n_k))
    for lb in range(lbar):
        l = 2 * lb
        kl = np.where(k == 0, 1.0 if l == 0 else 0.0, k ** l)
        F[lb] = 2.0 * mu * (-1.0) ** lb * kl
    rho = np.zeros(lbar)
    rho[0] = 1.0
    kkt = np.zeros((n_k + lbar, n_k + lbar))
    kkt[:n_k, :n_k] = S
    kkt[:n_k, n_k:] = F.T
    kkt[n_k:, :n_k] = F
    c = np.linalg.solve(kkt, np.concatenate([np.zeros(n_k), rho]))[:n_k]
    dsol = np.linalg.solve(kkt, np.concatenate([-(dS @ c), np.zeros(lbar)]))
    dc = dsol[:n_k]
    return np.array([dc[abs(m)] for m in range(-K, K + 1)])


# --------------------------------------------------------------------------
# High-pass interpolating differentiators (Section 3.1, Eq 8, Table I)
# --------------------------------------------------------------------------

def hpf_taps(d: int) -> dict:
    """Eq 8: H_d(z) = (z - 1)^d (z + 1)^{Delta_d} / ((Delta_d + 1) z^{K_hpf}),
    K_hpf = (d + Delta_d)/2.  Expanding and reading H(z) = sum_m h(m) z^{-m}
    gives the central-difference taps of Table I.  Returns {m: h_d(m)}."""
    delta = d % 2
    poly = {0: mp.mpf(1)}
    for _ in range(d):
        poly = _lmul(poly, {1: mp.mpf(1), 0: mp.mpf(-1)})
    for _ in range(delta):
        poly = _lmul(poly, {1: mp.mpf(1), 0: mp.mpf(1)})
    k_hpf = (d + delta) // 2
    # divide by (Delta_d + 1) z^{K_hpf}; coefficient of z^e is h(-(e - K_hpf))
    return {-(e - k_hpf): float(v) / (delta + 1) for e, v in poly.items() if v != 0}
