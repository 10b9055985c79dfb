// Host-side filter design (float64) for the blob-detection filter bank.
//
//  * Repeated-pole IIR blur, Section 4.3 / Table IV (K = 3) and the same
//    constrained design with a single Nyquist constraint (K = 2).  The Table IV
//    polynomials are evaluated in factored form in terms of p and e = 1 - p so
//    that nothing cancels as p -> 1 (coarse scales).
//  * Cascade realisation (float64) of the same transfer function.
//  * Coloured Savitzky-Golay FIR (Section 4.2, Eqs 20-22) and sampled Gaussian
//    FIR (Eqs 9c, 11).
#include <cmath>
#include <complex>
#include <vector>

#include "fdvm_internal.h"

namespace fdvm {

namespace {

// value and derivative with respect to the pole p (forward-mode derivative of
// the closed forms below)
struct Dual {
    double v, d;
};
inline Dual operator+(Dual a, Dual b) { return {a.v + b.v, a.d + b.d}; }
inline Dual operator-(Dual a, Dual b) { return {a.v - b.v, a.d - b.d}; }
inline Dual operator-(Dual a) { return {-a.v, -a.d}; }
inline Dual operator*(Dual a, Dual b) { return {a.v * b.v, a.d * b.v + a.v * b.d}; }
inline Dual operator/(Dual a, Dual b) { return {a.v / b.v, (a.d * b.v - a.v * b.d) / (b.v * b.v)}; }
inline Dual operator*(double c, Dual a) { return {c * a.v, c * a.d}; }
inline Dual operator+(double c, Dual a) { return {c + a.v, a.d}; }
inline Dual operator-(double c, Dual a) { return {c - a.v, -a.d}; }
inline Dual operator/(Dual a, double c) { return {a.v / c, a.d / c}; }
inline Dual operator+(Dual a, double c) { return {a.v + c, a.d}; }
inline Dual operator-(Dual a, double c) { return {a.v - c, a.d}; }
inline double val(double x) { return x; }
inline double val(Dual x) { return x.v; }

// DE coefficients of the repeated-pole blur at pole p (e = 1 - p supplied
// separately so it keeps full relative precision).
//
// K = 3 (Table IV, factored):
//   b0    = e (8 - p - p^2) / 16
//   b+_1  = 3 e (1 + p) (3 - p^2) / 32
//   b+_2  = -3 p e (1 + p) (5 - p^2) / 32
//   b+_3  = -e (1 + p) (p^4 - 8 p^2 + 1) / 32
//   a+    = [1, -3p, 3p^2, -p^3]
// K = 2 (unit dc gain, zero 2nd moment, H(pi) = 0 on the basis
//        {p^|m|, |m| p^|m|, delta(m)}):
//   b0    = e (5 + p) / 8
//   b+_1  = e (1 + p) (2 + p) / 8
//   b+_2  = -e (1 + p) (p^2 + 4p + 1) / 16
//   a+    = [1, -2p, p^2]
template <typename T>
void de_coefficients_t(int K, T p, T e, T *b0, T bp[4], T ap[4]) {
    for (int i = 0; i < 4; ++i) bp[i] = ap[i] = 0.0 * p;
    ap[0] = 1.0 + 0.0 * p;
    const T q = 1.0 + p;
    if (K == 3) {
        *b0 = e * (8.0 - p - p * p) / 16.0;
        bp[1] = 3.0 * (e * q * (3.0 - p * p)) / 32.0;
        bp[2] = -3.0 * (p * e * q * (5.0 - p * p)) / 32.0;
        bp[3] = -(e * q * (p * p * p * p - 8.0 * (p * p) + 1.0)) / 32.0;
        ap[1] = -3.0 * p;
        ap[2] = 3.0 * (p * p);
        ap[3] = -(p * p * p);
    } else {
        *b0 = e * (5.0 + p) / 8.0;
        bp[1] = e * q * (2.0 + p) / 8.0;
        bp[2] = -(e * q * (p * p + 4.0 * p + 1.0)) / 16.0;
        ap[1] = -2.0 * p;
        ap[2] = p * p;
    }
}

// Output weights of the cascade form.  With v_k = x / (1 - p z^-1)^k and
// y+(n) = sum_k W_k v_k(n-1), matching B+(z) = sum_m b+_m z^-m gives
//   K = 3: W_1 = -e (1+p)(p^4 - 8p^2 + 1) / (32 p^2)
//          W_2 =  e^2 (1+p)^2 (p^2 + 2) / (32 p^2)
//          W_3 = -e^3 (1+p)^3 / (32 p^2)
//   K = 2: W_1 =  e (1+p)(p^2 + 4p + 1) / (16 p)
//          W_2 = -e^2 (1+p)^2 / (16 p)
template <typename T>
void cascade_weights_t(int K, T p, T e, T W[3]) {
    const T q = 1.0 + p;
    W[0] = W[1] = W[2] = 0.0 * p;
    if (K == 3) {
        W[0] = -(e * q * (p * p * p * p - 8.0 * (p * p) + 1.0)) / (32.0 * (p * p));
        W[1] = e * e * q * q * (p * p + 2.0) / (32.0 * (p * p));
        W[2] = -(e * e * e * q * q * q) / (32.0 * (p * p));
    } else {
        W[0] = e * q * (p * p + 4.0 * p + 1.0) / (16.0 * p);
        W[1] = -(e * e * q * q) / (16.0 * p);
    }
}

void de_coefficients(int K, double p, double e, double *b0, double bp[4], double ap[4]) {
    de_coefficients_t<double>(K, p, e, b0, bp, ap);
}

}  // namespace

void repeated_pole_de(int K, double p, double e, double *b0, double bp[4], double ap[4]) {
    de_coefficients(K, p, e, b0, bp, ap);
}

Cascade cascade_realisation(int K, double sigma) {
    Cascade c{};
    const double p = std::exp(-1.0 / sigma);
    const double e = -std::expm1(-1.0 / sigma);  // 1 - p to full relative precision
    double b0, bp[4], ap[4], W[3];
    de_coefficients(K, p, e, &b0, bp, ap);
    cascade_weights_t<double>(K, p, e, W);
    c.p = p;
    c.b0 = b0;
    c.sections = K;
    double ss = 1.0;
    for (int k = 0; k < MAX_SECTIONS; ++k) {
        ss /= e;
        c.w[k] = k < 3 ? W[k] : 0.0;
        c.ss[k] = ss;
    }
    c.lnp = -1.0 / sigma;
    return c;
}

// Butterworth blur, L_B = 4 (Section 4.4; the procedure of Eqs A26-A31 for
// one fewer pole pair).  Prototype H(s) = 1 / (1 + (s / wc)^4) (Eq 25 with
// L_B = 4), wc = sqrt(2 ln 2) / sigma, bilinear s = 2 (z - 1) / (z + 1).  The
// left-half-plane poles s1, conj(s1) with s1 = wc (-1 + i) / sqrt(2) map to
// p = (2 + s1) / (2 - s1) and conj(p) inside the unit circle, and
//     H(z) = K0 z^-2 (1 + z)^4 / ((1 - p/z)(1 - p'/z)(1 - p z)(1 - p' z)),
// K0 = |1 - p|^4 / 16 (unit dc gain).  Residues of H(z) z^(n-1) at p, p' (and
// at 0 for n = 0) give the two-sided impulse response
//     h(n) = 2 Re(R p^(|n| - 1)), |n| >= 1;   h(0) = 2 Re(R / p) + K0 / |p|^2,
//     R = K0 (1 + p)^4 / ((p - p')(1 - p^2)(1 - |p|^2)).
// 1 - p, Im p and 1 - |p|^2 are formed from s1 directly so that they keep full
// relative precision at coarse scales (p close to 1).
Cascade butterworth_realisation(double sigma, double *omega_c, double de_b[3], double de_a[3]) {
    using cd = std::complex<double>;
    const double wc = std::sqrt(2.0 * std::log(2.0)) / sigma;
    const cd s1 = wc * cd(-1.0, 1.0) / std::sqrt(2.0);
    const double den = std::norm(2.0 - s1);                   // |2 - s1|^2
    const cd p = (2.0 + s1) / (2.0 - s1);
    const cd omp = -2.0 * s1 / (2.0 - s1);                    // 1 - p
    const double im2 = 2.0 * 4.0 * s1.imag() / den;           // 2 Im p = (p - p') / i
    const double om2 = -8.0 * s1.real() / den;                // 1 - |p|^2
    const double m2 = 1.0 - om2;
    const double K0 = std::pow(std::abs(omp), 4) / 16.0;
    const cd R = K0 * std::pow(1.0 + p, 4) / (cd(0.0, im2) * (omp * (1.0 + p)) * om2);
    Cascade c{};
    c.p = p.real();
    c.pim = p.imag();
    c.b0 = 2.0 * (R / p).real() + K0 / m2;
    c.w[0] = 2.0 * R.real();
    c.w[1] = -2.0 * R.imag();
    const cd ss = 1.0 / omp;
    c.ss[0] = ss.real();
    c.ss[1] = ss.imag();
    c.lnp = 0.5 * std::log(m2);   // log |p|
    c.sections = CPAIR;
    if (omega_c) *omega_c = wc;
    if (de_b && de_a) {
        // y+(n) = b1 x(n-1) + b2 x(n-2) - a1 y+(n-1) - a2 y+(n-2): the impulse
        // response h(1) = b1, h(2) = b2 - a1 b1
        de_a[0] = 1.0;
        de_a[1] = -2.0 * p.real();
        de_a[2] = m2;
        de_b[0] = 0.0;
        de_b[1] = 2.0 * R.real();
        de_b[2] = 2.0 * (R * p).real() + de_a[1] * de_b[1];
    }
    return c;
}

// d h(n) / d sigma with p = exp(-1/sigma), dp/dsigma = p / sigma^2:
//   h(0) = b0(p)                        -> b0'(p) dp/dsigma
//   h(n) = sum_k W_k(p) u_k(n - 1), n >= 1, u_k(m) = C(m + k - 1, k - 1) p^m
//   d u_k / dp = (k / p) (u_{k+1} - u_k)
// so dh(n)/dsigma = sum_{k=1}^{K+1} w'_k u_k(n - 1) with
//   w'_k = dp/dsigma (W_k'(p) - (k/p) W_k + ((k-1)/p) W_{k-1}),  W_0 = W_{K+1} = 0.
Cascade sigma_derivative_realisation(int K, double sigma) {
    Cascade c = cascade_realisation(K, sigma);
    const double p = c.p;
    const Dual pd{p, 1.0};
    const Dual ed{-std::expm1(-1.0 / sigma), -1.0};
    Dual b0, bp[4], ap[4], W[3];
    de_coefficients_t<Dual>(K, pd, ed, &b0, bp, ap);
    cascade_weights_t<Dual>(K, pd, ed, W);
    const double dps = p / (sigma * sigma);
    c.b0 = b0.d * dps;
    for (int k = 1; k <= K + 1; ++k) {
        const double Wk = k <= K ? W[k - 1].v : 0.0;
        const double dWk = k <= K ? W[k - 1].d : 0.0;
        const double Wkm = k >= 2 ? W[k - 2].v : 0.0;
        c.w[k - 1] = dps * (dWk - (k / p) * Wk + ((k - 1) / p) * Wkm);
    }
    c.sections = K + 1;
    return c;
}

// Coloured Savitzky-Golay blur, Section 4.2.  Unknowns c_0..c_K with
// h(0) = c_0, h(+-k) = c_k (unit-impulse pairs, Eq 16 with Delta_d = 0).
// Minimise c^T S c (the coloured-noise gain, Eq 21) subject to F c = rho,
// F rows: dc gain (c_0 + 2 sum c_k = 1) and zero second moment
// (sum_k 2 k^2 c_k = 0), S = T Sbar T^T with
//   Sbar(d) = (pi - omega_c)/pi (d = 0),  -sin(omega_c d)/(pi d) (d != 0).
// Solved through the Schur complement: Y = S^-1 F^T (Cholesky), then
// lambda = (F Y)^-1 rho and c = Y lambda, in long double.
namespace {
typedef long double ld;
const ld PI_L = 3.141592653589793238462643383279502884L;

// S (or, with dsbar, d S / d omega_c) of the K + 1 pair coefficients; Sbar
// depends only on the lag, so its 4 K + 1 values are evaluated once
template <class F>
std::vector<ld> pair_matrix(int K, F sbar) {
    const int n = K + 1;
    std::vector<ld> lag((size_t)(4 * K + 1));
    for (int d = -2 * K; d <= 2 * K; ++d) lag[(size_t)(d + 2 * K)] = sbar(d);
    std::vector<ld> S((size_t)n * n, 0.0L);
    for (int k1 = 0; k1 < n; ++k1) {
        for (int k2 = 0; k2 < n; ++k2) {
            ld acc = 0.0L;
            const int s1n = k1 == 0 ? 1 : 2, s2n = k2 == 0 ? 1 : 2;
            for (int a = 0; a < s1n; ++a)
                for (int b = 0; b < s2n; ++b) {
                    const int m1 = a == 0 ? k1 : -k1;
                    const int m2 = b == 0 ? k2 : -k2;
                    acc += lag[(size_t)(m1 - m2 + 2 * K)];
                }
            S[(size_t)k1 * n + k2] = acc;
        }
    }
    return S;
}

struct SgSystem {
    int n;
    std::vector<ld> L;        // Cholesky factor of S (lower triangle)
    std::vector<ld> y0, y2;   // S^-1 f0, S^-1 f2
    std::vector<ld> f0, f2;   // the rows of F
    ld m00, m01, m11;         // F Y
    std::vector<ld> c;        // the solution

    void solve(std::vector<ld> &v) const {
        for (int i = 0; i < n; ++i) {
            ld s = v[i];
            for (int k = 0; k < i; ++k) s -= L[(size_t)i * n + k] * v[k];
            v[i] = s / L[(size_t)i * n + i];
        }
        for (int i = n - 1; i >= 0; --i) {
            ld s = v[i];
            for (int k = i + 1; k < n; ++k) s -= L[(size_t)k * n + i] * v[k];
            v[i] = s / L[(size_t)i * n + i];
        }
    }

    bool build(int K, double omega_c) {
        n = K + 1;
        L = pair_matrix(K, [&](int d) -> ld {
            if (d == 0) return (PI_L - (ld)omega_c) / PI_L;
            return -std::sin((ld)omega_c * (ld)d) / (PI_L * (ld)d);
        });
        for (int j = 0; j < n; ++j) {   // Cholesky S = L L^T in place
            ld d = L[(size_t)j * n + j];
            for (int k = 0; k < j; ++k) d -= L[(size_t)j * n + k] * L[(size_t)j * n + k];
            if (!(d > 0.0L)) return false;
            d = std::sqrt(d);
            L[(size_t)j * n + j] = d;
            for (int i = j + 1; i < n; ++i) {
                ld s = L[(size_t)i * n + j];
                for (int k = 0; k < j; ++k) s -= L[(size_t)i * n + k] * L[(size_t)j * n + k];
                L[(size_t)i * n + j] = s / d;
            }
        }
        f0.assign(n, 0.0L);
        f2.assign(n, 0.0L);
        for (int k = 0; k < n; ++k) {
            f0[k] = k == 0 ? 1.0L : 2.0L;
            f2[k] = 2.0L * (ld)k * (ld)k;
        }
        y0 = f0;
        y2 = f2;
        solve(y0);
        solve(y2);
        m00 = m01 = m11 = 0.0L;
        for (int k = 0; k < n; ++k) {
            m00 += f0[k] * y0[k];
            m01 += f0[k] * y2[k];
            m11 += f2[k] * y2[k];
        }
        const ld det = m00 * m11 - m01 * m01;
        const ld l0 = m11 / det, l2 = -m01 / det;  // (F Y)^-1 [1, 0]^T
        c.assign(n, 0.0L);
        for (int k = 0; k < n; ++k) c[k] = y0[k] * l0 + y2[k] * l2;
        return true;
    }
};
}  // namespace

int colored_sg_taps(double sigma, int K, double omega_c, double *taps) {
    (void)sigma;
    SgSystem sys;
    if (!sys.build(K, omega_c)) return -1;
    for (int m = -K; m <= K; ++m) taps[m + K] = (double)sys.c[m < 0 ? -m : m];
    return 0;
}

// d h / d sigma of the coloured SG blur at fixed K, omega_c = 3 / sigma.
// Only S depends on sigma; differentiating S c + F^T lambda = 0, F c = rho:
//   S dc + F^T dlambda = -dS c,  F dc = 0,
// so with z = S^-1 (dS c):  dlambda = -(F Y)^-1 F z,  dc = -z - Y dlambda.
// dS = T dSbar T^T, dSbar(d) = -cos(omega_c d) / pi * d omega_c / d sigma.
int colored_sg_dtaps(double sigma, int K, double omega_c, double *dtaps) {
    SgSystem sys;
    if (!sys.build(K, omega_c)) return -1;
    const int n = K + 1;
    const ld dw = -3.0L / ((ld)sigma * (ld)sigma);
    const std::vector<ld> dS = pair_matrix(K, [&](int d) -> ld { return -std::cos((ld)omega_c * (ld)d) / PI_L * dw; });
    std::vector<ld> z(n, 0.0L);
    for (int i = 0; i < n; ++i) {
        ld acc = 0.0L;
        for (int k = 0; k < n; ++k) acc += dS[(size_t)i * n + k] * sys.c[k];
        z[i] = acc;
    }
    sys.solve(z);
    ld fz0 = 0.0L, fz2 = 0.0L;
    for (int k = 0; k < n; ++k) {
        fz0 += sys.f0[k] * z[k];
        fz2 += sys.f2[k] * z[k];
    }
    const ld det = sys.m00 * sys.m11 - sys.m01 * sys.m01;
    const ld u0 = (sys.m11 * fz0 - sys.m01 * fz2) / det;   // (F Y)^-1 F z = -dlambda
    const ld u2 = (-sys.m01 * fz0 + sys.m00 * fz2) / det;
    for (int m = -K; m <= K; ++m) {
        const int k = m < 0 ? -m : m;
        dtaps[m + K] = (double)(-z[k] + sys.y0[k] * u0 + sys.y2[k] * u2);
    }
    return 0;
}

// Sampled Gaussian (Eq 9c) on m = -K..K renormalised to unit dc gain (Eq 11).
int gaussian_taps(double sigma, int K, double *taps) {
    double sum = 0.0;
    for (int m = -K; m <= K; ++m) {
        taps[m + K] = std::exp(-(double)m * m / (2.0 * sigma * sigma));
        sum += taps[m + K];
    }
    for (int m = -K; m <= K; ++m) taps[m + K] /= sum;
    return 0;
}

// d h / d sigma of the sampled Gaussian at fixed K: with g(m) =
// exp(-m^2 / (2 sigma^2)) and h = g / sum g, dh(m) = h(m) (m^2 - sum_j h(j) j^2)
// / sigma^3.
int gaussian_dtaps(double sigma, int K, double *dtaps) {
    gaussian_taps(sigma, K, dtaps);
    double mom = 0.0;
    for (int m = -K; m <= K; ++m) mom += dtaps[m + K] * (double)m * m;
    const double s3 = sigma * sigma * sigma;
    for (int m = -K; m <= K; ++m) dtaps[m + K] *= ((double)m * m - mom) / s3;
    return 0;
}

}  // namespace fdvm
