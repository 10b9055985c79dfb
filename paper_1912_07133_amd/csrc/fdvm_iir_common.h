// Repeated-pole IIR blur on gfx950, shared by the row pass (fdvm_iir_rows.hip)
// and the column pass (fdvm_iir_cols.hip): causal + anti-causal recursions
// (Eqs A6-A10) along rows (x) and then columns (y), replicate (Eq A32 steady
// state) or zero start.
//
// Realisation.  Each one-sided part is a cascade of K first-order sections
// with the common pole p:
//     v_1(n) = p v_1(n-1) + x(n),   v_k(n) = p v_k(n-1) + v_{k-1}(n),
//     y+(n)  = sum_k w_k v_k(n-1)
// (2K multiply-adds per sample and direction).  The states and weights are
// float64: on CDNA3/CDNA4 a float64 FMA issues at the same rate as a
// (non-packed) float32 FMA, and float64 states keep the blur at the float32
// rounding floor even where the poles crowd z = 1, which the scale-normalised
// Laplacian (gain ~8 sigma^2) would otherwise amplify.  Planes are stored as
// float32.
//
// The x-pass intermediate between the two passes is either float32 planes
// (the public two-pass API) or, on the fused routes, int32 fixed point with one
// binary exponent per image row: q = rint(r 2^e_y), e_y chosen from the row's
// input maximum and an upper bound on the blur's l1 norm so that |q| < 2^31.
// Its absolute resolution is 32-64 times finer than float32 at the frame's
// full-scale value for the same 4 bytes per sample; that matters because the
// x-pass rounding is white along x and the scale-normalised second difference
// along x multiplies it by ~8 sigma^2.
//
// The zero-input transition over n samples is
//     A^n = p^n [[1,0,0],[n,1,0],[n(n+1)/2,n,1]]
// (K = 3; the upper-left block for K = 2), so a line cut into chunks is the
// chunks filtered from a zero state and stitched with
//     state_after(chunk) = A^len state_before + zero_state_end(chunk).
#pragma once

#include <cmath>
#include <type_traits>

#include "fdvm_internal.h"

namespace fdvm {
namespace {

constexpr int ROW_WPB = 8;   // wavefronts per row-pass work-group
constexpr int CT = 48;       // rows per column tile (a multiple of 16, at most 64): 48 keeps the
                             // final pass's LDS at 12.8 KB per wavefront, 12 wavefronts per CU
constexpr int COL_WPB = 4;   // wavefronts (tiles) per column work-group

struct ScaleArgs {
    double p, inv_p, b0, sig2;   // complex pair: p, inv_p are the real parts
    double pim, inv_pim;         // complex pair: imaginary parts of p and 1/p
    double w[MAX_SECTIONS];
    double ss[MAX_SECTIONS];
    double pbit[8];    // real pole: p^(2^k), k = 0..7
    double pchunk[7];  // real pole, row pass: p^(C 2^k), k = 0..6
};

struct Args {
    int nscales;
    int boundary;
    int direct;  // row pass: rows 16-byte aligned, lanes store their chunks directly
    int pad1;
    double l1;  // upper bound on the l1 norm of every scale's 1-D blur
    ScaleArgs s[FDVM_MAX_SCALES];
};

// the x-pass intermediate: float32 planes, or int32 fixed point with the
// per-row exponents rexp (sample = q 2^-rexp[y])
template <bool FX>
struct Mid {
    const void *base;
    int64_t pitch, pstride;
    const int *rexp;
    __device__ __forceinline__ double at(int s, int y, int x) const {
        return cvt(raw(s, y, x), row_scale(y));
    }
    __device__ __forceinline__ const uint32_t *ptr(int s, int y, int x) const {
        return static_cast<const uint32_t *>(base) + (int64_t)s * pstride + (int64_t)y * pitch + x;
    }
    __device__ __forceinline__ uint32_t raw(int s, int y, int x) const {
        const int64_t o = (int64_t)s * pstride + (int64_t)y * pitch + x;
        return static_cast<const uint32_t *>(base)[o];
    }
    // 2^-rexp[y] (1 for float planes)
    __device__ __forceinline__ double row_scale(int y) const {
        if constexpr (FX)
            return ldexp(1.0, -rexp[y]);
        else
            return 1.0;
    }
    __device__ __forceinline__ double cvt(uint32_t r, double scale) const {
        if constexpr (FX)
            return (double)(int)r * scale;
        else
            return (double)__uint_as_float(r);
    }
};

// lane l's value of a float64, as a wave-uniform value
__device__ __forceinline__ double read_lane_d(double v, int l) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
    return __hiloint2double(hi, lo);
}

// ------------------------------------------------------------ recursion
// Two realisations share the kernels, selected by K:
//  * K = 2..4 real sections with the repeated pole p (states v_1..v_K):
//      v_1(n) = p v_1(n-1) + x(n),  v_k(n) = p v_k(n-1) + v_{k-1}(n);
//  * K = CPAIR, one complex section with pole p (Butterworth pole pair), held
//    as the two real states (Re v, Im v):  v(n) = p v(n-1) + x(n).
// In both cases y+(n) = sum_k w_k v_k(n-1) over the real states.
template <int K>
__device__ __forceinline__ double cas_out(const ScaleArgs &c, const double (&v)[cascade_states(K)]) {
    double y = c.w[0] * v[0];
#pragma unroll
    for (int k = 1; k < cascade_states(K); ++k) y = fma(c.w[k], v[k], y);
    return y;
}

template <int K>
__device__ __forceinline__ void cas_step(const ScaleArgs &c, double (&v)[cascade_states(K)], double x) {
    if constexpr (K == CPAIR) {
        const double re = fma(c.p, v[0], fma(-c.pim, v[1], x));
        v[1] = fma(c.p, v[1], c.pim * v[0]);
        v[0] = re;
    } else {
        v[0] = fma(c.p, v[0], x);
#pragma unroll
        for (int k = 1; k < K; ++k) v[k] = fma(c.p, v[k], v[k - 1]);
    }
}

// one step back: the state before sample x, from the state after it
template <int K>
__device__ __forceinline__ void cas_unstep(const ScaleArgs &c, double (&v)[cascade_states(K)], double x) {
    if constexpr (K == CPAIR) {
        const double d = v[0] - x;   // (d + i v1) / p
        const double re = fma(d, c.inv_p, -v[1] * c.inv_pim);
        v[1] = fma(v[1], c.inv_p, d * c.inv_pim);
        v[0] = re;
    } else {
#pragma unroll
        for (int k = K - 1; k >= 1; --k) v[k] = (v[k] - v[k - 1]) * c.inv_p;
        v[0] = (v[0] - x) * c.inv_p;
    }
}

// The zero-input transition over n samples, A^n.  Real pole: a = p^n, b = n,
//   (A^n v)_k = p^n sum_{j <= k} C(n + k - j - 1, k - j) v_j;
// complex pair: a + i b = p^n.
struct Tr {
    double a, b;
};

// v <- A^n v + z
template <int K>
__device__ __forceinline__ void cas_advance_add(Tr t, double (&v)[cascade_states(K)],
                                                const double (&z)[cascade_states(K)]) {
    if constexpr (K == CPAIR) {
        const double re = fma(t.a, v[0], fma(-t.b, v[1], z[0]));
        v[1] = fma(t.a, v[1], fma(t.b, v[0], z[1]));
        v[0] = re;
    } else {
        static_assert(K >= 2 && K <= MAX_SECTIONS, "2 to 4 sections");
        const double pn = t.a, n = t.b;
        const double c1 = n, c2 = 0.5 * n * (n + 1.0);
        const double a = v[0], b = v[1];
        if constexpr (K == 4) {
            const double c3 = c2 * (n + 2.0) * (1.0 / 3.0);
            v[3] = fma(pn, fma(c3, a, fma(c2, b, fma(c1, v[2], v[3]))), z[3]);
        }
        if constexpr (K >= 3) v[2] = fma(pn, fma(c2, a, fma(c1, b, v[2])), z[2]);
        v[1] = fma(pn, fma(c1, a, b), z[1]);
        v[0] = fma(pn, a, z[0]);
    }
}

template <int N>
__device__ __forceinline__ void set_zero(double (&v)[N]) {
#pragma unroll
    for (int k = 0; k < N; ++k) v[k] = 0.0;
}

// p^n for 0 <= n < 256 from the binary powers
__device__ __forceinline__ double pow_bits(const ScaleArgs &c, int n) {
    double r = 1.0;
#pragma unroll
    for (int k = 0; k < 8; ++k)
        if ((n >> k) & 1) r *= c.pbit[k];
    return r;
}

// p^(C m) for 0 <= m < 128 from the chunk powers
__device__ __forceinline__ double pow_chunks(const ScaleArgs &c, int m) {
    double r = 1.0;
#pragma unroll
    for (int k = 0; k < 7; ++k)
        if ((m >> k) & 1) r *= c.pchunk[k];
    return r;
}

// p^n of the complex pole, n >= 0 (wave-uniform), by repeated squaring
__device__ __forceinline__ Tr cpow(const ScaleArgs &c, int n) {
    double rr = 1.0, ri = 0.0, br = c.p, bi = c.pim;
    for (; n > 0; n >>= 1) {
        if (n & 1) {
            const double t = fma(rr, br, -ri * bi);
            ri = fma(rr, bi, ri * br);
            rr = t;
        }
        const double t = fma(br, br, -bi * bi);
        bi = 2.0 * br * bi;
        br = t;
    }
    return {rr, ri};
}

// transitions over n < 256 samples, C m samples (m < 128), C 2^l samples
template <int K>
__device__ __forceinline__ Tr tr_n(const ScaleArgs &c, int n) {
    if constexpr (K == CPAIR)
        return cpow(c, n);
    else
        return {pow_bits(c, n), (double)n};
}
template <int K, int C>
__device__ __forceinline__ Tr tr_chunks(const ScaleArgs &c, int m) {
    if constexpr (K == CPAIR)
        return cpow(c, C * m);
    else
        return {pow_chunks(c, m), (double)(C * m)};
}
template <int K, int C>
__device__ __forceinline__ Tr tr_level(const ScaleArgs &c, int l) {
    if constexpr (K == CPAIR)
        return cpow(c, C << l);
    else
        return {c.pchunk[l], (double)(C << l)};
}

template <typename T>
__device__ __forceinline__ float load_as_float(const T *p);
template <>
__device__ __forceinline__ float load_as_float<uint16_t>(const uint16_t *p) { return (float)*p; }
template <>
__device__ __forceinline__ float load_as_float<float>(const float *p) { return *p; }
template <>
__device__ __forceinline__ float load_as_float<_Float16>(const _Float16 *p) { return (float)*p; }
struct bf16_t { uint16_t bits; };
template <>
__device__ __forceinline__ float load_as_float<bf16_t>(const bf16_t *p) {
    return __uint_as_float(((uint32_t)p->bits) << 16);
}

// Orders the LDS accesses of one wavefront (its lanes exchange data through a
// region no other wavefront touches): a compiler-level barrier plus a
// wavefront-scope fence; no s_barrier.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// index of the calling wavefront in its work-group, as a wave-uniform value
// (lets the compiler keep row offsets in scalar registers)
__device__ __forceinline__ int wave_id() { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }

// Upper bound on sum_n |h(n)| of the two-sided blur: the impulse response of
// every cascade section v_k is non-negative with sum ss[k] = 1/(1-p)^k, so
// sum |h| <= |b0| + 2 sum_k |w_k| ss[k].  Complex pair: |h(n)| = |2 Re(R p^(n-1))|
// <= |w| |p|^(n-1) with |w| = 2 |R|, so sum |h| <= |b0| + 2 |w| / (1 - |p|).
// Slightly enlarged against rounding.
double l1_bound(const IirParams &prm) {
    double m = 0.0;
    for (int s = 0; s < prm.nscales; ++s) {
        const IirScaleParams &q = prm.s[s];
        double b = std::fabs(q.b0);
        if (prm.order == CPAIR)
            b += 2.0 * std::hypot(q.w[0], q.w[1]) / (1.0 - std::hypot(q.p, q.pim));
        else
            for (int k = 0; k < prm.order; ++k) b += 2.0 * std::fabs(q.w[k]) * q.ss[k];
        m = std::fmax(m, b);
    }
    return m * (1.0 + 1e-9);
}

Args make_args(const IirParams &prm, int C) {
    Args a{};
    a.nscales = prm.nscales;
    a.boundary = prm.boundary;
    a.l1 = l1_bound(prm);
    for (int s = 0; s < prm.nscales; ++s) {
        const IirScaleParams &q = prm.s[s];
        ScaleArgs &d = a.s[s];
        d.p = q.p;
        d.pim = q.pim;
        const double m2 = q.p * q.p + q.pim * q.pim;   // |p|^2
        d.inv_p = q.p / m2;
        d.inv_pim = -q.pim / m2;
        d.b0 = q.b0;
        d.sig2 = q.sig2;
        for (int k = 0; k < MAX_SECTIONS; ++k) {
            d.w[k] = q.w[k];
            d.ss[k] = q.ss[k];
        }
        for (int k = 0; k < 8 && prm.order != CPAIR; ++k)   // complex powers are formed in the kernels
            d.pbit[k] = std::exp((double)(1 << k) * q.lnp);
        for (int k = 0; k < 7 && prm.order != CPAIR; ++k)
            d.pchunk[k] = std::exp((double)C * (double)(1 << k) * q.lnp);
    }
    return a;
}

}  // namespace
}  // namespace fdvm
