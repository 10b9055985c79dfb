// Repeated-pole IIR blur on gfx950: causal + anti-causal recursions (Eqs A6-A10)
// along rows (x) and then columns (y), replicate (Eq A32 steady state) or zero
// start.
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
//
// Row pass (x): one wavefront per image row (R wavefronts for wide rows).  The
// row is staged through LDS with coalesced loads, each lane owns C consecutive
// samples, the chunk states are combined by a log-step scan across lanes (and
// across the R wavefronts through LDS), outputs go back through LDS to
// coalesced stores.  All S scales are computed from one staged copy of the row.
//
// Column pass (y), lane = column (coalesced along the row), tiles of CT rows:
//   states  -- every tile's zero-state end states (forward and backward);
//   scan    -- per column, the states are chained into the true carries that
//              enter every tile (forward from the top, backward from the bottom);
//   final   -- every tile independently: backward sweep from its bottom carry,
//              forward sweep from its top carry, output.  Optionally the
//              scale-normalised Laplacian sigma^2 (D20 + D02) is formed here in
//              float64 from the unrounded blur: y-neighbours come from the
//              sweep itself (the rows just outside the tile are recovered by
//              inverting one step of the recursion), x-neighbours from the
//              adjacent lanes (tiles overlap by one column on each side).
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
    double pbit[7];    // real pole: p^(2^k), k = 0..6
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

// p^n for 0 <= n < 128 from the binary powers
__device__ __forceinline__ double pow_bits(const ScaleArgs &c, int n) {
    double r = 1.0;
#pragma unroll
    for (int k = 0; k < 7; ++k)
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

// transitions over n < 128 samples, C m samples (m < 128), C 2^l samples
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

// ------------------------------------------------------------ row pass
template <int K, int C, int R, typename TIn, bool FX>
__global__ __launch_bounds__(ROW_WPB * 64) void iir_rows_kernel(
    const TIn *__restrict__ in, int64_t in_pitch, void *__restrict__ out_v, int64_t out_pitch,
    int64_t plane_stride, int H, int W, int *__restrict__ rexp, Args a) {
    constexpr int NS = cascade_states(K);   // real states per direction
    using Acc = std::conditional_t<FX, double, float>;
    constexpr int LP = C + 1;  // padded lane stride in LDS: conflict-free chunk reads
    __shared__ __attribute__((aligned(16))) float buf[ROW_WPB][64 * LP];
    __shared__ double tot[ROW_WPB][2][NS];
    __shared__ float rmax[ROW_WPB];
    __shared__ ScaleArgs sargs[FDVM_MAX_SCALES];

    // the scales' coefficients, copied once per work-group (a per-scale read
    // of the kernel arguments is a chain of dependent scalar loads)
    {
        constexpr int NWD = sizeof(ScaleArgs) / sizeof(double);
        const double *from = reinterpret_cast<const double *>(a.s);
        double *to = reinterpret_cast<double *>(sargs);
        for (int i = threadIdx.x; i < a.nscales * NWD; i += ROW_WPB * 64) to[i] = from[i];
    }

    const int lane = threadIdx.x & 63;
    const int wv = wave_id();
    const int r = wv % R;
    const int row = blockIdx.x * (ROW_WPB / R) + wv / R;
    const bool row_ok = row < H;
    const int seg0 = r * 64 * C;
    const int g = r * 64 + lane;          // chunk index along the row
    const int c0 = g * C;                 // first column of this lane's chunk
    const int nv = max(0, min(C, W - c0));
    const int g_last = (W - 1) / C;       // chunk holding column W-1

    const TIn *src = in + (int64_t)(row_ok ? row : 0) * in_pitch;
    float *lds = buf[wv];

    // stage the wavefront's part of the row: element j of the segment goes to
    // lds[j + j / C] (lane j / C, position j % C)
    float amax = 0.0f;
#pragma unroll 4
    for (int i = 0; i < C; ++i) {
        const int j = i * 64 + lane;
        const int col = seg0 + j;
        const float v = load_as_float(src + min(col, W - 1));
        const float t = (row_ok && col < W) ? v : 0.0f;
        lds[j + j / C] = t;
        amax = fmaxf(amax, fabsf(t));
    }
    const double x_first = load_as_float(src);
    const double x_last = load_as_float(src + (W - 1));
    if constexpr (FX) {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) amax = fmaxf(amax, __shfl_xor(amax, o, 64));
        if (lane == 0) rmax[wv] = amax;
    }
    // each wavefront stages its own segment; the R > 1 exponent needs the
    // others' row maxima, and every wavefront needs the copied coefficients
    __syncthreads();
    // fixed-point exponent of this row: |out| <= max|x| * l1 < 2^(ilogb + 1)
    int ex = 0;
    if constexpr (FX) {
        float m = 0.0f;
#pragma unroll
        for (int q = 0; q < R; ++q) m = fmaxf(m, rmax[wv - r + q]);
        const double bound = (double)m * a.l1;
        ex = bound > 0.0 ? 30 - ilogb(bound) : 0;
        if (row_ok && r == 0 && lane == 0) rexp[row] = ex;
    }
    float xs[C];
#pragma unroll
    for (int j = 0; j < C; ++j) xs[j] = lds[lane * LP + j];
    const bool full_wave = __all(nv == C);

    // wavefronts start at different scales so that their stores do not all
    // arrive at once (the R wavefronts of a row step through the scales together)
    const int rot = (R == 1 ? row : (int)blockIdx.x) % a.nscales;
    for (int si = 0; si < a.nscales; ++si) {
        const int s = si + rot < a.nscales ? si + rot : si + rot - a.nscales;
        const ScaleArgs &cf = sargs[s];
        // ---- zero-state chunk states
        double zf[NS], zb[NS];
        set_zero(zf);
        set_zero(zb);
#pragma unroll
        for (int j = 0; j < C; ++j) cas_step<K>(cf, zf, (double)xs[j]);
#pragma unroll
        for (int j = C - 1; j >= 0; --j) cas_step<K>(cf, zb, (double)xs[j]);

        double init_l[NS], init_r[NS];
#pragma unroll
        for (int k = 0; k < NS; ++k) {
            init_l[k] = a.boundary == FDVM_BC_REPLICATE ? x_first * cf.ss[k] : 0.0;
            init_r[k] = a.boundary == FDVM_BC_REPLICATE ? x_last * cf.ss[k] : 0.0;
        }
        // forward elements: chunk 0 absorbs the left start state
        double sf[NS];
#pragma unroll
        for (int k = 0; k < NS; ++k) sf[k] = zf[k];
        if (g == 0) {
            double t[NS];
#pragma unroll
            for (int k = 0; k < NS; ++k) t[k] = init_l[k];
            cas_advance_add<K>(tr_level<K, C>(cf, 0), t, zf);
#pragma unroll
            for (int k = 0; k < NS; ++k) sf[k] = t[k];
        }
        // backward elements: the chunk holding column W-1 absorbs the right
        // start state; chunks past the end contribute nothing
        double sb[NS];
#pragma unroll
        for (int k = 0; k < NS; ++k) sb[k] = g > g_last ? 0.0 : zb[k];
        if (g == g_last) {
            double t[NS];
#pragma unroll
            for (int k = 0; k < NS; ++k) t[k] = init_r[k];
            cas_advance_add<K>(tr_n<K>(cf, nv), t, zb);
#pragma unroll
            for (int k = 0; k < NS; ++k) sb[k] = t[k];
        }
        // ---- intra-wavefront inclusive scans (forward from the left,
        // backward from the right): S_l <- A^(C d) S_(l-d) + S_l
#pragma unroll
        for (int lvl = 0; lvl < 6; ++lvl) {
            const int d = 1 << lvl;
            const Tr tl = tr_level<K, C>(cf, lvl);
            double tf[NS], tb[NS];
#pragma unroll
            for (int k = 0; k < NS; ++k) {
                tf[k] = __shfl_up(sf[k], d, 64);
                tb[k] = __shfl_down(sb[k], d, 64);
            }
            cas_advance_add<K>(tl, tf, sf);
            cas_advance_add<K>(tl, tb, sb);
#pragma unroll
            for (int k = 0; k < NS; ++k) {
                if (lane >= d) sf[k] = tf[k];
                if (lane + d < 64) sb[k] = tb[k];
            }
        }
        // ---- across the R wavefronts of the row
        double cwf[NS], cwb[NS];  // states entering this wavefront's segment
        set_zero(cwf);
        set_zero(cwb);
        if constexpr (R > 1) {
            if (lane == 63) {
#pragma unroll
                for (int k = 0; k < NS; ++k) tot[wv][0][k] = sf[k];
            }
            if (lane == 0) {
#pragma unroll
                for (int k = 0; k < NS; ++k) tot[wv][1][k] = sb[k];
            }
            __syncthreads();
            const int base = wv - r;
            const Tr tw = tr_level<K, C>(cf, 6);
            for (int q = 0; q < r; ++q) {
                double z[NS];
#pragma unroll
                for (int k = 0; k < NS; ++k) z[k] = tot[base + q][0][k];
                cas_advance_add<K>(tw, cwf, z);
            }
            for (int q = R - 1; q > r; --q) {
                double z[NS];
#pragma unroll
                for (int k = 0; k < NS; ++k) z[k] = tot[base + q][1][k];
                cas_advance_add<K>(tw, cwb, z);
            }
            __syncthreads();
            double t1[NS], t2[NS];
#pragma unroll
            for (int k = 0; k < NS; ++k) {
                t1[k] = cwf[k];
                t2[k] = cwb[k];
            }
            cas_advance_add<K>(tr_chunks<K, C>(cf, lane + 1), t1, sf);
            cas_advance_add<K>(tr_chunks<K, C>(cf, 64 - lane), t2, sb);
#pragma unroll
            for (int k = 0; k < NS; ++k) {
                sf[k] = t1[k];
                sb[k] = t2[k];
            }
        }
        // carry into each chunk: exclusive scans
        double vf[NS], vb[NS];
#pragma unroll
        for (int k = 0; k < NS; ++k) {
            const double up = __shfl_up(sf[k], 1, 64);
            const double dn = __shfl_down(sb[k], 1, 64);
            vf[k] = lane == 0 ? cwf[k] : up;
            vb[k] = lane == 63 ? cwb[k] : dn;
            if (g == 0) vf[k] = init_l[k];
            if (g == g_last) vb[k] = init_r[k];
        }
        // ---- final outputs of the chunk
        // y-(n) + b0 x(n) is kept as float32 until y+(n) is added in float64
        // (its rounding adds ~1/4 ulp to the 1/2 ulp of the stored output)
        // (float64 throughout for the fixed-point intermediate)
        Acc ys[C];
        if (full_wave) {
#pragma unroll
            for (int j = C - 1; j >= 0; --j) {
                ys[j] = (Acc)fma(cf.b0, (double)xs[j], cas_out<K>(cf, vb));
                cas_step<K>(cf, vb, (double)xs[j]);
            }
#pragma unroll
            for (int j = 0; j < C; ++j) {
                ys[j] = (Acc)((double)ys[j] + cas_out<K>(cf, vf));
                cas_step<K>(cf, vf, (double)xs[j]);
            }
        } else {
#pragma unroll
            for (int j = C - 1; j >= 0; --j) {
                if (j < nv) {
                    ys[j] = (Acc)fma(cf.b0, (double)xs[j], cas_out<K>(cf, vb));
                    cas_step<K>(cf, vb, (double)xs[j]);
                } else {
                    ys[j] = (Acc)0;
                }
            }
#pragma unroll
            for (int j = 0; j < C; ++j) {
                if (j < nv) {
                    ys[j] = (Acc)((double)ys[j] + cas_out<K>(cf, vf));
                    cas_step<K>(cf, vf, (double)xs[j]);
                }
            }
        }
        uint32_t *dst = static_cast<uint32_t *>(out_v) + (int64_t)s * plane_stride +
                        (int64_t)(row_ok ? row : 0) * out_pitch;
        auto word = [&](int j) -> uint32_t {
            if constexpr (FX)
                return (uint32_t)(int)rint(ldexp((double)ys[j], ex));   // |ys 2^ex| < 2^31 by the choice of ex
            else
                return __float_as_uint(ys[j]);
        };
        if (a.direct) {
            // 16-byte aligned rows.  Groups of NB = C / 4 lanes exchange their
            // 16-byte blocks through this wavefront's LDS segment (an NB x NB
            // transpose, XOR-swizzled against bank conflicts), so that every
            // store instruction writes whole runs of 16 NB bytes; a group that
            // reaches past the row's end stores its own words instead.
            constexpr int NB = C / 4;
            uint4 *l16 = reinterpret_cast<uint4 *>(lds);
            const int gr = lane % NB;  // lane within its group
            const int gl = lane - gr;  // first lane of the group
#pragma unroll
            for (int i = 0; i < NB; ++i)
                l16[lane * NB + (i ^ gr)] = make_uint4(word(4 * i), word(4 * i + 1), word(4 * i + 2), word(4 * i + 3));
            wave_lds_sync();
            if (row_ok) {
                if (seg0 + (gl + NB) * C <= W) {
#pragma unroll
                    for (int i = 0; i < NB; ++i)
                        *reinterpret_cast<uint4 *>(dst + seg0 + (gl + i) * C + 4 * gr) = l16[(gl + i) * NB + (gr ^ i)];
                } else {
#pragma unroll
                    for (int j = 0; j < C; ++j)
                        if (j < nv) dst[c0 + j] = word(j);
                }
            }
            wave_lds_sync();
            continue;
        }
        // ---- back through LDS (as raw 32-bit words) to coalesced stores
#pragma unroll
        for (int j = 0; j < C; ++j) lds[lane * LP + j] = __uint_as_float(word(j));
        wave_lds_sync();  // the segment in LDS belongs to this wavefront alone
#pragma unroll 4
        for (int i = 0; i < C; ++i) {
            const int j = i * 64 + lane;
            const int col = seg0 + j;
            if (row_ok && col < W) dst[col] = __float_as_uint(lds[j + j / C]);
        }
        wave_lds_sync();
    }
}

// ------------------------------------------------------------ column pass
// (a) zero-state end states of every CT-row tile (float64).  st layout:
//     st[((s * nty + ty) * 2K + k) * W + x], k < K forward, k >= K backward.
template <int K, bool FX>
__global__ __launch_bounds__(COL_WPB * 64) void iir_col_states_kernel(Mid<FX> m, int H, int W, int nty,
                                                                      double *__restrict__ st, Args a) {
    constexpr int NS = cascade_states(K);
    const int lane = threadIdx.x & 63;
    const int ty = blockIdx.y * COL_WPB + wave_id();
    const int s = blockIdx.z;
    const int col = blockIdx.x * 64 + lane;
    if (ty >= nty) return;
    const int ccol = min(col, W - 1);
    const ScaleArgs &cf = a.s[s];
    const int y0 = ty * CT;
    static_assert(CT <= 64, "one row scale per lane");
    const double lsc = m.row_scale(min(y0 + lane, H - 1));  // lane j: scale of row y0 + j
    uint32_t xs[CT];
#pragma unroll
    for (int j = 0; j < CT; ++j) {
        const int y = y0 + j;
        const uint32_t v = m.raw(s, min(y, H - 1), ccol);
        xs[j] = y < H ? v : 0u;  // zeros (in either format) after the last row
    }                            // leave the backward zero state exact
    double zf[NS], zb[NS];
    set_zero(zf);
    set_zero(zb);
#pragma unroll
    for (int j = 0; j < CT; ++j) cas_step<K>(cf, zf, m.cvt(xs[j], read_lane_d(lsc, j)));
#pragma unroll
    for (int j = CT - 1; j >= 0; --j) cas_step<K>(cf, zb, m.cvt(xs[j], read_lane_d(lsc, j)));
    if (col < W) {
        double *o = st + ((int64_t)(s * nty + ty) * 2 * NS) * W + col;
#pragma unroll
        for (int k = 0; k < NS; ++k) {
            o[(int64_t)k * W] = zf[k];
            o[(int64_t)(NS + k) * W] = zb[k];
        }
    }
}

// (b) carries: in place, every tile's forward zero state becomes the forward
// state entering the tile from above, every backward zero state the backward
// state entering it from below.
constexpr int SCAN_T = 64;  // threads (columns) per scan work-group

template <int K, bool FX>
__global__ __launch_bounds__(SCAN_T) void iir_col_scan_kernel(Mid<FX> m, int H, int W, int nty,
                                                              double *__restrict__ st, Args a) {
    constexpr int NS = cascade_states(K);
    constexpr int U = 8;  // tiles whose states are fetched together
    const int col = blockIdx.x * SCAN_T + threadIdx.x;
    const int s = blockIdx.y;
    const int dir = blockIdx.z;  // 0: forward from the top, 1: backward from the bottom
    if (col >= W) return;
    const ScaleArgs &cf = a.s[s];
    const bool rep = a.boundary == FDVM_BC_REPLICATE;
    const double xe = m.at(s, dir == 0 ? 0 : H - 1, col);
    double *base = st + (int64_t)s * nty * 2 * NS * W + (int64_t)dir * NS * W + col;
    const int64_t tstride = (int64_t)2 * NS * W;
    double c[NS];
#pragma unroll
    for (int k = 0; k < NS; ++k) c[k] = rep ? xe * cf.ss[k] : 0.0;
    const Tr tt = tr_n<K>(cf, CT);  // A^64
    for (int i0 = 0; i0 < nty; i0 += U) {
        double z[U][NS];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = i0 + u;
            const int ty = dir == 0 ? i : nty - 1 - i;
#pragma unroll
            for (int k = 0; k < NS; ++k) z[u][k] = i < nty ? base[ty * tstride + (int64_t)k * W] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = i0 + u;
            if (i >= nty) break;
            const int ty = dir == 0 ? i : nty - 1 - i;
#pragma unroll
            for (int k = 0; k < NS; ++k) base[ty * tstride + (int64_t)k * W] = c[k];
            const int len = min(CT, H - ty * CT);
            cas_advance_add<K>(len == CT ? tt : tr_n<K>(cf, len), c, z[u]);
        }
    }
}

// value of lane l-1 (left) / l+1 (right) of a double across the whole
// wavefront (gfx9 DPP wave_shr:1 / wave_shl:1 on both halves); the end lanes
// read 0, which only reaches their own results (lanes 0 and 63 of a
// Laplacian tile are overlap columns that are never written)
__device__ __forceinline__ double lane_left_d(double v) {
    const int lo = __double2loint(v), hi = __double2hiint(v);
    return __hiloint2double(__builtin_amdgcn_mov_dpp(hi, 0x138, 0xf, 0xf, true),
                            __builtin_amdgcn_mov_dpp(lo, 0x138, 0xf, 0xf, true));
}
__device__ __forceinline__ double lane_right_d(double v) {
    const int lo = __double2loint(v), hi = __double2hiint(v);
    return __hiloint2double(__builtin_amdgcn_mov_dpp(hi, 0x130, 0xf, 0xf, true),
                            __builtin_amdgcn_mov_dpp(lo, 0x130, 0xf, 0xf, true));
}

// Hardware work-group ids are dealt round-robin to the 8 XCDs (each with its
// own L2).  Map them so that every XCD gets one contiguous run of logical
// tiles: neighbouring column tiles (which share the cache lines at their
// edges, both read and written) then meet in the same L2.
__device__ __forceinline__ int xcd_logical_block(int hw, int n) {
    constexpr int NX = 8;
    const int xcd = hw % NX, slot = hw / NX;
    const int q = n / NX, r = n % NX;
    return xcd * q + min(xcd, r) + slot;
}

// copy one row of 64 lanes x 4 bytes from global memory straight into LDS
// (no register round trip); the data is there after "s_waitcnt vmcnt(0)"
__device__ __forceinline__ void row_to_lds(const void *g, uint32_t *l) {
    __builtin_amdgcn_global_load_lds(g, (__attribute__((address_space(3))) void *)l, 4, 0, 0);
}
__device__ __forceinline__ void wait_lds_dma() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

// (c) final pass of one CT-row tile per wavefront.  LAP = false: writes the
// blur; in place is allowed (a tile reads and writes only its own rows, and it
// stages all of them before its first write).  LAP = true: writes
// sigma^2 (D20 + D02) of the blur; lanes cover columns x0 - 1 .. x0 + 62 and
// lanes 1..62 write (in and out must not overlap).
// The tile (plus the rows just above and below it for LAP) is first copied
// into LDS with direct global-to-LDS loads, so the whole tile is in flight at
// once and no registers hold it.  It is then finished in bands of 16 rows
// (QT) so that only 16 float64 partial outputs are live: one backward sweep
// over all bands but the first records the state entering each band from
// below; then every band, top first, is swept backwards from its recorded
// state and finished by the forward sweep, which runs through the whole tile.
constexpr int FIN_WPB = 4;  // wavefronts (tiles) per final-pass work-group
constexpr int FIN_BLUR = 0, FIN_LAPLACIAN = 1, FIN_HESSIAN = 2;

template <int K, int MODE, bool FX>
__global__ __launch_bounds__(FIN_WPB * 64) void iir_col_final_kernel(
    Mid<FX> m, float *out, int64_t out_pitch, int64_t out_plane_stride, int H, int W, int nty, int ntx,
    const double *__restrict__ st, Args a, HessArgs hz) {
    constexpr int NS = cascade_states(K);
    constexpr bool LAP = MODE != FIN_BLUR;   // second differences need the neighbour rows and columns
    constexpr int QT = 16;
    constexpr int NQ = CT / QT;
    constexpr int NR = LAP ? CT + 2 : CT;   // staged rows: (y0 - 1 if LAP) .. y0 + CT - 1 (.. y0 + CT if LAP)
    constexpr int R0 = LAP ? 1 : 0;         // LDS row of tile row 0
    __shared__ uint32_t tiles[FIN_WPB][NR * 64];
    const int lane = threadIdx.x & 63;
    const int wv = wave_id();
    // logical block -> (column tile, group of FIN_WPB row tiles, scale), column tile fastest
    const int ntyg = (nty + FIN_WPB - 1) / FIN_WPB;
    const int lb = xcd_logical_block(blockIdx.x, ntx * ntyg * a.nscales);
    const int tx = lb % ntx;
    const int s = lb / (ntx * ntyg);
    const int ty = ((lb / ntx) % ntyg) * FIN_WPB + wv;
    const int col = LAP ? tx * 62 - 1 + lane : tx * 64 + lane;
    if (ty >= nty) return;
    const int ccol = min(max(col, 0), W - 1);
    const ScaleArgs &cf = a.s[s];
    const int y0 = ty * CT;
    const int y1 = min(y0 + CT, H);
    const int len = y1 - y0;
    uint32_t *lt = tiles[wv];
    // rows outside the image are clamped copies; they are never used as data
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        const int y = min(max(y0 - R0 + r, 0), H - 1);
        row_to_lds(m.ptr(s, y, ccol), lt + r * 64);
    }
    const double lsc = m.row_scale(min(y0 + lane, H - 1));  // lane j: scale of row y0 + j
    double vf[NS], ub[NQ][NS];
    {
        const double *o = st + ((int64_t)(s * nty + ty) * 2 * NS) * W + ccol;
#pragma unroll
        for (int k = 0; k < NS; ++k) {
            vf[k] = o[(int64_t)k * W];
            ub[NQ - 1][k] = o[(int64_t)(NS + k) * W];
        }
    }
    double sc_above = 1.0, sc_below = 1.0;
    if constexpr (LAP && FX) {
        sc_above = m.row_scale(max(y0 - 1, 0));
        sc_below = m.row_scale(min(y1, H - 1));
    }
    wait_lds_dma();
    // sample of tile row j (j = -1 and j = len only with LAP)
    auto X = [&](int j) { return m.cvt(lt[(j + R0) * 64 + lane], read_lane_d(lsc, j)); };
    float *dst = out + (int64_t)s * out_plane_stride;
    const double sig2 = cf.sig2;
    const bool wr = LAP ? (lane >= 1 && lane <= 62 && col < W) : col < W;
    // y- of row y1 (below the tile) for the Laplacian's last row
    double t_bot = 0.0;
    if (LAP && y1 < H) {
        const double xb = m.cvt(lt[(len + R0) * 64 + lane], sc_below);
        double u[NS];
#pragma unroll
        for (int k = 0; k < NS; ++k) u[k] = ub[NQ - 1][k];
        cas_unstep<K>(cf, u, xb);  // state before row y1 (from below)
        t_bot = fma(cf.b0, xb, cas_out<K>(cf, u));
    }

    auto body = [&](auto full_tag) {
        constexpr bool FULL = decltype(full_tag)::value;
        auto valid = [&](int j) { return FULL || j < len; };
        double xd[QT];              // the samples of one quarter
        double t[QT];               // y-(n) + b0 x(n) of one quarter
        double bm = 0.0, bc = 0.0;  // sliding B(n-1), B(n) for the Laplacian
        auto load_q = [&](int q) {
#pragma unroll
            for (int i = 0; i < QT; ++i) xd[i] = valid(q * QT + i) ? X(q * QT + i) : 0.0;
        };
        auto emit = [&](int y, double bmv, double bcv, double bnv) {
            const double bl = lane_left_d(bcv);
            const double br = lane_right_d(bcv);
            if constexpr (MODE == FIN_LAPLACIAN) {
                const double v = sig2 * fma(-4.0, bcv, (bl + br) + (bmv + bnv));
                if (wr) dst[(int64_t)y * out_pitch + col] = (float)v;
            } else if constexpr (MODE == FIN_HESSIAN) {
                // Table I taps: d = 2 central second differences, d = 1 half
                // central differences, D11 = D10 of D01 (Eqs 26-27)
                const double d20 = (bl + br) - 2.0 * bcv;
                const double d02 = (bmv + bnv) - 2.0 * bcv;
                const double d10 = 0.5 * (br - bl);
                const double d01 = 0.5 * (bnv - bmv);
                const double d11 = 0.25 * ((lane_right_d(bnv) - lane_left_d(bnv)) - (lane_right_d(bmv) - lane_left_d(bmv)));
                const double det = fma(d20, d02, -d11 * d11);
                const double ndet = sig2 * sig2 * det;
                bool hit = ndet > (double)hz.t1;
                if (hz.t2 > 0.0f) {
                    const double dx = (d01 * d11 - d02 * d10) / det;
                    const double dy = (d10 * d11 - d20 * d01) / det;
                    hit = hit && dx * dx + dy * dy < (double)hz.t2 * (double)hz.t2;
                }
                const bool inside = wr && col >= hz.border && col < W - hz.border && y >= hz.border &&
                                    y < H - hz.border;
                hit = hit && inside;
                const unsigned long long bits = __ballot(hit) >> 1;            // lanes 1..62 -> bits 0..61
                const unsigned long long bright = __ballot(hit && d20 < 0.0) >> 1;
                if (wr) dst[(int64_t)y * out_pitch + col] = (float)ndet;
                if (lane == 0) {
                    const int64_t wi = ((int64_t)s * H + y) * ntx + tx;
                    hz.mask[wi] = bits;
                    hz.pmask[wi] = bright;
                }
            }
        };
        // states entering each quarter from below
#pragma unroll
        for (int q = NQ - 1; q >= 1; --q) {
#pragma unroll
            for (int k = 0; k < NS; ++k) ub[q - 1][k] = ub[q][k];
            if (FULL || q * QT < len) {
                load_q(q);
#pragma unroll
                for (int i = QT - 1; i >= 0; --i)
                    if (valid(q * QT + i)) cas_step<K>(cf, ub[q - 1], xd[i]);
            }
        }
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            if (!(FULL || q * QT < len)) break;
            load_q(q);
            double u[NS];
#pragma unroll
            for (int k = 0; k < NS; ++k) u[k] = ub[q][k];
#pragma unroll
            for (int i = QT - 1; i >= 0; --i) {
                if (valid(q * QT + i)) {
                    t[i] = fma(cf.b0, xd[i], cas_out<K>(cf, u));
                    cas_step<K>(cf, u, xd[i]);
                }
            }
            if constexpr (LAP) {
                if (q == 0 && y0 > 0) {  // B of the row above the tile; u is u(y0)
                    const double xa = m.cvt(lt[lane], sc_above);
                    const double ta = fma(cf.b0, xa, cas_out<K>(cf, u));
                    double v[NS];
#pragma unroll
                    for (int k = 0; k < NS; ++k) v[k] = vf[k];
                    cas_unstep<K>(cf, v, xa);  // forward state before row y0-1
                    bm = ta + cas_out<K>(cf, v);
                }
            }
#pragma unroll
            for (int i = 0; i < QT; ++i) {
                const int j = q * QT + i;
                if (valid(j)) {
                    const double b = t[i] + cas_out<K>(cf, vf);
                    cas_step<K>(cf, vf, xd[i]);
                    if constexpr (!LAP) {
                        if (wr) dst[(int64_t)(y0 + j) * out_pitch + col] = (float)b;
                    } else {
                        if (j == 0) {
                            bc = b;
                            if (y0 == 0) bm = b;  // clamp above the image
                        } else {
                            emit(y0 + j - 1, bm, bc, b);
                            bm = bc;
                            bc = b;
                        }
                    }
                }
            }
        }
        if constexpr (LAP) {
            // the row below the tile: B(y1) = y-(y1) + b0 x(y1) + W v(y1 - 1)
            const double bn = y1 < H ? t_bot + cas_out<K>(cf, vf) : bc;
            emit(y1 - 1, bm, bc, bn);
        }
    };
    if (len == CT)
        body(std::true_type{});
    else
        body(std::false_type{});
}

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
        for (int k = 0; k < 7 && prm.order != CPAIR; ++k) {   // complex powers are formed in the kernels
            d.pbit[k] = std::exp((double)(1 << k) * q.lnp);
            d.pchunk[k] = std::exp((double)C * (double)(1 << k) * q.lnp);
        }
    }
    return a;
}

template <int K, int C, int R, typename T, bool FX>
hipError_t launch_rows_t(const void *in, int64_t H, int64_t W, int64_t in_pitch, void *out, int64_t out_pitch,
                         int64_t plane_stride, int *rexp, const IirParams &prm, hipStream_t st) {
    Args a = make_args(prm, C);
    a.direct = ((uintptr_t)out % 16 == 0 && out_pitch % 4 == 0 && plane_stride % 4 == 0) ? 1 : 0;
    const int rows_per_block = ROW_WPB / R;
    dim3 grid((unsigned)((H + rows_per_block - 1) / rows_per_block));
    hipLaunchKernelGGL((iir_rows_kernel<K, C, R, T, FX>), grid, dim3(ROW_WPB * 64), 0, st,
                       static_cast<const T *>(in), in_pitch, out, out_pitch, plane_stride, (int)H, (int)W, rexp, a);
    return hipGetLastError();
}

// chunk length C per lane and wavefronts per row R with 64 C R >= W,
// R in {1, 2, 4, 8}: by default the smallest C in {8, 16, 32} (R = 1) or
// C = 32 with the smallest R; with chunk = 8, 16 or 32 (fixed-point
// intermediate only) that C with the smallest R
template <int K, typename T>
hipError_t launch_rows_k(const void *in, int64_t H, int64_t W, int64_t in_pitch, void *out, int64_t out_pitch,
                         int64_t plane_stride, int *rexp, int chunk, const IirParams &prm, hipStream_t st) {
#define FDVM_ROWS_CR(CC, RR, FXV)                                                                       \
    return launch_rows_t<K, CC, RR, T, FXV>(in, H, W, in_pitch, out, out_pitch, plane_stride, rexp, prm, st)
    if (rexp && chunk != 0) {
        const int64_t need = (W + 64 * chunk - 1) / (64 * chunk);  // wavefronts per row
        if (chunk == 8) {
            if (need <= 1) FDVM_ROWS_CR(8, 1, true);
            if (need <= 2) FDVM_ROWS_CR(8, 2, true);
            if (need <= 4) FDVM_ROWS_CR(8, 4, true);
            if (need <= 8) FDVM_ROWS_CR(8, 8, true);
        } else if (chunk == 16) {
            if (need <= 1) FDVM_ROWS_CR(16, 1, true);
            if (need <= 2) FDVM_ROWS_CR(16, 2, true);
            if (need <= 4) FDVM_ROWS_CR(16, 4, true);
            if (need <= 8) FDVM_ROWS_CR(16, 8, true);
        } else if (chunk == 32) {
            if (need <= 1) FDVM_ROWS_CR(32, 1, true);
            if (need <= 2) FDVM_ROWS_CR(32, 2, true);
            if (need <= 4) FDVM_ROWS_CR(32, 4, true);
            if (need <= 8) FDVM_ROWS_CR(32, 8, true);
        }
        return hipErrorInvalidValue;
    }
    if (rexp) {
        if (W <= 64 * 8) FDVM_ROWS_CR(8, 1, true);
        if (W <= 64 * 16) FDVM_ROWS_CR(16, 1, true);
        if (W <= 64 * 32) FDVM_ROWS_CR(32, 1, true);
        if (W <= 2 * 64 * 32) FDVM_ROWS_CR(32, 2, true);
        if (W <= 4 * 64 * 32) FDVM_ROWS_CR(32, 4, true);
        if (W <= 8 * 64 * 32) FDVM_ROWS_CR(32, 8, true);
    } else {
        if (W <= 64 * 8) FDVM_ROWS_CR(8, 1, false);
        if (W <= 64 * 16) FDVM_ROWS_CR(16, 1, false);
        if (W <= 64 * 32) FDVM_ROWS_CR(32, 1, false);
        if (W <= 2 * 64 * 32) FDVM_ROWS_CR(32, 2, false);
        if (W <= 4 * 64 * 32) FDVM_ROWS_CR(32, 4, false);
        if (W <= 8 * 64 * 32) FDVM_ROWS_CR(32, 8, false);
    }
#undef FDVM_ROWS_CR
    return hipErrorInvalidValue;
}

// float32-plane row pass only (used for the 4-section sigma derivative)
template <int K, typename T>
hipError_t launch_rows_f32out(const void *in, int64_t H, int64_t W, int64_t in_pitch, void *out, int64_t out_pitch,
                              int64_t plane_stride, const IirParams &prm, hipStream_t st) {
#define FDVM_ROWS_CR(CC, RR) \
    return launch_rows_t<K, CC, RR, T, false>(in, H, W, in_pitch, out, out_pitch, plane_stride, nullptr, prm, st)
    if (W <= 64 * 8) FDVM_ROWS_CR(8, 1);
    if (W <= 64 * 16) FDVM_ROWS_CR(16, 1);
    if (W <= 64 * 32) FDVM_ROWS_CR(32, 1);
    if (W <= 2 * 64 * 32) FDVM_ROWS_CR(32, 2);
    if (W <= 4 * 64 * 32) FDVM_ROWS_CR(32, 4);
    if (W <= 8 * 64 * 32) FDVM_ROWS_CR(32, 8);
#undef FDVM_ROWS_CR
    return hipErrorInvalidValue;
}

template <int K, bool FX>
hipError_t launch_cols_kx(Mid<FX> m, float *out, int64_t H, int64_t W, int64_t pitch, int64_t plane_stride,
                          int mode, const HessArgs *hp, const IirParams &prm, double *st, hipStream_t stream) {
    Args a = make_args(prm, 1);
    const int nty = (int)((H + CT - 1) / CT);
    const unsigned S = (unsigned)prm.nscales;
    dim3 g1((unsigned)((W + 63) / 64), (unsigned)((nty + COL_WPB - 1) / COL_WPB), S);
    hipLaunchKernelGGL((iir_col_states_kernel<K, FX>), g1, dim3(COL_WPB * 64), 0, stream, m, (int)H, (int)W, nty,
                       st, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    dim3 g2((unsigned)((W + SCAN_T - 1) / SCAN_T), S, 2);
    hipLaunchKernelGGL((iir_col_scan_kernel<K, FX>), g2, dim3(SCAN_T), 0, stream, m, (int)H, (int)W, nty, st, a);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int ntyg = (nty + FIN_WPB - 1) / FIN_WPB;
    const HessArgs hz = hp ? *hp : HessArgs{};
    if (mode != FIN_BLUR) {
        const int ntx = (int)((W + 61) / 62);
        const unsigned nb = (unsigned)ntx * (unsigned)ntyg * S;
        if (mode == FIN_HESSIAN)
            hipLaunchKernelGGL((iir_col_final_kernel<K, FIN_HESSIAN, FX>), dim3(nb), dim3(FIN_WPB * 64), 0, stream,
                               m, out, pitch, plane_stride, (int)H, (int)W, nty, ntx, st, a, hz);
        else
            hipLaunchKernelGGL((iir_col_final_kernel<K, FIN_LAPLACIAN, FX>), dim3(nb), dim3(FIN_WPB * 64), 0,
                               stream, m, out, pitch, plane_stride, (int)H, (int)W, nty, ntx, st, a, hz);
    } else {
        const int ntx = (int)((W + 63) / 64);
        const unsigned nb = (unsigned)ntx * (unsigned)ntyg * S;
        hipLaunchKernelGGL((iir_col_final_kernel<K, FIN_BLUR, FX>), dim3(nb), dim3(FIN_WPB * 64), 0, stream, m, out,
                           pitch, plane_stride, (int)H, (int)W, nty, ntx, st, a, hz);
    }
    return hipGetLastError();
}

template <int K>
hipError_t launch_cols_k(const void *in, int64_t in_pitch, int64_t in_plane_stride, const int *rexp, float *out,
                         int64_t H, int64_t W, int64_t pitch, int64_t plane_stride, int mode, const HessArgs *hp,
                         const IirParams &prm, double *st, hipStream_t stream) {
    if (rexp)
        return launch_cols_kx<K, true>(Mid<true>{in, in_pitch, in_plane_stride, rexp}, out, H, W, pitch,
                                       plane_stride, mode, hp, prm, st, stream);
    return launch_cols_kx<K, false>(Mid<false>{in, in_pitch, in_plane_stride, nullptr}, out, H, W, pitch,
                                    plane_stride, mode, hp, prm, st, stream);
}

}  // namespace

hipError_t launch_iir_rows(const void *in, int dtype, int64_t H, int64_t W, int64_t in_pitch, void *out,
                           int64_t out_pitch, int64_t plane_stride, int *rexp, int chunk, const IirParams &prm,
                           hipStream_t st) {
#define FDVM_ROWS_DT(KK)                                                                                    \
    switch (dtype) {                                                                                        \
        case FDVM_U16:                                                                                      \
            return launch_rows_k<KK, uint16_t>(in, H, W, in_pitch, out, out_pitch, plane_stride, rexp, chunk, prm, st); \
        case FDVM_F32:                                                                                      \
            return launch_rows_k<KK, float>(in, H, W, in_pitch, out, out_pitch, plane_stride, rexp, chunk, prm, st);    \
        case FDVM_F16:                                                                                      \
            return launch_rows_k<KK, _Float16>(in, H, W, in_pitch, out, out_pitch, plane_stride, rexp, chunk, prm, st); \
        case FDVM_BF16:                                                                                     \
            return launch_rows_k<KK, bf16_t>(in, H, W, in_pitch, out, out_pitch, plane_stride, rexp, chunk, prm, st);   \
        default: return hipErrorInvalidValue;                                                               \
    }
    if (prm.order == 3) { FDVM_ROWS_DT(3) }
    if (prm.order == 2) { FDVM_ROWS_DT(2) }
    if (prm.order == CPAIR) { FDVM_ROWS_DT(CPAIR) }
    if (prm.order == 4 && !rexp) {
        switch (dtype) {
            case FDVM_U16: return launch_rows_f32out<4, uint16_t>(in, H, W, in_pitch, out, out_pitch, plane_stride, prm, st);
            case FDVM_F32: return launch_rows_f32out<4, float>(in, H, W, in_pitch, out, out_pitch, plane_stride, prm, st);
            case FDVM_F16: return launch_rows_f32out<4, _Float16>(in, H, W, in_pitch, out, out_pitch, plane_stride, prm, st);
            case FDVM_BF16: return launch_rows_f32out<4, bf16_t>(in, H, W, in_pitch, out, out_pitch, plane_stride, prm, st);
            default: return hipErrorInvalidValue;
        }
    }
#undef FDVM_ROWS_DT
    return hipErrorInvalidValue;
}

size_t iir_cols_workspace_bytes(int64_t H, int64_t W, int nscales, int order) {
    const int64_t nty = (H + CT - 1) / CT;
    return ((size_t)nscales * nty * 2 * cascade_states(order) * W * sizeof(double) + 255) & ~(size_t)255;
}

hipError_t launch_iir_cols(const void *in, int64_t in_pitch, int64_t in_plane_stride, const int *rexp, float *out,
                           int64_t H, int64_t W, int64_t pitch, int64_t plane_stride, bool laplacian,
                           const IirParams &prm, void *ws, hipStream_t st) {
    return launch_iir_cols_mode(in, in_pitch, in_plane_stride, rexp, out, H, W, pitch, plane_stride,
                                laplacian ? FIN_LAPLACIAN : FIN_BLUR, nullptr, prm, ws, st);
}

hipError_t launch_iir_cols_mode(const void *in, int64_t in_pitch, int64_t in_plane_stride, const int *rexp,
                                float *out, int64_t H, int64_t W, int64_t pitch, int64_t plane_stride, int mode,
                                const HessArgs *hp, const IirParams &prm, void *ws, hipStream_t st) {
    double *states = static_cast<double *>(ws);
    if (mode == FIN_HESSIAN && !hp) return hipErrorInvalidValue;
    if (prm.order == 3)
        return launch_cols_k<3>(in, in_pitch, in_plane_stride, rexp, out, H, W, pitch, plane_stride, mode, hp, prm,
                                states, st);
    if (prm.order == 2)
        return launch_cols_k<2>(in, in_pitch, in_plane_stride, rexp, out, H, W, pitch, plane_stride, mode, hp, prm,
                                states, st);
    if (prm.order == CPAIR)
        return launch_cols_k<CPAIR>(in, in_pitch, in_plane_stride, rexp, out, H, W, pitch, plane_stride, mode, hp,
                                    prm, states, st);
    if (prm.order == 4 && !rexp && mode != FIN_HESSIAN)
        return launch_cols_kx<4, false>(Mid<false>{in, in_pitch, in_plane_stride, nullptr}, out, H, W, pitch,
                                        plane_stride, mode, hp, prm, states, st);
    return hipErrorInvalidValue;
}

}  // namespace fdvm
