// Row pass (x) of the repeated-pole IIR blur: one wavefront per image row (R
// wavefronts for wide rows).  The row is staged through LDS with coalesced
// loads, each lane owns C consecutive samples, the chunk states are combined
// by a log-step scan across lanes (and across the R wavefronts through LDS),
// outputs go back through LDS to coalesced stores.  All S scales are computed
// from one staged copy of the row.  Realisation and intermediate formats:
// fdvm_iir_common.h.  Instantiated once per input type by
// fdvm_iir_rows_<type>.hip (so the types compile in parallel), dispatched by
// launch_iir_rows (fdvm_iir_rows.hip).
#pragma once

#include "fdvm_iir_common.h"

namespace fdvm {
namespace {

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
        // |out| 2^ex <= bound 2^ex < 2^31; one step less where the bound lies
        // within 2 of 2^31, so that no output rounds to 2^31
        if (bound > 0.0 && ldexp(bound, ex) > 2147483646.0) --ex;
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
        // backward from the right): S_l <- A^(C d) S_(l-d) + S_l.  A lane
        // with no partner d lanes away takes the zero transition instead
        // (A^n S + S_l with p^n = 0 is S_l exactly), which is one select of
        // p^n per direction rather than one per state.
#pragma unroll
        for (int lvl = 0; lvl < 6; ++lvl) {
            const int d = 1 << lvl;
            const Tr tl = tr_level<K, C>(cf, lvl);
            Tr tlf = tl, tlb = tl;
            tlf.a = lane >= d ? tl.a : 0.0;
            tlb.a = lane + d < 64 ? tl.a : 0.0;
            if constexpr (K == CPAIR) {   // p^n = a + i b
                tlf.b = lane >= d ? tl.b : 0.0;
                tlb.b = lane + d < 64 ? tl.b : 0.0;
            }
            double tf[NS], tb[NS];
#pragma unroll
            for (int k = 0; k < NS; ++k) {
                tf[k] = __shfl_up(sf[k], d, 64);
                tb[k] = __shfl_down(sb[k], d, 64);
            }
            cas_advance_add<K>(tlf, tf, sf);
            cas_advance_add<K>(tlb, tb, sb);
#pragma unroll
            for (int k = 0; k < NS; ++k) {
                sf[k] = tf[k];
                sb[k] = tb[k];
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
        // (float64 throughout for the fixed-point intermediate, where the
        // output weights carry the row's 2^ex: scaling by a power of two
        // commutes with every rounding, so the sums are those of the
        // unscaled weights times 2^ex)
        double wo[NS], b0o = cf.b0;
#pragma unroll
        for (int k = 0; k < NS; ++k) wo[k] = cf.w[k];
        if constexpr (FX) {
            const double sc = ldexp(1.0, ex);
            b0o *= sc;
#pragma unroll
            for (int k = 0; k < NS; ++k) wo[k] *= sc;
        }
        auto out_of = [&](const double(&v)[NS]) {
            double y = wo[0] * v[0];
#pragma unroll
            for (int k = 1; k < NS; ++k) y = fma(wo[k], v[k], y);
            return y;
        };
        Acc ys[C];
        if (full_wave) {
#pragma unroll
            for (int j = C - 1; j >= 0; --j) {
                ys[j] = (Acc)fma(b0o, (double)xs[j], out_of(vb));
                cas_step<K>(cf, vb, (double)xs[j]);
            }
#pragma unroll
            for (int j = 0; j < C; ++j) {
                ys[j] = (Acc)((double)ys[j] + out_of(vf));
                cas_step<K>(cf, vf, (double)xs[j]);
            }
        } else {
#pragma unroll
            for (int j = C - 1; j >= 0; --j) {
                if (j < nv) {
                    ys[j] = (Acc)fma(b0o, (double)xs[j], out_of(vb));
                    cas_step<K>(cf, vb, (double)xs[j]);
                } else {
                    ys[j] = (Acc)0;
                }
            }
#pragma unroll
            for (int j = 0; j < C; ++j) {
                if (j < nv) {
                    ys[j] = (Acc)((double)ys[j] + out_of(vf));
                    cas_step<K>(cf, vf, (double)xs[j]);
                }
            }
        }
        uint32_t *dst = static_cast<uint32_t *>(out_v) + (int64_t)s * plane_stride +
                        (int64_t)(row_ok ? row : 0) * out_pitch;
        auto word = [&](int j) -> uint32_t {
            if constexpr (FX) {
                // rint(ys) as a two's-complement word: |ys| < 2^31 - 1 by the
                // choice of ex, so ys + 1.5 2^52 lies in [2^52, 2^53), where the
                // float64 spacing is 1 and the sum rounds ys to the nearest
                // integer (ties to even); its low 32 bits are that integer
                // modulo 2^32
                return (uint32_t)__double2loint((double)ys[j] + 6755399441055744.0);
            } else {
                return __float_as_uint(ys[j]);
            }
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

// the row pass for one input type T, every realisation
template <typename T>
hipError_t launch_rows_typed(const void *in, int64_t H, int64_t W, int64_t in_pitch, void *out, int64_t out_pitch,
                             int64_t plane_stride, int *rexp, int chunk, const IirParams &prm, hipStream_t st) {
    if (prm.order == 3) return launch_rows_k<3, T>(in, H, W, in_pitch, out, out_pitch, plane_stride, rexp, chunk, prm, st);
    if (prm.order == 2) return launch_rows_k<2, T>(in, H, W, in_pitch, out, out_pitch, plane_stride, rexp, chunk, prm, st);
    if (prm.order == CPAIR)
        return launch_rows_k<CPAIR, T>(in, H, W, in_pitch, out, out_pitch, plane_stride, rexp, chunk, prm, st);
    if (prm.order == 4 && !rexp)
        return launch_rows_f32out<4, T>(in, H, W, in_pitch, out, out_pitch, plane_stride, prm, st);
    return hipErrorInvalidValue;
}

}  // namespace

// one instantiation per input type (fdvm_iir_rows_<type>.hip)
#define FDVM_ROWS_DECL(NAME)                                                                                 \
    hipError_t NAME(const void *in, int64_t H, int64_t W, int64_t in_pitch, void *out, int64_t out_pitch,    \
                    int64_t plane_stride, int *rexp, int chunk, const IirParams &prm, hipStream_t st)
FDVM_ROWS_DECL(launch_iir_rows_u16);
FDVM_ROWS_DECL(launch_iir_rows_f32);
FDVM_ROWS_DECL(launch_iir_rows_f16);
FDVM_ROWS_DECL(launch_iir_rows_bf16);

}  // namespace fdvm
