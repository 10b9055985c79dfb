// Repeated-pole IIR blur on gfx950: causal + anti-causal recursions (Eqs A6-A10)
// along rows (x) and then columns (y), replicate (Eq A32 steady state) or zero
// start.
//
// Realisation.  Each one-sided part is a cascade of K first-order sections
// with the common pole p (float32):
//     v_1(n) = p v_1(n-1) + x(n),   v_k(n) = p v_k(n-1) + v_{k-1}(n),
//     y+(n)  = sum_k w_k v_k(n-1)
// (2K flops per sample and direction).  The zero-input transition over n
// samples is A^n = p^n [[1,0,0],[n,1,0],[n(n+1)/2,n,1]] (K = 3; the upper-left
// 2x2 block for K = 2), which is what lets a line be cut into chunks that are
// filtered independently from a zero state and then stitched together:
//     state_after(chunk) = A^len state_before + zero_state_end(chunk).
//
// Row pass (x): one wavefront per image row (R wavefronts for wide rows).  The
// row is staged through LDS with coalesced loads, each lane owns C consecutive
// samples, the per-lane chunk states are combined with a log-step scan across
// lanes (and across the R wavefronts through LDS), and the outputs go back
// through LDS to coalesced stores.  All S scales are computed from one staged
// copy of the row.
//
// Column pass (y): lane = column (coalesced along the row), the 8 wavefronts
// of a work-group split the column height into segments, each segment is
// walked in tiles of 64 rows held in registers; segment carries are exchanged
// in LDS.
#include <cmath>

#include "fdvm_internal.h"

namespace fdvm {
namespace {

constexpr int ROW_WPB = 8;   // wavefronts per row-pass work-group
constexpr int COL_NW = 8;    // wavefronts per column-pass work-group
constexpr int COL_TW = 64;   // rows per register tile in the column pass

struct ScaleArgs {
    float p, b0;
    float w[3];
    float ss[3];
    float pbit[7];    // p^(2^k), k = 0..6
    float pchunk[8];  // row pass: p^(C 2^k), k = 0..7
    float pseg;       // column pass: p^seg
    float pad;
};

struct Args {
    int nscales;
    int boundary;
    int pad0, pad1;
    ScaleArgs s[FDVM_MAX_SCALES];
};

// ------------------------------------------------------------ recursion
template <int K>
__device__ __forceinline__ float cas_out(const ScaleArgs &c, const float (&v)[K]) {
    float y = c.w[0] * v[0];
#pragma unroll
    for (int k = 1; k < K; ++k) y = fmaf(c.w[k], v[k], y);
    return y;
}

template <int K>
__device__ __forceinline__ void cas_step(float p, float (&v)[K], float x) {
    v[0] = fmaf(p, v[0], x);
#pragma unroll
    for (int k = 1; k < K; ++k) v[k] = fmaf(p, v[k], v[k - 1]);
}

// v <- A^n v + z, with pn = p^n
template <int K>
__device__ __forceinline__ void cas_advance_add(float pn, float n, float (&v)[K], const float (&z)[K]) {
    const float a = v[0], b = v[1];
    if constexpr (K == 3) {
        const float c = v[2];
        v[2] = fmaf(pn, fmaf(0.5f * n * (n + 1.0f), a, fmaf(n, b, c)), z[2]);
    }
    v[1] = fmaf(pn, fmaf(n, a, b), z[1]);
    v[0] = fmaf(pn, a, z[0]);
}

template <int K>
__device__ __forceinline__ void set_zero(float (&v)[K]) {
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = 0.0f;
}

// p^n for 0 <= n < 128 from the binary powers
__device__ __forceinline__ float pow_bits(const ScaleArgs &c, int n) {
    float r = 1.0f;
#pragma unroll
    for (int k = 0; k < 7; ++k)
        if ((n >> k) & 1) r *= c.pbit[k];
    return r;
}

// p^(C m) for 0 <= m < 256 from the chunk powers
__device__ __forceinline__ float pow_chunks(const ScaleArgs &c, int m) {
    float r = 1.0f;
#pragma unroll
    for (int k = 0; k < 8; ++k)
        if ((m >> k) & 1) r *= c.pchunk[k];
    return r;
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

// ------------------------------------------------------------ row pass
template <int K, int C, int R, typename TIn>
__global__ __launch_bounds__(ROW_WPB * 64) void iir_rows_kernel(
    const TIn *__restrict__ in, int64_t in_pitch, float *__restrict__ out, int64_t out_pitch,
    int64_t plane_stride, int H, int W, Args a) {
    constexpr int LP = C + 1;  // padded lane stride in LDS: conflict-free chunk reads
    __shared__ float buf[ROW_WPB][64 * LP];
    __shared__ float tot[ROW_WPB][2][K];

    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
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
#pragma unroll 4
    for (int i = 0; i < C; ++i) {
        const int j = i * 64 + lane;
        const int col = seg0 + j;
        float v = 0.0f;
        if (row_ok && col < W) v = load_as_float(src + col);
        lds[j + j / C] = v;
    }
    float x_first = 0.0f, x_last = 0.0f;
    if (row_ok) {
        x_first = load_as_float(src);
        x_last = load_as_float(src + (W - 1));
    }
    __syncthreads();
    float xs[C];
#pragma unroll
    for (int j = 0; j < C; ++j) xs[j] = lds[lane * LP + j];
    const bool full_wave = __all(nv == C);

    for (int s = 0; s < a.nscales; ++s) {
        const ScaleArgs &cf = a.s[s];
        const float p = cf.p;
        const float nC = (float)C;
        // ---- pass 1: zero-state chunk states
        float zf[K], zb[K];
        set_zero(zf);
        set_zero(zb);
#pragma unroll
        for (int j = 0; j < C; ++j) cas_step(p, zf, xs[j]);
#pragma unroll
        for (int j = C - 1; j >= 0; --j) cas_step(p, zb, xs[j]);

        float init_l[K], init_r[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            init_l[k] = a.boundary == FDVM_BC_REPLICATE ? x_first * cf.ss[k] : 0.0f;
            init_r[k] = a.boundary == FDVM_BC_REPLICATE ? x_last * cf.ss[k] : 0.0f;
        }
        // forward elements: w_0 absorbs the left start state
        float sf[K];
#pragma unroll
        for (int k = 0; k < K; ++k) sf[k] = zf[k];
        if (g == 0) {
            float t[K];
#pragma unroll
            for (int k = 0; k < K; ++k) t[k] = init_l[k];
            cas_advance_add(cf.pchunk[0], nC, t, zf);
#pragma unroll
            for (int k = 0; k < K; ++k) sf[k] = t[k];
        }
        // backward elements: the chunk holding column W-1 absorbs the right
        // start state; chunks past the end contribute nothing
        float sb[K];
#pragma unroll
        for (int k = 0; k < K; ++k) sb[k] = g > g_last ? 0.0f : zb[k];
        if (g == g_last) {
            float t[K];
#pragma unroll
            for (int k = 0; k < K; ++k) t[k] = init_r[k];
            cas_advance_add(pow_bits(cf, nv), (float)nv, t, zb);
#pragma unroll
            for (int k = 0; k < K; ++k) sb[k] = t[k];
        }
        // ---- intra-wavefront inclusive scans (forward: from the left,
        // backward: from the right)
#pragma unroll
        for (int lvl = 0; lvl < 6; ++lvl) {
            const int d = 1 << lvl;
            const float pn = cf.pchunk[lvl];
            const float n = (float)(C * d);
            float tf[K], tb[K];
#pragma unroll
            for (int k = 0; k < K; ++k) {
                tf[k] = __shfl_up(sf[k], d, 64);
                tb[k] = __shfl_down(sb[k], d, 64);
            }
            // S_l <- A^(C d) S_(l-d) + S_l   (and the mirror image)
            cas_advance_add(pn, n, tf, sf);
            cas_advance_add(pn, n, tb, sb);
#pragma unroll
            for (int k = 0; k < K; ++k) {
                if (lane >= d) sf[k] = tf[k];
                if (lane + d < 64) sb[k] = tb[k];
            }
        }
        // ---- across the R wavefronts of the row
        float cwf[K], cwb[K];  // state entering this wavefront's segment
        set_zero(cwf);
        set_zero(cwb);
        if constexpr (R > 1) {
            if (lane == 63) {
#pragma unroll
                for (int k = 0; k < K; ++k) tot[wv][0][k] = sf[k];
            }
            if (lane == 0) {
#pragma unroll
                for (int k = 0; k < K; ++k) tot[wv][1][k] = sb[k];
            }
            __syncthreads();
            const int base = wv - r;
            const float pn = cf.pchunk[6];
            const float n = (float)(C * 64);
            for (int q = 0; q < r; ++q) {
                float z[K];
#pragma unroll
                for (int k = 0; k < K; ++k) z[k] = tot[base + q][0][k];
                cas_advance_add(pn, n, cwf, z);
            }
            for (int q = R - 1; q > r; --q) {
                float z[K];
#pragma unroll
                for (int k = 0; k < K; ++k) z[k] = tot[base + q][1][k];
                cas_advance_add(pn, n, cwb, z);
            }
            __syncthreads();
            // fold the incoming segment state into the per-lane scans
            float t1[K], t2[K];
#pragma unroll
            for (int k = 0; k < K; ++k) { t1[k] = cwf[k]; t2[k] = cwb[k]; }
            cas_advance_add(pow_chunks(cf, lane + 1), (float)(C * (lane + 1)), t1, sf);
            cas_advance_add(pow_chunks(cf, 64 - lane), (float)(C * (64 - lane)), t2, sb);
#pragma unroll
            for (int k = 0; k < K; ++k) { sf[k] = t1[k]; sb[k] = t2[k]; }
        }
        // carry into each chunk: exclusive scans
        float vf[K], vb[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const float up = __shfl_up(sf[k], 1, 64);
            const float dn = __shfl_down(sb[k], 1, 64);
            vf[k] = lane == 0 ? cwf[k] : up;
            vb[k] = lane == 63 ? cwb[k] : dn;
            if (g == 0) vf[k] = init_l[k];
            if (g == g_last) vb[k] = init_r[k];
        }
        // ---- pass 2: final outputs of the chunk
        float ys[C];
        if (full_wave) {
#pragma unroll
            for (int j = C - 1; j >= 0; --j) {
                ys[j] = fmaf(cf.b0, xs[j], cas_out(cf, vb));
                cas_step(p, vb, xs[j]);
            }
#pragma unroll
            for (int j = 0; j < C; ++j) {
                ys[j] += cas_out(cf, vf);
                cas_step(p, vf, xs[j]);
            }
        } else {
#pragma unroll
            for (int j = C - 1; j >= 0; --j) {
                if (j < nv) {
                    ys[j] = fmaf(cf.b0, xs[j], cas_out(cf, vb));
                    cas_step(p, vb, xs[j]);
                } else {
                    ys[j] = 0.0f;
                }
            }
#pragma unroll
            for (int j = 0; j < C; ++j) {
                if (j < nv) {
                    ys[j] += cas_out(cf, vf);
                    cas_step(p, vf, xs[j]);
                }
            }
        }
        // ---- back through LDS to coalesced stores
#pragma unroll
        for (int j = 0; j < C; ++j) lds[lane * LP + j] = ys[j];
        __syncthreads();
        float *dst = out + (int64_t)s * plane_stride + (int64_t)(row_ok ? row : 0) * out_pitch;
#pragma unroll 4
        for (int i = 0; i < C; ++i) {
            const int j = i * 64 + lane;
            const int col = seg0 + j;
            if (row_ok && col < W) dst[col] = lds[j + j / C];
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------ column pass
template <int K>
__global__ __launch_bounds__(COL_NW * 64) void iir_cols_kernel(
    const float *in, int64_t in_pitch, int64_t in_plane_stride, float *out, int64_t pitch,
    int64_t plane_stride, int H, int W, int seg, Args a) {
    constexpr int TW = COL_TW;
    extern __shared__ float tst[];            // [COL_NW][ntmax][K][64]
    __shared__ float xz[COL_NW][2][K][64];

    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int s = blockIdx.y;
    const int col = blockIdx.x * 64 + lane;
    const bool col_ok = col < W;
    const int ccol = col_ok ? col : W - 1;
    const ScaleArgs &cf = a.s[s];
    const float p = cf.p;
    const int ntmax = seg / TW;
    const float *plane = in + (int64_t)s * in_plane_stride;   // read with in_pitch
    float *oplane = out + (int64_t)s * plane_stride;          // written with pitch

    const int r0 = wv * seg;
    const int r1 = min(r0 + seg, H);
    const int len = max(0, r1 - r0);
    const int nt = (len + TW - 1) / TW;
    float *my = tst + (size_t)wv * ntmax * K * 64;

    // ---- pass 1: zero-state states per tile and per segment
    float zf[K];
    set_zero(zf);
    for (int t = 0; t < nt; ++t) {
        const int rt = r0 + t * TW;
        const int lt = min(TW, r1 - rt);
        float xs[TW];
#pragma unroll
        for (int j = 0; j < TW; ++j)
            xs[j] = (j < lt) ? plane[(int64_t)(rt + j) * in_pitch + ccol] : 0.0f;
#pragma unroll
        for (int j = 0; j < TW; ++j) cas_step(p, zf, xs[j]);
        float u[K];
        set_zero(u);
#pragma unroll
        for (int j = TW - 1; j >= 0; --j) cas_step(p, u, xs[j]);
#pragma unroll
        for (int k = 0; k < K; ++k) my[(t * K + k) * 64 + lane] = u[k];
    }
    {
        float acc[K];
        set_zero(acc);
        for (int t = nt - 1; t >= 0; --t) {
            float u[K];
#pragma unroll
            for (int k = 0; k < K; ++k) u[k] = my[(t * K + k) * 64 + lane];
            cas_advance_add(cf.pbit[6], (float)TW, acc, u);
        }
#pragma unroll
        for (int k = 0; k < K; ++k) {
            xz[wv][0][k][lane] = zf[k];
            xz[wv][1][k][lane] = acc[k];
        }
    }
    __syncthreads();

    // ---- carries entering this segment from above (forward) and below
    const float x_top = plane[ccol];
    const float x_bot = plane[(int64_t)(H - 1) * in_pitch + ccol];
    float cfw[K], cbw[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        cfw[k] = a.boundary == FDVM_BC_REPLICATE ? x_top * cf.ss[k] : 0.0f;
        cbw[k] = a.boundary == FDVM_BC_REPLICATE ? x_bot * cf.ss[k] : 0.0f;
    }
    for (int q = 0; q < wv; ++q) {
        float z[K];
#pragma unroll
        for (int k = 0; k < K; ++k) z[k] = xz[q][0][k][lane];
        cas_advance_add(cf.pseg, (float)seg, cfw, z);
    }
    const int last = (H - 1) / seg;  // last segment holding data
    if (wv < last) {
        // through the (possibly short) last segment first
        const int lenL = H - last * seg;
        float pL = 1.0f;
        {
            int n = lenL;
            int full = n / TW;
            for (int i = 0; i < full; ++i) pL *= cf.pbit[6];
            pL *= pow_bits(cf, n - full * TW);
        }
        float z[K];
#pragma unroll
        for (int k = 0; k < K; ++k) z[k] = xz[last][1][k][lane];
        cas_advance_add(pL, (float)lenL, cbw, z);
        for (int q = last - 1; q > wv; --q) {
#pragma unroll
            for (int k = 0; k < K; ++k) z[k] = xz[q][1][k][lane];
            cas_advance_add(cf.pseg, (float)seg, cbw, z);
        }
    }
    // true backward state at the bottom edge of every tile
    {
        float acc[K];
#pragma unroll
        for (int k = 0; k < K; ++k) acc[k] = cbw[k];
        for (int t = nt - 1; t >= 0; --t) {
            const int lt = min(TW, r1 - (r0 + t * TW));
            float u[K];
#pragma unroll
            for (int k = 0; k < K; ++k) {
                u[k] = my[(t * K + k) * 64 + lane];
                my[(t * K + k) * 64 + lane] = acc[k];
            }
            cas_advance_add(lt == TW ? cf.pbit[6] : pow_bits(cf, lt), (float)lt, acc, u);
        }
    }

    // ---- pass 2
    float vf[K];
#pragma unroll
    for (int k = 0; k < K; ++k) vf[k] = cfw[k];
    for (int t = 0; t < nt; ++t) {
        const int rt = r0 + t * TW;
        const int lt = min(TW, r1 - rt);
        float xs[TW], ys[TW];
        float vb[K];
#pragma unroll
        for (int k = 0; k < K; ++k) vb[k] = my[(t * K + k) * 64 + lane];
        if (lt == TW) {
#pragma unroll
            for (int j = 0; j < TW; ++j) xs[j] = plane[(int64_t)(rt + j) * in_pitch + ccol];
#pragma unroll
            for (int j = TW - 1; j >= 0; --j) {
                ys[j] = fmaf(cf.b0, xs[j], cas_out(cf, vb));
                cas_step(p, vb, xs[j]);
            }
#pragma unroll
            for (int j = 0; j < TW; ++j) {
                ys[j] += cas_out(cf, vf);
                cas_step(p, vf, xs[j]);
            }
            if (col_ok) {
#pragma unroll
                for (int j = 0; j < TW; ++j) oplane[(int64_t)(rt + j) * pitch + col] = ys[j];
            }
        } else {
#pragma unroll
            for (int j = 0; j < TW; ++j)
                xs[j] = (j < lt) ? plane[(int64_t)(rt + j) * in_pitch + ccol] : 0.0f;
#pragma unroll
            for (int j = TW - 1; j >= 0; --j) {
                if (j < lt) {
                    ys[j] = fmaf(cf.b0, xs[j], cas_out(cf, vb));
                    cas_step(p, vb, xs[j]);
                } else {
                    ys[j] = 0.0f;
                }
            }
#pragma unroll
            for (int j = 0; j < TW; ++j) {
                if (j < lt) {
                    ys[j] += cas_out(cf, vf);
                    cas_step(p, vf, xs[j]);
                }
            }
            if (col_ok) {
#pragma unroll
                for (int j = 0; j < TW; ++j)
                    if (j < lt) oplane[(int64_t)(rt + j) * pitch + col] = ys[j];
            }
        }
    }
}

Args make_args(const IirParams &prm, int C, int seg) {
    Args a{};
    a.nscales = prm.nscales;
    a.boundary = prm.boundary;
    for (int s = 0; s < prm.nscales; ++s) {
        const IirScaleParams &q = prm.s[s];
        ScaleArgs &d = a.s[s];
        d.p = q.p;
        d.b0 = q.b0;
        for (int k = 0; k < 3; ++k) {
            d.w[k] = q.w[k];
            d.ss[k] = q.ss[k];
        }
        for (int k = 0; k < 7; ++k) d.pbit[k] = (float)std::exp((double)(1 << k) * q.lnp);
        for (int k = 0; k < 8; ++k) d.pchunk[k] = (float)std::exp((double)C * (double)(1 << k) * q.lnp);
        d.pseg = (float)std::exp((double)seg * q.lnp);
    }
    return a;
}

template <int K, int C, int R, typename T>
hipError_t launch_rows_t(const void *in, int64_t H, int64_t W, int64_t in_pitch, float *out,
                         int64_t out_pitch, int64_t plane_stride, const IirParams &prm, hipStream_t st) {
    Args a = make_args(prm, C, 0);
    const int rows_per_block = ROW_WPB / R;
    dim3 grid((unsigned)((H + rows_per_block - 1) / rows_per_block));
    hipLaunchKernelGGL((iir_rows_kernel<K, C, R, T>), grid, dim3(ROW_WPB * 64), 0, st,
                       static_cast<const T *>(in), in_pitch, out, out_pitch, plane_stride, (int)H,
                       (int)W, a);
    return hipGetLastError();
}

template <int K, typename T>
hipError_t launch_rows_k(const void *in, int64_t H, int64_t W, int64_t in_pitch, float *out,
                         int64_t out_pitch, int64_t plane_stride, const IirParams &prm, hipStream_t st) {
    // chunk length C per lane and wavefronts per row R: smallest C in
    // {8, 16, 32} with 64 C R >= W, R in {1, 2, 4, 8}
    if (W <= 64 * 8) return launch_rows_t<K, 8, 1, T>(in, H, W, in_pitch, out, out_pitch, plane_stride, prm, st);
    if (W <= 64 * 16) return launch_rows_t<K, 16, 1, T>(in, H, W, in_pitch, out, out_pitch, plane_stride, prm, st);
    if (W <= 64 * 32) return launch_rows_t<K, 32, 1, T>(in, H, W, in_pitch, out, out_pitch, plane_stride, prm, st);
    if (W <= 2 * 64 * 32) return launch_rows_t<K, 32, 2, T>(in, H, W, in_pitch, out, out_pitch, plane_stride, prm, st);
    if (W <= 4 * 64 * 32) return launch_rows_t<K, 32, 4, T>(in, H, W, in_pitch, out, out_pitch, plane_stride, prm, st);
    if (W <= 8 * 64 * 32) return launch_rows_t<K, 32, 8, T>(in, H, W, in_pitch, out, out_pitch, plane_stride, prm, st);
    return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_iir_rows(const void *in, int dtype, int64_t H, int64_t W, int64_t in_pitch,
                           float *out, int64_t out_pitch, int64_t plane_stride,
                           const IirParams &prm, hipStream_t st) {
#define FDVM_ROWS_DT(KK)                                                                                     \
    switch (dtype) {                                                                                         \
        case FDVM_U16: return launch_rows_k<KK, uint16_t>(in, H, W, in_pitch, out, out_pitch, plane_stride, prm, st); \
        case FDVM_F32: return launch_rows_k<KK, float>(in, H, W, in_pitch, out, out_pitch, plane_stride, prm, st);    \
        case FDVM_F16: return launch_rows_k<KK, _Float16>(in, H, W, in_pitch, out, out_pitch, plane_stride, prm, st); \
        case FDVM_BF16: return launch_rows_k<KK, bf16_t>(in, H, W, in_pitch, out, out_pitch, plane_stride, prm, st);  \
        default: return hipErrorInvalidValue;                                                                \
    }
    if (prm.order == 3) { FDVM_ROWS_DT(3) }
    if (prm.order == 2) { FDVM_ROWS_DT(2) }
#undef FDVM_ROWS_DT
    return hipErrorInvalidValue;
}

size_t iir_cols_lds_bytes(int64_t H, int order, int *seg_out) {
    const int64_t per = (H + COL_NW - 1) / COL_NW;
    const int seg = (int)(((per + COL_TW - 1) / COL_TW) * COL_TW);
    if (seg_out) *seg_out = seg;
    return (size_t)COL_NW * (seg / COL_TW) * order * 64 * sizeof(float);
}

hipError_t launch_iir_cols(const float *in, int64_t in_pitch, int64_t in_plane_stride, float *out,
                           int64_t H, int64_t W, int64_t pitch, int64_t plane_stride,
                           const IirParams &prm, hipStream_t st) {
    int seg = 0;
    const size_t lds = iir_cols_lds_bytes(H, prm.order, &seg);
    if (lds > 120 * 1024) return hipErrorInvalidValue;
    Args a = make_args(prm, 1, seg);
    dim3 grid((unsigned)((W + 63) / 64), (unsigned)prm.nscales);
    if (prm.order == 3) {
        hipLaunchKernelGGL((iir_cols_kernel<3>), grid, dim3(COL_NW * 64), lds, st, in, in_pitch,
                           in_plane_stride, out, pitch, plane_stride, (int)H, (int)W, seg, a);
    } else if (prm.order == 2) {
        hipLaunchKernelGGL((iir_cols_kernel<2>), grid, dim3(COL_NW * 64), lds, st, in, in_pitch,
                           in_plane_stride, out, pitch, plane_stride, (int)H, (int)W, seg, a);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace fdvm
