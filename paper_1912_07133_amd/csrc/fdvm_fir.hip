// Non-recursive FIR blur on gfx950 (Eq A5: y(n) = sum_{m=-K..K} h(m) x(n-m)),
// separable, x then y, replicate or zero extension.
//
// Both passes use an input-stationary register block: a thread owns R
// consecutive outputs along the filter direction and walks the 2K + R inputs
// that reach them once; every input is multiplied into all R accumulators, so
// each input read feeds R fused multiply-adds.  Taps are kept in LDS as a
// zero-padded table so the walk needs no edge tests.
//   row pass:    one work-group per row segment, the segment (with its K-pixel
//                halo, boundary-extended) staged in LDS with one pad word per
//                R words so the per-thread strided reads are conflict-free;
//                output to the workspace plane.
//   column pass: lane = column (coalesced), inputs read from global memory.
// The Toeplitz-block form on the matrix cores is in fdvm_fir_mfma.hip.
#include <cmath>
#include <vector>

#include "fdvm_internal.h"

namespace fdvm {

namespace {

constexpr int FIR_R = 8;          // outputs per thread
constexpr int ROW_BLOCK = 256;    // threads per row-pass work-group
constexpr int ROW_SPAN = ROW_BLOCK * FIR_R;
constexpr int COL_R = 16;         // outputs per thread, column pass
constexpr int MAXK = FDVM_MAX_FIR_HALF;

struct Half {
    int K;
    float h[MAXK + 1];  // h(0..K)
};

template <typename T>
__device__ __forceinline__ float ldf(const T *p);
template <>
__device__ __forceinline__ float ldf<uint16_t>(const uint16_t *p) { return (float)*p; }
template <>
__device__ __forceinline__ float ldf<float>(const float *p) { return *p; }
template <>
__device__ __forceinline__ float ldf<_Float16>(const _Float16 *p) { return (float)*p; }
struct bf16_t { uint16_t bits; };
template <>
__device__ __forceinline__ float ldf<bf16_t>(const bf16_t *p) { return __uint_as_float(((uint32_t)p->bits) << 16); }

// zero-padded tap table: hz[t] = h(t - T0) for |t - T0| <= K, else 0,
// T0 = K + 2R; size 2K + 4R + 1
template <int R>
__device__ __forceinline__ void fill_taps(float *hz, const Half &hh) {
    const int K = hh.K;
    const int n = 2 * K + 4 * R + 1;
    for (int t = threadIdx.x; t < n; t += blockDim.x) {
        const int m = t - (K + 2 * R);
        const int am = m < 0 ? -m : m;
        hz[t] = am <= K ? hh.h[am] : 0.0f;
    }
}

__device__ __forceinline__ int lds_pad(int q) { return q + q / FIR_R; }

template <typename TIn>
__global__ __launch_bounds__(ROW_BLOCK) void fir_rows_kernel(const TIn *__restrict__ in, int64_t in_pitch,
                                                              float *__restrict__ out, int64_t out_pitch,
                                                              int H, int W, int boundary, int accumulate,
                                                              Half hh) {
    constexpr int R = FIR_R;
    extern __shared__ float smem[];
    const int K = hh.K;
    const int nblk = (2 * K + R + R - 1) / R;       // ceil((2K + R) / R) input blocks of R
    const int span = ROW_SPAN + R * nblk;           // staged inputs
    float *hz = smem;
    float *xs = smem + (2 * K + 4 * R + 1);
    const int y = blockIdx.y;
    const int xb = blockIdx.x * ROW_SPAN;           // first output column
    fill_taps<R>(hz, hh);
    const TIn *src = in + (int64_t)y * in_pitch;
    for (int q = threadIdx.x; q < span; q += ROW_BLOCK) {
        int col = xb - K + q;
        float v;
        if (col < 0 || col >= W) {
            if (boundary == FDVM_BC_REPLICATE) {
                col = min(max(col, 0), W - 1);
                v = ldf(src + col);
            } else {
                v = 0.0f;
            }
        } else {
            v = ldf(src + col);
        }
        xs[lds_pad(q)] = v;
    }
    __syncthreads();
    // thread t: outputs n0 + j, n0 = xb + t R; input i (0-based) is column
    // n0 - K + i; its tap for output j is h(j + K - i) = hz[j + 2K + 2R - i]
    const int t = threadIdx.x;
    float acc[R];
#pragma unroll
    for (int j = 0; j < R; ++j) acc[j] = 0.0f;
    for (int ib = 0; ib < nblk; ++ib) {
        const int tb = 2 * K + 2 * R - ib * R;  // hz index for (ii = 0, j = 0)
        float tw[2 * R];
#pragma unroll
        for (int u = 0; u < 2 * R; ++u) tw[u] = hz[tb - R + 1 + u];  // uniform (broadcast) reads
        float xv[R];
#pragma unroll
        for (int ii = 0; ii < R; ++ii) xv[ii] = xs[lds_pad(t * R + ib * R + ii)];
#pragma unroll
        for (int ii = 0; ii < R; ++ii) {
#pragma unroll
            for (int j = 0; j < R; ++j) acc[j] = fmaf(tw[R - 1 + j - ii], xv[ii], acc[j]);
        }
    }
    float *dst = out + (int64_t)y * out_pitch;
#pragma unroll
    for (int j = 0; j < R; ++j) {
        const int col = xb + t * R + j;
        if (col < W) dst[col] = accumulate ? dst[col] + acc[j] : acc[j];
    }
}

__global__ __launch_bounds__(256) void fir_cols_kernel(const float *__restrict__ in, int64_t in_pitch,
                                                        float *__restrict__ out, int64_t out_pitch, int H,
                                                        int W, int boundary, int accumulate, Half hh) {
    constexpr int R = COL_R;
    extern __shared__ float hz[];
    const int K = hh.K;
    fill_taps<R>(hz, hh);
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int col = blockIdx.x * 64 + lane;
    const int y0 = (blockIdx.y * 4 + wv) * R;     // first output row of this thread
    if (y0 >= H) return;
    const int ccol = min(col, W - 1);
    const int nblk = (2 * K + R + R - 1) / R;
    float acc[R];
#pragma unroll
    for (int j = 0; j < R; ++j) acc[j] = 0.0f;
    for (int ib = 0; ib < nblk; ++ib) {
        const int tb = 2 * K + 2 * R - ib * R;
        float tw[2 * R];
#pragma unroll
        for (int u = 0; u < 2 * R; ++u) tw[u] = hz[tb - R + 1 + u];
        float xv[R];
#pragma unroll
        for (int ii = 0; ii < R; ++ii) {
            int row = y0 - K + ib * R + ii;
            float v;
            if (row < 0 || row >= H) {
                if (boundary == FDVM_BC_REPLICATE) {
                    row = min(max(row, 0), H - 1);
                    v = in[(int64_t)row * in_pitch + ccol];
                } else {
                    v = 0.0f;
                }
            } else {
                v = in[(int64_t)row * in_pitch + ccol];
            }
            xv[ii] = v;
        }
#pragma unroll
        for (int ii = 0; ii < R; ++ii) {
#pragma unroll
            for (int j = 0; j < R; ++j) acc[j] = fmaf(tw[R - 1 + j - ii], xv[ii], acc[j]);
        }
    }
    if (col < W) {
#pragma unroll
        for (int j = 0; j < R; ++j)
            if (y0 + j < H) {
                float *o = out + (int64_t)(y0 + j) * out_pitch + col;
                *o = accumulate ? *o + acc[j] : acc[j];
            }
    }
}

template <typename T>
hipError_t rows_t(const void *in, int64_t H, int64_t W, int64_t in_pitch, float *tmp, int64_t tmp_pitch,
                  int boundary, const Half &hh, hipStream_t st, int accumulate = 0) {
    const int K = hh.K;
    const int nblk = (2 * K + 2 * FIR_R - 1) / FIR_R;
    const int span = ROW_SPAN + FIR_R * nblk;
    const size_t lds = sizeof(float) * ((2 * K + 4 * FIR_R + 1) + span + span / FIR_R + 1);
    dim3 grid((unsigned)((W + ROW_SPAN - 1) / ROW_SPAN), (unsigned)H);
    hipLaunchKernelGGL(fir_rows_kernel<T>, grid, dim3(ROW_BLOCK), lds, st, static_cast<const T *>(in),
                       in_pitch, tmp, tmp_pitch, (int)H, (int)W, boundary, accumulate, hh);
    return hipGetLastError();
}

hipError_t cols_f(const float *in, int64_t in_pitch, float *out, int64_t out_pitch, int64_t H, int64_t W,
                  int boundary, const Half &hh, hipStream_t st, int accumulate = 0) {
    const size_t lds = sizeof(float) * (2 * hh.K + 4 * COL_R + 1);
    dim3 grid((unsigned)((W + 63) / 64), (unsigned)((H + 4 * COL_R - 1) / (4 * COL_R)));
    hipLaunchKernelGGL(fir_cols_kernel, grid, dim3(256), lds, st, in, in_pitch, out, out_pitch, (int)H, (int)W,
                       boundary, accumulate, hh);
    return hipGetLastError();
}

}  // namespace

size_t fir_workspace_bytes(int64_t H, int64_t W, int nscales, int max_half) {
    (void)max_half;
    // direct: one row-pass plane; Toeplitz/MFMA: one transposed plane per
    // scale (float32 operands) or tap tables and a transposed pair of half
    // planes per scale (half operands)
    const size_t direct = ((size_t)H * (size_t)W * sizeof(float) + 255) & ~(size_t)255;
    const size_t mfma = fir_mfma_workspace_bytes(H, W, nscales);
    const size_t half = fir_mfma_half_workspace_bytes(H, W, nscales);
    const size_t m = direct > mfma ? direct : mfma;
    return m > half ? m : half;
}

hipError_t launch_fir(const void *in, int dtype, int64_t H, int64_t W, int64_t in_pitch, float *out,
                      int64_t out_pitch, int64_t plane_stride, const double *taps, const int32_t *half_len,
                      const int32_t *tap_offset, int nscales, int boundary, int algo, void *ws,
                      size_t ws_bytes, hipStream_t st) {
    (void)ws_bytes;
    float *tmp = static_cast<float *>(ws);
    const int64_t tmp_pitch = W;
    if (algo == FDVM_FIR_TOEPLITZ_MFMA)
        return launch_fir_mfma(in, dtype, H, W, in_pitch, tmp, out, out_pitch, plane_stride, taps, half_len,
                               tap_offset, nscales, boundary, st);
    if (algo == FDVM_FIR_TOEPLITZ_MFMA_HALF)
        return launch_fir_mfma_half(in, dtype, H, W, in_pitch, ws, out, out_pitch, plane_stride, taps, half_len,
                                    tap_offset, nscales, boundary, st);
    for (int s = 0; s < nscales; ++s) {
        float *dst = out + (int64_t)s * plane_stride;
        Half hh;
        hh.K = half_len[s];
        for (int m = 0; m <= hh.K; ++m) hh.h[m] = (float)taps[tap_offset[s] + hh.K + m];
        hipError_t e = hipSuccess;
        switch (dtype) {
            case FDVM_U16: e = rows_t<uint16_t>(in, H, W, in_pitch, tmp, tmp_pitch, boundary, hh, st); break;
            case FDVM_F32: e = rows_t<float>(in, H, W, in_pitch, tmp, tmp_pitch, boundary, hh, st); break;
            case FDVM_F16: e = rows_t<_Float16>(in, H, W, in_pitch, tmp, tmp_pitch, boundary, hh, st); break;
            case FDVM_BF16: e = rows_t<bf16_t>(in, H, W, in_pitch, tmp, tmp_pitch, boundary, hh, st); break;
            default: return hipErrorInvalidValue;
        }
        if (e != hipSuccess) return e;
        e = cols_f(tmp, tmp_pitch, dst, out_pitch, H, W, boundary, hh, st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_fir_pass(const void *in, int dtype, int64_t H, int64_t W, int64_t in_pitch, float *out,
                           int64_t out_pitch, int axis, int boundary, const double *h, int K, bool accumulate,
                           hipStream_t st) {
    if (K < 0 || K > MAXK) return hipErrorInvalidValue;
    Half hh;
    hh.K = K;
    for (int m = 0; m <= K; ++m) hh.h[m] = (float)h[m];
    const int acc = accumulate ? 1 : 0;
    if (axis == 1) {
        if (dtype != FDVM_F32) return hipErrorInvalidValue;
        return cols_f(static_cast<const float *>(in), in_pitch, out, out_pitch, H, W, boundary, hh, st, acc);
    }
    switch (dtype) {
        case FDVM_U16: return rows_t<uint16_t>(in, H, W, in_pitch, out, out_pitch, boundary, hh, st, acc);
        case FDVM_F32: return rows_t<float>(in, H, W, in_pitch, out, out_pitch, boundary, hh, st, acc);
        case FDVM_F16: return rows_t<_Float16>(in, H, W, in_pitch, out, out_pitch, boundary, hh, st, acc);
        case FDVM_BF16: return rows_t<bf16_t>(in, H, W, in_pitch, out, out_pitch, boundary, hh, st, acc);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace fdvm
