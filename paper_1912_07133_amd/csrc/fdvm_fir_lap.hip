// FIR blur fused with the scale-normalised Laplacian, for detection on the
// FIR form of the filter bank (Eq A5 blur, then sigma^2 (D20 + D02) from the
// Table I d = 2 taps on the replicate extension of the blur).
//
// The blur is formed without rounding before the second differences: the
// scale-normalised Laplacian multiplies any rounding of the blur by about
// 8 sigma^2 (3 10^4 at sigma = 64), so a float32 blur plane followed by a
// separate high-pass step turns float32 rounding into spurious extrema at
// coarse scales.  Here
//   x pass: P = h (*) X along rows, accumulated in float64, stored as float64
//           planes (the FIR is bound by its multiply-adds, not by the extra
//           4 bytes a sample);
//   y pass: B = h (*) P along columns for the rows y0 - 1 .. y0 + R of a
//           thread's block, accumulated in float64; the Laplacian is formed
//           from those float64 values, x-neighbours from the adjacent lanes
//           (a wavefront covers columns x0 - 1 .. x0 + 62 and writes 62), the
//           replicate extension of B at the image's edges taken on B itself.
// Both passes use an input-stationary register block (every input feeds all
// the block's accumulators) with the taps in LDS as a zero-padded float64
// table, read as wave-uniform broadcasts.
#include <cmath>

#include "fdvm_internal.h"

namespace fdvm {

namespace {

constexpr int LX_R = 8;            // outputs per thread, x pass
constexpr int LX_BLOCK = 256;      // threads per x-pass work-group
constexpr int LX_SPAN = LX_BLOCK * LX_R;
constexpr int LY_R = 16;           // output rows per thread, y pass
constexpr int LY_WAVES = 4;        // wavefronts (row blocks) per y-pass work-group

template <typename T>
__device__ __forceinline__ double ldd(const T *p);
template <>
__device__ __forceinline__ double ldd<uint16_t>(const uint16_t *p) { return (double)*p; }
template <>
__device__ __forceinline__ double ldd<float>(const float *p) { return (double)*p; }
template <>
__device__ __forceinline__ double ldd<_Float16>(const _Float16 *p) { return (double)(float)*p; }
struct bf16_t { uint16_t bits; };
template <>
__device__ __forceinline__ double ldd<bf16_t>(const bf16_t *p) {
    return (double)__uint_as_float(((uint32_t)p->bits) << 16);
}

// zero-padded float64 tap table hz[t] = h(t - T0) for |t - T0| <= K, else 0,
// T0 = K + 2 R, t = 0 .. 2K + 4R; taps = h(-K..K)
template <int R>
__device__ __forceinline__ void fill_taps_d(double *hz, const double *__restrict__ taps, int K) {
    const int n = 2 * K + 4 * R + 1;
    for (int t = threadIdx.x; t < n; t += blockDim.x) {
        const int m = t - (K + 2 * R);
        hz[t] = (m >= -K && m <= K) ? taps[K + m] : 0.0;
    }
}

// x pass: one work-group per segment of LX_SPAN outputs of one row; the
// segment plus its K-sample halo (boundary-extended) staged in LDS as
// float64, every thread LX_R consecutive outputs.
template <typename TIn>
__global__ __launch_bounds__(LX_BLOCK) void fir_lap_rows_kernel(const TIn *__restrict__ in, int64_t in_pitch,
                                                                 double *__restrict__ P, int H, int W, int boundary,
                                                                 const double *__restrict__ taps, int K) {
    constexpr int R = LX_R;
    extern __shared__ double lds[];
    const int nblk = (2 * K + R + R - 1) / R;       // input blocks of R per thread
    const int span = LX_SPAN + R * nblk;            // staged inputs
    double *hz = lds;
    double *xs = lds + (2 * K + 4 * R + 1);
    const int y = blockIdx.y;
    const int xb = blockIdx.x * LX_SPAN;            // first output column of the segment
    fill_taps_d<R>(hz, taps, K);
    const TIn *src = in + (int64_t)y * in_pitch;
    for (int q = threadIdx.x; q < span; q += LX_BLOCK) {
        const int col = xb - K + q;
        double v;
        if (col >= 0 && col < W)
            v = ldd(src + col);
        else
            v = boundary == FDVM_BC_REPLICATE ? ldd(src + min(max(col, 0), W - 1)) : 0.0;
        xs[q + q / R] = v;   // one pad word per R: the strided block reads are conflict-free
    }
    __syncthreads();
    // thread t: outputs n0 + j, n0 = xb + t R; input i is column n0 - K + i,
    // its tap for output j is h(j + K - i) = hz[j + 2K + 2R - i]
    const int t = threadIdx.x;
    double acc[R];
#pragma unroll
    for (int j = 0; j < R; ++j) acc[j] = 0.0;
    for (int ib = 0; ib < nblk; ++ib) {
        const int tb = 2 * K + 2 * R - ib * R;
        double tw[2 * R];
#pragma unroll
        for (int u = 0; u < 2 * R; ++u) tw[u] = hz[tb - R + 1 + u];
        double xv[R];
#pragma unroll
        for (int ii = 0; ii < R; ++ii) {
            const int q = t * R + ib * R + ii;
            xv[ii] = xs[q + q / R];
        }
#pragma unroll
        for (int ii = 0; ii < R; ++ii) {
#pragma unroll
            for (int j = 0; j < R; ++j) acc[j] = fma(tw[R - 1 + j - ii], xv[ii], acc[j]);
        }
    }
    double *dst = P + (int64_t)y * W;
#pragma unroll
    for (int j = 0; j < R; ++j) {
        const int col = xb + t * R + j;
        if (col < W) dst[col] = acc[j];
    }
}

// value of lane l-1 / l+1 of a double (DPP wave_shr:1 / wave_shl:1); the end
// lanes read 0, which reaches only the overlap columns that are not written
__device__ __forceinline__ double left_d(double v) {
    const int lo = __double2loint(v), hi = __double2hiint(v);
    return __hiloint2double(__builtin_amdgcn_mov_dpp(hi, 0x138, 0xf, 0xf, true),
                            __builtin_amdgcn_mov_dpp(lo, 0x138, 0xf, 0xf, true));
}
__device__ __forceinline__ double right_d(double v) {
    const int lo = __double2loint(v), hi = __double2hiint(v);
    return __hiloint2double(__builtin_amdgcn_mov_dpp(hi, 0x130, 0xf, 0xf, true),
                            __builtin_amdgcn_mov_dpp(lo, 0x130, 0xf, 0xf, true));
}

// y pass + Laplacian: lane = column x0 - 1 + lane of a 62-column strip, each
// wavefront a block of LY_R output rows; the blur of rows y0 - 1 .. y0 + LY_R
// (LY_R + 2 values) from one walk over the 2K + LY_R + 2 input rows.
__global__ __launch_bounds__(LY_WAVES * 64) void fir_lap_cols_kernel(const double *__restrict__ P, float *__restrict__ V,
                                                                      int64_t out_pitch, int H, int W, int boundary,
                                                                      const double *__restrict__ taps, int K,
                                                                      double sig2) {
    constexpr int R = LY_R;
    constexpr int NO = R + 2;               // blur values per thread: rows y0 - 1 .. y0 + R
    extern __shared__ double hz[];
    // table for NO outputs: hz[t] = h(t - T0), T0 = K + 2 NO
    {
        const int n = 2 * K + 4 * NO + 1;
        for (int t = threadIdx.x; t < n; t += blockDim.x) {
            const int m = t - (K + 2 * NO);
            hz[t] = (m >= -K && m <= K) ? taps[K + m] : 0.0;
        }
    }
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int col = blockIdx.x * 62 - 1 + lane;
    const int ccol = min(max(col, 0), W - 1);   // the replicate extension of B in x: B(-1) = B(0)
    const int y0 = (blockIdx.y * LY_WAVES + wv) * R;
    if (y0 >= H) return;
    const int yb = y0 - 1;                       // row of blur value 0
    // input i is row yb - K + i; its tap for output o (row yb + o) is
    // h(o + K - i) = hz[o + 2K + 2NO - i]... walked in blocks of NO inputs
    const int nblk = (2 * K + NO + NO - 1) / NO;
    double acc[NO];
#pragma unroll
    for (int o = 0; o < NO; ++o) acc[o] = 0.0;
    for (int ib = 0; ib < nblk; ++ib) {
        const int tb = 2 * K + 2 * NO - ib * NO;
        double tw[2 * NO];
#pragma unroll
        for (int u = 0; u < 2 * NO; ++u) tw[u] = hz[tb - NO + 1 + u];
        double xv[NO];
#pragma unroll
        for (int ii = 0; ii < NO; ++ii) {
            const int row = yb - K + ib * NO + ii;
            double v;
            if (row >= 0 && row < H)
                v = P[(int64_t)row * W + ccol];
            else
                v = boundary == FDVM_BC_REPLICATE ? P[(int64_t)min(max(row, 0), H - 1) * W + ccol] : 0.0;
            xv[ii] = v;
        }
#pragma unroll
        for (int ii = 0; ii < NO; ++ii) {
#pragma unroll
            for (int o = 0; o < NO; ++o) acc[o] = fma(tw[NO - 1 + o - ii], xv[ii], acc[o]);
        }
    }
    // the replicate extension of B in y: B(-1) = B(0), B(H) = B(H - 1)
    if (yb < 0) acc[0] = acc[1];
#pragma unroll
    for (int o = 1; o < NO; ++o)
        if (yb + o == H) acc[o] = acc[o - 1];
    const bool wr = lane >= 1 && lane <= 62 && col < W;
#pragma unroll
    for (int o = 1; o <= R; ++o) {
        const int y = yb + o;
        const double bc = acc[o];
        const double lap = (left_d(bc) + right_d(bc)) + (acc[o - 1] + acc[o + 1]) - 4.0 * bc;
        if (wr && y < H) V[(int64_t)y * out_pitch + col] = (float)(sig2 * lap);
    }
}

template <typename T>
hipError_t rows_lap_t(const void *in, int64_t H, int64_t W, int64_t in_pitch, double *P, int boundary,
                      const double *taps, int K, hipStream_t st) {
    const int nblk = (2 * K + 2 * LX_R - 1) / LX_R;
    const int span = LX_SPAN + LX_R * nblk;
    const size_t lds = sizeof(double) * ((2 * K + 4 * LX_R + 1) + span + span / LX_R + 1);
    dim3 grid((unsigned)((W + LX_SPAN - 1) / LX_SPAN), (unsigned)H);
    hipLaunchKernelGGL(fir_lap_rows_kernel<T>, grid, dim3(LX_BLOCK), lds, st, static_cast<const T *>(in), in_pitch,
                       P, (int)H, (int)W, boundary, taps, K);
    return hipGetLastError();
}

}  // namespace

size_t fir_laplacian_workspace_bytes(int64_t H, int64_t W) {
    return ((size_t)H * (size_t)W * sizeof(double) + 255) & ~(size_t)255;
}

hipError_t launch_fir_laplacian(const void *in, int dtype, int64_t H, int64_t W, int64_t in_pitch, float *out,
                                int64_t out_pitch, int64_t plane_stride, const double *taps_dev,
                                const int32_t *half_len, const int32_t *tap_offset, const double *sigmas,
                                int nscales, int boundary, void *ws, hipStream_t st) {
    double *P = static_cast<double *>(ws);
    for (int s = 0; s < nscales; ++s) {
        const int K = half_len[s];
        const double *taps = taps_dev + tap_offset[s];
        hipError_t e;
        switch (dtype) {
            case FDVM_U16: e = rows_lap_t<uint16_t>(in, H, W, in_pitch, P, boundary, taps, K, st); break;
            case FDVM_F32: e = rows_lap_t<float>(in, H, W, in_pitch, P, boundary, taps, K, st); break;
            case FDVM_F16: e = rows_lap_t<_Float16>(in, H, W, in_pitch, P, boundary, taps, K, st); break;
            case FDVM_BF16: e = rows_lap_t<bf16_t>(in, H, W, in_pitch, P, boundary, taps, K, st); break;
            default: return hipErrorInvalidValue;
        }
        if (e != hipSuccess) return e;
        constexpr int NO = LY_R + 2;
        const size_t lds = sizeof(double) * (2 * K + 4 * NO + 1);
        dim3 grid((unsigned)((W + 61) / 62), (unsigned)((H + LY_WAVES * LY_R - 1) / (LY_WAVES * LY_R)));
        hipLaunchKernelGGL(fir_lap_cols_kernel, grid, dim3(LY_WAVES * 64), lds, st, P,
                           out + (int64_t)s * plane_stride, out_pitch, (int)H, (int)W, boundary, taps, K,
                           sigmas[s] * sigmas[s]);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace fdvm
