// High-pass stage (Table I central differences) and multi-scale blob
// detection on gfx950.
//
// Detection is deterministic without atomics or sorting:
//   1. one work-group per (scale, row) evaluates the strict 3 x 3 x 3 extremum
//      test for every pixel of the row, packs the results into 64-bit masks
//      (one per wavefront-wide span of the row) and writes the row's count;
//   2. one work-group scans the S*H row counts (exclusive prefix sums), which
//      also yields the total;
//   3. one work-group per (scale, row) turns its masks into records at the
//      row's offset, in x order.
// Rows are visited in (scale, y) order, so the list comes out ordered by
// (scale, y, x).
#include <cmath>

#include "fdvm_internal.h"

namespace fdvm {
namespace {

constexpr int HP_BLOCK = 256;
constexpr int DET_BLOCK = 256;
constexpr int SCAN_BLOCK = 1024;

struct Norms {
    float v[FDVM_MAX_SCALES];
};

__device__ __forceinline__ float ld_clamped(const float *plane, int64_t pitch, int y, int x, int H, int W) {
    y = min(max(y, 0), H - 1);
    x = min(max(x, 0), W - 1);
    return plane[(int64_t)y * pitch + x];
}

__global__ __launch_bounds__(HP_BLOCK) void highpass_kernel(const float *__restrict__ blur, int64_t pitch,
                                                             int64_t plane_stride, int H, int W,
                                                             unsigned what, int nout, Norms norms,
                                                             float *__restrict__ out,
                                                             int64_t out_plane_stride) {
    const int x = blockIdx.x * HP_BLOCK + threadIdx.x;
    const int y = blockIdx.y;
    const int s = blockIdx.z;
    if (x >= W) return;
    const float *B = blur + (int64_t)s * plane_stride;
    const float c = B[(int64_t)y * pitch + x];
    const float xm = ld_clamped(B, pitch, y, x - 1, H, W);
    const float xp = ld_clamped(B, pitch, y, x + 1, H, W);
    const float ym = ld_clamped(B, pitch, y - 1, x, H, W);
    const float yp = ld_clamped(B, pitch, y + 1, x, H, W);
    const float d20 = (xp - c) + (xm - c);
    const float d02 = (yp - c) + (ym - c);
    const int64_t o = (int64_t)y * pitch + x;
    int j = 0;
    float *dst = out + (int64_t)s * nout * out_plane_stride;
    if (what & FDVM_HP_LAPLACIAN) dst[(j++) * out_plane_stride + o] = norms.v[s] * (d20 + d02);
    if (what & FDVM_HP_D20) dst[(j++) * out_plane_stride + o] = d20;
    if (what & FDVM_HP_D02) dst[(j++) * out_plane_stride + o] = d02;
    if (what & FDVM_HP_D11) {
        // D10 along x of the rows y-1 and y+1, then D01 along y
        const float a = ld_clamped(B, pitch, y + 1, x + 1, H, W) - ld_clamped(B, pitch, y + 1, x - 1, H, W);
        const float b = ld_clamped(B, pitch, y - 1, x + 1, H, W) - ld_clamped(B, pitch, y - 1, x - 1, H, W);
        dst[(j++) * out_plane_stride + o] = 0.25f * (a - b);
    }
    if (what & FDVM_HP_D10) dst[(j++) * out_plane_stride + o] = 0.5f * (xp - xm);
    if (what & FDVM_HP_D01) dst[(j++) * out_plane_stride + o] = 0.5f * (yp - ym);
}

// strict extremum test of pixel (s, y, x); returns +1 (bright), -1 (dark), 0
__device__ __forceinline__ int extremum(const float *__restrict__ V, int64_t pitch, int64_t plane_stride,
                                        int S, int H, int W, int s, int y, int x, float tau, int border,
                                        float *val) {
    if (y < border || y >= H - border || x < border || x >= W - border) return 0;
    const float v = V[(int64_t)s * plane_stride + (int64_t)y * pitch + x];
    *val = v;
    if (!(v <= -tau || v >= tau)) return 0;
    float lo = INFINITY, hi = -INFINITY;
    const int s0 = max(s - 1, 0), s1 = min(s + 1, S - 1);
    const int y0 = max(y - 1, 0), y1 = min(y + 1, H - 1);
    const int x0 = max(x - 1, 0), x1 = min(x + 1, W - 1);
    for (int s2 = s0; s2 <= s1; ++s2) {
        const float *P = V + (int64_t)s2 * plane_stride;
        for (int y2 = y0; y2 <= y1; ++y2) {
            for (int x2 = x0; x2 <= x1; ++x2) {
                if (s2 == s && y2 == y && x2 == x) continue;
                const float u = P[(int64_t)y2 * pitch + x2];
                lo = fminf(lo, u);
                hi = fmaxf(hi, u);
            }
        }
    }
    if (v < lo && v <= -tau) return 1;
    if (v > hi && v >= tau) return -1;
    return 0;
}

__global__ __launch_bounds__(DET_BLOCK) void detect_mask_kernel(const float *__restrict__ V, int64_t pitch,
                                                                 int64_t plane_stride, int S, int H, int W,
                                                                 float tau, int border,
                                                                 unsigned long long *__restrict__ mask,
                                                                 int nwords, int *__restrict__ counts) {
    const int y = blockIdx.x;
    const int s = blockIdx.y;
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    __shared__ int part[DET_BLOCK / 64];
    int cnt = 0;
    unsigned long long *mrow = mask + ((int64_t)s * H + y) * nwords;
    for (int x0 = 0; x0 < W; x0 += DET_BLOCK) {
        const int x = x0 + threadIdx.x;
        float v = 0.0f;
        const int pol = x < W ? extremum(V, pitch, plane_stride, S, H, W, s, y, x, tau, border, &v) : 0;
        const unsigned long long bits = __ballot(pol != 0);
        const int word = (x0 >> 6) + wv;
        if (lane == 0 && word < nwords) mrow[word] = bits;
        cnt += __popcll(bits);
    }
    if (lane == 0) part[wv] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) {
        int t = 0;
        for (int i = 0; i < DET_BLOCK / 64; ++i) t += part[i];
        counts[(int64_t)s * H + y] = t;
    }
}

__global__ __launch_bounds__(SCAN_BLOCK) void scan_counts_kernel(const int *__restrict__ counts, int n,
                                                                  int *__restrict__ offsets,
                                                                  int *__restrict__ total) {
    __shared__ int sh[SCAN_BLOCK];
    const int per = (n + SCAN_BLOCK - 1) / SCAN_BLOCK;
    const int b = threadIdx.x * per;
    const int e = min(b + per, n);
    int local = 0;
    for (int i = b; i < e; ++i) local += counts[i];
    sh[threadIdx.x] = local;
    __syncthreads();
    for (int d = 1; d < SCAN_BLOCK; d <<= 1) {
        const int t = threadIdx.x >= d ? sh[threadIdx.x - d] : 0;
        __syncthreads();
        sh[threadIdx.x] += t;
        __syncthreads();
    }
    int run = sh[threadIdx.x] - local;  // exclusive
    for (int i = b; i < e; ++i) {
        offsets[i] = run;
        run += counts[i];
    }
    if (threadIdx.x == SCAN_BLOCK - 1) *total = sh[SCAN_BLOCK - 1];
}

__global__ __launch_bounds__(DET_BLOCK) void detect_emit_kernel(const float *__restrict__ V, int64_t pitch,
                                                                 int64_t plane_stride, int H, int W,
                                                                 const unsigned long long *__restrict__ mask,
                                                                 int nwords, const int *__restrict__ offsets,
                                                                 fdvm_blob *__restrict__ out, int cap) {
    const int y = blockIdx.x;
    const int s = blockIdx.y;
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    __shared__ int part[DET_BLOCK / 64];
    const unsigned long long *mrow = mask + ((int64_t)s * H + y) * nwords;
    int base = offsets[(int64_t)s * H + y];
    for (int x0 = 0; x0 < W; x0 += DET_BLOCK) {
        const int word = (x0 >> 6) + wv;
        const unsigned long long bits = word < nwords ? mrow[word] : 0ull;
        if (lane == 0) part[wv] = __popcll(bits);
        __syncthreads();
        int before = 0, all = 0;
        for (int i = 0; i < DET_BLOCK / 64; ++i) {
            if (i < wv) before += part[i];
            all += part[i];
        }
        const int x = x0 + threadIdx.x;
        if ((bits >> lane) & 1ull) {
            const unsigned long long below = lane == 0 ? 0ull : (bits & ((~0ull) >> (64 - lane)));
            const int idx = base + before + __popcll(below);
            if (idx < cap) {
                const float v = V[(int64_t)s * plane_stride + (int64_t)y * pitch + x];
                fdvm_blob b;
                b.y = y;
                b.x = x;
                b.scale = s;
                b.polarity = v < 0.0f ? 1 : -1;
                b.value = v;
                out[idx] = b;
            }
        }
        base += all;
        __syncthreads();
    }
}

}  // namespace

hipError_t launch_highpass(const float *blur, int64_t H, int64_t W, int64_t pitch, int64_t plane_stride,
                           int nscales, const float *norms, unsigned what, float *out,
                           int64_t out_plane_stride, hipStream_t st) {
    Norms n{};
    for (int s = 0; s < nscales; ++s) n.v[s] = norms[s];
    int nout = 0;
    for (unsigned b = what; b; b >>= 1) nout += (int)(b & 1u);
    dim3 grid((unsigned)((W + HP_BLOCK - 1) / HP_BLOCK), (unsigned)H, (unsigned)nscales);
    hipLaunchKernelGGL(highpass_kernel, grid, dim3(HP_BLOCK), 0, st, blur, pitch, plane_stride, (int)H,
                       (int)W, what, nout, n, out, out_plane_stride);
    return hipGetLastError();
}

size_t detect_workspace_bytes(int64_t H, int64_t W, int nscales) {
    const int64_t nwords = (W + 63) / 64 + 4;
    const int64_t rows = (int64_t)nscales * H;
    size_t bytes = (size_t)rows * nwords * sizeof(unsigned long long);
    bytes += 2 * (size_t)rows * sizeof(int);
    return (bytes + 255) & ~(size_t)255;
}

hipError_t launch_detect(const float *resp, int64_t H, int64_t W, int64_t pitch, int64_t plane_stride,
                         int nscales, float tau, int border, fdvm_blob *out, int32_t cap, int32_t *count,
                         void *ws, hipStream_t st) {
    const int nwords = (int)((W + 63) / 64 + 4);
    const int64_t rows = (int64_t)nscales * H;
    unsigned long long *mask = static_cast<unsigned long long *>(ws);
    int *counts = reinterpret_cast<int *>(mask + rows * nwords);
    int *offsets = counts + rows;
    dim3 grid((unsigned)H, (unsigned)nscales);
    hipLaunchKernelGGL(detect_mask_kernel, grid, dim3(DET_BLOCK), 0, st, resp, pitch, plane_stride, nscales,
                       (int)H, (int)W, tau, border, mask, nwords, counts);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(scan_counts_kernel, dim3(1), dim3(SCAN_BLOCK), 0, st, counts, (int)rows, offsets,
                       count);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(detect_emit_kernel, grid, dim3(DET_BLOCK), 0, st, resp, pitch, plane_stride, (int)H,
                       (int)W, mask, nwords, offsets, out, cap);
    return hipGetLastError();
}

}  // namespace fdvm
