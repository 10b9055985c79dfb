// High-pass stage (Table I central differences) and multi-scale blob
// detection on gfx950.
//
// Detection (strict extremum over the 3 x 3 x 3 block of (scale, y, x)
// neighbours, thresholded) runs in four kernels, deterministic, with no
// atomics and no sort:
//   mask  -- lane = column, each wavefront owns an 8-row band of a 62-column
//            tile (tiles overlap by one column on each side so every output
//            column has both x-neighbours in the wavefront) and walks the
//            scales; x-neighbours come from wavefront shifts, the separable
//            3 x 3 minimum / maximum of the previous, current and next plane
//            stay in registers.  Output: one 64-bit mask word per
//            (scale, row, tile), words ordered by (scale, y, x).
//   sums  -- popcount totals of consecutive blocks of words;
//   scan  -- exclusive prefix of the block totals (one work-group), total count;
//   emit  -- every block rescans its words and writes the records.
// The list therefore comes out ordered by (scale, y, x).
#include <cmath>

#include "fdvm_internal.h"

namespace fdvm {
namespace {

constexpr int HP_BLOCK = 256;
constexpr int DT_W = 62;          // output columns per detection tile
constexpr int DT_ROWS = 8;        // rows per wavefront
constexpr int DT_WAVES = 4;       // wavefronts per work-group
constexpr int SUM_THREADS = 256;
constexpr int SUM_WORDS = 4;      // words per thread in sums / emit
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

// value of lane (l - 1) / (l + 1) across the whole wavefront (gfx9 DPP
// wave_shr:1 / wave_shl:1); the end lanes get a copy of their own value
__device__ __forceinline__ float lane_left(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(v), __float_as_int(v), 0x138, 0xf, 0xf, false));
}
__device__ __forceinline__ float lane_right(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(v), __float_as_int(v), 0x130, 0xf, 0xf, false));
}

// NaN marks a missing neighbour (outside the stack); fminf/fmaxf skip it.
__global__ __launch_bounds__(DT_WAVES * 64) void detect_mask_kernel(const float *__restrict__ V, int64_t pitch,
                                                                     int64_t plane_stride, int S, int H, int W,
                                                                     float tau, int border,
                                                                     unsigned long long *__restrict__ mask,
                                                                     int ntx) {
    constexpr int RB = DT_ROWS;
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int tx = blockIdx.x;
    const int x = tx * DT_W - 1 + lane;           // lanes 1..62 are output columns
    const int y0 = (blockIdx.y * DT_WAVES + wv) * RB;
    if (y0 >= H) return;
    const bool xin = x >= 0 && x < W;
    const int cx = min(max(x, 0), W - 1);
    const float qnan = __int_as_float(0x7fc00000);
    // rows y0-1 .. y0+RB of the plane, NaN outside the image
    auto load_plane = [&](int s, float (&v)[RB + 2]) {
        const float *P = V + (int64_t)s * plane_stride;   // wave-uniform
#pragma unroll
        for (int r = 0; r < RB + 2; ++r) {
            const int y = y0 - 1 + r;
            const float t = P[(int64_t)min(max(y, 0), H - 1) * pitch + cx];
            v[r] = (xin && y >= 0 && y < H) ? t : qnan;
        }
    };
    // separable 3x3 min / max (centre included) for rows y0 .. y0+RB-1, and
    // the 8-neighbour min / max (centre excluded)
    float cur[RB + 2], nxt[RB + 2], pre[RB + 2];
    float m9p[RB], M9p[RB];             // previous plane's 3x3 min / max
    float m9c[RB], M9c[RB], m8c[RB], M8c[RB];
    bool have_prev = false;
    load_plane(0, cur);
    if (S > 1) load_plane(1, pre);      // raw samples one plane ahead
    auto planes_stats = [&](const float (&v)[RB + 2], float (&m9)[RB], float (&M9)[RB], float (&m8)[RB],
                            float (&M8)[RB]) {
        float rmin[RB + 2], rmax[RB + 2];
#pragma unroll
        for (int r = 0; r < RB + 2; ++r) {
            const float l = lane_left(v[r]);
            const float rr = lane_right(v[r]);
            const float lr_min = fminf(l, rr), lr_max = fmaxf(l, rr);
            rmin[r] = fminf(lr_min, v[r]);
            rmax[r] = fmaxf(lr_max, v[r]);
            if (r >= 1 && r <= RB) {
                m8[r - 1] = lr_min;   // completed below with the rows above / below
                M8[r - 1] = lr_max;
            }
        }
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            const float a = fminf(rmin[r], rmin[r + 2]);
            const float b = fmaxf(rmax[r], rmax[r + 2]);
            m8[r] = fminf(m8[r], a);
            M8[r] = fmaxf(M8[r], b);
            m9[r] = fminf(a, rmin[r + 1]);
            M9[r] = fmaxf(b, rmax[r + 1]);
        }
    };
    planes_stats(cur, m9c, M9c, m8c, M8c);
    const bool xout = lane >= 1 && lane <= 62 && x < W && x >= border && x < W - border;
    for (int s = 0; s < S; ++s) {
        float m9n[RB], M9n[RB], m8n[RB], M8n[RB];
        const bool have_next = s + 1 < S;
        if (have_next) {
#pragma unroll
            for (int r = 0; r < RB + 2; ++r) nxt[r] = pre[r];
            if (s + 2 < S) load_plane(s + 2, pre);   // in flight while s + 1 is used
            planes_stats(nxt, m9n, M9n, m8n, M8n);
        }
        unsigned long long *mrow = mask + ((int64_t)s * H + y0) * ntx + tx;
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            const int y = y0 + r;
            const float v = cur[r + 1];
            float lo = m8c[r], hi = M8c[r];
            if (have_prev) {
                lo = fminf(lo, m9p[r]);
                hi = fmaxf(hi, M9p[r]);
            }
            if (have_next) {
                lo = fminf(lo, m9n[r]);
                hi = fmaxf(hi, M9n[r]);
            }
            const bool inside = xout && y < H && y >= border && y < H - border;
            // no neighbour at all (1 x 1 x 1 stack) compares as "strict" too
            const bool bright = inside && v <= -tau && !(v >= lo);
            const bool dark = inside && v >= tau && !(v <= hi);
            const unsigned long long bits = __ballot(bright || dark) >> 1;  // lanes 1..62 -> bits 0..61
            if (lane == 0 && y < H) mrow[(int64_t)r * ntx] = bits;
        }
        if (have_next) {
#pragma unroll
            for (int r = 0; r < RB; ++r) {
                m9p[r] = m9c[r];
                M9p[r] = M9c[r];
                m9c[r] = m9n[r];
                M9c[r] = M9n[r];
                m8c[r] = m8n[r];
                M8c[r] = M8n[r];
            }
#pragma unroll
            for (int r = 0; r < RB + 2; ++r) cur[r] = nxt[r];
            have_prev = true;
        }
    }
}

// popcount totals of SUM_THREADS * SUM_WORDS consecutive words
__global__ __launch_bounds__(SUM_THREADS) void detect_sums_kernel(const unsigned long long *__restrict__ mask,
                                                                  int64_t nwords, int *__restrict__ bsum) {
    constexpr int NW = SUM_THREADS * SUM_WORDS;
    __shared__ int part[SUM_THREADS / 64];
    const int64_t bbase = (int64_t)blockIdx.x * NW;
    int c = 0;
    for (int i = threadIdx.x; i < NW; i += SUM_THREADS)  // coalesced
        if (bbase + i < nwords) c += __popcll(mask[bbase + i]);
    for (int o = 32; o > 0; o >>= 1) c += __shfl_down(c, o, 64);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        int t = 0;
        for (int i = 0; i < SUM_THREADS / 64; ++i) t += part[i];
        bsum[blockIdx.x] = t;
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

__global__ __launch_bounds__(SUM_THREADS) void detect_emit_kernel(const float *__restrict__ V, int64_t pitch,
                                                                   int64_t plane_stride, int H, int W, int ntx,
                                                                   const unsigned long long *__restrict__ mask,
                                                                   int64_t nwords, const int *__restrict__ boff,
                                                                   fdvm_blob *__restrict__ out, int cap) {
    constexpr int NW = SUM_THREADS * SUM_WORDS;
    __shared__ unsigned long long wbuf[NW];
    __shared__ int part[SUM_THREADS / 64];
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int64_t bbase = (int64_t)blockIdx.x * NW;
    // coalesced staging of the block's words
    for (int i = threadIdx.x; i < NW; i += SUM_THREADS)
        wbuf[i] = bbase + i < nwords ? mask[bbase + i] : 0ull;
    __syncthreads();
    const int first = threadIdx.x * SUM_WORDS;
    int c = 0;
#pragma unroll
    for (int i = 0; i < SUM_WORDS; ++i) c += __popcll(wbuf[first + i]);
    // exclusive prefix of c over the block
    int incl = c;
    for (int o = 1; o < 64; o <<= 1) {
        const int t = __shfl_up(incl, o, 64);
        if (lane >= o) incl += t;
    }
    if (lane == 63) part[wv] = incl;
    __syncthreads();
    int before = 0;
    for (int i = 0; i < wv; ++i) before += part[i];
    int idx = boff[blockIdx.x] + before + incl - c;
    if (c == 0) return;
    for (int i = 0; i < SUM_WORDS; ++i) {
        unsigned long long bits = wbuf[first + i];
        if (!bits) continue;
        const unsigned word = (unsigned)(bbase + first + i);  // = (s * H + y) * ntx + tx
        const unsigned sy = word / (unsigned)ntx;
        const int tx = (int)(word - sy * (unsigned)ntx);
        const int s = (int)(sy / (unsigned)H);
        const int y = (int)(sy - (unsigned)s * (unsigned)H);
        while (bits) {
            const int b = __ffsll((long long)bits) - 1;
            bits &= bits - 1;
            if (idx < cap) {
                const int xx = tx * DT_W + b;
                const float v = V[(int64_t)s * plane_stride + (int64_t)y * pitch + xx];
                fdvm_blob rec;
                rec.y = y;
                rec.x = xx;
                rec.scale = s;
                rec.polarity = v < 0.0f ? 1 : -1;
                rec.value = v;
                out[idx] = rec;
            }
            ++idx;
        }
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

namespace {
struct DetectLayout {
    int ntx;
    int64_t nwords;
    int64_t nblocks;
    size_t mask_bytes, sums_bytes;
};
DetectLayout detect_layout(int64_t H, int64_t W, int nscales) {
    DetectLayout d;
    d.ntx = (int)((W + DT_W - 1) / DT_W);
    const int64_t hpad = ((H + DT_ROWS * DT_WAVES - 1) / (DT_ROWS * DT_WAVES)) * DT_ROWS * DT_WAVES;
    // words for rows up to the padded height are written (as zero) too
    d.nwords = (int64_t)nscales * H * d.ntx;
    const int64_t alloc_words = (int64_t)nscales * hpad * d.ntx + (int64_t)d.ntx * DT_ROWS;
    d.nblocks = (d.nwords + SUM_THREADS * SUM_WORDS - 1) / (SUM_THREADS * SUM_WORDS);
    d.mask_bytes = ((size_t)alloc_words * 8 + 255) & ~(size_t)255;
    d.sums_bytes = ((size_t)(2 * d.nblocks + 1) * sizeof(int) + 255) & ~(size_t)255;
    return d;
}
}  // namespace

size_t detect_workspace_bytes(int64_t H, int64_t W, int nscales) {
    const DetectLayout d = detect_layout(H, W, nscales);
    return d.mask_bytes + d.sums_bytes;
}

hipError_t launch_detect(const float *resp, int64_t H, int64_t W, int64_t pitch, int64_t plane_stride,
                         int nscales, float tau, int border, fdvm_blob *out, int32_t cap, int32_t *count,
                         void *ws, hipStream_t st) {
    const DetectLayout d = detect_layout(H, W, nscales);
    unsigned long long *mask = static_cast<unsigned long long *>(ws);
    int *bsum = reinterpret_cast<int *>(static_cast<char *>(ws) + d.mask_bytes);
    int *boff = bsum + d.nblocks;
    dim3 g1((unsigned)d.ntx, (unsigned)((H + DT_ROWS * DT_WAVES - 1) / (DT_ROWS * DT_WAVES)));
    hipLaunchKernelGGL(detect_mask_kernel, g1, dim3(DT_WAVES * 64), 0, st, resp, pitch, plane_stride, nscales,
                       (int)H, (int)W, tau, border, mask, d.ntx);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(detect_sums_kernel, dim3((unsigned)d.nblocks), dim3(SUM_THREADS), 0, st, mask, d.nwords,
                       bsum);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(scan_counts_kernel, dim3(1), dim3(SCAN_BLOCK), 0, st, bsum, (int)d.nblocks, boff, count);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(detect_emit_kernel, dim3((unsigned)d.nblocks), dim3(SUM_THREADS), 0, st, resp, pitch,
                       plane_stride, (int)H, (int)W, d.ntx, mask, d.nwords, boff, out, cap);
    return hipGetLastError();
}

}  // namespace fdvm
