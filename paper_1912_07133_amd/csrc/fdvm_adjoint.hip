// Adjoint (transposed) operators of the filter bank, for gradients:
//
//  * Blur.  One pass along an axis of length N with the replicate extension is
//    G = P H E (extend, convolve with the symmetric h, restrict to [0, N)).
//    Its transpose is E^T H P^T: convolve the zero-extended signal with h (the
//    same recursions run with the zero start: causal and anti-causal parts
//    swap roles, h being symmetric) and fold what lands outside [0, N) back
//    onto the end samples.  The folded amounts are
//        sum_{n<0} (h * g)(n) = sum_m g(m) T(m),  T(m) = sum_{k>m} h(k),
//    and the mirror image at N - 1.  fold_kernel adds them, generating T(m)
//    from T(0) = (1 - b0) / 2 and T(m) = T(m-1) - h(m), h(m) from the impulse
//    response of the cascade sections.  With the zero extension G^T is the
//    zero-start pass itself.
//  * Scale-normalised Laplacian V = sigma^2 (D20 + D02) with the replicate
//    extension of B (the Table I d = 2 taps along x and y): its transpose at
//    (y, x) gathers g from the samples whose clamped neighbours are (y, x).
//  * Plane inner products <a_s, b_s> in float64, fixed order (deterministic).
#include <cmath>

#include "fdvm_internal.h"

namespace fdvm {
namespace {

struct FoldScale {
    double p, b0;
    double w[MAX_SECTIONS];
    int mtail;  // T(m) is negligible from here on
    int pad;
};
struct FoldArgs {
    int nscales, sections;
    FoldScale s[FDVM_MAX_SCALES];
};

// AXIS 1 (y): thread = column x of plane s; AXIS 0 (x): thread = row y.
// Adds the folded tails of `src` to the end samples of `dst`.
template <int AXIS>
__global__ __launch_bounds__(256) void fold_kernel(const float *__restrict__ src, int64_t src_pitch,
                                                   int64_t src_plane, float *__restrict__ dst, int64_t dst_pitch,
                                                   int64_t dst_plane, int H, int W, FoldArgs a) {
    const int t = blockIdx.x * 256 + threadIdx.x;
    const int s = blockIdx.y;
    const int lines = AXIS == 1 ? W : H;   // columns or rows
    const int N = AXIS == 1 ? H : W;       // samples along the folded axis
    if (t >= lines) return;
    const FoldScale &c = a.s[s];
    const float *g = src + (int64_t)s * src_plane;
    const int64_t step = AXIS == 1 ? src_pitch : 1;
    const int64_t base = AXIS == 1 ? (int64_t)t : (int64_t)t * src_pitch;
    const int M = min(N, c.mtail);
    double u[MAX_SECTIONS];
#pragma unroll
    for (int k = 0; k < MAX_SECTIONS; ++k) u[k] = 1.0;   // sections' response at lag 0
    double T = 0.5 * (1.0 - c.b0);                        // sum_{k >= 1} h(k)
    double lo = 0.0, hi = 0.0;
    for (int m = 0; m < M; ++m) {
        lo = fma((double)g[base + (int64_t)m * step], T, lo);
        hi = fma((double)g[base + (int64_t)(N - 1 - m) * step], T, hi);
        // h(m + 1) = sum_k w_k u_k(m), then advance the sections one lag
        double h = 0.0;
#pragma unroll
        for (int k = 0; k < MAX_SECTIONS; ++k)
            if (k < a.sections) h = fma(c.w[k], u[k], h);
        T -= h;
        u[0] *= c.p;
#pragma unroll
        for (int k = 1; k < MAX_SECTIONS; ++k) u[k] = fma(c.p, u[k], u[k - 1]);
    }
    float *d = dst + (int64_t)s * dst_plane;
    const int64_t dstep = AXIS == 1 ? dst_pitch : 1;
    const int64_t dbase = AXIS == 1 ? (int64_t)t : (int64_t)t * dst_pitch;
    if (N == 1) {
        d[dbase] = (float)((double)d[dbase] + lo + hi);
    } else {
        d[dbase] = (float)((double)d[dbase] + lo);
        d[dbase + (int64_t)(N - 1) * dstep] = (float)((double)d[dbase + (int64_t)(N - 1) * dstep] + hi);
    }
}

struct Sig2 {
    float v[FDVM_MAX_SCALES];
};

// out = sigma^2 Lap^T g with clamp-to-edge Laplacian taps
__global__ __launch_bounds__(256) void laplacian_adjoint_kernel(const float *__restrict__ g, int64_t pitch,
                                                                int64_t plane, int H, int W, Sig2 sg,
                                                                float *__restrict__ out, int64_t out_pitch,
                                                                int64_t out_plane) {
    const int x = blockIdx.x * 256 + threadIdx.x;
    const int y = blockIdx.y;
    const int s = blockIdx.z;
    if (x >= W) return;
    const float *G = g + (int64_t)s * plane + (int64_t)y * pitch;
    // samples whose right / left neighbour clamps to x, and the same along y
    float acc = -4.0f * G[x];
    if (x + 1 < W) acc += G[x + 1];
    if (x == 0) acc += G[0];
    if (x >= 1) acc += G[x - 1];
    if (x == W - 1) acc += G[W - 1];
    if (y + 1 < H) acc += G[pitch + x];
    if (y == 0) acc += G[x];
    if (y >= 1) acc += G[x - pitch];
    if (y == H - 1) acc += G[x];
    out[(int64_t)s * out_plane + (int64_t)y * out_pitch + x] = sg.v[s] * acc;
}

constexpr int DOT_ROWS = 8;   // rows per partial sum
constexpr int DOT_T = 256;

__global__ __launch_bounds__(DOT_T) void dots_partial_kernel(const float *__restrict__ a, const float *__restrict__ b,
                                                             int64_t pitch, int64_t plane, int H, int W,
                                                             double *__restrict__ part, int nchunks) {
    __shared__ double red[DOT_T / 64];
    const int chunk = blockIdx.x, s = blockIdx.y;
    const int y0 = chunk * DOT_ROWS;
    double acc = 0.0;
    for (int y = y0; y < min(H, y0 + DOT_ROWS); ++y) {
        const int64_t o = (int64_t)s * plane + (int64_t)y * pitch;
        for (int x = threadIdx.x; x < W; x += DOT_T) acc = fma((double)a[o + x], (double)b[o + x], acc);
    }
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int i = 0; i < DOT_T / 64; ++i) t += red[i];
        part[(int64_t)s * nchunks + chunk] = t;
    }
}

__global__ __launch_bounds__(64) void dots_final_kernel(const double *__restrict__ part, int nchunks,
                                                        double *__restrict__ out) {
    const int s = blockIdx.x;
    double acc = 0.0;
    for (int i = threadIdx.x; i < nchunks; i += 64) acc += part[(int64_t)s * nchunks + i];
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
    if (threadIdx.x == 0) out[s] = acc;
}

}  // namespace

hipError_t launch_fold(const float *src, int64_t src_pitch, int64_t src_plane, float *dst, int64_t dst_pitch,
                       int64_t dst_plane, int64_t H, int64_t W, const IirParams &prm, int axis, hipStream_t st) {
    FoldArgs a{};
    a.nscales = prm.nscales;
    a.sections = prm.order;
    for (int s = 0; s < prm.nscales; ++s) {
        const IirScaleParams &q = prm.s[s];
        FoldScale &f = a.s[s];
        f.p = q.p;
        f.b0 = q.b0;
        for (int k = 0; k < MAX_SECTIONS; ++k) f.w[k] = q.w[k];
        // p^m m^3 < 1e-20 beyond m = sigma (46 + 3 ln m); sigma = -1 / ln p
        const double sigma = -1.0 / q.lnp;
        double m = 60.0 * sigma + 8.0;
        for (int it = 0; it < 4; ++it) m = sigma * (46.1 + 3.0 * std::log(m + 1.0)) + 8.0;
        f.mtail = (int)std::min(m, 2.0e9);
    }
    const int lines = (int)(axis == 1 ? W : H);
    dim3 grid((unsigned)((lines + 255) / 256), (unsigned)prm.nscales);
    if (axis == 1)
        hipLaunchKernelGGL(fold_kernel<1>, grid, dim3(256), 0, st, src, src_pitch, src_plane, dst, dst_pitch,
                           dst_plane, (int)H, (int)W, a);
    else
        hipLaunchKernelGGL(fold_kernel<0>, grid, dim3(256), 0, st, src, src_pitch, src_plane, dst, dst_pitch,
                           dst_plane, (int)H, (int)W, a);
    return hipGetLastError();
}

hipError_t launch_laplacian_adjoint(const float *g, int64_t H, int64_t W, int64_t pitch, int64_t plane, int nscales,
                                    const double *sigmas, float *out, int64_t out_pitch, int64_t out_plane,
                                    hipStream_t st) {
    Sig2 sg{};
    for (int s = 0; s < nscales; ++s) sg.v[s] = (float)(sigmas[s] * sigmas[s]);
    dim3 grid((unsigned)((W + 255) / 256), (unsigned)H, (unsigned)nscales);
    hipLaunchKernelGGL(laplacian_adjoint_kernel, grid, dim3(256), 0, st, g, pitch, plane, (int)H, (int)W, sg, out,
                       out_pitch, out_plane);
    return hipGetLastError();
}

size_t dots_workspace_bytes(int64_t H, int nscales) {
    const int64_t nchunks = (H + DOT_ROWS - 1) / DOT_ROWS;
    return ((size_t)nscales * nchunks * sizeof(double) + 255) & ~(size_t)255;
}

hipError_t launch_plane_dots(const float *a, const float *b, int64_t H, int64_t W, int64_t pitch, int64_t plane,
                             int nscales, double *out, void *ws, hipStream_t st) {
    const int nchunks = (int)((H + DOT_ROWS - 1) / DOT_ROWS);
    double *part = static_cast<double *>(ws);
    hipLaunchKernelGGL(dots_partial_kernel, dim3((unsigned)nchunks, (unsigned)nscales), dim3(DOT_T), 0, st, a, b,
                       pitch, plane, (int)H, (int)W, part, nchunks);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(dots_final_kernel, dim3((unsigned)nscales), dim3(64), 0, st, part, nchunks, out);
    return hipGetLastError();
}

}  // namespace fdvm
