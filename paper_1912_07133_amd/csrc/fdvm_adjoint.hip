// Adjoint (transposed) operators of the filter bank, for gradients:
//
//  * Blur.  One pass along an axis of length N with the replicate extension is
//    G = P H E (extend, convolve with the symmetric h, restrict to [0, N)).
//    Its transpose is E^T H P^T: convolve the zero-extended signal with h (the
//    same recursions run with the zero start: causal and anti-causal parts
//    swap roles, h being symmetric) and fold what lands outside [0, N) back
//    onto the end samples.  The folded amounts are
//        sum_{n<0} (h * g)(n) = sum_m g(m) T(m),  T(m) = sum_{k>m} h(k),
//    and the mirror image at N - 1.  fold_table_kernel tabulates T(m) per
//    scale (T(0) = (1 - b0) / 2, T(m) = T(m-1) - h(m), h from the impulse
//    response of the cascade sections); fold_cols_kernel / fold_rows_kernel
//    form the two dot products of every column / row and add them.  With the
//    zero extension G^T is the zero-start pass itself.
//  * Scale-normalised Laplacian V = sigma^2 (D20 + D02) with the replicate
//    extension of B (the Table I d = 2 taps along x and y): its transpose at
//    (y, x) gathers g from the samples whose clamped neighbours are (y, x).
//  * Plane inner products <a_s, b_s> in float64, fixed order (deterministic).
#include <algorithm>
#include <cmath>

#include "fdvm_internal.h"

namespace fdvm {
namespace {

struct FoldScale {
    double lnp, b0;
    double w[MAX_SECTIONS];
    int mtail;  // T(m) is negligible from here on
    int pad;
};
struct FoldArgs {
    int nscales, sections;
    FoldScale s[FDVM_MAX_SCALES];
};

constexpr int TAB_T = 1024;   // threads of the table kernel (one block per scale)
constexpr int FOLD_WAVES = 16;  // waves splitting the samples of a 64-column strip

// T_s(m) for m < min(len, mtail): T(0) = (1 - b0) / 2 (half the off-centre
// mass), T(m) = T(m-1) - h(m).  For lags n >= 0 the cascade's causal
// response is h(n + 1) = sum_k w_k C(n + k, k) p^n (k + 1 repeated poles at
// p), so every h is formed on its own and the running sum is a block scan
// in float64, in a fixed order.
__global__ __launch_bounds__(TAB_T) void fold_table_kernel(FoldArgs a, int len, int64_t stride,
                                                           double *__restrict__ tab) {
    __shared__ double wsum[TAB_T / 64];
    const int s = blockIdx.x;
    const FoldScale &c = a.s[s];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int M = min(len, c.mtail);
    double carry = 0.5 * (1.0 - c.b0);
    for (int m0 = 0; m0 < M; m0 += TAB_T) {
        const int n = m0 + (int)threadIdx.x;
        double binom = 1.0, h = c.w[0];
        for (int k = 1; k < a.sections; ++k) {
            binom *= (double)(n + k) / (double)k;
            h = fma(c.w[k], binom, h);
        }
        h *= exp((double)n * c.lnp);  // h(n + 1)
        double v = h;
        for (int off = 1; off < 64; off <<= 1) {
            const double t = __shfl_up(v, off, 64);
            if (lane >= off) v += t;
        }
        if (lane == 63) wsum[wv] = v;
        __syncthreads();
        double pre = 0.0, tot = 0.0;
        for (int i = 0; i < TAB_T / 64; ++i) {
            if (i < wv) pre += wsum[i];
            tot += wsum[i];
        }
        // sum_{j = m0+1}^{n} h(j) = (inclusive sum up to h(n + 1)) - h(n + 1)
        if (n < M) tab[(int64_t)s * stride + n] = carry - ((pre + v) - h);
        carry -= tot;
        __syncthreads();
    }
}

// Fold along y (axis 1): lane = column x of a 64-column strip, the waves of
// the block split the samples m; their float64 partials are added in wave
// order.  dst(0, x) += sum_m g(m, x) T(m), dst(H-1, x) += sum_m g(H-1-m, x) T(m).
__global__ __launch_bounds__(64 * FOLD_WAVES) void fold_cols_kernel(const float *__restrict__ src,
                                                                    int64_t src_pitch, int64_t src_plane,
                                                                    float *__restrict__ dst, int64_t dst_pitch,
                                                                    int64_t dst_plane, int H, int W, FoldArgs a,
                                                                    const double *__restrict__ tab,
                                                                    int64_t tab_stride) {
    __shared__ double part[2][FOLD_WAVES][64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int x = blockIdx.x * 64 + lane;
    const int s = blockIdx.y;
    const int M = min(H, a.s[s].mtail);
    const float *g = src + (int64_t)s * src_plane + x;
    const double *T = tab + (int64_t)s * tab_stride;
    double lo = 0.0, hi = 0.0;
    if (x < W) {
        for (int m = wv; m < M; m += FOLD_WAVES) {
            const double t = T[m];
            lo = fma((double)g[(int64_t)m * src_pitch], t, lo);
            hi = fma((double)g[(int64_t)(H - 1 - m) * src_pitch], t, hi);
        }
    }
    part[0][wv][lane] = lo;
    part[1][wv][lane] = hi;
    __syncthreads();
    if (wv != 0 || x >= W) return;
    lo = 0.0;
    hi = 0.0;
    for (int i = 0; i < FOLD_WAVES; ++i) {
        lo += part[0][i][lane];
        hi += part[1][i][lane];
    }
    float *d = dst + (int64_t)s * dst_plane + x;
    if (H == 1) {
        d[0] = (float)((double)d[0] + lo + hi);
    } else {
        d[0] = (float)((double)d[0] + lo);
        d[(int64_t)(H - 1) * dst_pitch] = (float)((double)d[(int64_t)(H - 1) * dst_pitch] + hi);
    }
}

// Fold along x (axis 0): one wave per row y; lanes stride the samples, the
// wave sum is a fixed butterfly.
__global__ __launch_bounds__(256) void fold_rows_kernel(const float *__restrict__ src, int64_t src_pitch,
                                                        int64_t src_plane, float *__restrict__ dst,
                                                        int64_t dst_pitch, int64_t dst_plane, int H, int W,
                                                        FoldArgs a, const double *__restrict__ tab,
                                                        int64_t tab_stride) {
    const int lane = threadIdx.x & 63;
    const int y = blockIdx.x * 4 + (int)(threadIdx.x >> 6);
    const int s = blockIdx.y;
    if (y >= H) return;  // uniform per wave
    const int M = min(W, a.s[s].mtail);
    const float *g = src + (int64_t)s * src_plane + (int64_t)y * src_pitch;
    const double *T = tab + (int64_t)s * tab_stride;
    double lo = 0.0, hi = 0.0;
    for (int m = lane; m < M; m += 64) {
        const double t = T[m];
        lo = fma((double)g[m], t, lo);
        hi = fma((double)g[W - 1 - m], t, hi);
    }
    for (int off = 32; off > 0; off >>= 1) {
        lo += __shfl_xor(lo, off, 64);
        hi += __shfl_xor(hi, off, 64);
    }
    if (lane != 0) return;
    float *d = dst + (int64_t)s * dst_plane + (int64_t)y * dst_pitch;
    if (W == 1) {
        d[0] = (float)((double)d[0] + lo + hi);
    } else {
        d[0] = (float)((double)d[0] + lo);
        d[W - 1] = (float)((double)d[W - 1] + hi);
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

// up to three independent sets of inner products in one launch (blockIdx.z:
// the set); each set as its own launch would compute it
struct DotSets {
    const float *a[3], *b[3];
    int64_t pitch[3], plane[3];
};

__global__ __launch_bounds__(DOT_T) void dots_partial_kernel(DotSets d, int H, int W, int nscales,
                                                             double *__restrict__ part, int nchunks) {
    __shared__ double red[DOT_T / 64];
    const int chunk = blockIdx.x, s = blockIdx.y, q = blockIdx.z;
    const float *a = d.a[q], *b = d.b[q];
    const int64_t pitch = d.pitch[q], plane = d.plane[q];
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
        part[((int64_t)q * nscales + s) * nchunks + chunk] = t;
    }
}

// out[q nscales + s]: the chunk partials of set q, plane s, summed
__global__ __launch_bounds__(64) void dots_final_kernel(const double *__restrict__ part, int nchunks,
                                                        double *__restrict__ out) {
    const int s = blockIdx.x;
    double acc = 0.0;
    for (int i = threadIdx.x; i < nchunks; i += 64) acc += part[(int64_t)s * nchunks + i];
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
    if (threadIdx.x == 0) out[s] = acc;
}

}  // namespace

namespace {
FoldArgs fold_args(const IirParams &prm) {
    FoldArgs a{};
    a.nscales = prm.nscales;
    a.sections = prm.order;
    for (int s = 0; s < prm.nscales; ++s) {
        const IirScaleParams &q = prm.s[s];
        FoldScale &f = a.s[s];
        f.lnp = q.lnp;
        f.b0 = q.b0;
        for (int k = 0; k < MAX_SECTIONS; ++k) f.w[k] = q.w[k];
        // p^m m^3 < 1e-20 beyond m = sigma (46 + 3 ln m); sigma = -1 / ln p
        const double sigma = -1.0 / q.lnp;
        double m = 60.0 * sigma + 8.0;
        for (int it = 0; it < 4; ++it) m = sigma * (46.1 + 3.0 * std::log(m + 1.0)) + 8.0;
        f.mtail = (int)std::min(m, 2.0e9);
    }
    return a;
}
}  // namespace

size_t fold_workspace_bytes(int64_t H, int64_t W, int nscales) {
    return ((size_t)std::max(H, W) * nscales * sizeof(double) + 255) & ~(size_t)255;
}

hipError_t launch_fold_table(int64_t H, int64_t W, const IirParams &prm, double *tab, hipStream_t st) {
    const int64_t len = std::max(H, W);
    hipLaunchKernelGGL(fold_table_kernel, dim3((unsigned)prm.nscales), dim3(TAB_T), 0, st, fold_args(prm),
                       (int)len, len, tab);
    return hipGetLastError();
}

hipError_t launch_fold(const float *src, int64_t src_pitch, int64_t src_plane, float *dst, int64_t dst_pitch,
                       int64_t dst_plane, int64_t H, int64_t W, const IirParams &prm, const double *tab, int axis,
                       hipStream_t st) {
    const FoldArgs a = fold_args(prm);
    const int64_t tstride = std::max(H, W);
    if (axis == 1)
        hipLaunchKernelGGL(fold_cols_kernel, dim3((unsigned)((W + 63) / 64), (unsigned)prm.nscales),
                           dim3(64 * FOLD_WAVES), 0, st, src, src_pitch, src_plane, dst, dst_pitch, dst_plane,
                           (int)H, (int)W, a, tab, tstride);
    else
        hipLaunchKernelGGL(fold_rows_kernel, dim3((unsigned)((H + 3) / 4), (unsigned)prm.nscales), dim3(256), 0,
                           st, src, src_pitch, src_plane, dst, dst_pitch, dst_plane, (int)H, (int)W, a, tab,
                           tstride);
    return hipGetLastError();
}

namespace {
struct FirTail {
    int K;
    float h[FDVM_MAX_FIR_HALF + 1];
};

// tab[m] = sum_{k = m+1..K} h(k), m = 0..K-1: the tap mass of the FIR that
// lies beyond lag m, each entry summed on its own in a fixed order
__global__ __launch_bounds__(256) void fir_tail_kernel(FirTail ft, double *__restrict__ tab) {
    for (int m = blockIdx.x * 256 + threadIdx.x; m < ft.K; m += gridDim.x * 256) {
        double t = 0.0;
        for (int k = ft.K; k > m; --k) t += (double)ft.h[k];
        tab[m] = t;
    }
}
}  // namespace

hipError_t launch_fir_tail_table(const double *h, int K, double *tab, hipStream_t st) {
    if (K < 1 || K > FDVM_MAX_FIR_HALF) return hipErrorInvalidValue;
    FirTail ft;
    ft.K = K;
    for (int m = 0; m <= K; ++m) ft.h[m] = (float)h[m];
    hipLaunchKernelGGL(fir_tail_kernel, dim3((unsigned)((K + 255) / 256)), dim3(256), 0, st, ft, tab);
    return hipGetLastError();
}

hipError_t launch_fold_fir(const float *src, int64_t src_pitch, float *dst, int64_t dst_pitch, int64_t H, int64_t W,
                           int K, const double *tab, int axis, hipStream_t st) {
    FoldArgs a{};
    a.nscales = 1;
    a.s[0].mtail = K;   // tab[m] = 0 from m = K on
    if (axis == 1)
        hipLaunchKernelGGL(fold_cols_kernel, dim3((unsigned)((W + 63) / 64), 1u), dim3(64 * FOLD_WAVES), 0, st, src,
                           src_pitch, (int64_t)0, dst, dst_pitch, (int64_t)0, (int)H, (int)W, a, tab, (int64_t)0);
    else
        hipLaunchKernelGGL(fold_rows_kernel, dim3((unsigned)((H + 3) / 4), 1u), dim3(256), 0, st, src, src_pitch,
                           (int64_t)0, dst, dst_pitch, (int64_t)0, (int)H, (int)W, a, tab, (int64_t)0);
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

hipError_t launch_plane_dots_sets(int nsets, const float *const *a, const float *const *b, const int64_t *pitch,
                                  const int64_t *plane, int64_t H, int64_t W, int nscales, double *out, void *ws,
                                  hipStream_t st) {
    if (nsets < 1 || nsets > 3) return hipErrorInvalidValue;
    const int nchunks = (int)((H + DOT_ROWS - 1) / DOT_ROWS);
    double *part = static_cast<double *>(ws);
    DotSets d{};
    for (int q = 0; q < nsets; ++q) {
        d.a[q] = a[q];
        d.b[q] = b[q];
        d.pitch[q] = pitch[q];
        d.plane[q] = plane[q];
    }
    hipLaunchKernelGGL(dots_partial_kernel, dim3((unsigned)nchunks, (unsigned)nscales, (unsigned)nsets), dim3(DOT_T),
                       0, st, d, (int)H, (int)W, nscales, part, nchunks);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(dots_final_kernel, dim3((unsigned)(nsets * nscales)), dim3(64), 0, st, part, nchunks, out);
    return hipGetLastError();
}

hipError_t launch_plane_dots(const float *a, const float *b, int64_t H, int64_t W, int64_t pitch, int64_t plane,
                             int nscales, double *out, void *ws, hipStream_t st) {
    return launch_plane_dots_sets(1, &a, &b, &pitch, &plane, H, W, nscales, out, ws, st);
}

}  // namespace fdvm
