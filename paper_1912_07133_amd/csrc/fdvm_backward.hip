// Small kernels of the backward calls (gradients through the detection
// response V_s = sigma_s^2 (D20 + D02)(B_s), B_s = G_s x):
//   * the sum over scales of the per-scale transposed blurs, dL/dx = sum_s
//     G_s^T dL/dB_s, added in scale order (deterministic);
//   * the assembly of dL/dsigma_s = 2/sigma_s <dL/dV_s, V_s> + <dL/dB_s,
//     dB_s/dsigma_s> from the float64 plane inner products, summed over the
//     frames of a batch (per lane in frame order, then over the lanes in
//     order: deterministic).
#include "fdvm_internal.h"

namespace fdvm {
namespace {

__global__ __launch_bounds__(256) void sum_planes_kernel(const float *__restrict__ in, int64_t pitch, int64_t plane,
                                                         int nscales, int H, int W, float *__restrict__ out,
                                                         int64_t out_pitch) {
    const int x = blockIdx.x * 256 + threadIdx.x;
    const int y = blockIdx.y;
    if (x >= W) return;
    const float *p = in + (int64_t)y * pitch + x;
    float acc = p[0];
    for (int s = 1; s < nscales; ++s) acc += p[(int64_t)s * plane];
    out[(int64_t)y * out_pitch + x] = acc;
}

struct GsigArgs {
    int nscales;
    int accumulate;   // add to gsigma (later frames of a batch) instead of overwriting
    int nterms;       // inner products <gB_s, dB_s/dsigma> given (1 or 2)
    double two_over_sigma[FDVM_MAX_SCALES];
};

// gsigma[s] (+)= 2/sigma_s vv[s] + sum_t terms[t * nscales + s]
__global__ __launch_bounds__(64) void gsigma_kernel(const double *__restrict__ vv, const double *__restrict__ terms,
                                                    GsigArgs a, double *__restrict__ gsigma) {
    const int s = threadIdx.x;
    if (s >= a.nscales) return;
    double g = a.two_over_sigma[s] * vv[s];
    for (int t = 0; t < a.nterms; ++t) g += terms[t * a.nscales + s];
    gsigma[s] = a.accumulate ? gsigma[s] + g : g;
}

// out[s] = sum over lanes l of part[l nscales + s], lanes in order
__global__ __launch_bounds__(64) void sum_lanes_kernel(const double *__restrict__ part, int nlanes, int nscales,
                                                       double *__restrict__ out) {
    const int s = threadIdx.x;
    if (s >= nscales) return;
    double g = part[s];
    for (int l = 1; l < nlanes; ++l) g += part[l * nscales + s];
    out[s] = g;
}

}  // namespace

hipError_t launch_sum_lanes(const double *part, int nlanes, int nscales, double *out, hipStream_t st) {
    hipLaunchKernelGGL(sum_lanes_kernel, dim3(1), dim3(64), 0, st, part, nlanes, nscales, out);
    return hipGetLastError();
}

hipError_t launch_sum_planes(const float *in, int64_t pitch, int64_t plane, int nscales, int64_t H, int64_t W,
                             float *out, int64_t out_pitch, hipStream_t st) {
    hipLaunchKernelGGL(sum_planes_kernel, dim3((unsigned)((W + 255) / 256), (unsigned)H), dim3(256), 0, st, in, pitch,
                       plane, nscales, (int)H, (int)W, out, out_pitch);
    return hipGetLastError();
}

hipError_t launch_gsigma(const double *vv, const double *terms, int nterms, const double *sigmas, int nscales,
                         bool accumulate, double *gsigma, hipStream_t st) {
    GsigArgs a{};
    a.nscales = nscales;
    a.accumulate = accumulate ? 1 : 0;
    a.nterms = nterms;
    for (int s = 0; s < nscales; ++s) a.two_over_sigma[s] = 2.0 / sigmas[s];
    hipLaunchKernelGGL(gsigma_kernel, dim3(1), dim3(64), 0, st, vv, terms, a, gsigma);
    return hipGetLastError();
}

}  // namespace fdvm
