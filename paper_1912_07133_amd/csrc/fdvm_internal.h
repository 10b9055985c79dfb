// Internal declarations shared by the C-ABI layer and the HIP kernels of the
// blob-detection filter bank.  Not part of the public ABI (see include/fdvm.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fdvm.h"

namespace fdvm {

// ---------------------------------------------------------------- design
// Repeated-pole blur (Section 4.3): DE coefficients at pole p (float64);
// e = 1 - p is passed separately so it keeps full relative precision.
void repeated_pole_de(int K, double p, double e, double *b0, double bp[4], double ap[4]);

// Realisation of the repeated-pole blur as a cascade of K first-order
// sections sharing the pole p (float64):
//   v_1(n) = p v_1(n-1) + x(n),  v_k(n) = p v_k(n-1) + v_{k-1}(n),
//   y+(n)  = sum_k w[k-1] v_k(n-1)          (causal part of Eq A10a)
// and the mirror image for the anti-causal part.  ss[k-1] = 1/(1 - p)^k is
// the steady-state value of v_k for a unit constant input (Eq A32 read as
// replicate extension).
constexpr int MAX_SECTIONS = 4;  // K = 3 blur and its sigma derivative (4 sections)
struct Cascade {
    double p;
    double pim;   // imaginary part of the pole (complex pair), else 0
    double b0;
    double w[MAX_SECTIONS];
    double ss[MAX_SECTIONS];
    double lnp;  // log(p), for p^n at run-time lengths
    int sections;
};
Cascade cascade_realisation(int K, double sigma);
// Butterworth blur of order L_B = 4 (Section 4.4): one complex first-order
// section per direction, v(n) = p v(n-1) + x(n), y+(n) = 2 Re(R v(n-1)),
// held as the two real states (Re v, Im v) with weights w = (2 Re R, -2 Im R)
// and steady state ss = (Re, Im) of 1 / (1 - p); sections = CPAIR.
// omega_c receives the analogue cutoff.  de_b / de_a receive the three-term
// DE coefficients [0, b1, b2] / [1, a1, a2].
constexpr int CPAIR = 1;   // `sections` value of a complex pole pair
Cascade butterworth_realisation(double sigma, double *omega_c, double de_b[3], double de_a[3]);
// number of real states of a realisation with `sections` (CPAIR: 2)
constexpr int cascade_states(int sections) { return sections == CPAIR ? 2 : sections; }
// d h / d sigma of the same blur: b0 -> d b0 / d sigma and, since
// d/dp of a k-fold section is (k/p)(section k+1 - section k), a cascade of
// K + 1 sections with the same pole.
Cascade sigma_derivative_realisation(int K, double sigma);

// Coloured Savitzky-Golay / Gaussian FIR designs (float64, h(-K..K)).
int colored_sg_taps(double sigma, int K, double omega_c, double *taps);
int gaussian_taps(double sigma, int K, double *taps);
// d h / d sigma of those two designs at fixed K
int colored_sg_dtaps(double sigma, int K, double omega_c, double *dtaps);
int gaussian_dtaps(double sigma, int K, double *dtaps);

// ---------------------------------------------------------------- kernels
struct IirScaleParams {
    double p, pim, b0;
    double w[MAX_SECTIONS];
    double ss[MAX_SECTIONS];
    double lnp;
    double sig2;  // sigma^2, for the fused normalised Laplacian
};

struct IirParams {
    int nscales;
    int order;  // number of cascade sections (2 .. MAX_SECTIONS), or CPAIR
    int boundary;  // fdvm_boundary
    int pad;
    IirScaleParams s[FDVM_MAX_SCALES];
};

// Row pass.  rexp == nullptr: `out` receives float32 planes.  Otherwise `out`
// receives the int32 fixed-point intermediate and rexp[y] the exponent of row y
// (sample = q 2^-rexp[y]); then chunk (8, 16 or 32; 0 = from W) sets the
// samples per lane.
hipError_t launch_iir_rows(const void *in, int dtype, int64_t H, int64_t W, int64_t in_pitch,
                           void *out, int64_t out_pitch, int64_t plane_stride, int *rexp, int chunk,
                           const IirParams &prm, hipStream_t stream);
size_t iir_cols_workspace_bytes(int64_t H, int64_t W, int nscales, int order);
inline size_t iir_rexp_bytes(int64_t H) { return ((size_t)H * sizeof(int) + 255) & ~(size_t)255; }
// Column pass over either intermediate format (rexp as for launch_iir_rows).
hipError_t launch_iir_cols(const void *in, int64_t in_pitch, int64_t in_plane_stride, const int *rexp,
                           float *out, int64_t H, int64_t W, int64_t pitch, int64_t plane_stride,
                           bool laplacian, const IirParams &prm, void *ws, hipStream_t stream);
// The column pass finished as the Hessian detector (Section 5, Eqs 26-27):
// out receives sigma^4 |H| per pixel; mask / pmask (one word per (scale, row,
// 62-column tile), the detection words' layout) receive the pixels passing
// Threshold #1 (and #2 when t2 > 0) and, of those, the bright ones (D20 < 0).
struct HessArgs {
    float t1, t2;
    int border, pad;
    unsigned long long *mask, *pmask;
};
hipError_t launch_iir_cols_mode(const void *in, int64_t in_pitch, int64_t in_plane_stride, const int *rexp,
                                float *out, int64_t H, int64_t W, int64_t pitch, int64_t plane_stride, int mode,
                                const HessArgs *hp, const IirParams &prm, void *ws, hipStream_t stream);
constexpr int COLS_HESSIAN = 2;   // launch_iir_cols_mode: 0 blur, 1 Laplacian, 2 Hessian

hipError_t launch_highpass(const float *blur, int64_t H, int64_t W, int64_t pitch, int64_t plane_stride,
                           int nscales, const float *norms, unsigned what,
                           float *out, int64_t out_plane_stride, hipStream_t stream);

size_t detect_workspace_bytes(int64_t H, int64_t W, int nscales);
// the detection words (mask) of a workspace laid out by detect_workspace_bytes
unsigned long long *detect_mask_words(void *ws);
// compaction of given detection words into the ordered list; values read from
// resp, polarity from pmask (null: the sign of the value)
hipError_t launch_compact(const float *resp, int64_t H, int64_t W, int64_t pitch, int64_t plane_stride,
                          int nscales, const unsigned long long *pmask, fdvm_blob *out, int32_t cap,
                          int32_t *count, void *ws, hipStream_t stream);
// host-side argument checks of fdvm_detect_blobs, workspace aside
fdvm_status detect_check(const float *resp, int64_t H, int64_t W, int64_t pitch, int64_t plane_stride, int nscales,
                         float tau, int border, const void *out_dev, int32_t cap, const int32_t *count_dev);
hipError_t launch_detect(const float *resp, int64_t H, int64_t W, int64_t pitch, int64_t plane_stride,
                         int nscales, float tau, int border, fdvm_blob *out, int32_t cap,
                         int32_t *count, void *ws, hipStream_t stream);

// Adjoint pieces (fdvm_adjoint.hip): fold of the replicate extension's
// tails (axis 1: along y, axis 0: along x), transposed scale-normalised
// Laplacian, per-plane float64 inner products.
// tab: device float64, fold_workspace_bytes(H, W, nscales); written by
// launch_fold_table, read by both folds.
size_t fold_workspace_bytes(int64_t H, int64_t W, int nscales);
hipError_t launch_fold_table(int64_t H, int64_t W, const IirParams &prm, double *tab, hipStream_t st);
hipError_t launch_fold(const float *src, int64_t src_pitch, int64_t src_plane, float *dst, int64_t dst_pitch,
                       int64_t dst_plane, int64_t H, int64_t W, const IirParams &prm, const double *tab, int axis,
                       hipStream_t st);
// FIR fold (transpose of the replicate extension): tab[m] = sum_{k>m} h(k)
// for m < K (h = h(0..K) as float32, summed in float64), then the fold of
// launch_fold along y (axis 1) or x (axis 0) for one plane.
hipError_t launch_fir_tail_table(const double *h, int K, double *tab, hipStream_t st);
hipError_t launch_fold_fir(const float *src, int64_t src_pitch, float *dst, int64_t dst_pitch, int64_t H, int64_t W,
                           int K, const double *tab, int axis, hipStream_t st);
// out = sum_s in_s (float32, scale order); in: nscales planes
hipError_t launch_sum_planes(const float *in, int64_t pitch, int64_t plane, int nscales, int64_t H, int64_t W,
                             float *out, int64_t out_pitch, hipStream_t st);
// gsigma[s] (+)= 2/sigma_s vv[s] + sum_{t < nterms} terms[t nscales + s]
// (device float64 arrays; sigmas on the host)
hipError_t launch_gsigma(const double *vv, const double *terms, int nterms, const double *sigmas, int nscales,
                         bool accumulate, double *gsigma, hipStream_t st);
// out[s] = sum_{l < nlanes} part[l nscales + s] (device float64, lanes in order)
hipError_t launch_sum_lanes(const double *part, int nlanes, int nscales, double *out, hipStream_t st);
hipError_t launch_laplacian_adjoint(const float *g, int64_t H, int64_t W, int64_t pitch, int64_t plane, int nscales,
                                    const double *sigmas, float *out, int64_t out_pitch, int64_t out_plane,
                                    hipStream_t st);
size_t dots_workspace_bytes(int64_t H, int nscales);
hipError_t launch_plane_dots(const float *a, const float *b, int64_t H, int64_t W, int64_t pitch, int64_t plane,
                             int nscales, double *out, void *ws, hipStream_t st);
// nsets (1..3) sets of plane inner products in one launch pair: set q pairs
// a[q] and b[q] (pitch[q], plane stride plane[q]); out[q nscales + s];
// ws >= dots_workspace_bytes(H, nsets * nscales); each set's sums as
// launch_plane_dots gives them
hipError_t launch_plane_dots_sets(int nsets, const float *const *a, const float *const *b, const int64_t *pitch,
                                  const int64_t *plane, int64_t H, int64_t W, int nscales, double *out, void *ws,
                                  hipStream_t st);

// FIR blur fused with the normalised Laplacian (float64 accumulation and
// x-pass plane; ws: fir_laplacian_workspace_bytes)
size_t fir_laplacian_workspace_bytes(int64_t H, int64_t W);
hipError_t launch_fir_laplacian(const void *in, int dtype, int64_t H, int64_t W, int64_t in_pitch, float *out,
                                int64_t out_pitch, int64_t plane_stride, const double *taps_dev,
                                const int32_t *half_len, const int32_t *tap_offset, const double *sigmas,
                                int nscales, int boundary, void *ws, hipStream_t stream);

bool fir_mfma_available();
// Toeplitz-block FIR on the matrix cores: y pass of `in` into tmp (nscales
// transposed W x H planes), x pass of tmp transposed back into `out`.
size_t fir_mfma_workspace_bytes(int64_t H, int64_t W, int nscales);
hipError_t launch_fir_mfma(const void *in, int dtype, int64_t H, int64_t W, int64_t in_pitch, float *tmp,
                           float *out, int64_t out_pitch, int64_t plane_stride, const double *taps,
                           const int32_t *half_len, const int32_t *tap_offset, int nscales, int boundary,
                           hipStream_t stream);
// The same Toeplitz-block FIR with half-precision operands (float16 /
// bfloat16 frames as stored, uint16 frames split exactly into float16 pairs;
// taps and the intermediate split hi + scaled lo), float32 accumulation.
// Workspace: the tap tables and the transposed pair planes of the
// intermediate.
size_t fir_mfma_half_workspace_bytes(int64_t H, int64_t W, int nscales);
hipError_t launch_fir_mfma_half(const void *in, int dtype, int64_t H, int64_t W, int64_t in_pitch, void *ws,
                                float *out, int64_t out_pitch, int64_t plane_stride, const double *taps,
                                const int32_t *half_len, const int32_t *tap_offset, int nscales, int boundary,
                                hipStream_t stream);
// The FIR detection response on the matrix cores (half-precision operand
// pairs): both row filters (h, d = h * [1, -2, 1]) in one launch, both column
// filters into V (the second accumulating), the edge rows and columns
// corrected in float64.  Workspace: tap tables, 2 S transposed pair planes
// (at most FDVM_MAX_SCALES / 2 scales per launch), 2 S H edge sums.
size_t fir_laplacian_mfma_workspace_bytes(int64_t H, int64_t W, int nscales);
hipError_t launch_fir_laplacian_mfma(const void *in, int dtype, int64_t H, int64_t W, int64_t in_pitch, void *ws,
                                     float *out, int64_t out_pitch, int64_t plane_stride, const double *taps,
                                     const int32_t *half_len, const int32_t *tap_offset, const double *sigmas,
                                     int nscales, int boundary, hipStream_t stream);
size_t fir_workspace_bytes(int64_t H, int64_t W, int nscales, int max_half);
// One direct FIR pass along x (axis 0, frame of any input type) or y (axis 1,
// float32 input): out (+)= sum_m h(|m|) in_ext(n - m), h = h(0..K) (float64,
// used as float32), boundary FDVM_BC_REPLICATE or FDVM_BC_ZERO.
hipError_t launch_fir_pass(const void *in, int dtype, int64_t H, int64_t W, int64_t in_pitch, float *out,
                           int64_t out_pitch, int axis, int boundary, const double *h, int K, bool accumulate,
                           hipStream_t st);
hipError_t launch_fir(const void *in, int dtype, int64_t H, int64_t W, int64_t in_pitch,
                      float *out, int64_t out_pitch, int64_t plane_stride,
                      const double *taps, const int32_t *half_len, const int32_t *tap_offset,
                      int nscales, int boundary, int algo, void *ws, size_t ws_bytes,
                      hipStream_t stream);

}  // namespace fdvm
