/*
 * fdvm.h -- C ABI of the MI355X (gfx950) blob-detection filter bank of
 * H. L. Kennedy, "Digital filters with vanishing moments for shape analysis"
 * (arXiv:1912.07133).
 *
 * Pipeline per frame and scale s (Section 5 two-stage architecture):
 *   blur      B_s = separable low-pass blur, x (rows) then y (columns):
 *               fdvm_blur_iir -- repeated-pole IIR of Section 4.3 / Table IV,
 *                                realised as the causal + anti-causal
 *                                recursions of Eqs A6-A10 with the
 *                                steady-state start of Eq A32;
 *               fdvm_blur_fir -- non-recursive FIR of Eq A5 (coloured
 *                                Savitzky-Golay, Section 4.2, or sampled
 *                                Gaussian, Eqs 9 and 11);
 *   highpass  V_s = sigma_s^2 (D20 + D02) from the Table I d = 2 taps
 *             (and optionally D10, D01, D11 for the Hessian of Eq 26);
 *   detect    strict local extrema of V over 3 x 3 pixels x adjacent scales,
 *             thresholded, listed in (scale, y, x) order.
 *
 * Conventions shared by every entry point
 *   - Images are row-major, element (y, x) at base[y * pitch + x]; pitches and
 *     plane strides are in ELEMENTS of the buffer's type.  1 <= H <= 65535,
 *     1 <= W <= 16384.  x runs left to
 *     right, y top to bottom (Appendix, Eqs A7-A8).
 *   - Device pointers are plain HIP device addresses; the caller owns every
 *     buffer (inputs, outputs, workspace).  The library allocates no device
 *     memory and keeps no pointer after returning.  Its only state: per
 *     device, FDVM_MAX_LANES internal streams and events of the batch and
 *     backward calls (created on the first multi-lane batch call or backward
 *     call of several frames on that device, under a lock) and the fixed
 *     scratch array of the no-allocation calls (its device address looked up
 *     on their first call there), both kept until the process ends.  Calls
 *     on different streams are independent, except that multi-lane batch
 *     calls and backward calls of several frames that overlap on one device
 *     share those streams, and no-allocation calls that overlap on one device
 *     share that array: either must be serialised by the caller.
 *   - Device work is enqueued on `stream` (a hipStream_t passed as void*;
 *     NULL = the legacy default stream) and the call returns without waiting.
 *     Argument errors are detected on the host before anything is enqueued;
 *     launch errors are reported as FDVM_EDEVICE; faults inside kernels show
 *     up at the caller's next synchronisation.
 *   - Boundary extension FDVM_BC_REPLICATE holds edge pixels constant to
 *     infinity (the recursions start in the steady state of Eq A32; the FIR
 *     and the high-pass stage clamp); FDVM_BC_ZERO pads with zeros (the
 *     paper's FIR start-up, Section 5).
 */
#ifndef FDVM_H
#define FDVM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FDVM_OK = 0,
    FDVM_EINVAL = -1,       /* invalid argument (null pointer, bad size/pitch/enum) */
    FDVM_ERANGE = -2,       /* sigma / length / size outside the supported range */
    FDVM_ENOMEM = -3,       /* caller-provided buffer too small (taps, workspace) */
    FDVM_EDEVICE = -4,      /* a HIP call failed */
    FDVM_EOVERFLOW = -5,    /* more detections than the output capacity */
    FDVM_EUNSUPPORTED = -6  /* valid request the library does not implement  */
} fdvm_status;

typedef enum {
    FDVM_IIR_REPEATED_POLE = 0, /* Filter D, Section 4.3 (order K = 2 or 3)   */
    FDVM_IIR_REPEATED_POLE_DSIGMA = 3, /* d h / d sigma of that blur (K + 1
                                    cascade sections); fdvm_iir_pass only   */
    FDVM_FIR_COLORED_SG = 1,    /* Filter C, Section 4.2 (Eqs 20-22)          */
    FDVM_FIR_GAUSSIAN = 2,      /* Filter A, Eqs 9c and 11                    */
    FDVM_IIR_BUTTERWORTH = 4,   /* Filter E, Section 4.4 (order L_B = 4: one
                                   complex-conjugate pole pair per direction) */
    FDVM_FIR_COLORED_SG_DSIGMA = 5, /* d h / d sigma of Filter C at fixed K   */
    FDVM_FIR_GAUSSIAN_DSIGMA = 6    /* d h / d sigma of Filter A at fixed K   */
} fdvm_kind;

typedef enum { FDVM_BC_REPLICATE = 0, FDVM_BC_ZERO = 1 } fdvm_boundary;

typedef enum { FDVM_U16 = 0, FDVM_F32 = 1, FDVM_F16 = 2, FDVM_BF16 = 3 } fdvm_dtype;

typedef enum { FDVM_FIR_DIRECT = 0, FDVM_FIR_TOEPLITZ_MFMA = 1, FDVM_FIR_TOEPLITZ_MFMA_HALF = 2 } fdvm_fir_algo;

/* high-pass outputs (bit mask for fdvm_highpass `what`) */
enum {
    FDVM_HP_LAPLACIAN = 1, /* sigma^2 (D20 + D02) (or unnormalised, see below) */
    FDVM_HP_D20 = 2,
    FDVM_HP_D02 = 4,
    FDVM_HP_D11 = 8,
    FDVM_HP_D10 = 16,
    FDVM_HP_D01 = 32
};

#define FDVM_MAX_SCALES 16   /* scales per blur / high-pass / detect call */
#define FDVM_MAX_FIR_HALF 512

/*
 * One designed filter (one scale).  Produced by fdvm_filter_design.
 * IIR (Section 4.3): the DE of Eq A10 is
 *   y+(n) = sum_{m=1..K} bp[m] x(n-m) - sum_{m=1..K} ap[m] y+(n-m)
 *   y-(n) = sum_{m=1..K} bp[m] x(n+m) - sum_{m=1..K} ap[m] y-(n+m)
 *   y(n)  = y+(n) + y-(n) + b0 x(n)
 * with ap[0] = 1, bp[0] = 0, all poles at p = exp(-1/sigma).
 * FIR: `order` is the half-length K, ntaps = 2K + 1; the taps themselves are
 * returned through fdvm_filter_design's `taps` argument.
 */
typedef struct {
    int32_t kind;      /* fdvm_kind                                          */
    int32_t order;     /* IIR: K (2 or 3); Butterworth: L_B (4); FIR: half-length K */
    double sigma;      /* scale parameter (pixels)                           */
    double p;          /* IIR: repeated pole exp(-1/sigma); Butterworth: real
                          part of the pole; FIR: 0                           */
    double b0;         /* IIR: central coefficient; FIR: h(0)                */
    double bp[4];      /* IIR: forward numerator, bp[0] = 0                  */
    double ap[4];      /* IIR: forward denominator, ap[0] = 1                */
    double side_gain;  /* IIR: B+(1)/A+(1) = (1 - b0)/2 (steady-state gain)  */
    double omega_c;    /* coloured SG: cutoff of Eq 21 (3/sigma); Butterworth:
                          analogue cutoff sqrt(2 ln 2)/sigma; else 0         */
    int32_t ntaps;     /* FIR: 2K + 1; IIR: 0                                */
    int32_t reserved;
} fdvm_filter;

/* One detection, produced by fdvm_detect_blobs. */
typedef struct {
    int32_t y, x;       /* pixel                                           */
    int32_t scale;      /* scale index s into the plane stack               */
    int32_t polarity;   /* +1 bright blob (minimum of V), -1 dark (maximum) */
    float value;        /* V at the pixel                                   */
} fdvm_blob;

/* Human-readable name of a status code (static string, never NULL). */
const char *fdvm_status_string(fdvm_status status);

/*
 * fdvm_filter_design -- host-only, pure function (Section 4).
 *   kind = FDVM_IIR_REPEATED_POLE: order K in {2, 3}.  K = 3 is the closed form
 *     of Table IV (L_D = 1, Lbar_pi = 2); K = 2 is the same constrained design
 *     with one Nyquist constraint (unit dc gain, zero second moment,
 *     H(pi) = 0).  sigma in [0.25, 4096].  `fir_half_len`, `taps`,
 *     `taps_cap` are ignored (taps may be NULL).
 *   kind = FDVM_IIR_REPEATED_POLE_DSIGMA: the derivative d h / d sigma of the
 *     order-K blur at sigma (p = exp(-1/sigma), dp/dsigma = p / sigma^2); b0
 *     receives d h(0) / d sigma.  Realised as K + 1 cascade sections with the
 *     same pole (a k-fold section differentiates into sections k and k + 1).
 *     Usable in fdvm_iir_pass (axes 0 and 1); with the replicate extension the
 *     pass is the sigma derivative of the blur pass of the extended input.
 *   kind = FDVM_IIR_BUTTERWORTH: order L_B = 4 (the blur of Filter E).  The
 *     analogue prototype of Eq 25 with omega_c = sqrt(2 ln 2) / sigma (its
 *     half-gain point matched to a Gaussian of scale sigma), discretised by
 *     the bilinear transform; per direction one complex-conjugate pole pair.
 *     Fills b0, bp = [0, b1, b2, 0], ap = [1, a1, a2, 0] of the three-term DE
 *     (Eq A17 form), p = real part of the pole, omega_c.  sigma in
 *     [0.5, 4096].
 *   kind = FDVM_FIR_COLORED_SG: Eq 20 solved in float64 with S from Eq 22,
 *     omega_c = 3/sigma and dc constraints rho = [1, 0] (D = 3); needs
 *     omega_c < pi (sigma > 3/pi), otherwise the stopband of Eq 21 is empty
 *     and the call returns FDVM_ERANGE;
 *     kind = FDVM_FIR_GAUSSIAN: Eq 9c sampled on m = -K..K, normalised by Eq 11.
 *     kind = FDVM_FIR_COLORED_SG_DSIGMA / FDVM_FIR_GAUSSIAN_DSIGMA: the
 *     derivatives d h(m) / d sigma of those two designs at fixed K (same K
 *     rule and ranges): the Gaussian's in closed form, h(m) (m^2 - sum_j
 *     h(j) j^2) / sigma^3; the coloured SG's from the Lagrange system of
 *     Eq 20 differentiated through Sbar (Eq 22b), omega_c = 3/sigma (only S
 *     depends on sigma, so the dc constraints hold: sum dh = 0 and
 *     sum m^2 dh = 0).  b0 receives dh(0)/dsigma.
 *     Half-length K = fir_half_len if > 0, else ceil(3 sigma) (length
 *     6 sigma + 1).  K must be in [1, FDVM_MAX_FIR_HALF]; sigma in [0.25, 1024].
 *     taps (host, float64, capacity taps_cap >= 2K + 1) receives
 *     h(-K), ..., h(K).  `order` argument ignored for FIR.
 * Returns FDVM_EINVAL (null out, bad kind/order), FDVM_ERANGE (sigma or K out
 * of range), FDVM_ENOMEM (taps too small).
 */
fdvm_status fdvm_filter_design(fdvm_kind kind, int order, double sigma, int fir_half_len,
                               fdvm_filter *out, double *taps, int taps_cap);

/*
 * fdvm_blur_iir -- separable repeated-pole IIR blur of one frame at nscales
 * scales (Eqs A6-A10, x then y; Sections 2 and 5).
 *   in        device, H x W elements of type dt, row pitch in_pitch (>= W)
 *             (u16, f16, bf16 and f32 are converted to float on load; u16 is
 *             exact for the 12-bit frames this is built for)
 *   out       device float32, nscales planes; plane s, pixel (y, x) at
 *             out[s * plane_stride + y * out_pitch + x]; out_pitch >= W,
 *             plane_stride >= H * out_pitch.  Must not overlap `in`.
 *   filters   host array of nscales IIR designs (fdvm_filter_design output);
 *             all FDVM_IIR_REPEATED_POLE with the same order (2 or 3), or all
 *             FDVM_IIR_BUTTERWORTH (order 4).
 *   bc        boundary extension (see conventions).
 *   ws        device workspace of at least
 *             fdvm_workspace_bytes(FDVM_OP_BLUR_IIR, H, W, nscales, 0) bytes
 *             (the chunk states of the column pass); contents on entry do not
 *             matter.
 *   The recursions run as a cascade of K first-order sections with float64
 *   states and weights; the planes are stored as float32.
 * Returns FDVM_EINVAL on bad arguments (H, W out of range, nscales outside
 * [1, FDVM_MAX_SCALES], mixed orders, pitch/stride too small, null pointers),
 * FDVM_ENOMEM (workspace too small), FDVM_EDEVICE if a launch fails.
 */
fdvm_status fdvm_blur_iir(const void *in, fdvm_dtype dt, int64_t H, int64_t W, int64_t in_pitch,
                          float *out, int64_t out_pitch, int64_t plane_stride,
                          const fdvm_filter *filters, int nscales, fdvm_boundary bc,
                          void *ws, size_t ws_bytes, void *stream);

/*
 * fdvm_iir_pass -- one of the two 1-D passes that fdvm_blur_iir chains
 * (Section 2: two sequential 1-D filtering operations, x then y).
 *   axis = 0 (x, along rows): `in` is one frame of type dt (row pitch
 *             in_pitch, in_plane_stride ignored); writes nscales float32
 *             planes to `out` (as fdvm_blur_iir).  `in` and `out` must not
 *             overlap.  ws may be NULL.
 *   axis = 1 (y, along columns): `in` holds nscales float32 planes (dt must be
 *             FDVM_F32, pitch in_pitch, plane stride in_plane_stride); each
 *             plane s is filtered with filters[s] into out plane s.  In-place
 *             operation (in == out with equal pitch and stride) is allowed;
 *             other overlaps are not.  ws as for fdvm_blur_iir.
 *   axis = 2 (y, then the high-pass stage): as axis = 1, but out plane s
 *             receives sigma_s^2 (D20 + D02) of the blurred plane (see
 *             fdvm_iir_laplacian); `in` and `out` must not overlap.
 * Errors as fdvm_blur_iir.
 */
fdvm_status fdvm_iir_pass(const void *in, fdvm_dtype dt, int64_t H, int64_t W, int64_t in_pitch,
                          int64_t in_plane_stride, float *out, int64_t out_pitch, int64_t plane_stride,
                          const fdvm_filter *filters, int nscales, fdvm_boundary bc, int axis,
                          void *ws, size_t ws_bytes, void *stream);

/*
 * fdvm_iir_laplacian -- the IIR blur and the high-pass stage in one call:
 * writes V_s = sigma_s^2 (D20 + D02) of the IIR blur B_s (Table I
 * d = 2 taps along x and along y, clamp-to-edge extension of B_s), i.e. what
 * fdvm_blur_iir followed by fdvm_highpass(FDVM_HP_LAPLACIAN, normalize = 1)
 * computes, without storing B_s: the Laplacian is formed in float64 from the
 * unrounded blur.
 *   Arguments as fdvm_blur_iir; `out` receives the V planes; ws of at least
 *   fdvm_workspace_bytes(FDVM_OP_IIR_LAPLACIAN, H, W, nscales, 0) bytes (holds
 *   the x-pass planes and the column-pass states).
 */
fdvm_status fdvm_iir_laplacian(const void *in, fdvm_dtype dt, int64_t H, int64_t W, int64_t in_pitch,
                               float *out, int64_t out_pitch, int64_t plane_stride,
                               const fdvm_filter *filters, int nscales, fdvm_boundary bc,
                               void *ws, size_t ws_bytes, void *stream);

/*
 * fdvm_blur_fir -- separable FIR blur (Eq A5), x then y, nscales scales.
 *   Same image arguments as fdvm_blur_iir.
 *   taps      host float64 array: the taps of scale s are taps[tap_offset[s] ..
 *             tap_offset[s] + 2 K_s], K_s = half_len[s] (h(-K)..h(K), as
 *             written by fdvm_filter_design).  Taps must be symmetric.
 *   half_len  host int32[nscales], each in [1, FDVM_MAX_FIR_HALF].
 *   tap_offset host int32[nscales].
 *   algo      FDVM_FIR_DIRECT (LDS-staged direct convolution, float32, x then
 *             y), FDVM_FIR_TOEPLITZ_MFMA (Toeplitz-block products on the
 *             matrix cores, float32 operands and accumulation, y then x: the
 *             two orders agree up to rounding for a separable filter with a
 *             separable extension, Section 2) or FDVM_FIR_TOEPLITZ_MFMA_HALF
 *             (the same products with half-precision operands, float32
 *             accumulation, x then y: float16 and bfloat16 frames are the
 *             operands as stored, uint16 frames are split exactly into a
 *             float16 pair; the taps and the intermediate are each carried
 *             as a hi + lo pair of the operand type, so the dc gain and
 *             moments of the taps hold to ~2^-22 (float16 operands) /
 *             ~2^-16 (bfloat16); dt FDVM_F32 gives FDVM_EINVAL).
 *   ws, ws_bytes device workspace of at least
 *             fdvm_workspace_bytes(FDVM_OP_BLUR_FIR, H, W, nscales, maxK) bytes
 *             (the first-pass planes: one for FDVM_FIR_DIRECT, nscales
 *             transposed ones for the Toeplitz forms, plus the half form's
 *             tap tables).
 * Returns FDVM_EINVAL / FDVM_ERANGE / FDVM_ENOMEM (workspace too small) /
 * FDVM_EDEVICE.
 */
fdvm_status fdvm_blur_fir(const void *in, fdvm_dtype dt, int64_t H, int64_t W, int64_t in_pitch,
                          float *out, int64_t out_pitch, int64_t plane_stride,
                          const double *taps, const int32_t *half_len, const int32_t *tap_offset,
                          int nscales, fdvm_boundary bc, int algo,
                          void *ws, size_t ws_bytes, void *stream);

/*
 * fdvm_fir_laplacian -- the FIR form of the detection response:
 *   V_s = sigma_s^2 (D20 + D02) B_s with B_s the separable FIR blur of Eq A5
 *   (x then y, extension bc) and the Table I d = 2 differences taken on the
 *   replicate extension of B_s (as fdvm_highpass), in one call.  Both FIR
 *   passes accumulate in float64 and the x-pass planes are float64, so the
 *   blur is never rounded before the second differences (the normalised
 *   Laplacian multiplies a rounding of B by about 8 sigma^2); only V is
 *   rounded, to float32.  This is the FIR counterpart of fdvm_iir_laplacian,
 *   the input of fdvm_detect_blobs (Section 5, the low-pass then high-pass
 *   stages of the two-stage filter bank).
 *   Image arguments and out as fdvm_iir_laplacian.
 *   taps_dev  DEVICE float64 array: the taps of scale s are taps_dev[tap_offset[s]
 *             .. tap_offset[s] + 2 K_s] = h(-K_s) .. h(K_s) (as written by
 *             fdvm_filter_design); read by the kernels, not modified.
 *   half_len, tap_offset  host int32[nscales]; K_s in [1, FDVM_MAX_FIR_HALF].
 *   sigmas    host float64[nscales], > 0: the normalisation sigma_s^2.
 *   ws, ws_bytes device workspace of at least
 *             fdvm_workspace_bytes(FDVM_OP_FIR_LAPLACIAN, H, W, nscales, 0)
 *             bytes (one float64 x-pass plane, reused scale by scale).
 * Returns FDVM_EINVAL / FDVM_ERANGE / FDVM_ENOMEM / FDVM_EDEVICE.
 */
fdvm_status fdvm_fir_laplacian(const void *in, fdvm_dtype dt, int64_t H, int64_t W, int64_t in_pitch, float *out,
                               int64_t out_pitch, int64_t plane_stride, const double *taps_dev,
                               const int32_t *half_len, const int32_t *tap_offset, const double *sigmas,
                               int nscales, fdvm_boundary bc, void *ws, size_t ws_bytes, void *stream);

/*
 * fdvm_iir_hessian -- the paper's blob detector (Section 5, Eqs 26-27) on the
 * IIR blur (repeated-pole or Butterworth designs), fused like
 * fdvm_iir_laplacian: per scale and pixel the
 * Hessian H = [[D20, D11], [D11, D02]] of the blur B_s (Table I taps, d = 2
 * central second differences, D11 the d = 1 difference along x of the d = 1
 * difference along y, clamp-to-edge extension), formed in float64 from the
 * unrounded blur.  `out` plane s receives sigma_s^4 |H|.  A pixel with
 * border <= y < H - border, border <= x < W - border is a detection when
 * sigma^4 |H| > t1 (Threshold #1) and, if t2 > 0, the Newton offset
 * (dx, dy) = ((D01 D11 - D02 D10) / |H|, (D10 D11 - D20 D01) / |H|) has
 * length < t2 (Threshold #2).  Detections go to out_dev in (scale, y, x)
 * order with value sigma^4 |H| and polarity +1 where D20 < 0 (a maximum of
 * the blur: bright blob), else -1; count_dev as fdvm_detect_blobs.
 *   Other arguments as fdvm_iir_laplacian; ws of at least
 *   fdvm_workspace_bytes(FDVM_OP_IIR_HESSIAN, H, W, nscales, 0) bytes.
 */
fdvm_status fdvm_iir_hessian(const void *in, fdvm_dtype dt, int64_t H, int64_t W, int64_t in_pitch, float *out,
                             int64_t out_pitch, int64_t plane_stride, const fdvm_filter *filters, int nscales,
                             fdvm_boundary bc, float t1, float t2, int border, fdvm_blob *out_dev, int32_t cap,
                             int32_t *count_dev, void *ws, size_t ws_bytes, void *stream);

/* ------------------------------------------------------------------ adjoints
 * Transposed operators for gradients (the paper's filters are linear; these
 * are the exact transposes of the float64-defined operators).
 *
 * fdvm_blur_iir_adjoint -- out_s = G_s^T g_s for the separable repeated-pole
 *   blur G_s of fdvm_blur_iir (rows then columns, extension bc): the
 *   zero-start recursions along columns then rows (h is symmetric), and, for
 *   the replicate extension, the tails that the transposed extension folds
 *   back onto the first and last sample of every column and row,
 *   sum_m g(m) T(m) with T(m) = sum_{k>m} h(k).
 *   g, out: device float32 planes (pitch, plane stride as in fdvm_blur_iir;
 *   must not overlap).  filters: FDVM_IIR_REPEATED_POLE designs (Butterworth
 *   designs return FDVM_EUNSUPPORTED).  ws: device,
 *   >= fdvm_workspace_bytes(FDVM_OP_BLUR_IIR_ADJOINT, H, W, nscales, 0).
 */
fdvm_status fdvm_blur_iir_adjoint(const float *g, int64_t H, int64_t W, int64_t pitch, int64_t plane_stride,
                                  float *out, int64_t out_pitch, int64_t out_plane_stride,
                                  const fdvm_filter *filters, int nscales, fdvm_boundary bc, void *ws,
                                  size_t ws_bytes, void *stream);

/*
 * fdvm_laplacian_adjoint -- out_s = sigma_s^2 Lap^T g_s, the transpose of the
 *   normalised Laplacian of fdvm_highpass(FDVM_HP_LAPLACIAN, normalize = 1)
 *   (Table I d = 2 taps along x and y, clamp-to-edge extension).
 *   g, out: device float32 planes, must not overlap.
 */
fdvm_status fdvm_laplacian_adjoint(const float *g, int64_t H, int64_t W, int64_t pitch, int64_t plane_stride,
                                   int nscales, const double *sigmas, float *out, int64_t out_pitch,
                                   int64_t out_plane_stride, void *stream);

/*
 * fdvm_plane_dots -- out_dev[s] = sum_{y,x} a_s(y, x) b_s(y, x) in float64,
 *   summed in a fixed order (the same result on every run).  a, b: device
 *   float32 planes with the same pitch and plane stride.  ws: device,
 *   >= fdvm_workspace_bytes(FDVM_OP_PLANE_DOTS, H, W, nscales, 0).
 */
fdvm_status fdvm_plane_dots(const float *a, const float *b, int64_t H, int64_t W, int64_t pitch,
                            int64_t plane_stride, int nscales, double *out_dev, void *ws, size_t ws_bytes,
                            void *stream);

/* ------------------------------------------------------------------ backward
 * Gradients of a loss L through the detection response of a batch of
 * nframes frames of one size,
 *     V_s = sigma_s^2 (D20 + D02)(B_s),   B_s = G_s x
 * (fdvm_iir_laplacian / fdvm_fir_laplacian), given gV = dL/dV:
 *     gB_s     = sigma_s^2 Lap^T gV_s                     (as fdvm_laplacian_adjoint)
 *     gx       = sum_s G_s^T gB_s                         (what & FDVM_GRAD_X)
 *     gsigma_s = sum over frames of
 *                2/sigma_s <gV_s, V_s> + <gB_s, dB_s/dsigma_s>   (what & FDVM_GRAD_SIGMA)
 * For the separable blur dB_s/dsigma = (G'_y G_x + G_y G'_x) x, G' the pass
 * with the sigma-derivative filter (the extension does not depend on sigma).
 * All of it runs on the device in float32 planes with float64 inner
 * products (fixed summation order: deterministic); nothing is copied to the
 * host and the call does not synchronise.
 *   x        device, frame f at x + f * x_frame_stride elements (dt, row
 *            pitch x_pitch); read only for FDVM_GRAD_SIGMA (may be NULL
 *            otherwise).
 *   V, gV    device float32; frame f, scale s, pixel (y, x) at
 *            [f * v_frame_stride + s * plane_stride + y * pitch + x]; V is
 *            read only for FDVM_GRAD_SIGMA (may be NULL otherwise).
 *   gx       device float32, frame f pixel (y, x) at
 *            [f * gx_frame_stride + y * gx_pitch + x], overwritten
 *            (FDVM_GRAD_X; may be NULL otherwise).  Must not overlap the
 *            inputs.
 *   gsigma   device float64 [nscales], overwritten with the batch sum
 *            (FDVM_GRAD_SIGMA; may be NULL otherwise).
 *   ws       device workspace >= fdvm_workspace_bytes(
 *            FDVM_OP_IIR_LAPLACIAN_BACKWARD / FDVM_OP_FIR_LAPLACIAN_BACKWARD,
 *            H, W, nscales, max K).  The frames run on up to four lanes
 *            (internal streams that wait on an event recorded on `stream`,
 *            and on which `stream` waits in turn; frame f on lane f mod 4),
 *            each with its own part of the workspace; the sigma gradient is
 *            summed per lane in frame order, then over the lanes in order.
 * Errors as the forward calls; what = 0 or any other bit is FDVM_EINVAL.
 */
enum { FDVM_GRAD_X = 1, FDVM_GRAD_SIGMA = 2 };

/* IIR form (Sections 4.3 and 5: the transposes of the recursions of Eqs
 * A6-A10 with the replicate start of Eq A32, as fdvm_blur_iir_adjoint, and the
 * sigma-derivative cascade of fdvm_iir_pass).  filters: FDVM_IIR_REPEATED_POLE designs of
 * one order; their sigma derivatives are designed inside the call
 * (FDVM_IIR_REPEATED_POLE_DSIGMA).  Butterworth designs: FDVM_EUNSUPPORTED. */
fdvm_status fdvm_iir_laplacian_backward(const void *x, fdvm_dtype dt, int64_t H, int64_t W, int64_t x_pitch,
                                        int64_t x_frame_stride, const float *V, const float *gV, int64_t pitch,
                                        int64_t plane_stride, int64_t v_frame_stride, int nframes,
                                        const fdvm_filter *filters, int nscales, fdvm_boundary bc, unsigned what,
                                        float *gx, int64_t gx_pitch, int64_t gx_frame_stride, double *gsigma,
                                        void *ws, size_t ws_bytes, void *stream);

/* FIR form (Eq A5 transposed: the zero-extension FIR of the symmetric taps
 * plus, for the replicate extension, the folded tails sum_m g(m) T(m),
 * T(m) = sum_{k>m} h(k), added to the first and last sample of every column
 * and row).  taps / half_len / tap_offset: host, as fdvm_blur_fir;
 * dtaps: host, dh/dsigma in the same layout (fdvm_filter_design with
 * FDVM_FIR_COLORED_SG_DSIGMA / FDVM_FIR_GAUSSIAN_DSIGMA; needed only for
 * FDVM_GRAD_SIGMA); sigmas: host, the scales of the sigma^2 factor. */
fdvm_status fdvm_fir_laplacian_backward(const void *x, fdvm_dtype dt, int64_t H, int64_t W, int64_t x_pitch,
                                        int64_t x_frame_stride, const float *V, const float *gV, int64_t pitch,
                                        int64_t plane_stride, int64_t v_frame_stride, int nframes,
                                        const double *taps, const double *dtaps, const int32_t *half_len,
                                        const int32_t *tap_offset, const double *sigmas, int nscales,
                                        fdvm_boundary bc, unsigned what, float *gx, int64_t gx_pitch,
                                        int64_t gx_frame_stride, double *gsigma, void *ws, size_t ws_bytes,
                                        void *stream);

/* workspace sizes */
enum { FDVM_OP_BLUR_IIR = 0, FDVM_OP_BLUR_FIR = 1, FDVM_OP_DETECT = 2, FDVM_OP_IIR_LAPLACIAN = 3,
       FDVM_OP_BLUR_IIR_ADJOINT = 4, FDVM_OP_PLANE_DOTS = 5, FDVM_OP_IIR_HESSIAN = 6,
       FDVM_OP_FIR_LAPLACIAN = 7, FDVM_OP_IIR_LAPLACIAN_BACKWARD = 8, FDVM_OP_FIR_LAPLACIAN_BACKWARD = 9,
       FDVM_OP_FIR_LAPLACIAN_MFMA = 10 };

/* Bytes of device workspace `op` needs for an H x W frame with nscales
 * scales and maximum FIR half-length max_half_len (0 if unused). */
size_t fdvm_workspace_bytes(int op, int64_t H, int64_t W, int nscales, int max_half_len);

/* Largest FIR half-length of fdvm_fir_laplacian_mfma: the difference taps
 * reach K + 1, which must fit the matrix-core tap tables (512 at most). */
#define FDVM_MAX_FIR_LAP_MFMA_HALF 511

/*
 * fdvm_fir_laplacian_mfma -- the FIR detection response of
 *   fdvm_fir_laplacian (the same V_s = sigma_s^2 (D20 + D02) B_s, Section 5
 *   and Table I on the blur of Eq A5) on the matrix cores with
 *   half-precision operands, as the two-stage band-pass of Section 5:
 *   with d_s = h_s * [1, -2, 1], V_s = sigma_s^2 (h_s(y) d_s(x) x +
 *   d_s(y) h_s(x) x), the x pass forming both row filters and the y pass
 *   both column filters (FDVM_FIR_TOEPLITZ_MFMA_HALF's operand pairs and
 *   float32 accumulation); no blur plane is formed or rounded.  The
 *   first and last rows and columns, where the differences of
 *   fdvm_fir_laplacian take the replicate extension of B_s and these
 *   filters the extension of the frame, are corrected in float64.
 *   Error against the float64 response: at most sigma_s^2 (sum |h_s|)
 *   (sum |d_s|) max |x| (12 2^-2p + (4 n + 2) 2^-24), p = 11 (float16 operands:
 *   F16 and U16 frames) or 8 (BF16), n = 2 K_s + 3 accumulated terms per pass
 *   (split taps and samples, the stored split intermediate, float32 sums and
 *   the float32 partial response between the two y filters).
 *   in, dt   F16, BF16 or U16 (F32 is rejected with FDVM_EINVAL, as for
 *            FDVM_FIR_TOEPLITZ_MFMA_HALF); image arguments and out as
 *            fdvm_iir_laplacian.
 *   taps, half_len, tap_offset  HOST, as fdvm_blur_fir (symmetric taps);
 *            K_s in [1, FDVM_MAX_FIR_LAP_MFMA_HALF].
 *   sigmas   host float64[nscales], > 0.
 *   ws, ws_bytes device workspace of at least
 *            fdvm_workspace_bytes(FDVM_OP_FIR_LAPLACIAN_MFMA, H, W, nscales, 0).
 * Returns FDVM_EINVAL / FDVM_ERANGE / FDVM_ENOMEM / FDVM_EUNSUPPORTED (no
 * matrix cores) / FDVM_EDEVICE.
 */
fdvm_status fdvm_fir_laplacian_mfma(const void *in, fdvm_dtype dt, int64_t H, int64_t W, int64_t in_pitch,
                                    float *out, int64_t out_pitch, int64_t plane_stride, const double *taps,
                                    const int32_t *half_len, const int32_t *tap_offset, const double *sigmas,
                                    int nscales, fdvm_boundary bc, void *ws, size_t ws_bytes, void *stream);

/*
 * fdvm_highpass -- Table I interpolating differences of blur planes with
 * clamp-to-edge extension.  For each scale s and each bit in `what`
 * (FDVM_HP_*, in increasing bit order) one output plane is written:
 *   LAPLACIAN: norm_s (D20 + D02), norm_s = sigmas[s]^2 if normalize else 1
 *   D20 = B(x+1) - 2B + B(x-1), D02 likewise along y,
 *   D10 = (B(x+1) - B(x-1))/2, D01 likewise, D11 = D10 applied along y.
 *   blur      device float32 planes (pitch, plane_stride as in blur_iir)
 *   sigmas    host float64[nscales]
 *   out       device float32; output plane j of scale s (j counts the set bits
 *             of `what`) at out[(s * nout + j) * out_plane_stride + y * pitch + x]
 *             where nout = number of bits set.  Must not overlap `blur`.
 */
fdvm_status fdvm_highpass(const float *blur, int64_t H, int64_t W, int64_t pitch, int64_t plane_stride,
                          int nscales, const double *sigmas, unsigned what, int normalize,
                          float *out, int64_t out_plane_stride, void *stream);

/*
 * fdvm_detect_blobs -- multi-scale strict extrema of the response planes.
 * A pixel (s, y, x) with border <= y < H - border, border <= x < W - border
 * is a detection when V is strictly below every existing neighbour in the
 * 3 x 3 x 3 block of (scale, y, x) offsets and V <= -tau (bright blob,
 * polarity +1), or strictly above every neighbour and V >= tau (dark blob,
 * polarity -1).  Neighbours outside the stack are ignored; ties never detect.
 *   resp      device float32 planes (as blur_iir's out)
 *   out_dev   device fdvm_blob[cap], filled in (scale, y, x) order
 *   count_dev device int32[1]: receives the TRUE number of detections (may
 *             exceed cap; only the first cap are written)
 *   ws        device workspace >= fdvm_workspace_bytes(FDVM_OP_DETECT, ...)
 * The call is asynchronous; the caller reads *count_dev after synchronising
 * and treats count > cap as overflow.  tau >= 0, border >= 0.  The planes
 * must hold no NaN (the comparisons run on order-preserving integer keys).
 */
fdvm_status fdvm_detect_blobs(const float *resp, int64_t H, int64_t W, int64_t pitch, int64_t plane_stride,
                              int nscales, float tau, int border, fdvm_blob *out_dev, int32_t cap,
                              int32_t *count_dev, void *ws, size_t ws_bytes, void *stream);

/* ------------------------------------------------------------------ batch
 * One call over many frames of uneven size (Section 2's filter bank per frame,
 * the same scales for all): for every frame, the fused repeated-pole blur and
 * normalised Laplacian (as fdvm_iir_laplacian) and the multi-scale extrema
 * (as fdvm_detect_blobs).  The frames are spread over up to nlanes internal
 * streams that fork from and join back into `stream` through events, so the
 * whole batch can be captured into one HIP graph by capturing `stream`.
 */
typedef struct {
    const void *data;     /* device, H x W elements of type dtype, row pitch `pitch` */
    int32_t dtype;        /* fdvm_dtype */
    int32_t H, W;         /* 1 <= H <= 65535, 1 <= W <= 16384 */
    int32_t row_chunk;    /* row-pass samples per lane: 0 = chosen from W, else 8, 16 or 32 */
    int64_t pitch;        /* elements, >= W */
    fdvm_blob *out;       /* device, capacity cap, filled in (scale, y, x) order */
    int32_t *count;       /* device int32[1]: true number of detections of this frame */
    int32_t cap;
    int32_t reserved;
} fdvm_frame;

#define FDVM_MAX_LANES 16

/* Workspace for fdvm_batch_detect: per lane, the largest frame's x-pass
 * planes, column states, row exponents, V planes and detection words. */
size_t fdvm_batch_workspace_bytes(const fdvm_frame *frames, int nframes, int nscales, int nlanes);

/*
 * fdvm_batch_detect -- frames[i] (host array of nframes descriptors) with the
 *   nscales IIR designs `filters`, boundary bc, threshold tau, border margin.
 *   nlanes in [1, FDVM_MAX_LANES] concurrent lanes (frame i runs on lane
 *   i % nlanes).  ws: device, >= fdvm_batch_workspace_bytes(...).  Frame
 *   outputs as fdvm_detect_blobs (count may exceed cap).
 *   The internal streams and events are created once per device and reused;
 *   calls that overlap on one device must not share them (serialise them).
 *   Every lane forked from `stream` is joined back into it on every return
 *   after the fork, also after a failed launch.
 * Returns FDVM_EINVAL / FDVM_ERANGE / FDVM_ENOMEM / FDVM_EUNSUPPORTED /
 * FDVM_EDEVICE as the single-frame calls; nothing is enqueued on a
 * validation error.
 */
fdvm_status fdvm_batch_detect(const fdvm_frame *frames, int nframes, const fdvm_filter *filters, int nscales,
                              fdvm_boundary bc, float tau, int border, int nlanes, void *ws, size_t ws_bytes,
                              void *stream);

/* ------------------------------------------------------------------ no allocation
 * For callers that cannot allocate device memory or pass a workspace: code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  The library keeps one fixed scratch array of
 * FDVM_NOALLOC_SCRATCH_BYTES in the memory of every device it runs on (from
 * the first use on that device until the process ends); no call here
 * allocates anything.
 */
#define FDVM_NOALLOC_SCRATCH_BYTES (32u << 20)

/* Size of the fixed scratch array of each device, in bytes. */
size_t fdvm_noalloc_scratch_bytes(void);

/*
 * fdvm_detect_blobs_noalloc -- fdvm_detect_blobs (same arguments, same
 *   results, same kernels) with its workspace taken from the device's fixed
 *   scratch array instead of a caller buffer.  The caller still passes resp,
 *   out_dev and count_dev.
 * Returns FDVM_ERANGE when the call would need more than
 *   FDVM_NOALLOC_SCRATCH_BYTES of workspace, i.e. when
 *   fdvm_workspace_bytes(FDVM_OP_DETECT, H, W, nscales, 0) exceeds it (about
 *   nscales * H * ceil(W / 62) * 8 bytes: 2048 x 2048 x 8 scales takes 4.5 MB,
 *   4096 columns x 3072 rows x 12 scales 19.8 MB); otherwise as
 *   fdvm_detect_blobs.  All calls on one device share its scratch array:
 *   calls that overlap on one device (several streams or threads) race and
 *   must be serialised by the caller.
 */
fdvm_status fdvm_detect_blobs_noalloc(const float *resp, int64_t H, int64_t W, int64_t pitch, int64_t plane_stride,
                                      int nscales, float tau, int border, fdvm_blob *out_dev, int32_t cap,
                                      int32_t *count_dev, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* FDVM_H */
