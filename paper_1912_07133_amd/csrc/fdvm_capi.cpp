// C ABI of the blob-detection filter bank: argument validation on the host,
// then dispatch to the HIP kernels.  See include/fdvm.h for the contract.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "fdvm_internal.h"

using namespace fdvm;

namespace {

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

fdvm_status from_hip(hipError_t e) { return e == hipSuccess ? FDVM_OK : FDVM_EDEVICE; }

fdvm_status check_image(const void *in, int64_t H, int64_t W, int64_t in_pitch) {
    if (!in) return FDVM_EINVAL;
    if (H < 1 || W < 1 || H > 65535 || W > 16384) return FDVM_EINVAL;
    if (in_pitch < W) return FDVM_EINVAL;
    return FDVM_OK;
}

fdvm_status check_planes(const void *out, int64_t H, int64_t W, int64_t pitch, int64_t plane_stride,
                         int nscales) {
    if (!out) return FDVM_EINVAL;
    if (nscales < 1 || nscales > FDVM_MAX_SCALES) return FDVM_EINVAL;
    if (pitch < W) return FDVM_EINVAL;
    if (nscales > 1 && plane_stride < H * pitch) return FDVM_EINVAL;
    if (nscales == 1 && plane_stride < 0) return FDVM_EINVAL;
    return FDVM_OK;
}

}  // namespace

namespace fdvm {
fdvm_status detect_check(const float *resp, int64_t H, int64_t W, int64_t pitch, int64_t plane_stride, int nscales,
                         float tau, int border, const void *out_dev, int32_t cap, const int32_t *count_dev) {
    fdvm_status st = check_image(resp, H, W, pitch);
    if (st != FDVM_OK) return st;
    if (!out_dev || !count_dev) return FDVM_EINVAL;
    if (nscales < 1 || nscales > FDVM_MAX_SCALES) return FDVM_EINVAL;
    if (nscales > 1 && plane_stride < H * pitch) return FDVM_EINVAL;
    if (!(tau >= 0.0f) || !std::isfinite(tau) || border < 0 || cap < 0) return FDVM_EINVAL;
    return FDVM_OK;
}
}  // namespace fdvm

extern "C" {

const char *fdvm_status_string(fdvm_status s) {
    switch (s) {
        case FDVM_OK: return "ok";
        case FDVM_EINVAL: return "invalid argument";
        case FDVM_ERANGE: return "parameter out of the supported range";
        case FDVM_ENOMEM: return "buffer too small";
        case FDVM_EDEVICE: return "HIP device error";
        case FDVM_EOVERFLOW: return "detection list overflow";
        case FDVM_EUNSUPPORTED: return "not supported";
    }
    return "unknown status";
}

fdvm_status fdvm_filter_design(fdvm_kind kind, int order, double sigma, int fir_half_len,
                               fdvm_filter *out, double *taps, int taps_cap) {
    if (!out) return FDVM_EINVAL;
    if (!std::isfinite(sigma)) return FDVM_ERANGE;
    fdvm_filter f;
    std::memset(&f, 0, sizeof(f));
    f.kind = kind;
    f.sigma = sigma;
    if (kind == FDVM_IIR_REPEATED_POLE_DSIGMA) {
        if (order != 2 && order != 3) return FDVM_EINVAL;
        if (!(sigma >= 0.25 && sigma <= 4096.0)) return FDVM_ERANGE;
        const Cascade d = sigma_derivative_realisation(order, sigma);
        f.order = order;
        f.p = d.p;
        f.b0 = d.b0;
        *out = f;
        return FDVM_OK;
    }
    if (kind == FDVM_IIR_BUTTERWORTH) {
        if (order != 4) return FDVM_EINVAL;
        if (!(sigma >= 0.5 && sigma <= 4096.0)) return FDVM_ERANGE;
        double wc, db[3], da[3];
        const Cascade c = butterworth_realisation(sigma, &wc, db, da);
        f.order = order;
        f.p = c.p;
        f.b0 = c.b0;
        for (int m = 0; m < 3; ++m) {
            f.bp[m] = db[m];
            f.ap[m] = da[m];
        }
        f.side_gain = 0.5 * (1.0 - c.b0);
        f.omega_c = wc;
        *out = f;
        return FDVM_OK;
    }
    if (kind == FDVM_IIR_REPEATED_POLE) {
        if (order != 2 && order != 3) return FDVM_EINVAL;
        if (!(sigma >= 0.25 && sigma <= 4096.0)) return FDVM_ERANGE;
        f.order = order;
        f.p = std::exp(-1.0 / sigma);
        const double e = -std::expm1(-1.0 / sigma);  // 1 - p to full relative precision
        double b0, bp[4], ap[4];
        repeated_pole_de(order, f.p, e, &b0, bp, ap);
        f.b0 = b0;
        for (int m = 0; m < 4; ++m) {
            f.bp[m] = bp[m];
            f.ap[m] = ap[m];
        }
        f.side_gain = 0.5 * (1.0 - b0);
        *out = f;
        return FDVM_OK;
    }
    if (kind == FDVM_FIR_COLORED_SG || kind == FDVM_FIR_GAUSSIAN || kind == FDVM_FIR_COLORED_SG_DSIGMA ||
        kind == FDVM_FIR_GAUSSIAN_DSIGMA) {
        if (!(sigma >= 0.25 && sigma <= 1024.0)) return FDVM_ERANGE;
        const int K = fir_half_len > 0 ? fir_half_len : (int)std::ceil(3.0 * sigma - 1e-9);
        if (K < 1 || K > FDVM_MAX_FIR_HALF) return FDVM_ERANGE;
        if (!taps) return FDVM_EINVAL;
        if (taps_cap < 2 * K + 1) return FDVM_ENOMEM;
        f.order = K;
        f.ntaps = 2 * K + 1;
        int rc;
        if (kind == FDVM_FIR_COLORED_SG || kind == FDVM_FIR_COLORED_SG_DSIGMA) {
            f.omega_c = 3.0 / sigma;
            if (!(f.omega_c < 3.141592653589793)) return FDVM_ERANGE;
            rc = kind == FDVM_FIR_COLORED_SG ? colored_sg_taps(sigma, K, f.omega_c, taps)
                                             : colored_sg_dtaps(sigma, K, f.omega_c, taps);
        } else {
            rc = kind == FDVM_FIR_GAUSSIAN ? gaussian_taps(sigma, K, taps) : gaussian_dtaps(sigma, K, taps);
        }
        if (rc != 0) return FDVM_ERANGE;
        f.b0 = taps[K];
        *out = f;
        return FDVM_OK;
    }
    return FDVM_EINVAL;
}

namespace {
size_t plane_bytes(int64_t H, int64_t W, int n) { return ((size_t)H * W * sizeof(float) * n + 255) & ~(size_t)255; }

// IIR backward: gB | P1 | P2 (nscales planes each) | inner | 3 nscales doubles.
// inner: column states + tail table (blur adjoint, P2 as its u planes) or
// column states of the derivative passes, or the inner-product partials.
size_t iir_backward_inner_bytes(int64_t H, int64_t W, int nscales) {
    const size_t a = iir_cols_workspace_bytes(H, W, nscales, MAX_SECTIONS) + fold_workspace_bytes(H, W, nscales);
    const size_t b = dots_workspace_bytes(H, 3 * nscales);   // the three sets of inner products
    return a > b ? a : b;
}
size_t iir_backward_frame_bytes(int64_t H, int64_t W, int nscales) {
    return 3 * plane_bytes(H, W, nscales) + iir_backward_inner_bytes(H, W, nscales) +
           (((size_t)3 * nscales * sizeof(double) + 255) & ~(size_t)255);
}
// FIR backward: gB (nscales planes) | three single planes | tail table |
// inner-product partials | 2 nscales doubles
size_t fir_backward_frame_bytes(int64_t H, int64_t W, int nscales) {
    return plane_bytes(H, W, nscales) + 3 * plane_bytes(H, W, 1) +
           ((((size_t)std::max(H, W)) * sizeof(double) + 255) & ~(size_t)255) + dots_workspace_bytes(H, nscales) +
           (((size_t)2 * nscales * sizeof(double) + 255) & ~(size_t)255);
}
// The backward calls run the frames of a batch on BWD_LANES lanes (frame f on
// lane f mod BWD_LANES): one frame's kernels are too small to fill the GPU.
// Workspace: one frame's part per lane, then each lane's sigma-gradient
// partial sums (BWD_LANES x nscales doubles).
constexpr int BWD_LANES = 4;
size_t backward_workspace_bytes(size_t frame_bytes, int nscales) {
    return BWD_LANES * frame_bytes + (((size_t)BWD_LANES * nscales * sizeof(double) + 255) & ~(size_t)255);
}
size_t iir_backward_workspace_bytes(int64_t H, int64_t W, int nscales) {
    return backward_workspace_bytes(iir_backward_frame_bytes(H, W, nscales), nscales);
}
size_t fir_backward_workspace_bytes(int64_t H, int64_t W, int nscales) {
    return backward_workspace_bytes(fir_backward_frame_bytes(H, W, nscales), nscales);
}
}  // namespace

size_t fdvm_workspace_bytes(int op, int64_t H, int64_t W, int nscales, int max_half_len) {
    if (H < 1 || W < 1 || nscales < 1) return 0;
    switch (op) {
        case FDVM_OP_BLUR_IIR: return iir_cols_workspace_bytes(H, W, nscales, MAX_SECTIONS) + iir_rexp_bytes(H);
        case FDVM_OP_IIR_LAPLACIAN:
            return (((size_t)H * W * sizeof(int32_t) + 255) & ~(size_t)255) * nscales +
                   iir_cols_workspace_bytes(H, W, nscales, 3) + iir_rexp_bytes(H);
        case FDVM_OP_BLUR_FIR: return fir_workspace_bytes(H, W, nscales, max_half_len);
        case FDVM_OP_DETECT: return detect_workspace_bytes(H, W, nscales);
        case FDVM_OP_BLUR_IIR_ADJOINT:
            return (((size_t)H * W * sizeof(float) * nscales + 255) & ~(size_t)255) +
                   iir_cols_workspace_bytes(H, W, nscales, MAX_SECTIONS) + fold_workspace_bytes(H, W, nscales);
        case FDVM_OP_PLANE_DOTS: return dots_workspace_bytes(H, nscales);
        case FDVM_OP_FIR_LAPLACIAN: return fir_laplacian_workspace_bytes(H, W);
        case FDVM_OP_IIR_LAPLACIAN_BACKWARD: return iir_backward_workspace_bytes(H, W, nscales);
        case FDVM_OP_FIR_LAPLACIAN_BACKWARD: return fir_backward_workspace_bytes(H, W, nscales);
        case FDVM_OP_FIR_LAPLACIAN_MFMA: return fir_laplacian_mfma_workspace_bytes(H, W, nscales);
        case FDVM_OP_IIR_HESSIAN:
            return (((size_t)H * W * sizeof(int32_t) + 255) & ~(size_t)255) * nscales +
                   iir_cols_workspace_bytes(H, W, nscales, 3) + iir_rexp_bytes(H) +
                   2 * detect_workspace_bytes(H, W, nscales);
        default: return 0;
    }
}

namespace {
// Realisations of the nscales designs: all of one kind (the blur, or with
// allow_dsigma its sigma derivative) and one order.
fdvm_status iir_params(const fdvm_filter *filters, int nscales, fdvm_boundary bc, IirParams *prm,
                       bool allow_dsigma = false) {
    if (!filters) return FDVM_EINVAL;
    if (bc != FDVM_BC_REPLICATE && bc != FDVM_BC_ZERO) return FDVM_EINVAL;
    const int order = filters[0].order;
    const int kind = filters[0].kind;
    if (kind == FDVM_IIR_BUTTERWORTH) {
        if (order != 4) return FDVM_EINVAL;
    } else {
        if (order != 2 && order != 3) return FDVM_EINVAL;
        if (kind != FDVM_IIR_REPEATED_POLE && !(allow_dsigma && kind == FDVM_IIR_REPEATED_POLE_DSIGMA))
            return FDVM_EINVAL;
    }
    std::memset(prm, 0, sizeof(*prm));
    prm->nscales = nscales;
    prm->boundary = bc;
    for (int s = 0; s < nscales; ++s) {
        const fdvm_filter &f = filters[s];
        if (f.kind != kind || f.order != order) return FDVM_EINVAL;
        if (!(f.sigma >= (kind == FDVM_IIR_BUTTERWORTH ? 0.5 : 0.25) && f.sigma <= 4096.0)) return FDVM_ERANGE;
        const Cascade c = kind == FDVM_IIR_BUTTERWORTH     ? butterworth_realisation(f.sigma, nullptr, nullptr, nullptr)
                          : kind == FDVM_IIR_REPEATED_POLE ? cascade_realisation(order, f.sigma)
                                                           : sigma_derivative_realisation(order, f.sigma);
        prm->order = c.sections;
        IirScaleParams &q = prm->s[s];
        q.p = c.p;
        q.pim = c.pim;
        q.b0 = c.b0;
        for (int k = 0; k < MAX_SECTIONS; ++k) {
            q.w[k] = c.w[k];
            q.ss[k] = c.ss[k];
        }
        q.lnp = c.lnp;
        q.sig2 = f.sigma * f.sigma;
    }
    return FDVM_OK;
}

fdvm_status check_dtype(fdvm_dtype dt) {
    return (dt == FDVM_U16 || dt == FDVM_F32 || dt == FDVM_F16 || dt == FDVM_BF16) ? FDVM_OK : FDVM_EINVAL;
}
}  // namespace

fdvm_status fdvm_iir_pass(const void *in, fdvm_dtype dt, int64_t H, int64_t W, int64_t in_pitch,
                          int64_t in_plane_stride, float *out, int64_t out_pitch, int64_t plane_stride,
                          const fdvm_filter *filters, int nscales, fdvm_boundary bc, int axis, void *ws,
                          size_t ws_bytes, void *stream) {
    fdvm_status st = check_image(in, H, W, in_pitch);
    if (st != FDVM_OK) return st;
    st = check_planes(out, H, W, out_pitch, plane_stride, nscales);
    if (st != FDVM_OK) return st;
    if (check_dtype(dt) != FDVM_OK) return FDVM_EINVAL;
    IirParams prm;
    st = iir_params(filters, nscales, bc, &prm, axis != 2);
    if (st != FDVM_OK) return st;
    hipStream_t hs = static_cast<hipStream_t>(stream);
    if (axis == 0) {
        if (W > 8 * 64 * 32) return FDVM_EUNSUPPORTED;
        return from_hip(launch_iir_rows(in, dt, H, W, in_pitch, out, out_pitch, plane_stride, nullptr, 0, prm, hs));
    }
    if (axis == 1 || axis == 2) {
        if (dt != FDVM_F32) return FDVM_EINVAL;
        if (nscales > 1 && in_plane_stride < H * in_pitch) return FDVM_EINVAL;
        const bool same = in == static_cast<const void *>(out);
        if (same && (axis == 2 || in_pitch != out_pitch || (nscales > 1 && in_plane_stride != plane_stride)))
            return FDVM_EINVAL;
        if (!ws) return FDVM_EINVAL;
        if (ws_bytes < iir_cols_workspace_bytes(H, W, nscales, prm.order)) return FDVM_ENOMEM;
        return from_hip(launch_iir_cols(in, in_pitch, in_plane_stride, nullptr, out, H, W, out_pitch, plane_stride,
                                        axis == 2, prm, ws, hs));
    }
    return FDVM_EINVAL;
}

fdvm_status fdvm_blur_iir(const void *in, fdvm_dtype dt, int64_t H, int64_t W, int64_t in_pitch, float *out,
                          int64_t out_pitch, int64_t plane_stride, const fdvm_filter *filters, int nscales,
                          fdvm_boundary bc, void *ws, size_t ws_bytes, void *stream) {
    // validate everything (both passes) before enqueueing anything
    fdvm_status st = check_image(in, H, W, in_pitch);
    if (st != FDVM_OK) return st;
    st = check_planes(out, H, W, out_pitch, plane_stride, nscales);
    if (st != FDVM_OK) return st;
    if (check_dtype(dt) != FDVM_OK) return FDVM_EINVAL;
    IirParams prm;
    st = iir_params(filters, nscales, bc, &prm);
    if (st != FDVM_OK) return st;
    if (!ws) return FDVM_EINVAL;
    const size_t st_bytes = iir_cols_workspace_bytes(H, W, nscales, prm.order);
    if (ws_bytes < st_bytes + iir_rexp_bytes(H)) return FDVM_ENOMEM;
    if (W > 8 * 64 * 32) return FDVM_EUNSUPPORTED;
    hipStream_t hs = static_cast<hipStream_t>(stream);
    // the fixed-point intermediate lives in `out` and is replaced in place
    int *rexp = reinterpret_cast<int *>(static_cast<char *>(ws) + st_bytes);
    hipError_t e = launch_iir_rows(in, dt, H, W, in_pitch, out, out_pitch, plane_stride, rexp, 0, prm, hs);
    if (e != hipSuccess) return FDVM_EDEVICE;
    return from_hip(launch_iir_cols(out, out_pitch, plane_stride, rexp, out, H, W, out_pitch, plane_stride, false,
                                    prm, ws, hs));
}

fdvm_status fdvm_iir_laplacian(const void *in, fdvm_dtype dt, int64_t H, int64_t W, int64_t in_pitch, float *out,
                               int64_t out_pitch, int64_t plane_stride, const fdvm_filter *filters, int nscales,
                               fdvm_boundary bc, void *ws, size_t ws_bytes, void *stream) {
    fdvm_status st = check_image(in, H, W, in_pitch);
    if (st != FDVM_OK) return st;
    st = check_planes(out, H, W, out_pitch, plane_stride, nscales);
    if (st != FDVM_OK) return st;
    if (check_dtype(dt) != FDVM_OK) return FDVM_EINVAL;
    IirParams prm;
    st = iir_params(filters, nscales, bc, &prm);
    if (st != FDVM_OK) return st;
    if (!ws) return FDVM_EINVAL;
    const size_t plane_bytes = ((size_t)H * W * sizeof(int32_t) + 255) & ~(size_t)255;
    const size_t st_bytes = iir_cols_workspace_bytes(H, W, nscales, prm.order);
    const size_t need = plane_bytes * nscales + st_bytes + iir_rexp_bytes(H);
    if (ws_bytes < need) return FDVM_ENOMEM;
    if (W > 8 * 64 * 32) return FDVM_EUNSUPPORTED;
    hipStream_t hs = static_cast<hipStream_t>(stream);
    // ws: x-pass fixed-point planes (pitch W) | column states | row exponents
    int32_t *rows = static_cast<int32_t *>(ws);
    const int64_t rstride = (int64_t)(plane_bytes / sizeof(int32_t));
    void *states = static_cast<char *>(ws) + plane_bytes * nscales;
    int *rexp = reinterpret_cast<int *>(static_cast<char *>(states) + st_bytes);
    hipError_t e = launch_iir_rows(in, dt, H, W, in_pitch, rows, W, rstride, rexp, 0, prm, hs);
    if (e != hipSuccess) return FDVM_EDEVICE;
    return from_hip(
        launch_iir_cols(rows, W, rstride, rexp, out, H, W, out_pitch, plane_stride, true, prm, states, hs));
}

fdvm_status fdvm_iir_hessian(const void *in, fdvm_dtype dt, int64_t H, int64_t W, int64_t in_pitch, float *out,
                             int64_t out_pitch, int64_t plane_stride, const fdvm_filter *filters, int nscales,
                             fdvm_boundary bc, float t1, float t2, int border, fdvm_blob *out_dev, int32_t cap,
                             int32_t *count_dev, void *ws, size_t ws_bytes, void *stream) {
    fdvm_status st = check_image(in, H, W, in_pitch);
    if (st != FDVM_OK) return st;
    st = check_planes(out, H, W, out_pitch, plane_stride, nscales);
    if (st != FDVM_OK) return st;
    if (check_dtype(dt) != FDVM_OK) return FDVM_EINVAL;
    if (!out_dev || !count_dev || cap < 0 || border < 0 || !std::isfinite(t1) || !std::isfinite(t2))
        return FDVM_EINVAL;
    IirParams prm;
    st = iir_params(filters, nscales, bc, &prm);
    if (st != FDVM_OK) return st;
    if (!ws) return FDVM_EINVAL;
    const size_t plane_bytes = ((size_t)H * W * sizeof(int32_t) + 255) & ~(size_t)255;
    const size_t st_bytes = iir_cols_workspace_bytes(H, W, nscales, prm.order);
    const size_t rx_bytes = iir_rexp_bytes(H);
    const size_t det_bytes = detect_workspace_bytes(H, W, nscales);
    if (ws_bytes < plane_bytes * nscales + st_bytes + rx_bytes + 2 * det_bytes) return FDVM_ENOMEM;
    if (W > 8 * 64 * 32) return FDVM_EUNSUPPORTED;
    hipStream_t hs = static_cast<hipStream_t>(stream);
    // ws: x-pass fixed-point planes | column states | row exponents |
    //     detection words + counts | bright-polarity words
    char *w = static_cast<char *>(ws);
    int32_t *rows = reinterpret_cast<int32_t *>(w);
    const int64_t rstride = (int64_t)(plane_bytes / sizeof(int32_t));
    void *states = w + plane_bytes * nscales;
    int *rexp = reinterpret_cast<int *>(w + plane_bytes * nscales + st_bytes);
    void *det = w + plane_bytes * nscales + st_bytes + rx_bytes;
    unsigned long long *pmask = reinterpret_cast<unsigned long long *>(static_cast<char *>(det) + det_bytes);
    HessArgs hz{t1, t2, border, 0, detect_mask_words(det), pmask};
    hipError_t e = launch_iir_rows(in, dt, H, W, in_pitch, rows, W, rstride, rexp, 0, prm, hs);
    if (e == hipSuccess)
        e = launch_iir_cols_mode(rows, W, rstride, rexp, out, H, W, out_pitch, plane_stride, COLS_HESSIAN, &hz, prm,
                                 states, hs);
    if (e == hipSuccess)
        e = launch_compact(out, H, W, out_pitch, plane_stride, nscales, pmask, out_dev, cap, count_dev, det, hs);
    return from_hip(e);
}

namespace {
size_t align256(size_t n) { return (n + 255) & ~(size_t)255; }

// G^T = (fold_x + zero-start x pass) (fold_y + zero-start y pass), u: nscales
// planes of pitch W (G_y^T g), states: column-pass states, tab: the tails
hipError_t blur_iir_adjoint_core(const float *g, int64_t pitch, int64_t plane_stride, int64_t H, int64_t W,
                                 float *out, int64_t out_pitch, int64_t out_plane_stride, const IirParams &prm,
                                 fdvm_boundary bc, float *u, void *states, double *tab, hipStream_t hs) {
    const int nscales = prm.nscales;
    IirParams zp = prm;
    zp.boundary = FDVM_BC_ZERO;
    hipError_t e = launch_iir_cols(g, pitch, plane_stride, nullptr, u, H, W, W, H * W, false, zp, states, hs);
    if (e == hipSuccess && bc == FDVM_BC_REPLICATE) e = launch_fold_table(H, W, prm, tab, hs);
    if (e == hipSuccess && bc == FDVM_BC_REPLICATE)
        e = launch_fold(g, pitch, plane_stride, u, W, H * W, H, W, prm, tab, 1, hs);
    for (int s = 0; e == hipSuccess && s < nscales; ++s) {
        IirParams one = zp;
        one.nscales = 1;
        one.s[0] = zp.s[s];
        e = launch_iir_rows(u + (int64_t)s * H * W, FDVM_F32, H, W, W, out + (int64_t)s * out_plane_stride, out_pitch,
                            out_plane_stride, nullptr, 0, one, hs);
    }
    if (e == hipSuccess && bc == FDVM_BC_REPLICATE)
        e = launch_fold(u, W, H * W, out, out_pitch, out_plane_stride, H, W, prm, tab, 0, hs);
    return e;
}
}  // namespace

fdvm_status fdvm_blur_iir_adjoint(const float *g, int64_t H, int64_t W, int64_t pitch, int64_t plane_stride,
                                  float *out, int64_t out_pitch, int64_t out_plane_stride,
                                  const fdvm_filter *filters, int nscales, fdvm_boundary bc, void *ws,
                                  size_t ws_bytes, void *stream) {
    fdvm_status st = check_image(g, H, W, pitch);
    if (st != FDVM_OK) return st;
    if (nscales > 1 && plane_stride < H * pitch) return FDVM_EINVAL;
    st = check_planes(out, H, W, out_pitch, out_plane_stride, nscales);
    if (st != FDVM_OK) return st;
    if (static_cast<const void *>(g) == static_cast<const void *>(out)) return FDVM_EINVAL;
    IirParams prm;
    st = iir_params(filters, nscales, bc, &prm);
    if (st != FDVM_OK) return st;
    if (prm.order == CPAIR) return FDVM_EUNSUPPORTED;   // folded tails are built for real-pole sections
    if (!ws) return FDVM_EINVAL;
    const size_t ubytes = align256((size_t)H * W * sizeof(float) * nscales);
    const size_t sbytes = iir_cols_workspace_bytes(H, W, nscales, prm.order);
    if (ws_bytes < ubytes + sbytes + fold_workspace_bytes(H, W, nscales)) return FDVM_ENOMEM;
    if (W > 8 * 64 * 32) return FDVM_EUNSUPPORTED;
    // ws: G_y^T g (pitch W) | column states | tail table T_s(m)
    float *u = static_cast<float *>(ws);
    void *states = static_cast<char *>(ws) + ubytes;
    double *tab = reinterpret_cast<double *>(static_cast<char *>(ws) + ubytes + sbytes);
    return from_hip(blur_iir_adjoint_core(g, pitch, plane_stride, H, W, out, out_pitch, out_plane_stride, prm, bc, u,
                                          states, tab, static_cast<hipStream_t>(stream)));
}

fdvm_status fdvm_laplacian_adjoint(const float *g, int64_t H, int64_t W, int64_t pitch, int64_t plane_stride,
                                   int nscales, const double *sigmas, float *out, int64_t out_pitch,
                                   int64_t out_plane_stride, void *stream) {
    fdvm_status st = check_image(g, H, W, pitch);
    if (st != FDVM_OK) return st;
    if (nscales > 1 && plane_stride < H * pitch) return FDVM_EINVAL;
    st = check_planes(out, H, W, out_pitch, out_plane_stride, nscales);
    if (st != FDVM_OK) return st;
    if (!sigmas || static_cast<const void *>(g) == static_cast<const void *>(out)) return FDVM_EINVAL;
    for (int s = 0; s < nscales; ++s)
        if (!finite_pos(sigmas[s])) return FDVM_ERANGE;
    return from_hip(launch_laplacian_adjoint(g, H, W, pitch, plane_stride, nscales, sigmas, out, out_pitch,
                                             out_plane_stride, static_cast<hipStream_t>(stream)));
}

fdvm_status fdvm_plane_dots(const float *a, const float *b, int64_t H, int64_t W, int64_t pitch,
                            int64_t plane_stride, int nscales, double *out_dev, void *ws, size_t ws_bytes,
                            void *stream) {
    fdvm_status st = check_image(a, H, W, pitch);
    if (st != FDVM_OK) return st;
    if (!b || !out_dev || !ws) return FDVM_EINVAL;
    if (nscales < 1 || nscales > FDVM_MAX_SCALES) return FDVM_EINVAL;
    if (nscales > 1 && plane_stride < H * pitch) return FDVM_EINVAL;
    if (ws_bytes < dots_workspace_bytes(H, nscales)) return FDVM_ENOMEM;
    return from_hip(launch_plane_dots(a, b, H, W, pitch, plane_stride, nscales, out_dev, ws,
                                      static_cast<hipStream_t>(stream)));
}

fdvm_status fdvm_blur_fir(const void *in, fdvm_dtype dt, int64_t H, int64_t W, int64_t in_pitch, float *out,
                          int64_t out_pitch, int64_t plane_stride, const double *taps, const int32_t *half_len,
                          const int32_t *tap_offset, int nscales, fdvm_boundary bc, int algo, void *ws,
                          size_t ws_bytes, void *stream) {
    fdvm_status st = check_image(in, H, W, in_pitch);
    if (st != FDVM_OK) return st;
    st = check_planes(out, H, W, out_pitch, plane_stride, nscales);
    if (st != FDVM_OK) return st;
    if (!taps || !half_len || !tap_offset || !ws) return FDVM_EINVAL;
    if (dt != FDVM_U16 && dt != FDVM_F32 && dt != FDVM_F16 && dt != FDVM_BF16) return FDVM_EINVAL;
    if (bc != FDVM_BC_REPLICATE && bc != FDVM_BC_ZERO) return FDVM_EINVAL;
    if (algo != FDVM_FIR_DIRECT && algo != FDVM_FIR_TOEPLITZ_MFMA && algo != FDVM_FIR_TOEPLITZ_MFMA_HALF)
        return FDVM_EINVAL;
    if (algo == FDVM_FIR_TOEPLITZ_MFMA_HALF && dt == FDVM_F32) return FDVM_EINVAL;
    int maxK = 0;
    for (int s = 0; s < nscales; ++s) {
        if (half_len[s] < 1 || half_len[s] > FDVM_MAX_FIR_HALF) return FDVM_ERANGE;
        if (tap_offset[s] < 0) return FDVM_EINVAL;
        if (half_len[s] > maxK) maxK = half_len[s];
        const double *h = taps + tap_offset[s];
        const int K = half_len[s];
        for (int m = 1; m <= K; ++m)
            if (h[K + m] != h[K - m]) return FDVM_EINVAL;  // symmetric taps only
    }
    if (ws_bytes < fir_workspace_bytes(H, W, nscales, maxK)) return FDVM_ENOMEM;
    if (algo != FDVM_FIR_DIRECT && !fir_mfma_available()) return FDVM_EUNSUPPORTED;
    hipError_t e = launch_fir(in, dt, H, W, in_pitch, out, out_pitch, plane_stride, taps, half_len, tap_offset,
                              nscales, bc, algo, ws, ws_bytes, static_cast<hipStream_t>(stream));
    return from_hip(e);
}

fdvm_status fdvm_fir_laplacian(const void *in, fdvm_dtype dt, int64_t H, int64_t W, int64_t in_pitch, float *out,
                               int64_t out_pitch, int64_t plane_stride, const double *taps_dev,
                               const int32_t *half_len, const int32_t *tap_offset, const double *sigmas,
                               int nscales, fdvm_boundary bc, void *ws, size_t ws_bytes, void *stream) {
    fdvm_status st = check_image(in, H, W, in_pitch);
    if (st != FDVM_OK) return st;
    st = check_planes(out, H, W, out_pitch, plane_stride, nscales);
    if (st != FDVM_OK) return st;
    if (check_dtype(dt) != FDVM_OK) return FDVM_EINVAL;
    if (bc != FDVM_BC_REPLICATE && bc != FDVM_BC_ZERO) return FDVM_EINVAL;
    if (!taps_dev || !half_len || !tap_offset || !sigmas || !ws) return FDVM_EINVAL;
    for (int s = 0; s < nscales; ++s) {
        if (half_len[s] < 1 || half_len[s] > FDVM_MAX_FIR_HALF) return FDVM_ERANGE;
        if (tap_offset[s] < 0) return FDVM_EINVAL;
        if (!finite_pos(sigmas[s])) return FDVM_ERANGE;
    }
    if (ws_bytes < fir_laplacian_workspace_bytes(H, W)) return FDVM_ENOMEM;
    return from_hip(launch_fir_laplacian(in, dt, H, W, in_pitch, out, out_pitch, plane_stride, taps_dev, half_len,
                                         tap_offset, sigmas, nscales, bc, ws, static_cast<hipStream_t>(stream)));
}

fdvm_status fdvm_fir_laplacian_mfma(const void *in, fdvm_dtype dt, int64_t H, int64_t W, int64_t in_pitch,
                                    float *out, int64_t out_pitch, int64_t plane_stride, const double *taps,
                                    const int32_t *half_len, const int32_t *tap_offset, const double *sigmas,
                                    int nscales, fdvm_boundary bc, void *ws, size_t ws_bytes, void *stream) {
    fdvm_status st = check_image(in, H, W, in_pitch);
    if (st != FDVM_OK) return st;
    st = check_planes(out, H, W, out_pitch, plane_stride, nscales);
    if (st != FDVM_OK) return st;
    if (dt != FDVM_U16 && dt != FDVM_F16 && dt != FDVM_BF16) return FDVM_EINVAL;
    if (bc != FDVM_BC_REPLICATE && bc != FDVM_BC_ZERO) return FDVM_EINVAL;
    if (!taps || !half_len || !tap_offset || !sigmas || !ws) return FDVM_EINVAL;
    for (int s = 0; s < nscales; ++s) {
        if (half_len[s] < 1 || half_len[s] > FDVM_MAX_FIR_LAP_MFMA_HALF) return FDVM_ERANGE;
        if (tap_offset[s] < 0) return FDVM_EINVAL;
        if (!finite_pos(sigmas[s])) return FDVM_ERANGE;
        const double *h = taps + tap_offset[s];
        const int K = half_len[s];
        for (int m = 1; m <= K; ++m)
            if (h[K + m] != h[K - m]) return FDVM_EINVAL;  // symmetric taps only
    }
    if (ws_bytes < fir_laplacian_mfma_workspace_bytes(H, W, nscales)) return FDVM_ENOMEM;
    if (!fir_mfma_available()) return FDVM_EUNSUPPORTED;
    return from_hip(launch_fir_laplacian_mfma(in, dt, H, W, in_pitch, ws, out, out_pitch, plane_stride, taps,
                                              half_len, tap_offset, sigmas, nscales, bc,
                                              static_cast<hipStream_t>(stream)));
}

fdvm_status fdvm_highpass(const float *blur, int64_t H, int64_t W, int64_t pitch, int64_t plane_stride,
                          int nscales, const double *sigmas, unsigned what, int normalize, float *out,
                          int64_t out_plane_stride, void *stream) {
    fdvm_status st = check_image(blur, H, W, pitch);
    if (st != FDVM_OK) return st;
    if (!out || !sigmas) return FDVM_EINVAL;
    if (nscales < 1 || nscales > FDVM_MAX_SCALES) return FDVM_EINVAL;
    if (nscales > 1 && plane_stride < H * pitch) return FDVM_EINVAL;
    if (what == 0 || (what & ~63u)) return FDVM_EINVAL;
    int nout = 0;
    for (unsigned b = what; b; b >>= 1) nout += (int)(b & 1u);
    if ((nout > 1 || nscales > 1) && out_plane_stride < H * pitch) return FDVM_EINVAL;
    float norms[FDVM_MAX_SCALES];
    for (int s = 0; s < nscales; ++s) {
        if (!finite_pos(sigmas[s])) return FDVM_ERANGE;
        norms[s] = normalize ? (float)(sigmas[s] * sigmas[s]) : 1.0f;
    }
    hipError_t e = launch_highpass(blur, H, W, pitch, plane_stride, nscales, norms, what, out, out_plane_stride,
                                   static_cast<hipStream_t>(stream));
    return from_hip(e);
}

fdvm_status fdvm_detect_blobs(const float *resp, int64_t H, int64_t W, int64_t pitch, int64_t plane_stride,
                              int nscales, float tau, int border, fdvm_blob *out_dev, int32_t cap,
                              int32_t *count_dev, void *ws, size_t ws_bytes, void *stream) {
    fdvm_status st = detect_check(resp, H, W, pitch, plane_stride, nscales, tau, border, out_dev, cap, count_dev);
    if (st != FDVM_OK) return st;
    if (!ws) return FDVM_EINVAL;
    if (ws_bytes < detect_workspace_bytes(H, W, nscales)) return FDVM_ENOMEM;
    hipError_t e = launch_detect(resp, H, W, pitch, plane_stride, nscales, tau, border, out_dev, cap, count_dev,
                                 ws, static_cast<hipStream_t>(stream));
    return from_hip(e);
}


}  // extern "C"

namespace {

// internal streams and events of the batch lanes, created once per device
struct Lanes {
    int device = -1;
    hipStream_t st[FDVM_MAX_LANES] = {};
    hipEvent_t done[FDVM_MAX_LANES] = {};
    hipEvent_t fork = nullptr;
};
std::mutex g_lanes_mu;
std::vector<Lanes *> g_lanes;

Lanes *lanes_for_current_device() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return nullptr;
    std::lock_guard<std::mutex> lock(g_lanes_mu);
    for (Lanes *l : g_lanes)
        if (l->device == dev) return l;
    Lanes *l = new Lanes();
    l->device = dev;
    // default priority, non-blocking with respect to the null stream
    for (int i = 0; i < FDVM_MAX_LANES; ++i)
        if (hipStreamCreateWithFlags(&l->st[i], hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&l->done[i], hipEventDisableTiming) != hipSuccess)
            return nullptr;
    if (hipEventCreateWithFlags(&l->fork, hipEventDisableTiming) != hipSuccess) return nullptr;
    g_lanes.push_back(l);
    return l;
}

// Lanes 0..used-1 forked from the caller's stream with an event, and joined
// back into it with one event per lane, also after a failure, so that a
// capture of the caller's stream stays well formed.  With no lanes forked
// every "lane" is the caller's stream.
struct LaneFork {
    hipStream_t origin;
    Lanes *lanes = nullptr;
    int forked = 0;
    explicit LaneFork(hipStream_t o) : origin(o) {}
    fdvm_status fork(int used) {
        lanes = lanes_for_current_device();
        if (!lanes) return FDVM_EDEVICE;
        if (hipEventRecord(lanes->fork, origin) != hipSuccess) return FDVM_EDEVICE;
        for (int l = 0; l < used; ++l) {
            if (hipStreamWaitEvent(lanes->st[l], lanes->fork, 0) != hipSuccess) return join(FDVM_EDEVICE);
            forked = l + 1;
        }
        return FDVM_OK;
    }
    hipStream_t stream(int l) const { return forked ? lanes->st[l] : origin; }
    fdvm_status join(fdvm_status status) {
        for (int l = 0; l < forked; ++l) {
            if (hipEventRecord(lanes->done[l], lanes->st[l]) != hipSuccess) status = FDVM_EDEVICE;
            else if (hipStreamWaitEvent(origin, lanes->done[l], 0) != hipSuccess) status = FDVM_EDEVICE;
        }
        forked = 0;
        return status;
    }
};

size_t round256(size_t b) { return (b + 255) & ~(size_t)255; }

// per-lane workspace, sized for the largest frame term by term
struct LaneLayout {
    size_t mid = 0, states = 0, rexp = 0, vplanes = 0, det = 0;
    size_t total() const { return mid + states + rexp + vplanes + det; }
};
LaneLayout lane_layout(const fdvm_frame *frames, int nframes, int nscales, int order) {
    LaneLayout L;
    for (int f = 0; f < nframes; ++f) {
        const int64_t H = frames[f].H, W = frames[f].W;
        const size_t plane = round256((size_t)H * W * sizeof(int32_t));
        L.mid = std::max(L.mid, plane * nscales);
        L.states = std::max(L.states, iir_cols_workspace_bytes(H, W, nscales, order));
        L.rexp = std::max(L.rexp, iir_rexp_bytes(H));
        L.vplanes = std::max(L.vplanes, round256((size_t)H * W * sizeof(float) * nscales));
        L.det = std::max(L.det, detect_workspace_bytes(H, W, nscales));
    }
    return L;
}

fdvm_status check_frame(const fdvm_frame &f) {
    if (!f.data || !f.out || !f.count || f.cap < 0) return FDVM_EINVAL;
    if (f.H < 1 || f.W < 1 || f.H > 65535 || f.W > 16384 || f.pitch < f.W) return FDVM_EINVAL;
    if (check_dtype((fdvm_dtype)f.dtype) != FDVM_OK) return FDVM_EINVAL;
    if (f.row_chunk != 0 && f.row_chunk != 8 && f.row_chunk != 16 && f.row_chunk != 32) return FDVM_EINVAL;
    const int64_t chunk = f.row_chunk ? f.row_chunk : 32;
    if (f.W > 8 * 64 * chunk) return FDVM_EUNSUPPORTED;
    return FDVM_OK;
}

}  // namespace

extern "C" {

size_t fdvm_batch_workspace_bytes(const fdvm_frame *frames, int nframes, int nscales, int nlanes) {
    if (!frames || nframes < 1 || nscales < 1 || nscales > FDVM_MAX_SCALES || nlanes < 1 ||
        nlanes > FDVM_MAX_LANES)
        return 0;
    for (int f = 0; f < nframes; ++f)
        if (frames[f].H < 1 || frames[f].W < 1) return 0;
    return lane_layout(frames, nframes, nscales, 3).total() * (size_t)std::min(nlanes, nframes);
}

fdvm_status fdvm_batch_detect(const fdvm_frame *frames, int nframes, const fdvm_filter *filters, int nscales,
                              fdvm_boundary bc, float tau, int border, int nlanes, void *ws, size_t ws_bytes,
                              void *stream) {
    if (!frames || nframes < 1 || !ws) return FDVM_EINVAL;
    if (nscales < 1 || nscales > FDVM_MAX_SCALES) return FDVM_EINVAL;
    if (nlanes < 1 || nlanes > FDVM_MAX_LANES) return FDVM_EINVAL;
    if (!(tau >= 0.0f) || !std::isfinite(tau) || border < 0) return FDVM_EINVAL;
    for (int f = 0; f < nframes; ++f) {
        const fdvm_status st = check_frame(frames[f]);
        if (st != FDVM_OK) return st;
    }
    IirParams prm;
    fdvm_status st = iir_params(filters, nscales, bc, &prm);
    if (st != FDVM_OK) return st;
    const LaneLayout L = lane_layout(frames, nframes, nscales, prm.order);
    const int used = std::min(nlanes, nframes);
    if (ws_bytes < L.total() * (size_t)used) return FDVM_ENOMEM;
    LaneFork lanes(static_cast<hipStream_t>(stream));
    if (used > 1) {
        st = lanes.fork(used);
        if (st != FDVM_OK) return st;
    }
    for (int f = 0; f < nframes; ++f) {
        const fdvm_frame &fr = frames[f];
        const int l = f % used;
        hipStream_t hs = lanes.stream(l);
        char *base = static_cast<char *>(ws) + L.total() * (size_t)l;
        const int64_t H = fr.H, W = fr.W;
        int32_t *mid = reinterpret_cast<int32_t *>(base);
        const int64_t mstride = (int64_t)(round256((size_t)H * W * sizeof(int32_t)) / sizeof(int32_t));
        void *states = base + L.mid;
        int *rexp = reinterpret_cast<int *>(base + L.mid + L.states);
        float *V = reinterpret_cast<float *>(base + L.mid + L.states + L.rexp);
        void *det = base + L.mid + L.states + L.rexp + L.vplanes;
        hipError_t e = launch_iir_rows(fr.data, fr.dtype, H, W, fr.pitch, mid, W, mstride, rexp, fr.row_chunk, prm, hs);
        if (e == hipSuccess)
            e = launch_iir_cols(mid, W, mstride, rexp, V, H, W, W, H * W, true, prm, states, hs);
        if (e == hipSuccess)
            e = launch_detect(V, H, W, W, H * W, nscales, tau, border, fr.out, fr.cap, fr.count, det, hs);
        if (e != hipSuccess) return lanes.join(FDVM_EDEVICE);
    }
    return lanes.join(FDVM_OK);
}

}  // extern "C"

namespace {
// shared argument checks of the two backward calls
fdvm_status backward_check(const void *x, fdvm_dtype dt, int64_t H, int64_t W, int64_t x_pitch,
                           int64_t x_frame_stride, const float *V, const float *gV, int64_t pitch,
                           int64_t plane_stride, int64_t v_frame_stride, int nframes, int nscales, fdvm_boundary bc,
                           unsigned what, const float *gx, int64_t gx_pitch, int64_t gx_frame_stride,
                           const double *gsigma, const void *ws) {
    if (what == 0 || (what & ~(unsigned)(FDVM_GRAD_X | FDVM_GRAD_SIGMA))) return FDVM_EINVAL;
    if (nframes < 1 || !ws) return FDVM_EINVAL;
    if (bc != FDVM_BC_REPLICATE && bc != FDVM_BC_ZERO) return FDVM_EINVAL;
    fdvm_status st = check_planes(gV, H, W, pitch, plane_stride, nscales);
    if (st != FDVM_OK) return st;
    if (H > 65535 || W > 16384) return FDVM_EINVAL;
    if (nframes > 1 && v_frame_stride < (int64_t)nscales * std::max(plane_stride, H * pitch)) return FDVM_EINVAL;
    if (what & FDVM_GRAD_SIGMA) {
        if (!V || !gsigma) return FDVM_EINVAL;
        st = check_image(x, H, W, x_pitch);
        if (st != FDVM_OK) return st;
        if (check_dtype(dt) != FDVM_OK) return FDVM_EINVAL;
        if (nframes > 1 && x_frame_stride < H * x_pitch) return FDVM_EINVAL;
    }
    if (what & FDVM_GRAD_X) {
        st = check_image(gx, H, W, gx_pitch);
        if (st != FDVM_OK) return st;
        if (nframes > 1 && gx_frame_stride < H * gx_pitch) return FDVM_EINVAL;
        if (static_cast<const void *>(gx) == static_cast<const void *>(gV)) return FDVM_EINVAL;
    }
    return FDVM_OK;
}

size_t elem_bytes(fdvm_dtype dt) { return dt == FDVM_F32 ? 4 : 2; }
}  // namespace

extern "C" fdvm_status fdvm_iir_laplacian_backward(const void *x, fdvm_dtype dt, int64_t H, int64_t W,
                                                   int64_t x_pitch, int64_t x_frame_stride, const float *V,
                                                   const float *gV, int64_t pitch, int64_t plane_stride,
                                                   int64_t v_frame_stride, int nframes, const fdvm_filter *filters,
                                                   int nscales, fdvm_boundary bc, unsigned what, float *gx,
                                                   int64_t gx_pitch, int64_t gx_frame_stride, double *gsigma,
                                                   void *ws, size_t ws_bytes, void *stream) {
    fdvm_status st = backward_check(x, dt, H, W, x_pitch, x_frame_stride, V, gV, pitch, plane_stride, v_frame_stride,
                                    nframes, nscales, bc, what, gx, gx_pitch, gx_frame_stride, gsigma, ws);
    if (st != FDVM_OK) return st;
    IirParams prm, dprm;
    st = iir_params(filters, nscales, bc, &prm);
    if (st != FDVM_OK) return st;
    if (prm.order == CPAIR || filters[0].kind != FDVM_IIR_REPEATED_POLE) return FDVM_EUNSUPPORTED;
    if (W > 8 * 64 * 32) return FDVM_EUNSUPPORTED;
    if (ws_bytes < iir_backward_workspace_bytes(H, W, nscales)) return FDVM_ENOMEM;
    double sig[FDVM_MAX_SCALES];
    for (int s = 0; s < nscales; ++s) sig[s] = filters[s].sigma;
    if (what & FDVM_GRAD_SIGMA) {
        fdvm_filter df[FDVM_MAX_SCALES];
        for (int s = 0; s < nscales; ++s) {
            st = fdvm_filter_design(FDVM_IIR_REPEATED_POLE_DSIGMA, filters[s].order, filters[s].sigma, 0, &df[s],
                                    nullptr, 0);
            if (st != FDVM_OK) return st;
        }
        st = iir_params(df, nscales, bc, &dprm, true);
        if (st != FDVM_OK) return st;
    }
    const int64_t P = H * W;   // workspace planes: pitch W, plane H W
    const size_t fbytes = iir_backward_frame_bytes(H, W, nscales);
    const size_t sbytes = iir_cols_workspace_bytes(H, W, nscales, MAX_SECTIONS);
    double *gpart = reinterpret_cast<double *>(static_cast<char *>(ws) + BWD_LANES * fbytes);
    const int used = std::min(BWD_LANES, nframes);
    LaneFork lanes(static_cast<hipStream_t>(stream));
    if (used > 1) {
        st = lanes.fork(used);
        if (st != FDVM_OK) return st;
    }
    hipError_t e = hipSuccess;
    for (int f = 0; e == hipSuccess && f < nframes; ++f) {
        const int l = f % used;
        hipStream_t hs = lanes.stream(l);
        char *w = static_cast<char *>(ws) + l * fbytes;
        float *gB = reinterpret_cast<float *>(w);
        float *P1 = reinterpret_cast<float *>(w + plane_bytes(H, W, nscales));
        float *P2 = reinterpret_cast<float *>(w + 2 * plane_bytes(H, W, nscales));
        char *inner = w + 3 * plane_bytes(H, W, nscales);
        double *res = reinterpret_cast<double *>(inner + iir_backward_inner_bytes(H, W, nscales));
        // the lane's own sigma-gradient sum (first frame of the lane: overwritten)
        double *gs = used > 1 ? gpart + (int64_t)l * nscales : gsigma;
        const float *gVf = gV + (int64_t)f * v_frame_stride;
        e = launch_laplacian_adjoint(gVf, H, W, pitch, plane_stride, nscales, sig, gB, W, P, hs);
        if (e == hipSuccess && (what & FDVM_GRAD_X)) {
            e = blur_iir_adjoint_core(gB, W, P, H, W, P1, W, P, prm, bc, P2, inner,
                                      reinterpret_cast<double *>(inner + sbytes), hs);
            if (e == hipSuccess)
                e = launch_sum_planes(P1, W, P, nscales, H, W, gx + (int64_t)f * gx_frame_stride, gx_pitch, hs);
        }
        if (e == hipSuccess && (what & FDVM_GRAD_SIGMA)) {
            const void *xf = static_cast<const char *>(x) + (int64_t)f * x_frame_stride * (int64_t)elem_bytes(dt);
            // P1 = G_x x, P2 = G'_x x, then in place P2 = G_y G'_x x, P1 = G'_y G_x x
            e = launch_iir_rows(xf, dt, H, W, x_pitch, P1, W, P, nullptr, 0, prm, hs);
            if (e == hipSuccess) e = launch_iir_rows(xf, dt, H, W, x_pitch, P2, W, P, nullptr, 0, dprm, hs);
            if (e == hipSuccess) e = launch_iir_cols(P2, W, P, nullptr, P2, H, W, W, P, false, prm, inner, hs);
            if (e == hipSuccess) e = launch_iir_cols(P1, W, P, nullptr, P1, H, W, W, P, false, dprm, inner, hs);
            if (e == hipSuccess) {
                // <gV, V>, <gB, G_y G'_x x>, <gB, G'_y G_x x> into res[0 .. 3 nscales)
                const float *da[3] = {gVf, gB, gB};
                const float *db[3] = {V + (int64_t)f * v_frame_stride, P2, P1};
                const int64_t dp[3] = {pitch, W, W}, dq[3] = {plane_stride, P, P};
                e = launch_plane_dots_sets(3, da, db, dp, dq, H, W, nscales, res, inner, hs);
            }
            if (e == hipSuccess) e = launch_gsigma(res, res + nscales, 2, sig, nscales, f >= used, gs, hs);
        }
    }
    st = lanes.join(from_hip(e));
    if (st == FDVM_OK && used > 1 && (what & FDVM_GRAD_SIGMA))
        st = from_hip(launch_sum_lanes(gpart, used, nscales, gsigma, static_cast<hipStream_t>(stream)));
    return st;
}

extern "C" fdvm_status fdvm_fir_laplacian_backward(const void *x, fdvm_dtype dt, int64_t H, int64_t W,
                                                   int64_t x_pitch, int64_t x_frame_stride, const float *V,
                                                   const float *gV, int64_t pitch, int64_t plane_stride,
                                                   int64_t v_frame_stride, int nframes, const double *taps,
                                                   const double *dtaps, const int32_t *half_len,
                                                   const int32_t *tap_offset, const double *sigmas, int nscales,
                                                   fdvm_boundary bc, unsigned what, float *gx, int64_t gx_pitch,
                                                   int64_t gx_frame_stride, double *gsigma, void *ws,
                                                   size_t ws_bytes, void *stream) {
    fdvm_status st = backward_check(x, dt, H, W, x_pitch, x_frame_stride, V, gV, pitch, plane_stride, v_frame_stride,
                                    nframes, nscales, bc, what, gx, gx_pitch, gx_frame_stride, gsigma, ws);
    if (st != FDVM_OK) return st;
    if (!taps || !half_len || !tap_offset || !sigmas) return FDVM_EINVAL;
    if ((what & FDVM_GRAD_SIGMA) && !dtaps) return FDVM_EINVAL;
    for (int s = 0; s < nscales; ++s) {
        if (half_len[s] < 1 || half_len[s] > FDVM_MAX_FIR_HALF) return FDVM_ERANGE;
        if (tap_offset[s] < 0) return FDVM_EINVAL;
        if (!finite_pos(sigmas[s])) return FDVM_ERANGE;
        const double *h = taps + tap_offset[s];
        const int K = half_len[s];
        for (int m = 1; m <= K; ++m)
            if (h[K + m] != h[K - m]) return FDVM_EINVAL;   // symmetric taps only
    }
    if (ws_bytes < fir_backward_workspace_bytes(H, W, nscales)) return FDVM_ENOMEM;
    const int64_t P = H * W;
    const size_t fbytes = fir_backward_frame_bytes(H, W, nscales);
    double *gpart = reinterpret_cast<double *>(static_cast<char *>(ws) + BWD_LANES * fbytes);
    const int used = std::min(BWD_LANES, nframes);
    LaneFork lanes(static_cast<hipStream_t>(stream));
    if (used > 1) {
        st = lanes.fork(used);
        if (st != FDVM_OK) return st;
    }
    const bool rep = bc == FDVM_BC_REPLICATE;
    hipError_t e = hipSuccess;
    for (int f = 0; e == hipSuccess && f < nframes; ++f) {
        const int l = f % used;
        hipStream_t hs = lanes.stream(l);
        char *w = static_cast<char *>(ws) + l * fbytes;
        float *gB = reinterpret_cast<float *>(w);
        float *Q0 = reinterpret_cast<float *>(w + plane_bytes(H, W, nscales));
        float *Q1 = reinterpret_cast<float *>(w + plane_bytes(H, W, nscales) + plane_bytes(H, W, 1));
        float *Q2 = reinterpret_cast<float *>(w + plane_bytes(H, W, nscales) + 2 * plane_bytes(H, W, 1));
        char *rest = w + plane_bytes(H, W, nscales) + 3 * plane_bytes(H, W, 1);
        double *tab = reinterpret_cast<double *>(rest);
        char *dots = rest + ((((size_t)std::max(H, W)) * sizeof(double) + 255) & ~(size_t)255);
        double *res = reinterpret_cast<double *>(dots + dots_workspace_bytes(H, nscales));
        double *gs = used > 1 ? gpart + (int64_t)l * nscales : gsigma;
        const float *gVf = gV + (int64_t)f * v_frame_stride;
        e = launch_laplacian_adjoint(gVf, H, W, pitch, plane_stride, nscales, sigmas, gB, W, P, hs);
        for (int s = 0; e == hipSuccess && s < nscales; ++s) {
            const int K = half_len[s];
            const double *h = taps + tap_offset[s] + K;   // h(0..K)
            const float *g = gB + (int64_t)s * P;
            if (what & FDVM_GRAD_X) {
                float *gxf = gx + (int64_t)f * gx_frame_stride;
                // G^T = (fold_x + zero-extension x pass) (fold_y + zero-extension y pass)
                e = launch_fir_pass(g, FDVM_F32, H, W, W, Q0, W, 1, FDVM_BC_ZERO, h, K, false, hs);
                if (e == hipSuccess && rep) e = launch_fir_tail_table(h, K, tab, hs);
                if (e == hipSuccess && rep) e = launch_fold_fir(g, W, Q0, W, H, W, K, tab, 1, hs);
                if (e == hipSuccess)
                    e = launch_fir_pass(Q0, FDVM_F32, H, W, W, gxf, gx_pitch, 0, FDVM_BC_ZERO, h, K, s > 0, hs);
                if (e == hipSuccess && rep) e = launch_fold_fir(Q0, W, gxf, gx_pitch, H, W, K, tab, 0, hs);
            }
            if (e == hipSuccess && (what & FDVM_GRAD_SIGMA)) {
                const void *xf = static_cast<const char *>(x) + (int64_t)f * x_frame_stride * (int64_t)elem_bytes(dt);
                const double *dh = dtaps + tap_offset[s] + K;
                // dB/dsigma = G'_y G_x x + G_y G'_x x, then <gB_s, dB_s/dsigma>
                e = launch_fir_pass(xf, dt, H, W, x_pitch, Q0, W, 0, bc, h, K, false, hs);
                if (e == hipSuccess) e = launch_fir_pass(xf, dt, H, W, x_pitch, Q1, W, 0, bc, dh, K, false, hs);
                if (e == hipSuccess) e = launch_fir_pass(Q0, FDVM_F32, H, W, W, Q2, W, 1, bc, dh, K, false, hs);
                if (e == hipSuccess) e = launch_fir_pass(Q1, FDVM_F32, H, W, W, Q2, W, 1, bc, h, K, true, hs);
                if (e == hipSuccess) e = launch_plane_dots(g, Q2, H, W, W, P, 1, res + nscales + s, dots, hs);
            }
        }
        if (e == hipSuccess && (what & FDVM_GRAD_SIGMA)) {
            e = launch_plane_dots(gVf, V + (int64_t)f * v_frame_stride, H, W, pitch, plane_stride, nscales, res, dots,
                                  hs);
            if (e == hipSuccess) e = launch_gsigma(res, res + nscales, 1, sigmas, nscales, f >= used, gs, hs);
        }
    }
    st = lanes.join(from_hip(e));
    if (st == FDVM_OK && used > 1 && (what & FDVM_GRAD_SIGMA))
        st = from_hip(launch_sum_lanes(gpart, used, nscales, gsigma, static_cast<hipStream_t>(stream)));
    return st;
}
