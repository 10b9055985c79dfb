// Toeplitz-block FIR on the gfx950 matrix cores (placeholder until the MFMA
// kernel lands; fdvm_blur_fir reports FDVM_EUNSUPPORTED for this algorithm).
#include "fdvm_internal.h"

namespace fdvm {

bool fir_mfma_available() { return false; }

hipError_t launch_fir_mfma(const float *src, int64_t H, int64_t W, int64_t pitch, float *dst,
                           int64_t out_pitch, const float *taps_half, int K, int boundary,
                           bool transpose_in, hipStream_t st) {
    (void)src; (void)H; (void)W; (void)pitch; (void)dst; (void)out_pitch;
    (void)taps_half; (void)K; (void)boundary; (void)transpose_in; (void)st;
    return hipErrorNotSupported;
}

}  // namespace fdvm
