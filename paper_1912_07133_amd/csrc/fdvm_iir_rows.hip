// Row pass of the repeated-pole IIR blur: dispatch on the frame's element type
// (kernels in fdvm_iir_rows.h, one translation unit per type).
#include "fdvm_iir_rows.h"

namespace fdvm {

hipError_t launch_iir_rows(const void *in, int dtype, int64_t H, int64_t W, int64_t in_pitch, void *out,
                           int64_t out_pitch, int64_t plane_stride, int *rexp, int chunk, const IirParams &prm,
                           hipStream_t st) {
    switch (dtype) {
        case FDVM_U16: return launch_iir_rows_u16(in, H, W, in_pitch, out, out_pitch, plane_stride, rexp, chunk, prm, st);
        case FDVM_F32: return launch_iir_rows_f32(in, H, W, in_pitch, out, out_pitch, plane_stride, rexp, chunk, prm, st);
        case FDVM_F16: return launch_iir_rows_f16(in, H, W, in_pitch, out, out_pitch, plane_stride, rexp, chunk, prm, st);
        case FDVM_BF16:
            return launch_iir_rows_bf16(in, H, W, in_pitch, out, out_pitch, plane_stride, rexp, chunk, prm, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace fdvm
