// Row pass of the repeated-pole IIR blur for f32 frames (kernels in fdvm_iir_rows.h).
#include "fdvm_iir_rows.h"

namespace fdvm {

FDVM_ROWS_DECL(launch_iir_rows_f32) {
    return launch_rows_typed<float>(in, H, W, in_pitch, out, out_pitch, plane_stride, rexp, chunk, prm, st);
}

}  // namespace fdvm
