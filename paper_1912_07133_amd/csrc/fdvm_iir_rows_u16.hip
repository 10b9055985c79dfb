// Row pass of the repeated-pole IIR blur for u16 frames (kernels in fdvm_iir_rows.h).
#include "fdvm_iir_rows.h"

namespace fdvm {

FDVM_ROWS_DECL(launch_iir_rows_u16) {
    return launch_rows_typed<uint16_t>(in, H, W, in_pitch, out, out_pitch, plane_stride, rexp, chunk, prm, st);
}

}  // namespace fdvm
