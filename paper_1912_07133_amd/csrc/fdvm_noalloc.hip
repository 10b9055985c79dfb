// fdvm_detect_blobs_noalloc: the multi-scale extremum detection of
// fdvm_detect_blobs for callers that cannot allocate device memory (code under
// HIP graph capture, serving loops, harnesses that forbid hipMalloc).  Its
// kernels are those of fdvm_detect_blobs; their scratch (the mask words and
// the per-block totals and offsets) lives in `scratch`, a fixed array of this
// library in every device's memory instead of a caller workspace.
//
// In host code `scratch` names a host-side stand-in, not device memory: its
// device address is looked up once per device (hipGetSymbolAddress, with that
// device current) and only that address is handed to kernels.  Every call on a
// device shares that device's array and leaves the last call's words in it;
// the detection kernels write every word they later read, so nothing needs
// clearing between calls.  Calls that overlap on one device (different
// streams, or threads) race on the array.
#include <mutex>

#include "fdvm_internal.h"

namespace {

__device__ __align__(256) unsigned char scratch[FDVM_NOALLOC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch[MAX_DEVICES];  // device address of `scratch` on each device (null until looked up)

// the current device's copy of `scratch`, looked up on the first call there
fdvm_status scratch_on_current_device(void **out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return FDVM_EDEVICE;
    if (dev < 0 || dev >= MAX_DEVICES) return FDVM_EUNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return FDVM_EDEVICE;
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return FDVM_OK;
}

}  // namespace

extern "C" {

size_t fdvm_noalloc_scratch_bytes(void) { return (size_t)FDVM_NOALLOC_SCRATCH_BYTES; }

fdvm_status fdvm_detect_blobs_noalloc(const float *resp, int64_t H, int64_t W, int64_t pitch, int64_t plane_stride,
                                      int nscales, float tau, int border, fdvm_blob *out_dev, int32_t cap,
                                      int32_t *count_dev, void *stream) {
    fdvm_status st = fdvm::detect_check(resp, H, W, pitch, plane_stride, nscales, tau, border, out_dev, cap,
                                        count_dev);
    if (st != FDVM_OK) return st;
    if (fdvm::detect_workspace_bytes(H, W, nscales) > (size_t)FDVM_NOALLOC_SCRATCH_BYTES) return FDVM_ERANGE;
    void *ws = nullptr;
    st = scratch_on_current_device(&ws);
    if (st != FDVM_OK) return st;
    const hipError_t e = fdvm::launch_detect(resp, H, W, pitch, plane_stride, nscales, tau, border, out_dev, cap,
                                             count_dev, ws, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? FDVM_OK : FDVM_EDEVICE;
}

}  // extern "C"
