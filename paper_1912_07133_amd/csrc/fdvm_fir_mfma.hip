// Toeplitz-block FIR (Eq A5) on the gfx950 matrix cores, float32 operands and
// float32 accumulation (v_mfma_f32_32x32x2f32).
//
// One kernel filters along y and writes its result transposed; run twice it is
// the separable blur (y, then x on the transposed intermediate, transposed
// back).  The separable product with a separable boundary extension does not
// depend on the order of the two 1-D passes (Section 2), so this equals the
// x-then-y form up to rounding.
//
// Per wavefront: 32 columns x0..x0+31 and 64 outputs y0..y0+63 along y, as
// two 32 x 32 blocks t = 0, 1.  For block t and the input rows r, r+1:
//     D_t[i][j] += sum_{kk=0,1} in(r + kk, x0 + i) * h(y0 + 32 t + j - r - kk)
// i.e. A = two input rows (32 x 2, lane i + 32 kk: coalesced loads along the
// row), B = a 2 x 32 slice of the Toeplitz matrix of the taps (read from a
// zero-padded tap table in LDS), D = the 32 x 32 block with lane j holding
// output y0 + 32 t + j: the transposed store out[x][y] is coalesced along y.
// With the half-length rounded up to K' (a multiple of 8, taps beyond K zero),
// the row pairs p = 0 .. 31 + K' starting at y0 - K' meet block 0 for
// p < 16 + K' and block 1 for p >= 16, so the loop runs in three branch-free
// phases (block 0 only, both, block 1 only): 32 + 2K' instructions of 4096
// flops per wavefront for 64 x 32 outputs of 2 (2K + 1) useful flops each.
#include <type_traits>

#include "fdvm_internal.h"

namespace fdvm {
namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));

constexpr int MF_TN = 64;          // outputs per wavefront along the filtered axis (two blocks)
constexpr int MF_WPB = 4;          // wavefronts per work-group
constexpr int MF_U = 8;            // row pairs per group
constexpr int MF_RING = 32;        // row pairs held per wavefront in its LDS ring
constexpr int MF_DIST = 24;        // row pairs requested ahead of the one being used
constexpr int MF_KMAX = ((FDVM_MAX_FIR_HALF + MF_U - 1) / MF_U) * MF_U;
constexpr int MF_HZ = 2 * MF_KMAX + 68;
constexpr int MF_ARG_TAPS = 880;   // tap words that fit in the kernel arguments

// the half tap tables h(0..K_s) of all scales of one launch
struct TapSet {
    int nscales;
    int K[FDVM_MAX_SCALES];
    int off[FDVM_MAX_SCALES];
    float h[MF_ARG_TAPS];
};

template <typename T>
__device__ __forceinline__ float ldx(const T *p);
template <>
__device__ __forceinline__ float ldx<uint16_t>(const uint16_t *p) { return (float)*p; }
template <>
__device__ __forceinline__ float ldx<float>(const float *p) { return *p; }
template <>
__device__ __forceinline__ float ldx<_Float16>(const _Float16 *p) { return (float)*p; }
struct bf16_t { uint16_t bits; };
template <>
__device__ __forceinline__ float ldx<bf16_t>(const bf16_t *p) { return __uint_as_float(((uint32_t)p->bits) << 16); }

// hardware work-group ids go round-robin to the 8 XCDs; give every XCD one
// contiguous run of logical blocks
__device__ __forceinline__ int xcd_logical(int hw, int n) {
    constexpr int NX = 8;
    const int xcd = hw % NX, slot = hw / NX;
    const int q = n / NX, r = n % NX;
    return xcd * q + min(xcd, r) + slot;
}

// Filters H x W frames along y, scale s of the tap set from input plane s
// (in_plane_stride may be 0: one frame for all scales); out plane s (W rows of
// pitch out_pitch >= H) receives the transpose: out[s * out_plane_stride + x * out_pitch + y].
// Logical blocks are ordered (x group, y tile, scale), scale fastest, so that
// each XCD gets a balanced mix of tap lengths and the blocks that read the
// same input rows meet in one L2.
static_assert(MF_DIST + MF_U <= MF_RING && MF_DIST <= 63 && MF_DIST % MF_U == 0, "ring and vmcnt limits");

// copy one element per lane from global memory straight into LDS: lane n's
// element lands in the 32-bit word l[n] (2-byte elements zero-extended);
// complete once vmcnt has dropped past it
template <typename T>
__device__ __forceinline__ void to_lds(const T *g, uint32_t *l) {
    static_assert(sizeof(T) == 2 || sizeof(T) == 4, "2- or 4-byte elements");
    auto *ld = (__attribute__((address_space(3))) void *)l;
    if constexpr (sizeof(T) == 2)
        __builtin_amdgcn_global_load_lds((const void *)g, ld, 2, 0, 0);
    else
        __builtin_amdgcn_global_load_lds((const void *)g, ld, 4, 0, 0);
}
// Eight LDS words at a + k * STRIDE (k = 0..7), read and waited for in one
// block.  The compiler cannot tell LDS reads from the direct global-to-LDS
// copies still in flight and would wait for every one of them before a plain
// LDS load; these reads touch only data whose copies have been waited for.
#define FDVM_DS8(OP, S)                                                                                  \
    asm volatile(OP " %0, %8\n " OP " %1, %8 offset:" #S "*1\n " OP " %2, %8 offset:" #S "*2\n " OP    \
                    " %3, %8 offset:" #S "*3\n " OP " %4, %8 offset:" #S "*4\n " OP " %5, %8 offset:" #S \
                    "*5\n " OP " %6, %8 offset:" #S "*6\n " OP " %7, %8 offset:" #S "*7\n s_waitcnt lgkmcnt(0)" \
                 : "=&v"(r[0]), "=&v"(r[1]), "=&v"(r[2]), "=&v"(r[3]), "=&v"(r[4]), "=&v"(r[5]), "=&v"(r[6]),   \
                   "=&v"(r[7])                                                                          \
                 : "v"(a)                                                                               \
                 : "memory")
__device__ __forceinline__ uint32_t lds_addr(const void *p) {
    return (uint32_t)(uintptr_t)(const __attribute__((address_space(3))) void *)p;
}
// ring words of pairs p0 .. p0 + 7 (consecutive slots of 64 words) for the calling lane
__device__ __forceinline__ void ring_read8(const uint32_t *p, uint32_t (&r)[8]) {
    const uint32_t a = lds_addr(p);
    FDVM_DS8("ds_read_b32", 256);
}
// taps for pairs p0 .. p0 + 7 of one block: q points at the entry of pair
// p0 + 7; the entry of pair p0 + u lies 2 (7 - u) words above it
__device__ __forceinline__ void taps_read8(const float *q, float (&b)[8]) {
    const uint32_t a = lds_addr(q);
    uint32_t r[8];
    FDVM_DS8("ds_read_b32", 8);
#pragma unroll
    for (int u = 0; u < 8; ++u) b[u] = __uint_as_float(r[7 - u]);
}
#undef FDVM_DS8

template <typename T>
__device__ __forceinline__ float bits_to_float(uint32_t b);
template <>
__device__ __forceinline__ float bits_to_float<float>(uint32_t b) { return __uint_as_float(b); }
template <>
__device__ __forceinline__ float bits_to_float<uint16_t>(uint32_t b) { return (float)(b & 0xffffu); }
template <>
__device__ __forceinline__ float bits_to_float<_Float16>(uint32_t b) {
    return (float)__builtin_bit_cast(_Float16, (uint16_t)(b & 0xffffu));
}
template <>
__device__ __forceinline__ float bits_to_float<bf16_t>(uint32_t b) { return __uint_as_float(b << 16); }

template <int N>
__device__ __forceinline__ void wait_vm() {
    asm volatile("s_waitcnt vmcnt(%0)" ::"n"(N) : "memory");
}

template <typename TIn>
__global__ __launch_bounds__(MF_WPB * 64) void fir_mfma_kernel(const TIn *__restrict__ in, int64_t in_pitch,
                                                                int64_t in_plane_stride, int H, int W,
                                                                float *__restrict__ out, int64_t out_pitch,
                                                                int64_t out_plane_stride, int boundary, TapSet ts) {
    __shared__ float hz[MF_HZ];
    __shared__ uint32_t ring[MF_WPB][MF_RING * 64];  // one 32-bit word per element
    const int nyt = (H + MF_TN - 1) / MF_TN;
    const int nxg = (W + 32 * MF_WPB - 1) / (32 * MF_WPB);
    const int S = ts.nscales;
    const int lb = xcd_logical(blockIdx.x, nyt * nxg * S);
    const int s = lb % S;
    const int yt = (lb / S) % nyt;
    const int xg = lb / (S * nyt);
    const int K = ts.K[s];
    const int KP = ((K + MF_U - 1) / MF_U) * MF_U;  // K' >= K, multiple of MF_U
    const float *h = ts.h + ts.off[s];
    const int OFF = KP + 33;  // hz[OFF + d] = h(d) for |d| <= K, 0 for K < |d| <= K' + 33
    for (int t = threadIdx.x; t < 2 * KP + 67; t += blockDim.x) {
        const int d = t - OFF;
        const int ad = d < 0 ? -d : d;
        hz[t] = ad <= K ? h[ad] : 0.0f;
    }
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int x0 = (xg * MF_WPB + wv) * 32;
    const int y0 = yt * MF_TN;
    if (x0 >= W) return;
    const int i = lane & 31;   // A: column x0 + i; B and D: output y0 + 32 t + i
    const int kk = lane >> 5;  // row of the pair
    const int xc = min(x0 + i, W - 1);
    const bool rep = boundary == FDVM_BC_REPLICATE;
    const TIn *colp = in + (int64_t)s * in_plane_stride + xc;

    floatx16 acc0, acc1;
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        acc0[e] = 0.0f;
        acc1[e] = 0.0f;
    }
    // pair p covers rows r_begin + 2p (+ kk); block t at pair p takes
    // h(32 t + K' - 2p + j - kk), i.e. hz[OFF + 32 t + K' - 2p + i - kk]
    const int r_begin = y0 - KP;
    const float *hz0 = hz + OFF + KP + i - kk;   // block 0 at pair p: hz0[-2p]
    const float *hz1 = hz0 + 32;                 // block 1 at pair p: hz1[-2p]
    // Input rows go through a per-wavefront ring in LDS by direct
    // global-to-LDS copies issued MF_DIST pairs ahead, so a long stretch of the
    // window is in flight without holding registers.  Lane i + 32 kk copies
    // (and later reads) element (r_begin + 2p + kk, x0 + i) of pair p.  Rows
    // outside the image are clamped copies, zeroed on use for the zero
    // extension.  Requests past the window's end are clamped reads that keep
    // the in-flight count uniform.
    uint32_t *rg = ring[wv];
    auto request = [&](int p) {
        const int row = r_begin + 2 * p + kk;
        const int cr = min(max(row, 0), H - 1);
        to_lds(colp + (int64_t)cr * in_pitch, rg + (p % MF_RING) * 64);
    };
    static_assert(MF_U == 8 && MF_RING % MF_U == 0, "ring_read8 reads one group");
    for (int p = 0; p < MF_DIST; ++p) request(p);
    // one phase: pairs [pa, pb) in groups of MF_U; before a group is used the
    // group MF_DIST pairs later is requested and all but the last MF_DIST
    // requests are waited for
    auto phase = [&](int pa, int pb, auto blocks_tag) {
        constexpr int BL = decltype(blocks_tag)::value;  // 1: block 0, 2: block 1, 3: both
        for (int p0 = pa; p0 < pb; p0 += MF_U) {
#pragma unroll
            for (int u = 0; u < MF_U; ++u) request(p0 + MF_DIST + u);
            wait_vm<MF_DIST>();
            uint32_t raw[MF_U];
            ring_read8(rg + (p0 % MF_RING) * 64 + lane, raw);
            float a[MF_U];
#pragma unroll
            for (int u = 0; u < MF_U; ++u) {
                const int row = r_begin + 2 * (p0 + u) + kk;
                a[u] = (rep || (row >= 0 && row < H)) ? bits_to_float<TIn>(raw[u]) : 0.0f;
            }
            float b0[MF_U], b1[MF_U];
            if constexpr (BL & 1) taps_read8(hz0 - 2 * (p0 + MF_U - 1), b0);
            if constexpr (BL & 2) taps_read8(hz1 - 2 * (p0 + MF_U - 1), b1);
#pragma unroll
            for (int u = 0; u < MF_U; ++u) {
                if constexpr (BL & 1) acc0 = __builtin_amdgcn_mfma_f32_32x32x2f32(a[u], b0[u], acc0, 0, 0, 0);
                if constexpr (BL & 2) acc1 = __builtin_amdgcn_mfma_f32_32x32x2f32(a[u], b1[u], acc1, 0, 0, 0);
            }
        }
    };
    phase(0, 16, std::integral_constant<int, 1>{});
    phase(16, 16 + KP, std::integral_constant<int, 3>{});
    phase(16 + KP, 32 + KP, std::integral_constant<int, 2>{});
    wait_vm<0>();  // no copy may land in LDS after this wavefront is gone
    floatx16 acc[2] = {acc0, acc1};
    // D[i][j] of block t sits in lane j + 32 ((i / 4) % 2), register (i / 8) 4 + i % 4
    float *o = out + (int64_t)s * out_plane_stride;
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        const int y = y0 + 32 * t + i;
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            const int x = x0 + (e / 4) * 8 + kk * 4 + (e % 4);
            if (x < W && y < H) o[(int64_t)x * out_pitch + y] = acc[t][e];
        }
    }
}

template <typename T>
hipError_t pass_t(const void *in, int64_t in_pitch, int64_t in_plane_stride, int64_t H, int64_t W, float *out,
                  int64_t out_pitch, int64_t out_plane_stride, int boundary, const TapSet &ts, hipStream_t st) {
    const int nyt = (int)((H + MF_TN - 1) / MF_TN);
    const int nxg = (int)((W + 32 * MF_WPB - 1) / (32 * MF_WPB));
    const unsigned nb = (unsigned)nyt * (unsigned)nxg * (unsigned)ts.nscales;
    hipLaunchKernelGGL(fir_mfma_kernel<T>, dim3(nb), dim3(MF_WPB * 64), 0, st, static_cast<const T *>(in),
                       in_pitch, in_plane_stride, (int)H, (int)W, out, out_pitch, out_plane_stride, boundary, ts);
    return hipGetLastError();
}

hipError_t run_set(const void *in, int dtype, int64_t H, int64_t W, int64_t in_pitch, float *tmp, float *out,
                   int64_t out_pitch, int64_t plane_stride, const TapSet &ts, int boundary, hipStream_t st) {
    const int64_t tstride = H * W;  // transposed planes W x H, pitch H
    hipError_t e;
    switch (dtype) {
        case FDVM_U16: e = pass_t<uint16_t>(in, in_pitch, 0, H, W, tmp, H, tstride, boundary, ts, st); break;
        case FDVM_F32: e = pass_t<float>(in, in_pitch, 0, H, W, tmp, H, tstride, boundary, ts, st); break;
        case FDVM_F16: e = pass_t<_Float16>(in, in_pitch, 0, H, W, tmp, H, tstride, boundary, ts, st); break;
        case FDVM_BF16: e = pass_t<bf16_t>(in, in_pitch, 0, H, W, tmp, H, tstride, boundary, ts, st); break;
        default: return hipErrorInvalidValue;
    }
    if (e != hipSuccess) return e;
    // x pass: plane s of tmp read as a W x H frame, filtered along its y (the
    // image's x), written transposed back into out plane s
    return pass_t<float>(tmp, H, tstride, W, H, out, out_pitch, plane_stride, boundary, ts, st);
}

}  // namespace

bool fir_mfma_available() { return true; }

size_t fir_mfma_workspace_bytes(int64_t H, int64_t W, int nscales) {
    return ((size_t)nscales * H * W * sizeof(float) + 255) & ~(size_t)255;
}

hipError_t launch_fir_mfma(const void *in, int dtype, int64_t H, int64_t W, int64_t in_pitch, float *tmp,
                           float *out, int64_t out_pitch, int64_t plane_stride, const double *taps,
                           const int32_t *half_len, const int32_t *tap_offset, int nscales, int boundary,
                           hipStream_t st) {
    // all scales in one launch per pass while their half tables fit in the
    // kernel arguments; otherwise one launch per scale
    int words = 0;
    for (int s = 0; s < nscales; ++s) words += half_len[s] + 1;
    const int per = words <= MF_ARG_TAPS ? nscales : 1;
    for (int s0 = 0; s0 < nscales; s0 += per) {
        TapSet ts{};
        ts.nscales = per;
        int pos = 0;
        for (int q = 0; q < per; ++q) {
            const int K = half_len[s0 + q];
            const double *hd = taps + tap_offset[s0 + q];
            ts.K[q] = K;
            ts.off[q] = pos;
            if (pos + K + 1 > MF_ARG_TAPS) return hipErrorInvalidValue;  // K <= FDVM_MAX_FIR_HALF < MF_ARG_TAPS
            for (int m = 0; m <= K; ++m) ts.h[pos + m] = (float)hd[K + m];
            pos += K + 1;
        }
        hipError_t e = run_set(in, dtype, H, W, in_pitch, tmp, out + (int64_t)s0 * plane_stride, out_pitch,
                               plane_stride, ts, boundary, st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace fdvm
