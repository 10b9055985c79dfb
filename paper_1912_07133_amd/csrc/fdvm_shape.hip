// High-pass stage (Table I central differences) and multi-scale blob
// detection on gfx950.
//
// Detection (strict extremum over the 3 x 3 x 3 block of (scale, y, x)
// neighbours, thresholded) runs in four kernels, deterministic, with no
// atomics and no sort:
//   mask  -- lane = column, each wavefront owns an 8-row band of a 62-column
//            tile (tiles overlap by one column on each side so every output
//            column has both x-neighbours in the wavefront) and walks the
//            scales; x-neighbours come from wavefront shifts, the separable
//            3 x 3 minimum / maximum of the previous, current and next plane
//            stay in registers.  Output: one 64-bit mask word per
//            (scale, row, tile), words ordered by (scale, y, x).
//   sums  -- popcount totals of consecutive blocks of words;
//   scan  -- exclusive prefix of the block totals (one work-group), total count;
//   emit  -- every block rescans its words and writes the records.
// The list therefore comes out ordered by (scale, y, x).
#include <cmath>
#include <type_traits>

#include "fdvm_internal.h"

namespace fdvm {
namespace {

constexpr int HP_BLOCK = 256;
constexpr int DT_W = 62;          // output columns per detection tile
constexpr int DT_ROWS = 8;        // rows per wavefront
constexpr int DT_WAVES = 4;       // wavefronts per work-group
constexpr int SUM_THREADS = 256;
constexpr int SUM_WORDS = 4;      // words per thread in sums / emit
constexpr int SCAN_BLOCK = 1024;

struct Norms {
    float v[FDVM_MAX_SCALES];
};

__device__ __forceinline__ float ld_clamped(const float *plane, int64_t pitch, int y, int x, int H, int W) {
    y = min(max(y, 0), H - 1);
    x = min(max(x, 0), W - 1);
    return plane[(int64_t)y * pitch + x];
}

__global__ __launch_bounds__(HP_BLOCK) void highpass_kernel(const float *__restrict__ blur, int64_t pitch,
                                                             int64_t plane_stride, int H, int W,
                                                             unsigned what, int nout, Norms norms,
                                                             float *__restrict__ out,
                                                             int64_t out_plane_stride) {
    const int x = blockIdx.x * HP_BLOCK + threadIdx.x;
    const int y = blockIdx.y;
    const int s = blockIdx.z;
    if (x >= W) return;
    const float *B = blur + (int64_t)s * plane_stride;
    const float c = B[(int64_t)y * pitch + x];
    const float xm = ld_clamped(B, pitch, y, x - 1, H, W);
    const float xp = ld_clamped(B, pitch, y, x + 1, H, W);
    const float ym = ld_clamped(B, pitch, y - 1, x, H, W);
    const float yp = ld_clamped(B, pitch, y + 1, x, H, W);
    const float d20 = (xp - c) + (xm - c);
    const float d02 = (yp - c) + (ym - c);
    const int64_t o = (int64_t)y * pitch + x;
    int j = 0;
    float *dst = out + (int64_t)s * nout * out_plane_stride;
    if (what & FDVM_HP_LAPLACIAN) dst[(j++) * out_plane_stride + o] = norms.v[s] * (d20 + d02);
    if (what & FDVM_HP_D20) dst[(j++) * out_plane_stride + o] = d20;
    if (what & FDVM_HP_D02) dst[(j++) * out_plane_stride + o] = d02;
    if (what & FDVM_HP_D11) {
        // D10 along x of the rows y-1 and y+1, then D01 along y
        const float a = ld_clamped(B, pitch, y + 1, x + 1, H, W) - ld_clamped(B, pitch, y + 1, x - 1, H, W);
        const float b = ld_clamped(B, pitch, y - 1, x + 1, H, W) - ld_clamped(B, pitch, y - 1, x - 1, H, W);
        dst[(j++) * out_plane_stride + o] = 0.25f * (a - b);
    }
    if (what & FDVM_HP_D10) dst[(j++) * out_plane_stride + o] = 0.5f * (xp - xm);
    if (what & FDVM_HP_D01) dst[(j++) * out_plane_stride + o] = 0.5f * (yp - ym);
}

// value of lane (l - 1) / (l + 1) across the whole wavefront (gfx9 DPP
// wave_shr:1 / wave_shl:1); the end lanes get a copy of their own value
__device__ __forceinline__ float lane_left(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(v), __float_as_int(v), 0x138, 0xf, 0xf, false));
}
__device__ __forceinline__ float lane_right(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(v), __float_as_int(v), 0x130, 0xf, 0xf, false));
}

__device__ __forceinline__ int xcd_logical_block(int hw, int n) {
    constexpr int NX = 8;   // XCDs
    const int xcd = hw % NX, slot = hw / NX;
    const int q = n / NX, r = n % NX;
    return xcd * q + min(xcd, r) + slot;
}

// planes in each wavefront's LDS ring: the one awaited and the next in flight
// (rings of 3 and 4 planes measured slower on a 2048 x 2048 x 8-scale stack)
constexpr int DT_NPL = 2;

// copy 64 lanes x 4 bytes from global memory straight into LDS (lane n to
// l[n]); complete once vmcnt has dropped past it
__device__ __forceinline__ void row_to_lds(const float *g, uint32_t *l) {
    __builtin_amdgcn_global_load_lds((const void *)g, (__attribute__((address_space(3))) void *)l, 4, 0, 0);
}
template <int N>
__device__ __forceinline__ void wait_vm() {
    asm volatile("s_waitcnt vmcnt(%0)" ::"n"(N) : "memory");
}
// the calling lane's word of the DT_ROWS + 2 staged rows of one plane, read
// and waited for in one block: a plain LDS load would make the compiler wait
// for every copy still in flight (it cannot tell which LDS words they write)
static_assert(DT_ROWS + 2 == 10, "read10 reads ten rows");
__device__ __forceinline__ void read10(const uint32_t *p, uint32_t (&r)[10]) {
    const uint32_t a = (uint32_t)(uintptr_t)(const __attribute__((address_space(3))) uint32_t *)p;
    asm volatile(
        "ds_read_b32 %0, %10\n ds_read_b32 %1, %10 offset:256\n ds_read_b32 %2, %10 offset:512\n"
        " ds_read_b32 %3, %10 offset:768\n ds_read_b32 %4, %10 offset:1024\n ds_read_b32 %5, %10 offset:1280\n"
        " ds_read_b32 %6, %10 offset:1536\n ds_read_b32 %7, %10 offset:1792\n ds_read_b32 %8, %10 offset:2048\n"
        " ds_read_b32 %9, %10 offset:2304\n s_waitcnt lgkmcnt(0)"
        : "=&v"(r[0]), "=&v"(r[1]), "=&v"(r[2]), "=&v"(r[3]), "=&v"(r[4]), "=&v"(r[5]), "=&v"(r[6]), "=&v"(r[7]),
          "=&v"(r[8]), "=&v"(r[9])
        : "v"(a)
        : "memory");
}

// lane L of v <- the wave-uniform value u (v_writelane_b32)
template <int L>
__device__ __forceinline__ void write_lane(int &v, uint32_t u) {
    asm volatile("v_writelane_b32 %0, %1, %2" : "+v"(v) : "s"(u), "n"(L));
}
// f(integral_constant<int, 0>) .. f(integral_constant<int, N - 1>), in order
template <int N, int I = 0, typename F>
__device__ __forceinline__ void static_for(F &&f) {
    if constexpr (I < N) {
        f(std::integral_constant<int, I>{});
        static_for<N, I + 1>(f);
    }
}

// Order-preserving integer key of a float32 (finite or infinite): k(a) < k(b)
// exactly when a < b, and k(+0) = k(-0) = 0.  Integer minima and maxima then
// need no NaN handling, and a missing neighbour is a sentinel key that can
// never win: INT32_MAX for minima, INT32_MIN for maxima.
__device__ __forceinline__ int fkey(float v) {
    const int b = __float_as_int(v);
    const int sgn = b >> 31;
    return ((b & 0x7fffffff) ^ sgn) - sgn;
}
// key of lane (l - 1) / (l + 1) (gfx9 DPP wave_shr:1 / wave_shl:1); the end
// lanes read 0, which only ever feeds their own (unused) results
__device__ __forceinline__ int key_left(int k) { return __builtin_amdgcn_mov_dpp(k, 0x138, 0xf, 0xf, true); }
__device__ __forceinline__ int key_right(int k) { return __builtin_amdgcn_mov_dpp(k, 0x130, 0xf, 0xf, true); }

// The planes reach LDS by direct global-to-LDS copies issued DT_NPL - 1
// planes ahead of use; the mask words of the wavefront collect in LDS and are
// written once at the end (no stores interleave with the counted copies).
// Per plane and output row the kernel keeps the centre and the two 3 x 3
// statistics without it (those with it are formed where a neighbouring
// scale's decision needs them); the planes rotate through three register
// roles (previous, current, next), so the scale loop is unrolled by three.  A
// missing plane (before the first, after the last) drops out of the decision.
//
// RAW (tau > 0): a bright candidate is negative and a dark one positive, and
// for such a centre the float order against any neighbour is an integer order
// of the raw bit patterns: for c < 0, c < n exactly when bits(c) > bits(n) as
// unsigned integers (negative floats above every non-negative one, larger
// magnitude higher); for c > 0, c > n exactly when bits(c) > bits(n) as signed
// integers.  The statistics are then the unsigned and the signed maximum of
// the raw bits, and no key transform is needed; a sample outside the image
// enters as +0 (bits 0), which lies below both threshold floors below.
// The thresholds join them the same way: c <= -tau exactly when bits(c) >
// bits(-tau) - 1 unsigned, c >= tau exactly when bits(c) > bits(tau) - 1
// signed; taken into every row's left/right maximum, they reach each
// decision through the centre plane's 8-neighbour statistic, and a candidate
// is one unsigned and one signed comparison.
// Otherwise (tau = 0, where a zero centre may be an extremum) they are the
// minimum and maximum of order-preserving keys (fkey; sentinels INT32_MAX and
// INT32_MIN).
template <bool RAW>
__global__ __launch_bounds__(DT_WAVES * 64) void detect_mask_kernel(const float *__restrict__ V, int64_t pitch,
                                                                     int64_t plane_stride, int S, int H, int W,
                                                                     float tau, int border,
                                                                     unsigned long long *__restrict__ mask,
                                                                     int ntx) {
    constexpr int RB = DT_ROWS;
    constexpr int IMAX = 0x7fffffff, IMIN = (int)0x80000000;
    // sentinels of the two statistics: lo (bright test) and hi (dark test)
    constexpr int LO_NONE = RAW ? 0 : IMAX;
    constexpr int HI_NONE = IMIN;
    __shared__ uint32_t ring[DT_WAVES][DT_NPL][(RB + 2) * 64];
    __shared__ unsigned long long words[DT_WAVES][FDVM_MAX_SCALES * RB];
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    // hardware work-group ids go round-robin to the 8 XCDs (each with its own
    // L2); give every XCD one contiguous run of tiles (column tile fastest) so
    // that the halo columns and rows that neighbouring tiles share are fetched
    // from HBM once
    const int nby = (H + DT_ROWS * DT_WAVES - 1) / (DT_ROWS * DT_WAVES);
    const int lb = xcd_logical_block(blockIdx.x, ntx * nby);
    const int tx = lb % ntx;
    const int by = lb / ntx;
    const int x = tx * DT_W - 1 + lane;           // lanes 1..62 are output columns
    const int y0 = (by * DT_WAVES + wv) * RB;
    if (y0 >= H) return;
    const bool xin = x >= 0 && x < W;
    const int cx = min(max(x, 0), W - 1);
    uint32_t *rg = &ring[wv][0][0];
    // rows y0-1 .. y0+RB of plane min(s, S - 1) into ring slot s % DT_NPL
    // (a wave-uniform row address plus the lane's 32-bit byte offset, which
    // the copy takes as its scalar base and vector offset)
    const uint32_t xoff = (uint32_t)cx * 4u;
    auto request = [&](int s) {
        const char *P = reinterpret_cast<const char *>(V + (int64_t)min(s, S - 1) * plane_stride);
        uint32_t *slot = rg + (s % DT_NPL) * (RB + 2) * 64;
#pragma unroll
        for (int r = 0; r < RB + 2; ++r) {
            const int y = min(max(y0 - 1 + r, 0), H - 1);
            row_to_lds(reinterpret_cast<const float *>(P + (int64_t)y * pitch * 4 + xoff), slot + r * 64);
        }
    };
    constexpr int AHEAD = (DT_NPL - 1) * (RB + 2);  // copies issued after the plane awaited
    // per plane and output row: the centre and the two 3 x 3 statistics
    // without it; a neighbouring plane's 3 x 3 statistic with its centre is
    // formed where a decision needs it (one more max per statistic there, none
    // for it in the plane's own pass, and three planes' worth of registers less)
    struct Plane {
        int c[RB];               // centre (raw bits or key) of the output rows
        int lo8[RB], hi8[RB];    // 3 x 3 statistics without the centre
    };
    // the two statistics of a pair / triple of values
    auto lo2 = [](int a, int b) {
        if constexpr (RAW) return (int)max((unsigned)a, (unsigned)b);
        else return min(a, b);
    };
    auto lo3 = [](int a, int b, int c) {
        if constexpr (RAW) return (int)max(max((unsigned)a, (unsigned)b), (unsigned)c);
        else return min(min(a, b), c);
    };
    auto hi2 = [](int a, int b) { return max(a, b); };
    auto hi3 = [](int a, int b, int c) { return max(max(a, b), c); };
    // RAW: the thresholds as raw-bit floors of the two statistics (below);
    // otherwise the statistics' sentinels, which change nothing
    const int tlo = RAW ? (int)(__float_as_uint(-tau) - 1u) : LO_NONE;
    const int thi = RAW ? __float_as_int(tau) - 1 : HI_NONE;
    // statistics of plane s (its copies must have landed).  EDGE: the band
    // touches the image border (some rows or lanes outside get sentinels);
    // otherwise every staged sample is inside and no test is needed.
    auto stats = [&](int s, Plane &pl, auto edge_tag) {
        constexpr bool EDGE = decltype(edge_tag)::value;
        uint32_t raw[RB + 2];
        read10(rg + (s % DT_NPL) * (RB + 2) * 64 + lane, raw);
        int rlo[RB + 2], rhi[RB + 2], llo[RB + 2], lhi[RB + 2];
#pragma unroll
        for (int r = 0; r < RB + 2; ++r) {
            int k = RAW ? (int)raw[r] : fkey(__uint_as_float(raw[r]));
            if constexpr (EDGE && RAW) {
                // with tau > 0 a sample outside the image can be +0 for both
                // statistics: it is below both threshold floors, which every
                // decision's statistics already hold, so it never changes one
                // (and the decisions of lanes and rows outside are masked)
                const int y = y0 - 1 + r;
                k = (xin && y >= 0 && y < H) ? k : 0;
            }
            if constexpr (EDGE && !RAW) {
                const int y = y0 - 1 + r;
                const bool yin = y >= 0 && y < H;   // wave-uniform
                const int klo = xin ? k : LO_NONE, khi = xin ? k : HI_NONE;
                const int l = lo3(key_left(klo), key_right(klo), tlo);
                const int h = hi3(key_left(khi), key_right(khi), thi);
                llo[r] = yin ? l : LO_NONE;
                lhi[r] = yin ? h : HI_NONE;
                rlo[r] = yin ? lo2(l, klo) : LO_NONE;
                rhi[r] = yin ? hi2(h, khi) : HI_NONE;
            } else {
                // the row statistics carry the threshold floors as well (as on
                // the edge path): every decision's statistic already holds
                // them through the centre plane, so they change no decision
                const int kl = key_left(k), kr = key_right(k);
                llo[r] = lo3(kl, kr, tlo);
                lhi[r] = hi3(kl, kr, thi);
                rlo[r] = lo2(llo[r], k);
                rhi[r] = hi2(lhi[r], k);
            }
            if (r >= 1 && r <= RB) pl.c[r - 1] = k;
        }
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            pl.lo8[r] = lo3(rlo[r], llo[r + 1], rlo[r + 2]);
            pl.hi8[r] = hi3(rhi[r], lhi[r + 1], rhi[r + 2]);
        }
    };
    const int kneg = fkey(-tau), kpos = fkey(tau);
    const bool xout = lane >= 1 && lane <= 62 && x < W && x >= border && x < W - border;
    unsigned long long *wd = words[wv];
    // decisions at plane s from its neighbours in scale (a plane's 3 x 3
    // statistic with its centre is the one without it joined with the centre:
    // the centre row's left/right maximum already holds the threshold floor,
    // on both paths, and a lane outside the image decides nothing).  The
    // first plane has no plane before it; after the last plane its own
    // 8-neighbour statistics stand in for the missing ones (the maximum of a
    // value with itself changes nothing), so that term is dropped.
    // The decided columns as a lane mask; ballots are taken of single
    // comparisons and combined on the scalar unit (a ballot of a combined
    // condition is rebuilt through a vector register)
    const unsigned long long xmask = __builtin_amdgcn_ballot_w64(xout);
    // lo/hi of plane s joined with plane s - 1's statistics (formed before
    // plane s + 1's statistics, so that plane s - 1 is no longer live then)
    auto join_prev = [&](const Plane &pv, const Plane &pc, int (&lo)[RB], int (&hi)[RB], auto has_pv) {
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            lo[r] = pc.lo8[r];
            hi[r] = pc.hi8[r];
            if constexpr (decltype(has_pv)::value) {
                lo[r] = lo3(lo[r], pv.lo8[r], pv.c[r]);
                hi[r] = hi3(hi[r], pv.hi8[r], pv.c[r]);
            }
        }
    };
    auto decide = [&](int s, const int (&plo)[RB], const int (&phi)[RB], const Plane &pc, const Plane &pn,
                      auto has_pn) {
        constexpr bool HPN = decltype(has_pn)::value;
        // row r's mask word goes to lane r of (whi, wlo); lanes 0..RB-1 store them
        int wlo = 0, whi = 0;
        static_for<RB>([&](auto rc) {
            constexpr int r = decltype(rc)::value;
            const int y = y0 + r;
            int lo = plo[r], hi = phi[r];
            if constexpr (HPN) {
                lo = lo3(lo, pn.lo8[r], pn.c[r]);
                hi = hi3(hi, pn.hi8[r], pn.c[r]);
            }
            const int k = pc.c[r];
            const bool yin = y < H && y >= border && y < H - border;   // wave-uniform
            // no neighbour at all (1 x 1 x 1 stack) compares as "strict" too
            unsigned long long hit;
            if constexpr (RAW) {   // the thresholds are inside lo and hi
                hit = __builtin_amdgcn_ballot_w64((unsigned)k > (unsigned)lo) | __builtin_amdgcn_ballot_w64(k > hi);
            } else {
                hit = (__builtin_amdgcn_ballot_w64(k <= kneg) & __builtin_amdgcn_ballot_w64(k < lo)) |
                      (__builtin_amdgcn_ballot_w64(k >= kpos) & __builtin_amdgcn_ballot_w64(k > hi));
            }
            const unsigned long long bits = yin ? (hit & xmask) >> 1 : 0ull;   // lanes 1..62 -> bits 0..61
            write_lane<r>(wlo, (uint32_t)bits);
            write_lane<r>(whi, (uint32_t)(bits >> 32));
        });
        if (lane < RB) wd[s * RB + lane] = ((unsigned long long)(uint32_t)whi << 32) | (uint32_t)wlo;
    };
#pragma unroll
    for (int q = 0; q < DT_NPL; ++q) request(q);
    auto run = [&](auto edge_tag) {
        Plane P0, P1, P2;
        wait_vm<AHEAD>();   // plane 0
        stats(0, P0, edge_tag);
        // step at plane s: plane s + 1 is needed now; plane s's slot is free
        // (its statistics are in registers)
        auto step = [&](int s, Plane &pv, Plane &pc, Plane &pn, auto has_pv) {
            int plo[RB], phi[RB];
            join_prev(pv, pc, plo, phi, has_pv);
            request(s + DT_NPL);
            wait_vm<AHEAD>();
            if (s + 1 < S) {
                stats(s + 1, pn, edge_tag);
                decide(s, plo, phi, pc, pn, std::true_type{});
            } else {
                decide(s, plo, phi, pc, pn, std::false_type{});
            }
        };
        step(0, P2, P0, P1, std::false_type{});
        for (int s = 1; s < S; s += 3) {
            step(s, P0, P1, P2, std::true_type{});
            if (s + 1 >= S) break;
            step(s + 1, P1, P2, P0, std::true_type{});
            if (s + 2 >= S) break;
            step(s + 2, P2, P0, P1, std::true_type{});
        }
    };
    // a band is interior when its 64 lanes and RB + 2 rows all lie in the image
    const bool interior = x - lane >= 0 && x - lane + 63 < W && y0 >= 1 && y0 + RB < H;  // wave-uniform
    if (interior)
        run(std::false_type{});
    else
        run(std::true_type{});
    wait_vm<0>();  // no copy may land in LDS after this wavefront is gone
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    for (int k = lane; k < S * RB; k += 64) {
        const int s = k / RB, r = k % RB;
        if (y0 + r < H) mask[((int64_t)s * H + y0 + r) * ntx + tx] = wd[k];
    }
}

// popcount totals of SUM_THREADS * SUM_WORDS consecutive words
__global__ __launch_bounds__(SUM_THREADS) void detect_sums_kernel(const unsigned long long *__restrict__ mask,
                                                                  int64_t nwords, int *__restrict__ bsum) {
    constexpr int NW = SUM_THREADS * SUM_WORDS;
    __shared__ int part[SUM_THREADS / 64];
    const int64_t bbase = (int64_t)blockIdx.x * NW;
    int c = 0;
    for (int i = threadIdx.x; i < NW; i += SUM_THREADS)  // coalesced
        if (bbase + i < nwords) c += __popcll(mask[bbase + i]);
    for (int o = 32; o > 0; o >>= 1) c += __shfl_down(c, o, 64);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        int t = 0;
        for (int i = 0; i < SUM_THREADS / 64; ++i) t += part[i];
        bsum[blockIdx.x] = t;
    }
}

__global__ __launch_bounds__(SCAN_BLOCK) void scan_counts_kernel(const int *__restrict__ counts, int n,
                                                                  int *__restrict__ offsets,
                                                                  int *__restrict__ total) {
    __shared__ int sh[SCAN_BLOCK];
    const int per = (n + SCAN_BLOCK - 1) / SCAN_BLOCK;
    const int b = threadIdx.x * per;
    const int e = min(b + per, n);
    int local = 0;
    for (int i = b; i < e; ++i) local += counts[i];
    sh[threadIdx.x] = local;
    __syncthreads();
    for (int d = 1; d < SCAN_BLOCK; d <<= 1) {
        const int t = threadIdx.x >= d ? sh[threadIdx.x - d] : 0;
        __syncthreads();
        sh[threadIdx.x] += t;
        __syncthreads();
    }
    int run = sh[threadIdx.x] - local;  // exclusive
    for (int i = b; i < e; ++i) {
        offsets[i] = run;
        run += counts[i];
    }
    if (threadIdx.x == SCAN_BLOCK - 1) *total = sh[SCAN_BLOCK - 1];
}

// Writes the records of the words of one block.  The block's detections are
// first listed in LDS in output order (word, bit), then written one per
// thread, so that the reads of V are independent of each other; a block with
// more detections than the list holds walks its words thread by thread.
__device__ __forceinline__ void emit_one(const float *__restrict__ V, int64_t pitch, int64_t plane_stride, int H,
                                         int ntx, unsigned word, int b, const unsigned long long *__restrict__ pmask,
                                         fdvm_blob *__restrict__ out, int idx, int cap) {
    if (idx >= cap) return;
    const unsigned sy = word / (unsigned)ntx;                  // word = (s * H + y) * ntx + tx
    const int tx = (int)(word - sy * (unsigned)ntx);
    const int s = (int)(sy / (unsigned)H);
    const int y = (int)(sy - (unsigned)s * (unsigned)H);
    const int xx = tx * DT_W + b;
    const float v = V[(int64_t)s * plane_stride + (int64_t)y * pitch + xx];
    fdvm_blob rec;
    rec.y = y;
    rec.x = xx;
    rec.scale = s;
    rec.polarity = pmask ? (((pmask[word] >> b) & 1ull) ? 1 : -1) : (v < 0.0f ? 1 : -1);
    rec.value = v;
    out[idx] = rec;
}

constexpr int EMIT_LIST = 2048;   // detections per block listed in LDS
constexpr int EMIT_PREFIX_BLOCKS = 4096;   // emit forms its own block offsets up to this many blocks

__global__ __launch_bounds__(SUM_THREADS) void detect_emit_kernel(const float *__restrict__ V, int64_t pitch,
                                                                   int64_t plane_stride, int H, int W, int ntx,
                                                                   const unsigned long long *__restrict__ mask,
                                                                   const unsigned long long *__restrict__ pmask,
                                                                   int64_t nwords, const int *__restrict__ boff,
                                                                   const int *__restrict__ bsum,
                                                                   int32_t *__restrict__ count,
                                                                   fdvm_blob *__restrict__ out, int cap) {
    constexpr int NW = SUM_THREADS * SUM_WORDS;
    static_assert(NW <= (1 << 26), "word index in a list entry");
    __shared__ unsigned long long wbuf[NW];
    __shared__ uint32_t list[EMIT_LIST];   // (word in block << 6) | bit
    __shared__ int part[SUM_THREADS / 64];
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int64_t bbase = (int64_t)blockIdx.x * NW;
    // coalesced staging of the block's words
    for (int i = threadIdx.x; i < NW; i += SUM_THREADS)
        wbuf[i] = bbase + i < nwords ? mask[bbase + i] : 0ull;
    __syncthreads();
    const int first = threadIdx.x * SUM_WORDS;
    int c = 0;
#pragma unroll
    for (int i = 0; i < SUM_WORDS; ++i) c += __popcll(wbuf[first + i]);
    // exclusive prefix of c over the block
    int incl = c;
    for (int o = 1; o < 64; o <<= 1) {
        const int t = __shfl_up(incl, o, 64);
        if (lane >= o) incl += t;
    }
    if (lane == 63) part[wv] = incl;
    __syncthreads();
    int before = 0, total = 0;
    for (int i = 0; i < SUM_THREADS / 64; ++i) {
        before += i < wv ? part[i] : 0;
        total += part[i];
    }
    const int local = before + incl - c;   // this thread's first record within the block
    int base;
    if (bsum) {
        // few blocks: this block's offset is the sum of the totals of the
        // blocks before it (read straight from the per-block totals, fixed
        // order); the last block writes the total count
        int acc = 0;
        for (int i = threadIdx.x; i < (int)blockIdx.x; i += SUM_THREADS) acc += bsum[i];
        for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o, 64);
        __syncthreads();   // part[] is reused
        if (lane == 0) part[wv] = acc;
        __syncthreads();
        base = 0;
        for (int i = 0; i < SUM_THREADS / 64; ++i) base += part[i];
        if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) *count = base + total;
    } else {
        base = boff[blockIdx.x];
    }
    if (total == 0) return;                // block-uniform
    if (total <= EMIT_LIST) {
        int li = local;
        for (int i = 0; i < SUM_WORDS; ++i) {
            unsigned long long bits = wbuf[first + i];
            while (bits) {
                const int b = __ffsll((long long)bits) - 1;
                bits &= bits - 1;
                list[li++] = ((uint32_t)(first + i) << 6) | (uint32_t)b;
            }
        }
        __syncthreads();
        for (int t = threadIdx.x; t < total; t += SUM_THREADS) {
            const uint32_t e = list[t];
            emit_one(V, pitch, plane_stride, H, ntx, (unsigned)(bbase + (e >> 6)), (int)(e & 63u), pmask, out,
                     base + t, cap);
        }
    } else {
        int idx = base + local;
        for (int i = 0; i < SUM_WORDS; ++i) {
            unsigned long long bits = wbuf[first + i];
            while (bits) {
                const int b = __ffsll((long long)bits) - 1;
                bits &= bits - 1;
                emit_one(V, pitch, plane_stride, H, ntx, (unsigned)(bbase + first + i), b, pmask, out, idx, cap);
                ++idx;
            }
        }
    }
}

}  // namespace

hipError_t launch_highpass(const float *blur, int64_t H, int64_t W, int64_t pitch, int64_t plane_stride,
                           int nscales, const float *norms, unsigned what, float *out,
                           int64_t out_plane_stride, hipStream_t st) {
    Norms n{};
    for (int s = 0; s < nscales; ++s) n.v[s] = norms[s];
    int nout = 0;
    for (unsigned b = what; b; b >>= 1) nout += (int)(b & 1u);
    dim3 grid((unsigned)((W + HP_BLOCK - 1) / HP_BLOCK), (unsigned)H, (unsigned)nscales);
    hipLaunchKernelGGL(highpass_kernel, grid, dim3(HP_BLOCK), 0, st, blur, pitch, plane_stride, (int)H,
                       (int)W, what, nout, n, out, out_plane_stride);
    return hipGetLastError();
}

namespace {
struct DetectLayout {
    int ntx;
    int64_t nwords;
    int64_t nblocks;
    size_t mask_bytes, sums_bytes;
};
DetectLayout detect_layout(int64_t H, int64_t W, int nscales) {
    DetectLayout d;
    d.ntx = (int)((W + DT_W - 1) / DT_W);
    const int64_t hpad = ((H + DT_ROWS * DT_WAVES - 1) / (DT_ROWS * DT_WAVES)) * DT_ROWS * DT_WAVES;
    // words for rows up to the padded height are written (as zero) too
    d.nwords = (int64_t)nscales * H * d.ntx;
    const int64_t alloc_words = (int64_t)nscales * hpad * d.ntx + (int64_t)d.ntx * DT_ROWS;
    d.nblocks = (d.nwords + SUM_THREADS * SUM_WORDS - 1) / (SUM_THREADS * SUM_WORDS);
    d.mask_bytes = ((size_t)alloc_words * 8 + 255) & ~(size_t)255;
    d.sums_bytes = ((size_t)(2 * d.nblocks + 1) * sizeof(int) + 255) & ~(size_t)255;
    return d;
}
}  // namespace

size_t detect_workspace_bytes(int64_t H, int64_t W, int nscales) {
    const DetectLayout d = detect_layout(H, W, nscales);
    return d.mask_bytes + d.sums_bytes;
}

unsigned long long *detect_mask_words(void *ws) { return static_cast<unsigned long long *>(ws); }

hipError_t launch_compact(const float *resp, int64_t H, int64_t W, int64_t pitch, int64_t plane_stride,
                          int nscales, const unsigned long long *pmask, fdvm_blob *out, int32_t cap,
                          int32_t *count, void *ws, hipStream_t st) {
    const DetectLayout d = detect_layout(H, W, nscales);
    unsigned long long *mask = static_cast<unsigned long long *>(ws);
    int *bsum = reinterpret_cast<int *>(static_cast<char *>(ws) + d.mask_bytes);
    int *boff = bsum + d.nblocks;
    hipLaunchKernelGGL(detect_sums_kernel, dim3((unsigned)d.nblocks), dim3(SUM_THREADS), 0, st, mask, d.nwords,
                       bsum);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // up to EMIT_PREFIX_BLOCKS blocks every emit block sums the totals before
    // it itself (at most that many reads from L2 per block); beyond, a scan
    // kernel forms the offsets
    const bool in_emit = d.nblocks <= EMIT_PREFIX_BLOCKS;
    if (!in_emit) {
        hipLaunchKernelGGL(scan_counts_kernel, dim3(1), dim3(SCAN_BLOCK), 0, st, bsum, (int)d.nblocks, boff, count);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(detect_emit_kernel, dim3((unsigned)d.nblocks), dim3(SUM_THREADS), 0, st, resp, pitch,
                       plane_stride, (int)H, (int)W, d.ntx, mask, pmask, d.nwords, boff,
                       in_emit ? bsum : nullptr, count, out, cap);
    return hipGetLastError();
}

hipError_t launch_detect(const float *resp, int64_t H, int64_t W, int64_t pitch, int64_t plane_stride,
                         int nscales, float tau, int border, fdvm_blob *out, int32_t cap, int32_t *count,
                         void *ws, hipStream_t st) {
    const DetectLayout d = detect_layout(H, W, nscales);
    unsigned long long *mask = static_cast<unsigned long long *>(ws);
    dim3 g1((unsigned)(d.ntx * ((H + DT_ROWS * DT_WAVES - 1) / (DT_ROWS * DT_WAVES))));
    if (tau > 0.0f)
        hipLaunchKernelGGL(detect_mask_kernel<true>, g1, dim3(DT_WAVES * 64), 0, st, resp, pitch, plane_stride,
                           nscales, (int)H, (int)W, tau, border, mask, d.ntx);
    else
        hipLaunchKernelGGL(detect_mask_kernel<false>, g1, dim3(DT_WAVES * 64), 0, st, resp, pitch, plane_stride,
                           nscales, (int)H, (int)W, tau, border, mask, d.ntx);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_compact(resp, H, W, pitch, plane_stride, nscales, nullptr, out, cap, count, ws, st);
}

}  // namespace fdvm
