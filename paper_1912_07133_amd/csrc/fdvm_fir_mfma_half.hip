// Toeplitz-block FIR (Eq A5) on the gfx950 matrix cores with half-precision
// operands and float32 accumulation (v_mfma_f32_32x32x16_f16 / _bf16), for
// frames stored as float16 or bfloat16 (the operands are the stored samples,
// exactly) and as uint16 (each sample split exactly into a float16 pair).
//
// Precision.  Each tap h (scaled per scale by a power of two 2^e that brings
// the largest to [0.5, 1)) is carried as a pair of the operand type: hi = h
// rounded, lo' = (h - hi) 2^L rounded (L = 11 for float16, 8 for bfloat16),
// so the taps keep 22 / 16 significant bits and the unit dc gain and the
// vanishing moments of the design (Eqs 7, 11) hold to about 2^-22 / 2^-16.
// The intermediate between the passes is stored as the same kind of pair.
// Products of hi parts go to one accumulator, products with one lo' part to a
// second, and the result is main + 2^-L second: scaling lo' by 2^L keeps it a
// normal number of the half type (no bits lost to subnormals), and the
// dropped lo' x lo' product is 2^-2L of the terms.  float16 intermediates are
// stored times 2^-4 so that sums of samples up to 65504 stay finite.
//
// Geometry.  One kernel filters the rows of a plane along their length and
// writes the result transposed; run twice (frame -> transposed pair planes ->
// output planes) it is the separable blur.  Per wavefront 32 rows y0 + i and
// 64 outputs p0 .. p0 + 63 along the rows, as two 32 x 32 blocks t = 0, 1.
// One instruction takes 16 consecutive samples of each row:
//     D_t[i][j] += sum_{k=0..15} x(y0 + i, r + k) h(p0 + 32 t + j - r - k)
// A (32 x 16): lane i + 32 g holds samples r + 8 g .. r + 8 g + 7 of row
// y0 + i, one 16-byte load; B (16 x 32): lane j + 32 g holds h(c - 8 g - u),
// u = 0..7, c = p0 + 32 t + j - r, one 16-byte LDS read from a table whose
// entry c is h(c), h(c - 1), .., h(c - 7) (hi, and lo').  With the half-
// length rounded up to K' (a multiple of 32), groups g = 0 .. 2K'/16 + 3 of
// 16 samples from p0 - K' meet block 0 for g <= 2K'/16 + 1 and block 1 for
// g >= 2, and block 1 at group g + 2 uses block 0's B fragment of group g,
// so each group reads one fragment pair from LDS.  The tables are built once
// per call in the workspace and copied to LDS by every work-group.
#include <cmath>
#include <type_traits>

#include "fdvm_internal.h"

namespace fdvm {
namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int HT_ROWS = 32;       // rows per wavefront
constexpr int HT_POS = 64;        // outputs per wavefront along the rows (two blocks)
constexpr int HT_WPB = 4;         // wavefronts per work-group
// two wavefronts stacked across rows: a work-group writes 64 consecutive
// samples (128 bytes) of each transposed intermediate row, whole cache lines
constexpr int HT_WROW = 2;
constexpr int HT_WPOS = HT_WPB / HT_WROW;   // and two side by side along the rows
constexpr int HT_G = 16;          // samples per instruction
// row tiles taken together in the launch order (scale, then HT_RG row tiles,
// then position groups): the work-groups running at once write runs twice as
// long in each output row, and neighbours along the rows still share their
// input windows in L2 (1, 2, 4, 8 measured: 2 is best for both passes)
constexpr int HT_RG = 2;
constexpr int HT_ARG_TAPS = 880;  // tap words that fit in the kernel arguments
constexpr int HT_KP_MAX = ((FDVM_MAX_FIR_HALF + 31) / 32) * 32;
constexpr int HT_NE_MAX = 2 * HT_KP_MAX + 120;
constexpr size_t HT_TABLE_BYTES = (size_t)FDVM_MAX_SCALES * 2 * HT_NE_MAX * sizeof(u32x4);

enum { SRC_HALF = 0, SRC_U16 = 1, SRC_PAIR = 2 };

// K' = K rounded up to a multiple of 32, so that the groups meeting both
// output blocks (K'/8 of them) come in whole rounds of the four ring slots
constexpr int HT_KQ = 32;
__host__ __device__ constexpr int round_kp(int k) { return ((k + HT_KQ - 1) / HT_KQ) * HT_KQ; }
__host__ __device__ constexpr int table_entries(int kp) { return 2 * kp + 120; }

struct HalfTaps {   // table builder: taps of one launch's scales, times 2^e, centre first
    int nscales;
    int K[FDVM_MAX_SCALES];
    int off[FDVM_MAX_SCALES];
    int tab[FDVM_MAX_SCALES];   // table offset, in 16-byte entries
    float h[HT_ARG_TAPS];
};

struct HalfSet {    // filter kernel: per scale half-length, table, factor on the sums
    int nscales;
    int K[FDVM_MAX_SCALES];
    int tab[FDVM_MAX_SCALES];
    float post[FDVM_MAX_SCALES];
};

template <typename H>
struct Op;
template <>
struct Op<_Float16> {
    static constexpr float lo_scale = 2048.0f;   // 2^11
    __device__ static uint16_t bits(float v) { return __builtin_bit_cast(uint16_t, (_Float16)v); }
    __device__ static float value(uint16_t b) { return (float)__builtin_bit_cast(_Float16, b); }
    __device__ static floatx16 mfma(u32x4 a, u32x4 b, floatx16 c) {
        return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8, a), __builtin_bit_cast(f16x8, b), c,
                                                      0, 0, 0);
    }
};
template <>
struct Op<__bf16> {
    static constexpr float lo_scale = 256.0f;    // 2^8
    __device__ static uint16_t bits(float v) { return __builtin_bit_cast(uint16_t, (__bf16)v); }
    __device__ static float value(uint16_t b) { return __uint_as_float(((uint32_t)b) << 16); }
    __device__ static floatx16 mfma(u32x4 a, u32x4 b, floatx16 c) {
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b),
                                                       c, 0, 0, 0);
    }
};

// v = value(hi) + value(lo) / lo_scale to 2^-2p relative
template <typename H>
__device__ __forceinline__ void split(float v, uint16_t &hi, uint16_t &lo) {
    hi = Op<H>::bits(v);
    lo = Op<H>::bits((v - Op<H>::value(hi)) * Op<H>::lo_scale);
}

// wait until at most N vector-memory operations of this wavefront are in
// flight (s_waitcnt with the expcnt and lgkmcnt fields at their no-wait
// maxima; vmcnt split over bits 3:0 and 15:14).  The builtin, unlike an asm
// block, is seen by the compiler's own wait tracking, which then knows that
// the copies issued before those N operations have landed in LDS.
template <int N>
__device__ __forceinline__ void wait_vm() {
    static_assert(N >= 0 && N < 64, "vmcnt range");
    __builtin_amdgcn_s_waitcnt((N & 0xf) | (0x7 << 4) | (0xf << 8) | ((N >> 4) << 14));
}

__device__ __forceinline__ int xcd_logical(int hw, int n) {
    constexpr int NX = 8;
    const int xcd = hw % NX, slot = hw / NX;
    const int q = n / NX, r = n % NX;
    return xcd * q + min(xcd, r) + slot;
}

// one work-group per scale: entry e of the scale's table holds taps
// h(c) .. h(c - 7), c = e - K' - 56 (zero beyond the half-length), hi entries
// first, then lo'
template <typename H>
__global__ __launch_bounds__(256) void fir_half_tables_kernel(u32x4 *__restrict__ tables, HalfTaps ht) {
    const int s = blockIdx.x;
    const int K = ht.K[s];
    const int KP = round_kp(K);
    const int NE = table_entries(KP);
    const int C0 = KP + 56;
    const float *h = ht.h + ht.off[s];
    u32x4 *tab = tables + ht.tab[s];
    for (int e = threadIdx.x; e < NE; e += blockDim.x) {
        uint16_t hi[8], lo[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int d = e - C0 - u;
            const int ad = d < 0 ? -d : d;
            split<H>(ad <= K ? h[ad] : 0.0f, hi[u], lo[u]);
        }
        u32x4 vh, vl;
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            vh[w] = (uint32_t)hi[2 * w] | ((uint32_t)hi[2 * w + 1] << 16);
            vl[w] = (uint32_t)lo[2 * w] | ((uint32_t)lo[2 * w + 1] << 16);
        }
        tab[e] = vh;
        tab[NE + e] = vl;
    }
}

// Filters R rows (plane s of the source, or plane 0 for all scales when
// src_plane is 0) along their length: n outputs per row from the n_in samples
// held (n_in >= n: the intermediate's rows carry a padding already filled
// with the boundary extension); output p of row y goes to
// dst[p * dst_pitch + y] of plane s for y < R_out: a float32 plane (OUT_F32)
// or a pair of half planes (hi at dst, lo' at dst_lo), rows y >= R of the
// pair holding the extension (row R - 1, or zero).  FAST: every group of
// eight samples lies wholly inside [0, n_in) or wholly outside (n_in a
// multiple of 8, rows 16-byte aligned): one clamped 16-byte load and a
// select; otherwise eight clamped element loads.  Neither form branches
// around a load, so the loads of later groups stay in flight.  Logical blocks
// (scale, row tile within a group of HT_RG, position group, row-tile group),
// scale fastest, XCD-contiguous.
template <typename H, int SRC, bool OUT_F32, bool FAST, bool ACCUM = false>
__global__ __launch_bounds__(HT_WPB * 64) void fir_half_rows_kernel(
    const uint16_t *__restrict__ src, const uint16_t *__restrict__ src_lo, int64_t src_pitch, int64_t src_plane,
    int R, int n, int n_in, void *__restrict__ dst, uint16_t *__restrict__ dst_lo, int64_t dst_pitch,
    int64_t dst_plane, int R_out, int boundary, int vec_out, const u32x4 *__restrict__ tables, HalfSet hs,
    int stage_off) {
    constexpr bool SPLIT = SRC != SRC_HALF;   // A carries a lo' part
    constexpr bool PAIR = SRC == SRC_PAIR;
    // the scale's table (NE hi entries, NE lo' entries), then (FAST) each
    // wavefront's staging buffer from entry stage_off on
    extern __shared__ u32x4 lds[];
    const int nrt = (R_out + HT_ROWS * HT_WROW - 1) / (HT_ROWS * HT_WROW);
    const int npg = (n + HT_POS * HT_WPOS - 1) / (HT_POS * HT_WPOS);
    const int S = hs.nscales;
    const int lb = xcd_logical(blockIdx.x, nrt * npg * S);
    const int s = lb % S;
    const int r2 = lb / S;
    const int rq = r2 / (HT_RG * npg), rw = r2 % (HT_RG * npg);
    const int rgn = min(HT_RG, nrt - rq * HT_RG);   // row tiles in this group
    const int rt = rq * HT_RG + rw % rgn;
    const int pg = rw / rgn;
    const int KP = round_kp(hs.K[s]);
    const int NE = table_entries(KP);
    const int NG = KP / 8 + 4;   // groups: 2 K'/16 + 4
    const int C0 = KP + 56;
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int p0 = (pg * HT_WPOS + wv % HT_WPOS) * HT_POS;
    const int y0 = (rt * HT_WROW + wv / HT_WPOS) * HT_ROWS;
    const bool live = p0 < n && y0 < R_out;   // wave-uniform
    // FAST: chunks of four groups (64 samples of the wavefront's 32 rows) are
    // fetched with whole-line loads (lane l: row 8 j + l / 8, 16-byte segment
    // l % 8; every instruction reads 8 full 128-byte lines), AHEAD chunks in
    // flight, chunk c in slot c % AHEAD.  Two for pair sources; one for the
    // first pass, whose register budget would otherwise cost a wavefront per
    // SIMD.
    constexpr int AHEAD = PAIR ? 2 : 1;
    const int lr = lane >> 3, lq = lane & 7;
    int64_t roffs[4];
#pragma unroll
    for (int j = 0; j < 4; ++j)
        roffs[j] = (int64_t)s * src_plane + (int64_t)min(y0 + 8 * j + lr, R - 1) * src_pitch;
    u32x4 fa[4], fla[4], fb[4], flb[4];
    auto gload = [&](int c, u32x4(&fh)[4], u32x4(&fl)[4]) {
        const int c0 = p0 - KP + 64 * c + 8 * lq;
        const int cl = min(max(c0, 0), n_in - 8);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            fh[j] = *reinterpret_cast<const u32x4 *>(src + roffs[j] + cl);
            if constexpr (PAIR) fl[j] = *reinterpret_cast<const u32x4 *>(src_lo + roffs[j] + cl);
        }
    };
    {
        const u32x4 *tg = tables + hs.tab[s];
        if constexpr (FAST) {
            // the table straight into LDS, 16 bytes per lane (the last round's
            // spare lanes land in the padding before the staging buffers),
            // then the first chunks: only the table is waited for before the
            // barrier, so their latency overlaps the copy
            for (int e0 = 0; e0 < 2 * NE; e0 += HT_WPB * 64)
                __builtin_amdgcn_global_load_lds((const void *)(tg + min(e0 + (int)threadIdx.x, 2 * NE - 1)),
                                                 (__attribute__((address_space(3))) void *)(lds + e0 + wv * 64),
                                                 16, 0, 0);
            __builtin_amdgcn_sched_barrier(0);
            if (live) {
                gload(0, fa, fla);
                if constexpr (AHEAD == 2) gload(1, fb, flb);
                __builtin_amdgcn_sched_barrier(0);
                wait_vm<(PAIR ? 8 : 4) * AHEAD>();
            } else {
                wait_vm<0>();
            }
        } else {
            for (int e = threadIdx.x; e < 2 * NE; e += blockDim.x) lds[e] = tg[e];
        }
    }
    if constexpr (FAST) {
        // every wavefront has waited for its own copies of the table; a plain
        // barrier (no fence) lets the first chunks stay in flight across it
        asm volatile("" ::: "memory");
        __builtin_amdgcn_s_barrier();
        asm volatile("" ::: "memory");
    } else {
        __syncthreads();
    }
    if (!live) return;   // no barrier follows
    const int i = lane & 31;   // A: row y0 + i; B and D: output p0 + 32 t + i
    const int g8 = lane >> 5;  // which eight of the group's sixteen samples
    const int row = min(y0 + i, R - 1);
    const bool rep = boundary == FDVM_BC_REPLICATE;
    const int64_t roff = (int64_t)s * src_plane + (int64_t)row * src_pitch;
    const uint16_t *rh = src + roff;
    const uint16_t *rl = PAIR ? src_lo + roff : nullptr;
    const int cb = p0 - KP + 8 * g8;   // first sample of this lane's eight in group 0
    // the extension at samples outside [0, n_in): the clamped loads already
    // replicate in the element form; FAST chunks wholly outside take the
    // first / last sample of the clamped chunk, or zero
    auto extend = [&](int g, u32x4 &v) {
        const int c0 = cb + HT_G * g;
        if constexpr (FAST) {
            const bool left = c0 < 0, out = left || c0 >= n_in;
            uint32_t e = left ? (v[0] & 0xffffu) : (v[3] >> 16);
            e = rep ? (e | (e << 16)) : 0u;
#pragma unroll
            for (int w = 0; w < 4; ++w) v[w] = out ? e : v[w];
        } else {
#pragma unroll
            for (int w = 0; w < 4; ++w) {
                const int c = c0 + 2 * w;
                const uint32_t m = ((rep || (c >= 0 && c < n_in)) ? 0xffffu : 0u) |
                                   ((rep || (c + 1 >= 0 && c + 1 < n_in)) ? 0xffff0000u : 0u);
                v[w] &= m;
            }
        }
    };
    // uint16 samples -> float16 hi (rounded toward zero, so 65535 stays
    // finite) and lo' = (x - hi) 2^11, both exact
    auto split_u16 = [&](const u32x4 &raw, u32x4 &ah, u32x4 &al) {
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            const float fa = (float)(raw[w] & 0xffffu), fb = (float)(raw[w] >> 16);
            const auto hv = __builtin_amdgcn_cvt_pkrtz(fa, fb);
            const float la = (fa - (float)hv[0]) * 2048.0f, lb2 = (fb - (float)hv[1]) * 2048.0f;
            const auto lv = __builtin_amdgcn_cvt_pkrtz(la, lb2);
            ah[w] = __builtin_bit_cast(uint32_t, hv);
            al[w] = __builtin_bit_cast(uint32_t, lv);
        }
    };
    floatx16 m0, m1, l0, l1;   // hi x hi sums and lo' sums, blocks 0 and 1
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        m0[e] = 0.0f;
        m1[e] = 0.0f;
        l0[e] = 0.0f;
        l1[e] = 0.0f;
    }
    // block 0's tap fragment of group g is entry ebase - 16 g; block 1's is
    // block 0's of group g - 2, read again rather than kept (a register ring
    // of fragments would cost the kernel a wavefront per SIMD)
    const int ebase = C0 + KP + i - 8 * g8;   // block 0's entry at group 0
    // the products of group g from its raw samples vh (and vl)
    auto mma = [&](int g, u32x4 vh, u32x4 vl, auto slot_c, auto blocks_c) {
        constexpr int k = decltype(slot_c)::value;
        constexpr int BL = decltype(blocks_c)::value;   // 1: block 0, 2: block 1, 3: both
        u32x4 ah, al;
        extend(g, vh);
        if constexpr (PAIR) extend(g, vl);
        if constexpr (SRC == SRC_U16) {
            split_u16(vh, ah, al);
        } else {
            ah = vh;
            if constexpr (PAIR) al = vl;
        }
        if constexpr (BL & 1) {
            const u32x4 bh = lds[ebase - HT_G * g];
            const u32x4 bl = lds[NE + ebase - HT_G * g];
            m0 = Op<H>::mfma(ah, bh, m0);
            l0 = Op<H>::mfma(ah, bl, l0);
            if constexpr (SPLIT) l0 = Op<H>::mfma(al, bh, l0);
        }
        if constexpr (BL & 2) {
            const u32x4 bh = lds[ebase - HT_G * (g - 2)];
            const u32x4 bl = lds[NE + ebase - HT_G * (g - 2)];
            m1 = Op<H>::mfma(ah, bh, m1);
            l1 = Op<H>::mfma(ah, bl, l1);
            if constexpr (SPLIT) l1 = Op<H>::mfma(al, bh, l1);
        }
    };
    using I = std::integral_constant<int, 0>;
    using I1 = std::integral_constant<int, 1>;
    using I2 = std::integral_constant<int, 2>;
    using I3 = std::integral_constant<int, 3>;
    // block 0 alone for groups 0, 1; both for 2 .. NG - 3 (K'/8 groups, a
    // multiple of 4); block 1 alone for NG - 2, NG - 1
    if constexpr (FAST) {
        // Each chunk (fetched before the barrier for the first AHEAD) is
        // written to this wavefront's LDS buffer with the segment of row r at
        // slot segment ^ (r % 8), so that the A fragments (lane i + 32 g: row
        // i, segment 2 (g % 4) + g) come back conflict-free, and its slot is
        // refilled with chunk c + AHEAD (the last chunk again at the end: an
        // L1 hit).  The buffer is the wavefront's own and LDS operations of a
        // wavefront complete in order, so no barrier is needed between a
        // chunk's reads and the next write.
        u32x4 *sh = lds + stage_off + wv * (PAIR ? 512 : 256);
        u32x4 *sl = sh + 256;
        const int NC = NG / 4;   // >= 2 (K' >= 32)
        const int rsw = i & 7;
        auto chunk = [&](int c, auto kind_c, u32x4(&fh)[4], u32x4(&fl)[4]) {
            constexpr int KIND = decltype(kind_c)::value;   // 0 first, 1 middle, 2 last
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                sh[(8 * j + lr) * 8 + (lq ^ lr)] = fh[j];
                if constexpr (PAIR) sl[(8 * j + lr) * 8 + (lq ^ lr)] = fl[j];
            }
            // the refill after the writes: hoisted above them, it would be
            // waited for with them
            __builtin_amdgcn_sched_barrier(0);
            gload(min(c + AHEAD, NC - 1), fh, fl);
            // keep the refill here: the scheduler would otherwise sink it
            __builtin_amdgcn_sched_barrier(0);
            auto grp = [&](auto gi_c, auto blocks_c) {
                constexpr int gi = decltype(gi_c)::value;
                const int seg = 2 * gi + g8;
                const u32x4 vh = sh[i * 8 + (seg ^ rsw)];
                u32x4 vl;
                if constexpr (PAIR) vl = sl[i * 8 + (seg ^ rsw)];
                mma(4 * c + gi, vh, vl, gi_c, blocks_c);
            };
            using B0 = std::integral_constant<int, KIND == 0 ? 1 : 3>;
            using B1 = std::integral_constant<int, KIND == 2 ? 2 : 3>;
            grp(I{}, B0{});
            grp(I1{}, B0{});
            grp(I2{}, B1{});
            grp(I3{}, B1{});
        };
        using FIRST = std::integral_constant<int, 0>;
        using MID = std::integral_constant<int, 1>;
        using LAST = std::integral_constant<int, 2>;
        if constexpr (AHEAD == 2) {
            chunk(0, FIRST{}, fa, fla);
            int c = 1;
            for (; c + 2 < NC; c += 2) {
                chunk(c, MID{}, fb, flb);
                chunk(c + 1, MID{}, fa, fla);
            }
            if (c < NC - 1) chunk(c, MID{}, fb, flb);
            // both slots hold the last chunk by now (the refills are clamped to it)
        } else {
            chunk(0, FIRST{}, fa, fla);
            for (int c = 1; c < NC - 1; ++c) chunk(c, MID{}, fa, fla);
        }
        chunk(NC - 1, LAST{}, fa, fla);
    } else {
        // element loads into a 4-slot register ring, three groups ahead
        auto load = [&](int g, u32x4 &vh, u32x4 &vl) {
            const int c0 = cb + HT_G * g;
            uint32_t eh[8], el[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int cc = min(max(c0 + u, 0), n_in - 1);
                eh[u] = rh[cc];
                if constexpr (PAIR) el[u] = rl[cc];
            }
#pragma unroll
            for (int w = 0; w < 4; ++w) {
                vh[w] = eh[2 * w] | (eh[2 * w + 1] << 16);
                if constexpr (PAIR) vl[w] = el[2 * w] | (el[2 * w + 1] << 16);
            }
        };
        u32x4 ra[4], rla[4];
#pragma unroll
        for (int q = 0; q < 3; ++q) load(q, ra[q], rla[q]);
        auto step = [&](int g, auto slot_c, auto blocks_c, auto load_c) {
            constexpr int k = decltype(slot_c)::value;
            if constexpr (decltype(load_c)::value) {
                constexpr int kn = (k + 3) % 4;
                load(min(g + 3, NG - 1), ra[kn], rla[kn]);
            }
            __builtin_amdgcn_sched_barrier(0);
            mma(g, ra[k], rla[k], slot_c, blocks_c);
        };
        using LOAD = std::true_type;
        using NOLOAD = std::false_type;
        step(0, I{}, I1{}, LOAD{});
        step(1, I1{}, I1{}, LOAD{});
        for (int g = 2; g < NG - 2; g += 4) {
            step(g, I2{}, I3{}, LOAD{});
            step(g + 1, I3{}, I3{}, LOAD{});
            step(g + 2, I{}, I3{}, LOAD{});
            step(g + 3, I1{}, I3{}, LOAD{});
        }
        step(NG - 2, I2{}, I2{}, NOLOAD{});
        step(NG - 1, I3{}, I2{}, NOLOAD{});
    }
    // D[i][j] of block t sits in lane j + 32 ((i / 4) % 2), register
    // (i / 8) 4 + i % 4: each lane holds rows y0 + 8 q + 4 g8 + (0..3) of
    // output p0 + 32 t + (lane & 31)
    const float post = hs.post[s];
    constexpr float inv_lo = 1.0f / Op<H>::lo_scale;
    auto value = [&](const floatx16 &m, const floatx16 &l, int q, float (&v)[4]) {
        const int y = y0 + 8 * q + 4 * g8;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            v[u] = (m[4 * q + u] + l[4 * q + u] * inv_lo) * post;
            if (!OUT_F32 && !rep && y + u >= R) v[u] = 0.0f;   // zero extension rows
        }
    };
    if constexpr (FAST) {
        // Each block goes through the wavefront's staging buffer, one 128-byte
        // LDS row per output: 32 float32 samples (16-byte segment c: rows
        // y0 + 4 c .. + 3), or the 32 hi samples then the 32 lo' samples
        // (segment c: rows y0 + 8 (c % 4) .. + 7 of plane c / 4), segment c of
        // row j at slot c ^ (j % 8) and, for the 8-byte halves the pair form
        // writes, the half flipped in rows j with j / 8 odd: every group of
        // lanes that LDS serves together meets distinct banks.  Read back,
        // lane l holds segment l % 8 of output 8 k + l / 8, so that each store
        // instruction writes 8 outputs x 128 contiguous bytes (float32) or
        // 8 x 64 bytes of each plane, not 32 outputs x 32 or 16 bytes.
        u32x4 *ob = lds + stage_off + wv * (PAIR ? 512 : 256);
        const int lr = lane >> 3, lq = lane & 7;
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            const floatx16 &m = t ? m1 : m0;
            const floatx16 &l = t ? l1 : l0;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                float v[4];
                value(m, l, q, v);
                if constexpr (OUT_F32) {
                    ob[i * 8 + ((2 * q + g8) ^ (i & 7))] = __builtin_bit_cast(u32x4, f32x4{v[0], v[1], v[2], v[3]});
                } else {
                    uint16_t hi[4], lo[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) split<H>(v[u], hi[u], lo[u]);
                    u32x2 *ob2 = reinterpret_cast<u32x2 *>(ob);
                    const int hf = g8 ^ ((i >> 3) & 1);
                    ob2[2 * (i * 8 + (q ^ (i & 7))) + hf] =
                        u32x2{(uint32_t)hi[0] | ((uint32_t)hi[1] << 16), (uint32_t)hi[2] | ((uint32_t)hi[3] << 16)};
                    ob2[2 * (i * 8 + ((4 + q) ^ (i & 7))) + hf] =
                        u32x2{(uint32_t)lo[0] | ((uint32_t)lo[1] << 16), (uint32_t)lo[2] | ((uint32_t)lo[3] << 16)};
                }
            }
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int j = 8 * k + lr;
                u32x4 w = ob[j * 8 + (lq ^ lr)];
                const int p = p0 + 32 * t + j;
                if (p >= n) continue;
                const int64_t base = (int64_t)s * dst_plane + (int64_t)p * dst_pitch;
                if constexpr (OUT_F32) {
                    const int y = y0 + 4 * lq;
                    float *o = static_cast<float *>(dst) + base + y;
                    if (vec_out && y + 3 < R_out) {
                        if constexpr (ACCUM)
                            w = __builtin_bit_cast(u32x4, *reinterpret_cast<const f32x4 *>(o) +
                                                              __builtin_bit_cast(f32x4, w));
                        *reinterpret_cast<u32x4 *>(o) = w;
                    } else {
#pragma unroll
                        for (int u = 0; u < 4; ++u)
                            if (y + u < R_out) o[u] = (ACCUM ? o[u] : 0.0f) + __uint_as_float(w[u]);
                    }
                } else {
                    if (k & 1) w = u32x4{w[2], w[3], w[0], w[1]};
                    const int y = y0 + 8 * (lq & 3);
                    uint16_t *o = (lq < 4 ? static_cast<uint16_t *>(dst) : dst_lo) + base + y;
                    if (y + 7 < R_out) {
                        *reinterpret_cast<u32x4 *>(o) = w;
                    } else {
#pragma unroll
                        for (int u = 0; u < 8; ++u)
                            if (y + u < R_out) o[u] = (uint16_t)(w[u / 2] >> (16 * (u % 2)));
                    }
                }
            }
        }
        return;
    }
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        const int p = p0 + 32 * t + i;
        if (p >= n) continue;
        const floatx16 &m = t ? m1 : m0;
        const floatx16 &l = t ? l1 : l0;
        const int64_t base = (int64_t)s * dst_plane + (int64_t)p * dst_pitch;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int y = y0 + 8 * q + 4 * g8;
            float v[4];
            value(m, l, q, v);
            if constexpr (OUT_F32) {
                float *o = static_cast<float *>(dst) + base + y;
                if (vec_out && y + 3 < R_out) {
                    f32x4 a = f32x4{v[0], v[1], v[2], v[3]};
                    if constexpr (ACCUM) a += *reinterpret_cast<const f32x4 *>(o);
                    *reinterpret_cast<f32x4 *>(o) = a;
                } else {
#pragma unroll
                    for (int u = 0; u < 4; ++u)
                        if (y + u < R_out) o[u] = (ACCUM ? o[u] : 0.0f) + v[u];
                }
            } else {
                uint16_t hi[4], lo[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) split<H>(v[u], hi[u], lo[u]);
                uint16_t *oh = static_cast<uint16_t *>(dst) + base + y;
                uint16_t *ol = dst_lo + base + y;
                if (y + 3 < R_out) {
                    *reinterpret_cast<u32x2 *>(oh) =
                        u32x2{(uint32_t)hi[0] | ((uint32_t)hi[1] << 16), (uint32_t)hi[2] | ((uint32_t)hi[3] << 16)};
                    *reinterpret_cast<u32x2 *>(ol) =
                        u32x2{(uint32_t)lo[0] | ((uint32_t)lo[1] << 16), (uint32_t)lo[2] | ((uint32_t)lo[3] << 16)};
                } else {
#pragma unroll
                    for (int u = 0; u < 4; ++u)
                        if (y + u < R_out) {
                            oh[u] = hi[u];
                            ol[u] = lo[u];
                        }
                }
            }
        }
    }
}

template <typename H, int SRC, bool OUT_F32, bool FAST, bool ACCUM = false>
hipError_t rows_pass(const void *src, const void *src_lo, int64_t src_pitch, int64_t src_plane, int64_t R,
                     int64_t n, int64_t n_in, void *dst, void *dst_lo, int64_t dst_pitch, int64_t dst_plane,
                     int64_t R_out, int boundary, bool vec_out, const u32x4 *tables, const HalfSet &hs, int kp_max,
                     hipStream_t st) {
    const unsigned nrt = (unsigned)((R_out + HT_ROWS * HT_WROW - 1) / (HT_ROWS * HT_WROW));
    const unsigned npg = (unsigned)((n + HT_POS * HT_WPOS - 1) / (HT_POS * HT_WPOS));
    // the table's direct copies write whole rounds of HT_WPB * 64 entries
    const int stage_off = ((2 * table_entries(kp_max) + HT_WPB * 64 - 1) / (HT_WPB * 64)) * (HT_WPB * 64);
    const int stage = FAST ? HT_WPB * (SRC == SRC_PAIR ? 512 : 256) : 0;   // 16-byte entries
    const size_t lds = sizeof(u32x4) * (size_t)(stage_off + stage);
    hipLaunchKernelGGL((fir_half_rows_kernel<H, SRC, OUT_F32, FAST, ACCUM>), dim3(nrt * npg * (unsigned)hs.nscales),
                       dim3(HT_WPB * 64), lds, st, static_cast<const uint16_t *>(src),
                       static_cast<const uint16_t *>(src_lo), src_pitch, src_plane, (int)R, (int)n, (int)n_in, dst,
                       static_cast<uint16_t *>(dst_lo), dst_pitch, dst_plane, (int)R_out, boundary, (int)vec_out,
                       tables, hs, stage_off);
    return hipGetLastError();
}

// intermediate planes: W rows (one per frame column) of Hp >= H samples,
// an odd number of 128-byte lines: every row starts on a line (the staged
// chunk loads and the output runs then cover whole lines, not two halves),
// and the rows one instruction touches spread over the memory channels
int64_t pair_pitch(int64_t H) { return 64 * (((H + 63) / 64) | 1); }

template <typename T, int SRC1>
hipError_t run_chunk(const void *in, int64_t H, int64_t W, int64_t in_pitch, bool vec_in, void *ws, float *out,
                     int64_t out_pitch, int64_t plane_stride, bool vec_out, const HalfTaps &ht,
                     const float *unscale, int boundary, hipStream_t st) {
    constexpr float mid = std::is_same_v<T, _Float16> ? 0.0625f : 1.0f;   // intermediate factor
    u32x4 *tables = static_cast<u32x4 *>(ws);
    const int64_t hp = pair_pitch(H);
    uint16_t *ph = reinterpret_cast<uint16_t *>(static_cast<char *>(ws) + HT_TABLE_BYTES);
    uint16_t *pl = ph + (int64_t)ht.nscales * W * hp;
    HalfSet hs{};
    hs.nscales = ht.nscales;
    int kp_max = 0;
    for (int q = 0; q < ht.nscales; ++q) {
        hs.K[q] = ht.K[q];
        hs.tab[q] = ht.tab[q];
        hs.post[q] = unscale[q] * mid;
        kp_max = round_kp(ht.K[q]) > kp_max ? round_kp(ht.K[q]) : kp_max;
    }
    hipLaunchKernelGGL(fir_half_tables_kernel<T>, dim3(ht.nscales), dim3(256), 0, st, tables, ht);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // first pass: the frame's H rows of W samples -> W x hp pair planes, rows
    // H .. hp - 1 holding the extension; the 16-byte form needs aligned rows
    // of a multiple of 8 samples
    if (vec_in && W % 8 == 0)
        e = rows_pass<T, SRC1, false, true>(in, nullptr, in_pitch, 0, H, W, W, ph, pl, hp, W * hp, hp, boundary,
                                            true, tables, hs, kp_max, st);
    else
        e = rows_pass<T, SRC1, false, false>(in, nullptr, in_pitch, 0, H, W, W, ph, pl, hp, W * hp, hp, boundary,
                                             true, tables, hs, kp_max, st);
    if (e != hipSuccess) return e;
    // second pass: W rows of hp samples (H outputs each) -> the H x W planes
    for (int q = 0; q < ht.nscales; ++q) hs.post[q] = unscale[q] / mid;
    return rows_pass<T, SRC_PAIR, true, true>(ph, pl, hp, W * hp, W, H, hp, out, nullptr, out_pitch, plane_stride,
                                              W, boundary, vec_out, tables, hs, kp_max, st);
}


// ---------------------------------------------------------------- detection
// response on the matrix cores.  With d = h * [1, -2, 1] (Table I, d = 2),
// sigma^2 (D20 + D02) of the separable blur is sigma^2 (h_y (d_x x) +
// d_y (h_x x)): pass 1 filters the rows with h and with d (two tap sets per
// scale, both of half-length K + 1), pass 2 filters the columns of the
// h-plane with d and then, accumulating, those of the d-plane with h.  No
// blur is formed, so none is rounded before the differences.  The
// difference taps sum to zero and are small (about 1 / sigma^2 of h): the
// d-plane is stored times 2^(e_h - e_d) (the exponents of the two tap sets'
// largest magnitudes), so that it spans the h-plane's range and both pass-2
// products carry the same factor.  The second differences of the oracle
// clamp the blur at the image edge, where these filters see the extension:
// the first and last rows and columns are corrected afterwards in float64
// (lap_rows_fix_kernel, lap_edge_sums_kernel, lap_cols_fix_kernel).

constexpr int LAP_MAX = FDVM_MAX_SCALES / 2;   // scales per launch (two tap sets each)
constexpr int LAP_TAPS = HT_ARG_TAPS;   // the edge kernels' copy of h(0..K), all scales of a launch

struct LapFix {   // the blur taps h(0..K) of a launch's scales, float32, and sigma^2
    int q;
    int K[LAP_MAX];
    int off[LAP_MAX];
    float sig2[LAP_MAX];
    float h[LAP_TAPS];
};

__device__ __forceinline__ float tap_of(const LapFix &f, int s, int m) {
    const int a = m < 0 ? -m : m;
    return a <= f.K[s] ? f.h[f.off[s] + a] : 0.0f;
}

// The edge terms.  With B = h * P_ext (P extended by the boundary rule), the
// clamped difference at the first sample wants B(0) where the filters used
// B(-1): B(0) - B(-1) = sum_m h(m) [P_ext(-m) - P_ext(-1 - m)], whose terms
// with both indices outside vanish, leaving
//     e_first = [zero extension] h(0) P(0) + sum_{j=1..K} h(j) (P_ext(j) - P_ext(j - 1)),
// and the mirror image at the last sample.  One wavefront per line, lanes
// striding along it (coalesced), a butterfly sum at the end.
__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// e_first and e_last of one line of n samples, get(j) the sample j in [0, n)
template <typename G>
__device__ __forceinline__ void edge_terms(const LapFix &f, int s, int n, bool rep, G get, double &first,
                                           double &last) {
    const int K = f.K[s];
    const int lane = threadIdx.x & 63;
    const double p0 = get(0), pn = get(n - 1);
    auto ext = [&](int j, double inside_edge) { return j < n ? get(j) : (rep ? inside_edge : 0.0); };
    double a = 0.0, b = 0.0;
    for (int j = 1 + lane; j <= K; j += 64) {
        const double h = f.h[f.off[s] + j];
        a += h * (ext(j, pn) - ext(j - 1, pn));
        // mirror: P_ext(n - 1 - j) - P_ext(n - j), indices below 0 extended by P(0)
        const int i1 = n - 1 - j, i0 = n - j;
        const double v1 = i1 >= 0 ? get(i1) : (rep ? p0 : 0.0);
        const double v0 = i0 >= 0 ? get(i0) : (rep ? p0 : 0.0);
        b += h * (v1 - v0);
    }
    first = wave_sum_d(a);
    last = wave_sum_d(b);
    if (!rep) {
        first += (double)f.h[f.off[s]] * p0;
        last += (double)f.h[f.off[s]] * pn;
    }
}

// the D02 term at the first and last rows: e from the h-plane of pass 1
// (row x, samples along y), V(0, x) += sigma^2 e_first, V(H - 1, x) += sigma^2 e_last
template <typename T>
__global__ __launch_bounds__(256) void lap_rows_fix_kernel(const uint16_t *__restrict__ ph,
                                                           const uint16_t *__restrict__ pl, int64_t hp, int W, int H,
                                                           int boundary, float inv_mid, LapFix f, float *out,
                                                           int64_t out_pitch, int64_t plane_stride) {
    const int x = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int s = blockIdx.y;
    if (x >= W) return;
    const int64_t row = ((int64_t)(2 * s) * W + x) * hp;   // the h-plane of scale s
    auto get = [&](int j) -> double {
        return ((double)Op<T>::value(ph[row + j]) + (double)Op<T>::value(pl[row + j]) / Op<T>::lo_scale) *
               inv_mid;
    };
    double first, last;
    edge_terms(f, s, H, boundary == FDVM_BC_REPLICATE, get, first, last);
    if ((threadIdx.x & 63) != 0) return;
    float *o = out + (int64_t)s * plane_stride + x;
    const double sg = f.sig2[s];
    if (H == 1) {
        o[0] += (float)(sg * (first + last));
    } else {
        o[0] += (float)(sg * first);
        o[(int64_t)(H - 1) * out_pitch] += (float)(sg * last);
    }
}

template <typename TIn>
__device__ __forceinline__ double sample_at(const TIn *p) {
    if constexpr (std::is_same_v<TIn, uint16_t>)
        return (double)*p;
    else
        return (double)Op<TIn>::value(*reinterpret_cast<const uint16_t *>(p));
}

// the D20 term's row values: e_first and e_last of every frame row (the row
// filter's value at the edge column minus one column outside), per scale
template <typename TIn>
__global__ __launch_bounds__(256) void lap_edge_sums_kernel(const TIn *__restrict__ in, int64_t in_pitch, int W,
                                                            int H, int boundary, LapFix f, double *__restrict__ c) {
    const int y = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int s = blockIdx.y;
    if (y >= H) return;
    const TIn *r = in + (int64_t)y * in_pitch;
    double first, last;
    edge_terms(f, s, W, boundary == FDVM_BC_REPLICATE, [&](int j) { return sample_at<TIn>(r + j); }, first, last);
    if ((threadIdx.x & 63) != 0) return;
    c[((int64_t)s * 2) * H + y] = first;
    c[((int64_t)s * 2 + 1) * H + y] = last;
}

// V(y, 0) += sigma^2 (h_y * c_first)(y), V(y, W - 1) += sigma^2 (h_y * c_last)(y),
// c extended along y by the boundary rule; each block filters 256 rows from
// a window of both columns staged in LDS
constexpr int LAP_FIX_ROWS = 256;
__global__ __launch_bounds__(LAP_FIX_ROWS) void lap_cols_fix_kernel(const double *__restrict__ c, int W, int H,
                                                                    int boundary, LapFix f, float *out,
                                                                    int64_t out_pitch, int64_t plane_stride) {
    __shared__ double win[2][LAP_FIX_ROWS + 2 * FDVM_MAX_FIR_LAP_MFMA_HALF];
    const int s = blockIdx.y;
    const int y0 = blockIdx.x * LAP_FIX_ROWS;
    const int K = f.K[s];
    const bool rep = boundary == FDVM_BC_REPLICATE;
    const double *cl = c + ((int64_t)s * 2) * H;
    const double *cr = cl + H;
    for (int i = threadIdx.x; i < LAP_FIX_ROWS + 2 * K; i += LAP_FIX_ROWS) {
        int j = y0 - K + i;
        const bool in = j >= 0 && j < H;
        j = min(max(j, 0), H - 1);
        win[0][i] = (in || rep) ? cl[j] : 0.0;
        win[1][i] = (in || rep) ? cr[j] : 0.0;
    }
    __syncthreads();
    const int y = y0 + threadIdx.x;
    if (y >= H) return;
    double lft = 0.0, rgt = 0.0;
    for (int m = -K; m <= K; ++m) {
        const double h = f.h[f.off[s] + (m < 0 ? -m : m)];
        lft += h * win[0][threadIdx.x + K - m];
        rgt += h * win[1][threadIdx.x + K - m];
    }
    float *o = out + (int64_t)s * plane_stride + (int64_t)y * out_pitch;
    const double sg = f.sig2[s];
    if (W == 1) {
        o[0] += (float)(sg * (lft + rgt));
    } else {
        o[0] += (float)(sg * lft);
        o[W - 1] += (float)(sg * rgt);
    }
}

// one launch's scales: tap set 2 s is h_s, 2 s + 1 is d_s (half-length K_s + 1
// both); their tables are built by one or more builder launches (each within
// the builder's argument table)
struct LapPlan {
    int q;
    int K[2 * LAP_MAX];
    int tab[2 * LAP_MAX];
    float unscale[2 * LAP_MAX];
    int nbatch;
    HalfTaps batch[2 * LAP_MAX];
};

template <typename T, int SRC1, typename TIn>
hipError_t run_lap_chunk(const void *in, int64_t H, int64_t W, int64_t in_pitch, bool vec_in, void *ws, float *out,
                         int64_t out_pitch, int64_t plane_stride, bool vec_out, const LapPlan &pl_,
                         const LapFix &fx, int boundary, hipStream_t st) {
    constexpr float mid = std::is_same_v<T, _Float16> ? 0.0625f : 1.0f;
    const int q = fx.q;
    u32x4 *tables = static_cast<u32x4 *>(ws);
    const int64_t hp = pair_pitch(H);
    uint16_t *ph = reinterpret_cast<uint16_t *>(static_cast<char *>(ws) + HT_TABLE_BYTES);
    uint16_t *pl = ph + (int64_t)2 * q * W * hp;
    double *cb = reinterpret_cast<double *>(pl + (int64_t)2 * q * W * hp);
    int kp_max = 0;
    for (int e = 0; e < 2 * q; ++e) kp_max = std::max(kp_max, round_kp(pl_.K[e]));
    hipError_t e = hipSuccess;
    for (int b = 0; b < pl_.nbatch; ++b) {
        hipLaunchKernelGGL(fir_half_tables_kernel<T>, dim3(pl_.batch[b].nscales), dim3(256), 0, st, tables,
                           pl_.batch[b]);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    // pass 1: both tap sets, each plane in the h set's units (the d set is
    // scaled by 2^-e_d in its table, so 2^e_h leaves the d-plane times
    // 2^(e_h - e_d))
    HalfSet h1{};
    h1.nscales = 2 * q;
    for (int j = 0; j < 2 * q; ++j) {
        h1.K[j] = pl_.K[j];
        h1.tab[j] = pl_.tab[j];
        h1.post[j] = pl_.unscale[2 * (j / 2)] * mid;
    }
    if (vec_in && W % 8 == 0)
        e = rows_pass<T, SRC1, false, true>(in, nullptr, in_pitch, 0, H, W, W, ph, pl, hp, W * hp, hp, boundary, true,
                                            tables, h1, kp_max, st);
    else
        e = rows_pass<T, SRC1, false, false>(in, nullptr, in_pitch, 0, H, W, W, ph, pl, hp, W * hp, hp, boundary,
                                             true, tables, h1, kp_max, st);
    if (e != hipSuccess) return e;
    // pass 2: the h-planes' columns with d, then the d-planes' columns with h,
    // both products scaled by sigma^2 2^e_d / mid
    HalfSet h2{};
    h2.nscales = q;
    for (int j = 0; j < q; ++j) {
        h2.K[j] = pl_.K[2 * j + 1];
        h2.tab[j] = pl_.tab[2 * j + 1];
        h2.post[j] = fx.sig2[j] * pl_.unscale[2 * j + 1] / mid;
    }
    const int64_t pstride = 2 * W * hp;   // every other plane
    e = rows_pass<T, SRC_PAIR, true, true, false>(ph, pl, hp, pstride, W, H, hp, out, nullptr, out_pitch,
                                                 plane_stride, W, boundary, vec_out, tables, h2, kp_max, st);
    if (e != hipSuccess) return e;
    for (int j = 0; j < q; ++j) {
        h2.K[j] = pl_.K[2 * j];
        h2.tab[j] = pl_.tab[2 * j];
    }
    e = rows_pass<T, SRC_PAIR, true, true, true>(ph + W * hp, pl + W * hp, hp, pstride, W, H, hp, out, nullptr,
                                                out_pitch, plane_stride, W, boundary, vec_out, tables, h2, kp_max,
                                                st);
    if (e != hipSuccess) return e;
    // the edge rows and columns, in float64
    hipLaunchKernelGGL(lap_rows_fix_kernel<T>, dim3((unsigned)((W + 3) / 4), (unsigned)q), dim3(256), 0, st, ph,
                       pl, hp, (int)W, (int)H, boundary, 1.0f / mid, fx, out, out_pitch, plane_stride);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(lap_edge_sums_kernel<TIn>, dim3((unsigned)((H + 3) / 4), (unsigned)q), dim3(256), 0, st,
                       static_cast<const TIn *>(in), in_pitch, (int)W, (int)H, boundary, fx, cb);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(lap_cols_fix_kernel, dim3((unsigned)((H + LAP_FIX_ROWS - 1) / LAP_FIX_ROWS), (unsigned)q),
                       dim3(LAP_FIX_ROWS), 0, st, cb,
                       (int)W, (int)H, boundary, fx, out, out_pitch, plane_stride);
    return hipGetLastError();
}

}  // namespace

size_t fir_mfma_half_workspace_bytes(int64_t H, int64_t W, int nscales) {
    return HT_TABLE_BYTES + (size_t)nscales * (size_t)W * (size_t)pair_pitch(H) * 4;
}

hipError_t launch_fir_mfma_half(const void *in, int dtype, int64_t H, int64_t W, int64_t in_pitch, void *ws,
                                float *out, int64_t out_pitch, int64_t plane_stride, const double *taps,
                                const int32_t *half_len, const int32_t *tap_offset, int nscales, int boundary,
                                hipStream_t st) {
    if (dtype != FDVM_F16 && dtype != FDVM_BF16 && dtype != FDVM_U16) return hipErrorInvalidValue;
    const bool vec_in = (reinterpret_cast<uintptr_t>(in) % 16 == 0) && ((in_pitch * 2) % 16 == 0);
    for (int s0 = 0; s0 < nscales;) {
        // the longest run of scales whose taps fit in the builder's arguments
        HalfTaps ht{};
        float unscale[FDVM_MAX_SCALES];
        int pos = 0, tab = 0, q = 0;
        while (s0 + q < nscales && pos + half_len[s0 + q] + 1 <= HT_ARG_TAPS) {
            const int K = half_len[s0 + q];
            const double *hd = taps + tap_offset[s0 + q];
            double hmax = 0.0;
            for (int m = 0; m <= K; ++m) hmax = std::fmax(hmax, std::fabs(hd[K + m]));
            int ex = 0;
            if (hmax > 0.0) std::frexp(hmax, &ex);   // hmax = f 2^ex, f in [0.5, 1)
            unscale[q] = std::ldexp(1.0f, ex);
            ht.K[q] = K;
            ht.off[q] = pos;
            ht.tab[q] = tab;
            for (int m = 0; m <= K; ++m) ht.h[pos + m] = (float)std::ldexp(hd[K + m], -ex);
            pos += K + 1;
            tab += 2 * table_entries(round_kp(K));
            ++q;
        }
        if (q == 0) return hipErrorInvalidValue;   // a half-length beyond the argument table
        ht.nscales = q;
        float *o = out + (int64_t)s0 * plane_stride;
        const bool vec_out = (reinterpret_cast<uintptr_t>(o) % 16 == 0) && (out_pitch % 4 == 0) &&
                             (plane_stride % 4 == 0);
        hipError_t e;
        if (dtype == FDVM_F16)
            e = run_chunk<_Float16, SRC_HALF>(in, H, W, in_pitch, vec_in, ws, o, out_pitch, plane_stride, vec_out,
                                              ht, unscale, boundary, st);
        else if (dtype == FDVM_U16)
            e = run_chunk<_Float16, SRC_U16>(in, H, W, in_pitch, vec_in, ws, o, out_pitch, plane_stride, vec_out,
                                             ht, unscale, boundary, st);
        else
            e = run_chunk<__bf16, SRC_HALF>(in, H, W, in_pitch, vec_in, ws, o, out_pitch, plane_stride, vec_out,
                                            ht, unscale, boundary, st);
        if (e != hipSuccess) return e;
        s0 += q;
    }
    return hipSuccess;
}


size_t fir_laplacian_mfma_workspace_bytes(int64_t H, int64_t W, int nscales) {
    const int q = std::min(nscales, LAP_MAX);
    return HT_TABLE_BYTES + (size_t)2 * q * (size_t)W * (size_t)pair_pitch(H) * 4 +
           (size_t)2 * q * (size_t)H * sizeof(double);
}

hipError_t launch_fir_laplacian_mfma(const void *in, int dtype, int64_t H, int64_t W, int64_t in_pitch, void *ws,
                                     float *out, int64_t out_pitch, int64_t plane_stride, const double *taps,
                                     const int32_t *half_len, const int32_t *tap_offset, const double *sigmas,
                                     int nscales, int boundary, hipStream_t st) {
    if (dtype != FDVM_F16 && dtype != FDVM_BF16 && dtype != FDVM_U16) return hipErrorInvalidValue;
    const bool vec_in = (reinterpret_cast<uintptr_t>(in) % 16 == 0) && ((in_pitch * 2) % 16 == 0);
    for (int s0 = 0; s0 < nscales;) {
        // up to LAP_MAX scales per launch; their tap sets go to the table
        // builder in batches that fit its argument table
        static thread_local LapPlan plan;   // about 60 KB: not on the stack
        plan = LapPlan{};
        LapFix fx{};
        int fpos = 0, tab = 0, q = 0;
        HalfTaps *cur = &plan.batch[0];
        plan.nbatch = 1;
        int pos = 0;
        while (s0 + q < nscales && q < LAP_MAX && fpos + half_len[s0 + q] + 1 <= LAP_TAPS) {
            const int K = half_len[s0 + q];
            const double *hd = taps + tap_offset[s0 + q] + K;   // h(m) = hd[m], |m| <= K
            auto hv = [&](int m) { return (m < -K || m > K) ? 0.0 : hd[m]; };
            double hm = 0.0, dm = 0.0;
            for (int m = 0; m <= K + 1; ++m) {
                hm = std::fmax(hm, std::fabs(hv(m)));
                dm = std::fmax(dm, std::fabs(hv(m - 1) - 2.0 * hv(m) + hv(m + 1)));
            }
            int eh = 0, ed = 0;
            if (hm > 0.0) std::frexp(hm, &eh);
            if (dm > 0.0) std::frexp(dm, &ed);
            for (int t = 0; t < 2; ++t) {   // tap set 2 q: h (padded to K + 1), 2 q + 1: d
                const int ent = 2 * q + t;
                const int ex = t ? ed : eh;
                if (pos + K + 2 > HT_ARG_TAPS) {   // the next builder batch
                    cur = &plan.batch[plan.nbatch++];
                    pos = 0;
                }
                const int bi = cur->nscales++;
                plan.unscale[ent] = std::ldexp(1.0f, ex);
                plan.K[ent] = K + 1;
                plan.tab[ent] = tab;
                cur->K[bi] = K + 1;
                cur->off[bi] = pos;
                cur->tab[bi] = tab;
                for (int m = 0; m <= K + 1; ++m) {
                    const double v = t ? hv(m - 1) - 2.0 * hv(m) + hv(m + 1) : hv(m);
                    cur->h[pos + m] = (float)std::ldexp(v, -ex);
                }
                pos += K + 2;
                tab += 2 * table_entries(round_kp(K + 1));
            }
            fx.K[q] = K;
            fx.off[q] = fpos;
            fx.sig2[q] = (float)(sigmas[s0 + q] * sigmas[s0 + q]);
            for (int m = 0; m <= K; ++m) fx.h[fpos + m] = (float)hd[m];
            fpos += K + 1;
            ++q;
        }
        if (q == 0) return hipErrorInvalidValue;
        plan.q = q;
        fx.q = q;
        float *o = out + (int64_t)s0 * plane_stride;
        const bool vec_out = (reinterpret_cast<uintptr_t>(o) % 16 == 0) && (out_pitch % 4 == 0) &&
                             (plane_stride % 4 == 0);
        hipError_t e;
        if (dtype == FDVM_F16)
            e = run_lap_chunk<_Float16, SRC_HALF, _Float16>(in, H, W, in_pitch, vec_in, ws, o, out_pitch,
                                                            plane_stride, vec_out, plan, fx, boundary, st);
        else if (dtype == FDVM_U16)
            e = run_lap_chunk<_Float16, SRC_U16, uint16_t>(in, H, W, in_pitch, vec_in, ws, o, out_pitch,
                                                           plane_stride, vec_out, plan, fx, boundary, st);
        else
            e = run_lap_chunk<__bf16, SRC_HALF, __bf16>(in, H, W, in_pitch, vec_in, ws, o, out_pitch, plane_stride,
                                                        vec_out, plan, fx, boundary, st);
        if (e != hipSuccess) return e;
        s0 += q;
    }
    return hipSuccess;
}

}  // namespace fdvm
