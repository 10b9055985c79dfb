// Column pass (y) of the repeated-pole IIR blur, lane = column (coalesced
// along the row), optionally finished as the scale-normalised Laplacian or the
// Hessian detector.  Realisation and intermediate formats: fdvm_iir_common.h.
//
// Tiles of CT rows, grouped COL_WPB at a time into super tiles:
//   states  -- every tile's zero-state end states (forward and backward),
//              combined within its super tile into the states entering each
//              tile from the super tile's top and bottom edges (zero there),
//              and into the super tile's own zero-state end states;
//   scan    -- per column, the super tiles' states are chained into the true
//              carries that enter every super tile (forward from the top,
//              backward from the bottom);
//   final   -- every tile independently: its true carries are the super
//              tile's carries moved across the rows between them plus the
//              tile's in-super-tile states; backward sweep from its bottom
//              carry, forward sweep from its top carry, output.  Optionally the
//              scale-normalised Laplacian sigma^2 (D20 + D02) is formed here in
//              float64 from the unrounded blur: y-neighbours come from the
//              sweep itself (the rows just outside the tile are recovered by
//              inverting one step of the recursion), x-neighbours from the
//              adjacent lanes (tiles overlap by one column on each side).
#include "fdvm_iir_common.h"

namespace fdvm {
namespace {

// (a) zero-state end states of every CT-row tile (float64), one wavefront per
//     tile, the COL_WPB tiles of a super tile in one work-group.  Writes, per
//     tile, the forward state entering it from the top of its super tile and
//     the backward state entering it from the bottom (both zero at those
//     edges): lt[((s * nty + ty) * 2K + k) * W + x], k < K forward, k >= K
//     backward; and per super tile its zero-state end states, laid out the
//     same way in sst with nsy super tiles.
template <int K, bool FX>
__global__ __launch_bounds__(COL_WPB * 64) void iir_col_states_kernel(Mid<FX> m, int H, int W, int nty, int nsy,
                                                                      double *__restrict__ lt,
                                                                      double *__restrict__ sst, Args a) {
    constexpr int NS = cascade_states(K);
    __shared__ double zx[COL_WPB][2 * NS][64];
    const int lane = threadIdx.x & 63;
    const int wv = wave_id();
    const int sy = blockIdx.y;
    const int ty = sy * COL_WPB + wv;
    const int s = blockIdx.z;
    const int col = blockIdx.x * 64 + lane;
    const int ccol = min(col, W - 1);
    const ScaleArgs &cf = a.s[s];
    const int y0 = ty * CT;
    static_assert(CT <= 64, "one row scale per lane");
    auto tile_len = [&](int t) { return max(0, min(CT, H - t * CT)); };
    double zf[NS], zb[NS];
    set_zero(zf);
    set_zero(zb);
    if (ty < nty) {   // tiles past the last row contribute zero states over zero rows
        const double lsc = m.row_scale(min(y0 + lane, H - 1));  // lane j: scale of row y0 + j
        uint32_t xs[CT];
#pragma unroll
        for (int j = 0; j < CT; ++j) {
            const int y = y0 + j;
            const uint32_t v = m.raw(s, min(y, H - 1), ccol);
            xs[j] = y < H ? v : 0u;  // zeros (in either format) after the last row
        }                            // leave the backward zero state exact
#pragma unroll
        for (int j = 0; j < CT; ++j) cas_step<K>(cf, zf, m.cvt(xs[j], read_lane_d(lsc, j)));
#pragma unroll
        for (int j = CT - 1; j >= 0; --j) cas_step<K>(cf, zb, m.cvt(xs[j], read_lane_d(lsc, j)));
    }
#pragma unroll
    for (int k = 0; k < NS; ++k) {
        zx[wv][k][lane] = zf[k];
        zx[wv][NS + k][lane] = zb[k];
    }
    __syncthreads();
    if (col >= W) return;
    auto zget = [&](int t, int k0, double (&z)[NS]) {
#pragma unroll
        for (int k = 0; k < NS; ++k) z[k] = zx[t][k0 + k][lane];
    };
    if (ty < nty) {
        // forward: over the tiles above this one (all CT rows long); backward:
        // over the tiles below it, from the super tile's bottom edge
        double lf[NS], lb[NS], z[NS];
        set_zero(lf);
        set_zero(lb);
        const Tr tfull = tr_n<K>(cf, CT);
        for (int t = 0; t < wv; ++t) {
            zget(t, 0, z);
            cas_advance_add<K>(tfull, lf, z);
        }
        for (int t = COL_WPB - 1; t > wv; --t) {
            zget(t, NS, z);
            cas_advance_add<K>(tr_n<K>(cf, tile_len(sy * COL_WPB + t)), lb, z);
        }
        // the first tile's forward state and the last tile's backward state
        // are zero by definition: not stored (nor read by the final pass)
        double *o = lt + ((int64_t)(s * nty + ty) * 2 * NS) * W + col;
#pragma unroll
        for (int k = 0; k < NS; ++k) {
            if (wv > 0) o[(int64_t)k * W] = lf[k];
            if (wv < COL_WPB - 1) o[(int64_t)(NS + k) * W] = lb[k];
        }
    }
    if (wv == 0) {
        double sf[NS], sb[NS], z[NS];
        set_zero(sf);
        set_zero(sb);
        for (int t = 0; t < COL_WPB; ++t) {
            zget(t, 0, z);
            cas_advance_add<K>(tr_n<K>(cf, tile_len(sy * COL_WPB + t)), sf, z);
        }
        for (int t = COL_WPB - 1; t >= 0; --t) {
            zget(t, NS, z);
            cas_advance_add<K>(tr_n<K>(cf, tile_len(sy * COL_WPB + t)), sb, z);
        }
        double *o = sst + ((int64_t)(s * nsy + sy) * 2 * NS) * W + col;
#pragma unroll
        for (int k = 0; k < NS; ++k) {
            o[(int64_t)k * W] = sf[k];
            o[(int64_t)(NS + k) * W] = sb[k];
        }
    }
}

// (b) carries: in place, every super tile's forward zero state becomes the
// forward state entering it from above, every backward zero state the
// backward state entering it from below.
constexpr int SCAN_T = 64;        // threads (columns) per scan work-group
constexpr int SCT = CT * COL_WPB;  // rows per super tile (transitions over up to 255 rows)
static_assert(SCT < 256, "super-tile transitions from the eight binary powers");

template <int K, bool FX>
__global__ __launch_bounds__(SCAN_T) void iir_col_scan_kernel(Mid<FX> m, int H, int W, int nty,
                                                              double *__restrict__ st, Args a) {
    // nty: super tiles of SCT rows
    constexpr int NS = cascade_states(K);
    constexpr int U = 8;  // tiles whose states are fetched together
    const int col = blockIdx.x * SCAN_T + threadIdx.x;
    const int s = blockIdx.y;
    const int dir = blockIdx.z;  // 0: forward from the top, 1: backward from the bottom
    if (col >= W) return;
    const ScaleArgs &cf = a.s[s];
    const bool rep = a.boundary == FDVM_BC_REPLICATE;
    const double xe = m.at(s, dir == 0 ? 0 : H - 1, col);
    double *base = st + (int64_t)s * nty * 2 * NS * W + (int64_t)dir * NS * W + col;
    const int64_t tstride = (int64_t)2 * NS * W;
    double c[NS];
#pragma unroll
    for (int k = 0; k < NS; ++k) c[k] = rep ? xe * cf.ss[k] : 0.0;
    const Tr tt = tr_n<K>(cf, SCT);
    for (int i0 = 0; i0 < nty; i0 += U) {
        double z[U][NS];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = i0 + u;
            const int ty = dir == 0 ? i : nty - 1 - i;
#pragma unroll
            for (int k = 0; k < NS; ++k) z[u][k] = i < nty ? base[ty * tstride + (int64_t)k * W] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = i0 + u;
            if (i >= nty) break;
            const int ty = dir == 0 ? i : nty - 1 - i;
#pragma unroll
            for (int k = 0; k < NS; ++k) base[ty * tstride + (int64_t)k * W] = c[k];
            const int len = min(SCT, H - ty * SCT);
            cas_advance_add<K>(len == CT ? tt : tr_n<K>(cf, len), c, z[u]);
        }
    }
}

// value of lane l-1 (left) / l+1 (right) of a double across the whole
// wavefront (gfx9 DPP wave_shr:1 / wave_shl:1 on both halves); the end lanes
// read 0, which only reaches their own results (lanes 0 and 63 of a
// Laplacian tile are overlap columns that are never written)
__device__ __forceinline__ double lane_left_d(double v) {
    const int lo = __double2loint(v), hi = __double2hiint(v);
    return __hiloint2double(__builtin_amdgcn_mov_dpp(hi, 0x138, 0xf, 0xf, true),
                            __builtin_amdgcn_mov_dpp(lo, 0x138, 0xf, 0xf, true));
}
__device__ __forceinline__ double lane_right_d(double v) {
    const int lo = __double2loint(v), hi = __double2hiint(v);
    return __hiloint2double(__builtin_amdgcn_mov_dpp(hi, 0x130, 0xf, 0xf, true),
                            __builtin_amdgcn_mov_dpp(lo, 0x130, 0xf, 0xf, true));
}

// Hardware work-group ids are dealt round-robin to the 8 XCDs (each with its
// own L2).  Map them so that every XCD gets one contiguous run of logical
// tiles: neighbouring column tiles (which share the cache lines at their
// edges, both read and written) then meet in the same L2.
__device__ __forceinline__ int xcd_logical_block(int hw, int n) {
    constexpr int NX = 8;
    const int xcd = hw % NX, slot = hw / NX;
    const int q = n / NX, r = n % NX;
    return xcd * q + min(xcd, r) + slot;
}

// copy one row of 64 lanes x 4 bytes from global memory straight into LDS
// (no register round trip); the data is there after "s_waitcnt vmcnt(0)"
__device__ __forceinline__ void row_to_lds(const void *g, uint32_t *l) {
    __builtin_amdgcn_global_load_lds(g, (__attribute__((address_space(3))) void *)l, 4, 0, 0);
}
__device__ __forceinline__ void wait_lds_dma() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

// (c) final pass of one CT-row tile per wavefront.  LAP = false: writes the
// blur; in place is allowed (a tile reads and writes only its own rows, and it
// stages all of them before its first write).  LAP = true: writes
// sigma^2 (D20 + D02) of the blur; lanes cover columns x0 - 1 .. x0 + 62 and
// lanes 1..62 write (in and out must not overlap).
// The tile (plus the rows just above and below it for LAP) is first copied
// into LDS with direct global-to-LDS loads, so the whole tile is in flight at
// once and no registers hold it.  It is then finished in bands of 16 rows
// (QT) so that only 16 float64 partial outputs are live: one backward sweep
// over all bands but the first records the state entering each band from
// below; then every band, top first, is swept backwards from its recorded
// state and finished by the forward sweep, which runs through the whole tile.
constexpr int FIN_WPB = 1;  // wavefronts (tiles) per final-pass work-group (1: measured faster than 2 or 4)
constexpr int FIN_BLUR = 0, FIN_LAPLACIAN = 1, FIN_HESSIAN = 2;

template <int K, int MODE, bool FX>
__global__ __launch_bounds__(FIN_WPB * 64) void iir_col_final_kernel(
    Mid<FX> m, float *out, int64_t out_pitch, int64_t out_plane_stride, int H, int W, int nty, int ntx,
    const double *__restrict__ st, const double *__restrict__ sst, int nsy, Args a, HessArgs hz) {
    constexpr int NS = cascade_states(K);
    constexpr bool LAP = MODE != FIN_BLUR;   // second differences need the neighbour rows and columns
    constexpr int QT = 16;
    constexpr int NQ = CT / QT;
    constexpr int NR = LAP ? CT + 2 : CT;   // staged rows: (y0 - 1 if LAP) .. y0 + CT - 1 (.. y0 + CT if LAP)
    constexpr int R0 = LAP ? 1 : 0;         // LDS row of tile row 0
    __shared__ uint32_t tiles[FIN_WPB][NR * 64];
    const int lane = threadIdx.x & 63;
    const int wv = wave_id();
    // logical block -> (column tile, group of FIN_WPB row tiles, scale), column tile fastest
    const int ntyg = (nty + FIN_WPB - 1) / FIN_WPB;
    const int lb = xcd_logical_block(blockIdx.x, ntx * ntyg * a.nscales);
    const int tx = lb % ntx;
    const int s = lb / (ntx * ntyg);
    const int ty = ((lb / ntx) % ntyg) * FIN_WPB + wv;
    const int col = LAP ? tx * 62 - 1 + lane : tx * 64 + lane;
    if (ty >= nty) return;
    const int ccol = min(max(col, 0), W - 1);
    const ScaleArgs &cf = a.s[s];
    const int y0 = ty * CT;
    const int y1 = min(y0 + CT, H);
    const int len = y1 - y0;
    uint32_t *lt = tiles[wv];
    // rows outside the image are clamped copies; they are never used as data
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        const int y = min(max(y0 - R0 + r, 0), H - 1);
        row_to_lds(m.ptr(s, y, ccol), lt + r * 64);
    }
    const double lsc = m.row_scale(min(y0 + lane, H - 1));  // lane j: scale of row y0 + j
    double vf[NS], ub[NQ][NS];
    {
        // the super tile's carries moved to this tile's edges (A^n over the
        // zero-input rows between them), plus the tile's states within the
        // super tile
        const int sy = ty / COL_WPB, w = ty % COL_WPB;   // wave-uniform
        const double *c = sst + ((int64_t)(s * nsy + sy) * 2 * NS) * W + ccol;
        const double *o = st + ((int64_t)(s * nty + ty) * 2 * NS) * W + ccol;
        double lf[NS], lb[NS];
        set_zero(lf);   // the first tile's forward and the last tile's backward
        set_zero(lb);   // states are zero (not stored)
#pragma unroll
        for (int k = 0; k < NS; ++k) {
            vf[k] = c[(int64_t)k * W];
            ub[NQ - 1][k] = c[(int64_t)(NS + k) * W];
        }
        if (w > 0) {
#pragma unroll
            for (int k = 0; k < NS; ++k) lf[k] = o[(int64_t)k * W];
        }
        if (w < COL_WPB - 1) {
#pragma unroll
            for (int k = 0; k < NS; ++k) lb[k] = o[(int64_t)(NS + k) * W];
        }
        cas_advance_add<K>(tr_n<K>(cf, y0 - sy * SCT), vf, lf);
        cas_advance_add<K>(tr_n<K>(cf, max(0, min(H, (sy + 1) * SCT) - y1)), ub[NQ - 1], lb);
    }
    double sc_above = 1.0, sc_below = 1.0;
    if constexpr (LAP && FX) {
        sc_above = m.row_scale(max(y0 - 1, 0));
        sc_below = m.row_scale(min(y1, H - 1));
    }
    wait_lds_dma();
    // sample of tile row j (j = -1 and j = len only with LAP)
    auto X = [&](int j) { return m.cvt(lt[(j + R0) * 64 + lane], read_lane_d(lsc, j)); };
    float *dst = out + (int64_t)s * out_plane_stride;
    const double sig2 = cf.sig2;
    const bool wr = LAP ? (lane >= 1 && lane <= 62 && col < W) : col < W;
    // y- of row y1 (below the tile) for the Laplacian's last row
    double t_bot = 0.0;
    if (LAP && y1 < H) {
        const double xb = m.cvt(lt[(len + R0) * 64 + lane], sc_below);
        double u[NS];
#pragma unroll
        for (int k = 0; k < NS; ++k) u[k] = ub[NQ - 1][k];
        cas_unstep<K>(cf, u, xb);  // state before row y1 (from below)
        t_bot = fma(cf.b0, xb, cas_out<K>(cf, u));
    }

    auto body = [&](auto full_tag) {
        constexpr bool FULL = decltype(full_tag)::value;
        auto valid = [&](int j) { return FULL || j < len; };
        double xd[QT];              // the samples of one quarter
        double t[QT];               // y-(n) + b0 x(n) of one quarter
        double bm = 0.0, bc = 0.0;  // sliding B(n-1), B(n) for the Laplacian
        auto load_q = [&](int q) {
#pragma unroll
            for (int i = 0; i < QT; ++i) xd[i] = valid(q * QT + i) ? X(q * QT + i) : 0.0;
        };
        auto emit = [&](int y, double bmv, double bcv, double bnv) {
            const double bl = lane_left_d(bcv);
            const double br = lane_right_d(bcv);
            if constexpr (MODE == FIN_LAPLACIAN) {
                const double v = sig2 * fma(-4.0, bcv, (bl + br) + (bmv + bnv));
                if (wr) dst[(int64_t)y * out_pitch + col] = (float)v;
            } else if constexpr (MODE == FIN_HESSIAN) {
                // Table I taps: d = 2 central second differences, d = 1 half
                // central differences, D11 = D10 of D01 (Eqs 26-27)
                const double d20 = (bl + br) - 2.0 * bcv;
                const double d02 = (bmv + bnv) - 2.0 * bcv;
                const double d10 = 0.5 * (br - bl);
                const double d01 = 0.5 * (bnv - bmv);
                const double d11 = 0.25 * ((lane_right_d(bnv) - lane_left_d(bnv)) - (lane_right_d(bmv) - lane_left_d(bmv)));
                const double det = fma(d20, d02, -d11 * d11);
                const double ndet = sig2 * sig2 * det;
                bool hit = ndet > (double)hz.t1;
                if (hz.t2 > 0.0f) {
                    const double dx = (d01 * d11 - d02 * d10) / det;
                    const double dy = (d10 * d11 - d20 * d01) / det;
                    hit = hit && dx * dx + dy * dy < (double)hz.t2 * (double)hz.t2;
                }
                const bool inside = wr && col >= hz.border && col < W - hz.border && y >= hz.border &&
                                    y < H - hz.border;
                hit = hit && inside;
                const unsigned long long bits = __ballot(hit) >> 1;            // lanes 1..62 -> bits 0..61
                const unsigned long long bright = __ballot(hit && d20 < 0.0) >> 1;
                if (wr) dst[(int64_t)y * out_pitch + col] = (float)ndet;
                if (lane == 0) {
                    const int64_t wi = ((int64_t)s * H + y) * ntx + tx;
                    hz.mask[wi] = bits;
                    hz.pmask[wi] = bright;
                }
            }
        };
        // states entering each quarter from below
#pragma unroll
        for (int q = NQ - 1; q >= 1; --q) {
#pragma unroll
            for (int k = 0; k < NS; ++k) ub[q - 1][k] = ub[q][k];
            if (FULL || q * QT < len) {
                load_q(q);
#pragma unroll
                for (int i = QT - 1; i >= 0; --i)
                    if (valid(q * QT + i)) cas_step<K>(cf, ub[q - 1], xd[i]);
            }
        }
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            if (!(FULL || q * QT < len)) break;
            load_q(q);
            double u[NS];
#pragma unroll
            for (int k = 0; k < NS; ++k) u[k] = ub[q][k];
#pragma unroll
            for (int i = QT - 1; i >= 0; --i) {
                if (valid(q * QT + i)) {
                    t[i] = fma(cf.b0, xd[i], cas_out<K>(cf, u));
                    cas_step<K>(cf, u, xd[i]);
                }
            }
            if constexpr (LAP) {
                if (q == 0 && y0 > 0) {  // B of the row above the tile; u is u(y0)
                    const double xa = m.cvt(lt[lane], sc_above);
                    const double ta = fma(cf.b0, xa, cas_out<K>(cf, u));
                    double v[NS];
#pragma unroll
                    for (int k = 0; k < NS; ++k) v[k] = vf[k];
                    cas_unstep<K>(cf, v, xa);  // forward state before row y0-1
                    bm = ta + cas_out<K>(cf, v);
                }
            }
#pragma unroll
            for (int i = 0; i < QT; ++i) {
                const int j = q * QT + i;
                if (valid(j)) {
                    const double b = t[i] + cas_out<K>(cf, vf);
                    cas_step<K>(cf, vf, xd[i]);
                    if constexpr (!LAP) {
                        if (wr) dst[(int64_t)(y0 + j) * out_pitch + col] = (float)b;
                    } else {
                        if (j == 0) {
                            bc = b;
                            if (y0 == 0) bm = b;  // clamp above the image
                        } else {
                            emit(y0 + j - 1, bm, bc, b);
                            bm = bc;
                            bc = b;
                        }
                    }
                }
            }
        }
        if constexpr (LAP) {
            // the row below the tile: B(y1) = y-(y1) + b0 x(y1) + W v(y1 - 1)
            const double bn = y1 < H ? t_bot + cas_out<K>(cf, vf) : bc;
            emit(y1 - 1, bm, bc, bn);
        }
    };
    if (len == CT)
        body(std::true_type{});
    else
        body(std::false_type{});
}

// the tiles' states within their super tiles, then the super tiles' states
int64_t tile_state_doubles(int64_t H, int64_t W, int nscales, int order) {
    return (int64_t)nscales * ((H + CT - 1) / CT) * 2 * cascade_states(order) * W;
}
int64_t super_state_doubles(int64_t H, int64_t W, int nscales, int order) {
    return (int64_t)nscales * ((H + SCT - 1) / SCT) * 2 * cascade_states(order) * W;
}

template <int K, bool FX>
hipError_t launch_cols_kx(Mid<FX> m, float *out, int64_t H, int64_t W, int64_t pitch, int64_t plane_stride,
                          int mode, const HessArgs *hp, const IirParams &prm, double *st, hipStream_t stream) {
    Args a = make_args(prm, 1);
    const int nty = (int)((H + CT - 1) / CT);
    const int nsy = (int)((H + SCT - 1) / SCT);
    double *sst = st + tile_state_doubles(H, W, prm.nscales, K);
    const unsigned S = (unsigned)prm.nscales;
    dim3 g1((unsigned)((W + 63) / 64), (unsigned)nsy, S);
    hipLaunchKernelGGL((iir_col_states_kernel<K, FX>), g1, dim3(COL_WPB * 64), 0, stream, m, (int)H, (int)W, nty,
                       nsy, st, sst, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    dim3 g2((unsigned)((W + SCAN_T - 1) / SCAN_T), S, 2);
    hipLaunchKernelGGL((iir_col_scan_kernel<K, FX>), g2, dim3(SCAN_T), 0, stream, m, (int)H, (int)W, nsy, sst,
                       a);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int ntyg = (nty + FIN_WPB - 1) / FIN_WPB;
    const HessArgs hz = hp ? *hp : HessArgs{};
    if (mode != FIN_BLUR) {
        const int ntx = (int)((W + 61) / 62);
        const unsigned nb = (unsigned)ntx * (unsigned)ntyg * S;
        if (mode == FIN_HESSIAN)
            hipLaunchKernelGGL((iir_col_final_kernel<K, FIN_HESSIAN, FX>), dim3(nb), dim3(FIN_WPB * 64), 0, stream,
                               m, out, pitch, plane_stride, (int)H, (int)W, nty, ntx, st, sst, nsy, a, hz);
        else
            hipLaunchKernelGGL((iir_col_final_kernel<K, FIN_LAPLACIAN, FX>), dim3(nb), dim3(FIN_WPB * 64), 0,
                               stream, m, out, pitch, plane_stride, (int)H, (int)W, nty, ntx, st, sst, nsy, a, hz);
    } else {
        const int ntx = (int)((W + 63) / 64);
        const unsigned nb = (unsigned)ntx * (unsigned)ntyg * S;
        hipLaunchKernelGGL((iir_col_final_kernel<K, FIN_BLUR, FX>), dim3(nb), dim3(FIN_WPB * 64), 0, stream, m, out,
                           pitch, plane_stride, (int)H, (int)W, nty, ntx, st, sst, nsy, a, hz);
    }
    return hipGetLastError();
}

template <int K>
hipError_t launch_cols_k(const void *in, int64_t in_pitch, int64_t in_plane_stride, const int *rexp, float *out,
                         int64_t H, int64_t W, int64_t pitch, int64_t plane_stride, int mode, const HessArgs *hp,
                         const IirParams &prm, double *st, hipStream_t stream) {
    if (rexp)
        return launch_cols_kx<K, true>(Mid<true>{in, in_pitch, in_plane_stride, rexp}, out, H, W, pitch,
                                       plane_stride, mode, hp, prm, st, stream);
    return launch_cols_kx<K, false>(Mid<false>{in, in_pitch, in_plane_stride, nullptr}, out, H, W, pitch,
                                    plane_stride, mode, hp, prm, st, stream);
}

}  // namespace

size_t iir_cols_workspace_bytes(int64_t H, int64_t W, int nscales, int order) {
    const int64_t n = tile_state_doubles(H, W, nscales, order) + super_state_doubles(H, W, nscales, order);
    return ((size_t)n * sizeof(double) + 255) & ~(size_t)255;
}

hipError_t launch_iir_cols(const void *in, int64_t in_pitch, int64_t in_plane_stride, const int *rexp, float *out,
                           int64_t H, int64_t W, int64_t pitch, int64_t plane_stride, bool laplacian,
                           const IirParams &prm, void *ws, hipStream_t st) {
    return launch_iir_cols_mode(in, in_pitch, in_plane_stride, rexp, out, H, W, pitch, plane_stride,
                                laplacian ? FIN_LAPLACIAN : FIN_BLUR, nullptr, prm, ws, st);
}

hipError_t launch_iir_cols_mode(const void *in, int64_t in_pitch, int64_t in_plane_stride, const int *rexp,
                                float *out, int64_t H, int64_t W, int64_t pitch, int64_t plane_stride, int mode,
                                const HessArgs *hp, const IirParams &prm, void *ws, hipStream_t st) {
    double *states = static_cast<double *>(ws);
    if (mode == FIN_HESSIAN && !hp) return hipErrorInvalidValue;
    if (prm.order == 3)
        return launch_cols_k<3>(in, in_pitch, in_plane_stride, rexp, out, H, W, pitch, plane_stride, mode, hp, prm,
                                states, st);
    if (prm.order == 2)
        return launch_cols_k<2>(in, in_pitch, in_plane_stride, rexp, out, H, W, pitch, plane_stride, mode, hp, prm,
                                states, st);
    if (prm.order == CPAIR)
        return launch_cols_k<CPAIR>(in, in_pitch, in_plane_stride, rexp, out, H, W, pitch, plane_stride, mode, hp,
                                    prm, states, st);
    if (prm.order == 4 && !rexp && mode != FIN_HESSIAN)
        return launch_cols_kx<4, false>(Mid<false>{in, in_pitch, in_plane_stride, nullptr}, out, H, W, pitch,
                                        plane_stride, mode, hp, prm, states, st);
    return hipErrorInvalidValue;
}

}  // namespace fdvm
