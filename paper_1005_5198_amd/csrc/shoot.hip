// Deflection + binning kernel for inverse ray-shooting on gfx950.
//
// Computes, for every ray of a chunk of the ray window, the lens equation of
// Section 2, Eq. (sigma),
//     y = diag(1 - gamma - sigma_c, 1 + gamma - sigma_c) x - sum_k m_k (x - x_k)/|x - x_k|^2,
// and bins it into the source-plane count map of Eq. (mu_ij).
//
// Design (gfx950, FP32 VALU bound; no MFMA since the sum is not a contraction):
//  * A block owns a 64 x 32 patch of rays. Lenses stream through LDS in tiles
//    of LENS_TILE, converted once per block from FP64 to FP32 offsets relative
//    to the patch centre, so FP32 carries small numbers and the per-block
//    conversion is paid once per lens per 2048 rays.
//  * Each lane owns RX x RY rays (4x2, 4x4, 8x2 or 8x4: a tuned choice), its
//    rows in adjacent pairs; per lens it computes dx for RX columns and dy,
//    dy^2 for RY rows, then r^2 = fma(dx, dx, dy^2) per ray, one v_rcp_f32 per
//    four rays (two adjacent rows of two columns 16 apart, of the product of
//    their r^2) and nine multiplies, and two FMAs per ray. Every LDS read is a
//    16-byte broadcast of two lenses.
//  * The sum runs in FP32 over GROUP lenses, then each partial is folded
//    exactly into an FP64 accumulator, so FP32 rounding never sees the large
//    running total.
//  * Mixed mode: while staging lenses the block also sums a rigorous bound on
//    the FP32 error of every ray in the patch (lenses close to the patch are
//    bounded per ray instead). A ray whose bound reaches a pixel edge goes to a
//    queue that the FP64 re-check stages decide exactly as the definition does.
//  * Binning uses wave-aggregated atomics: lanes that hit the same pixel add
//    their count with one atomic.
#include "shoot_common.h"

namespace rs {
namespace {

// One lens's terms for this lane's RX x RY rays: dx per column, dy and dy^2 per
// row, then per ray r^2 = fma(dx, dx, dy^2), the reciprocal and two FMAs into the
// FP32 sums. The reciprocal issues at a fraction of the FMA rate, so rays share it
// through products of their r^2:
//  * QUAD: the rays of rows 2k, 2k+1 and columns c, c' = c + 16 (lane columns c
//    and c + CQ, CQ = 16 / stride) share one v_rcp_f32 of P = (a b)(c d):
//    1/a = b (R cd), 1/b = a (R cd), 1/c = d (R ab), 1/d = c (R ab) with
//    R = rcp(P), nine multiplies per four rays;
//  * otherwise rows 2k and 2k+1 of a column share one, of the product of their
//    r^2 (1/a = b/(ab), 1/b = a/(ab)), three multiplies per two rays.
// With masses each reciprocal is multiplied by the lens's mass last, so a unit
// mass gives the unit path's result. The partners do not depend on the thread
// shape, so neither does a ray's arithmetic.
template <int RX, int RY, bool UNIT, bool QUAD, int CQ>
__device__ __forceinline__ void lens_terms(float LX, float LY, float M, const float (&rxl)[RX],
                                           const float (&ryl)[RY], float (&sx)[RY][RX], float (&sy)[RY][RX]) {
    float dy[RY], dy2[RY], dx[RX];
#pragma unroll
    for (int r = 0; r < RY; ++r) {
        dy[r] = ryl[r] - LY;
        dy2[r] = dy[r] * dy[r];
    }
#pragma unroll
    for (int c = 0; c < RX; ++c) dx[c] = rxl[c] - LX;
#pragma unroll
    for (int r = 0; r < RY; r += 2)
#pragma unroll
        for (int c = 0; c < RX; ++c) {
            if (QUAD) {
                if ((c / CQ) % 2) continue;
                const int e = c + CQ;
                const float ra = __builtin_fmaf(dx[c], dx[c], dy2[r]);
                const float rb = __builtin_fmaf(dx[c], dx[c], dy2[r + 1]);
                const float rc = __builtin_fmaf(dx[e], dx[e], dy2[r]);
                const float rd = __builtin_fmaf(dx[e], dx[e], dy2[r + 1]);
                const float pab = ra * rb, pcd = rc * rd;
                const float R = __builtin_amdgcn_rcpf(pab * pcd);
                const float qab = R * pcd, qcd = R * pab;
                float ia = rb * qab, ib = ra * qab, ic = rd * qcd, id = rc * qcd;
                if (!UNIT) {
                    ia = M * ia;
                    ib = M * ib;
                    ic = M * ic;
                    id = M * id;
                }
                sx[r][c] = __builtin_fmaf(dx[c], ia, sx[r][c]);
                sy[r][c] = __builtin_fmaf(dy[r], ia, sy[r][c]);
                sx[r + 1][c] = __builtin_fmaf(dx[c], ib, sx[r + 1][c]);
                sy[r + 1][c] = __builtin_fmaf(dy[r + 1], ib, sy[r + 1][c]);
                sx[r][e] = __builtin_fmaf(dx[e], ic, sx[r][e]);
                sy[r][e] = __builtin_fmaf(dy[r], ic, sy[r][e]);
                sx[r + 1][e] = __builtin_fmaf(dx[e], id, sx[r + 1][e]);
                sy[r + 1][e] = __builtin_fmaf(dy[r + 1], id, sy[r + 1][e]);
            } else {
                const float ra = __builtin_fmaf(dx[c], dx[c], dy2[r]);
                const float rb = __builtin_fmaf(dx[c], dx[c], dy2[r + 1]);
                const float rab = __builtin_amdgcn_rcpf(ra * rb);
                float ia = rb * rab, ib = ra * rab;
                if (!UNIT) {
                    ia = M * ia;
                    ib = M * ib;
                }
                sx[r][c] = __builtin_fmaf(dx[c], ia, sx[r][c]);
                sy[r][c] = __builtin_fmaf(dy[r], ia, sy[r][c]);
                sx[r + 1][c] = __builtin_fmaf(dx[c], ib, sx[r + 1][c]);
                sy[r + 1][c] = __builtin_fmaf(dy[r + 1], ib, sy[r + 1][c]);
            }
        }
}

// FP32 sums over the N lenses of tile entries g .. g+N-1 for this lane's rays
// (lens_terms), folded into the FP64 accumulators. Every LDS read is a 16-byte
// broadcast: two lenses of unit mass, or one lens with its mass. The four-ray
// loop is unrolled by 8 reads, not fully (a full unroll makes the compiler spill);
// the two-ray loop fully.
template <int N, int RX, int RY, bool UNIT, bool QUAD, int CQ>
__device__ __forceinline__ void group_sums(const float4 *tile, int g, const float (&rxl)[RX], const float (&ryl)[RY],
                                           double (&Ax)[RY][RX], double (&Ay)[RY][RX]) {
    static_assert(RY % 2 == 0, "rows are paired for the shared reciprocal");
    static_assert(RX == 4 * CQ, "column partners are CQ lane columns apart");
    float sx[RY][RX], sy[RY][RX];
#pragma unroll
    for (int r = 0; r < RY; ++r)
#pragma unroll
        for (int c = 0; c < RX; ++c) {
            sx[r][c] = 0.0f;
            sy[r][c] = 0.0f;
        }
    if (UNIT) {
        if (QUAD) {
#pragma unroll 8
            for (int kk = 0; kk < N; kk += 2) {
                const float4 q = tile[(g + kk) >> 1];
                lens_terms<RX, RY, true, true, CQ>(q.x, q.y, 1.0f, rxl, ryl, sx, sy);
                lens_terms<RX, RY, true, true, CQ>(q.z, q.w, 1.0f, rxl, ryl, sx, sy);
            }
        } else {
#pragma unroll
            for (int kk = 0; kk < N; kk += 2) {
                const float4 q = tile[(g + kk) >> 1];
                lens_terms<RX, RY, true, false, CQ>(q.x, q.y, 1.0f, rxl, ryl, sx, sy);
                lens_terms<RX, RY, true, false, CQ>(q.z, q.w, 1.0f, rxl, ryl, sx, sy);
            }
        }
    } else {
        if (QUAD) {
#pragma unroll 8
            for (int kk = 0; kk < N; ++kk) {
                const float4 q = tile[g + kk];
                lens_terms<RX, RY, false, true, CQ>(q.x, q.y, q.z, rxl, ryl, sx, sy);
            }
        } else {
#pragma unroll
            for (int kk = 0; kk < N; ++kk) {
                const float4 q = tile[g + kk];
                lens_terms<RX, RY, false, false, CQ>(q.x, q.y, q.z, rxl, ryl, sx, sy);
            }
        }
    }
#pragma unroll
    for (int r = 0; r < RY; ++r)
#pragma unroll
        for (int c = 0; c < RX; ++c) {
            Ax[r][c] += (double)sx[r][c];
            Ay[r][c] += (double)sy[r][c];
        }
}

// One 64 x 32 ray patch. RX x RY rays per lane, WX x WY waves per block; every
// shape covers the same PATCH_X x PATCH_Y ray patch, so a ray's arithmetic
// (patch origin, lens offsets, operation order) does not depend on the shape.
template <int RX, int RY, int WX, int WY, bool UNIT, int MODE, bool PIX, class Sink>
__device__ __forceinline__ void shoot_patch(const ShootArgs &a, int64_t patch, ShootSmem &sm, const Sink &sink) {
    constexpr int BLOCK_THREADS = 64 * WX * WY;
    constexpr int STRIDE_X = LANES_X * WX;
    constexpr int STRIDE_Y = LANES_Y * WY;
    static_assert(RX * STRIDE_X == PATCH_X && RY * STRIDE_Y == PATCH_Y, "shape must tile the patch");
    static_assert(BLOCK_THREADS / 64 <= 16, "reduction buffer");
    float4 *tile = sm.tile;
    int &near_count = sm.near_count;
    double *red_bx = sm.red_bx;
    double *red_by = sm.red_by;

    const int tid = threadIdx.x;
    const int wave = tid >> 6;
    const int lane = tid & 63;
    const int wx = wave % WX, wy = wave / WX;
    const int lx = lane % LANES_X, ly = lane / LANES_X;
    __syncthreads();  // the previous patch of this block is done with the shared buffers

    // Patch of this block.
    const int64_t pbx = patch % a.nbx;
    const int64_t pby = patch / a.nbx;
    const int64_t ib = a.i0 + pbx * PATCH_X;
    const int64_t jb = a.jc0 + pby * PATCH_Y;
    // Patch origin and half-extents (with a spacing of slack on each side).
    const double ox = a.sx0 + ((double)ib + 0.5 * PATCH_X) * a.spx;
    const double oy = a.sy0 + ((double)jb + 0.5 * PATCH_Y) * a.spy;
    const double hx = (0.5 * PATCH_X + 1.0) * a.spx;
    const double hy = (0.5 * PATCH_Y + 1.0) * a.spy;
    const double h = sqrt(hx * hx + hy * hy);
    const double near_r2 = 4.0 * h * h;

    // This lane's rays: column i = i_lane + c * STRIDE_X and the rows below, held
    // as FP32 offsets from the patch origin.
    const int64_t i_lane = ib + wx * LANES_X + lx;
    // Rows come in adjacent pairs (2k, 2k+1) per lane, the pairs STRIDE_Y apart:
    // ray r of the lane is on row j_pair + 2 (r / 2) STRIDE_Y + (r % 2).
    const int64_t j_pair = jb + 2 * (wy * LANES_Y + ly);
    float rxl[RX], ryl[RY];
#pragma unroll
    for (int c = 0; c < RX; ++c) rxl[c] = (float)(ray_coord(a.sx0, i_lane + c * STRIDE_X, a.spx) - ox);
#pragma unroll
    for (int r = 0; r < RY; ++r) ryl[r] = (float)(ray_coord(a.sy0, j_pair + 2 * (r >> 1) * STRIDE_Y + (r & 1), a.spy) - oy);

    double Ax[RY][RX], Ay[RY][RX];
#pragma unroll
    for (int r = 0; r < RY; ++r)
#pragma unroll
        for (int c = 0; c < RX; ++c) {
            Ax[r][c] = 0.0;
            Ay[r][c] = 0.0;
        }

    if (tid == 0) {
        near_count = 0;
        sm.far_tile = -1;
    }
    double bx = 0.0, by = 0.0;  // this thread's share of the block error bound (units of u)
    const double k_term = UNIT ? K_TERM_QUAD : K_TERM_MASS_QUAD;
    // Four-ray reciprocals need the patch's half-diagonal in range (see QUAD_RANGE).
    const bool quad_patch = h >= QUAD_H_MIN && h <= QUAD_H_MAX;
    constexpr int CQ = 16 / STRIDE_X;

    for (int64_t t0 = 0; t0 < a.n_lens; t0 += LENS_TILE) {
        const int cnt = (int)((a.n_lens - t0) < LENS_TILE ? (a.n_lens - t0) : LENS_TILE);
        const int cnt_pad = (cnt + GROUP / 2 - 1) / (GROUP / 2) * (GROUP / 2);
        __syncthreads();  // previous tile fully consumed (and near_count initialised)
        stage_tile<UNIT, MODE, BLOCK_THREADS>(a, t0, cnt, cnt_pad, ox, oy, hx, hy, h, near_r2, k_term, sm, tid, bx,
                                              by);
        __syncthreads();

        // Whole groups of real lenses with four-ray reciprocals where the tile's lenses
        // and the patch allow them; then the rest (groups holding padding lenses, at
        // offset PAD_OFFSET, or every group of a tile out of range) with two-ray ones. The
        // last tile may end with half a group, summed by code of its own, so that the
        // loops' schedules are those of whole groups.
        const int tile_idx = (int)(t0 / LENS_TILE);
        const int full_q = (quad_patch && sm.far_tile != tile_idx) ? cnt / GROUP * GROUP : 0;
        const int full = cnt_pad / GROUP * GROUP;
        int g = 0;
        for (; g < full_q; g += GROUP) group_sums<GROUP, RX, RY, UNIT, true, CQ>(tile, g, rxl, ryl, Ax, Ay);
        for (; g < full; g += GROUP) group_sums<GROUP, RX, RY, UNIT, false, CQ>(tile, g, rxl, ryl, Ax, Ay);
        if (full < cnt_pad) group_sums<GROUP / 2, RX, RY, UNIT, false, CQ>(tile, full, rxl, ryl, Ax, Ay);
    }

    // Block-wide error bound (mixed mode).
    double Bx = 0.0, By = 0.0;
    int n_near = 0;
    bool all_flagged = false;
    if (MODE == 1) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            bx += __shfl_xor(bx, off);
            by += __shfl_xor(by, off);
        }
        __syncthreads();
        if (lane == 0) {
            red_bx[wave] = bx;
            red_by[wave] = by;
        }
        __syncthreads();
#pragma unroll
        for (int w = 0; w < BLOCK_THREADS / 64; ++w) {
            Bx += red_bx[w];
            By += red_by[w];
        }
        n_near = near_count;
        // (a patch under 1e-6 across could underflow the paired products of r^2)
        all_flagged = n_near > NEAR_MAX || h < 1.0e-6;
        if (all_flagged) n_near = 0;
    }

    // Epilogue: macro terms, pixel, classification, binning.
    const float h_f = (float)h;
    const float tiny_r2 = 1.0e-6f * h_f * h_f;
    unsigned long long n_in = 0, n_out = 0, n_sing = 0;
    const int64_t W = a.i1 - a.i0;
#pragma unroll
    for (int r = 0; r < RY; ++r)
#pragma unroll
        for (int c = 0; c < RX; ++c) {
            const int64_t i = i_lane + c * STRIDE_X, j = j_pair + 2 * (r >> 1) * STRIDE_Y + (r & 1);
            const bool valid = (i < a.i1) && (j < a.jc1);
            const double x1 = ray_coord(a.sx0, i, a.spx);
            const double x2 = ray_coord(a.sy0, j, a.spy);
            const double y1 = a.c1 * x1 - Ax[r][c];
            const double y2 = a.c2 * x2 - Ay[r][c];
            const double u = (y1 - a.tx0) * a.inv_pixw;
            const double v = (y2 - a.ty0) * a.inv_pixh;
            const int cp = ((c / CQ) % 2) ? c - CQ : c + CQ;   // the column partner of the four-ray reciprocal
            int code = classify_ray<MODE>(a, x1, x2, Ax[r][c], Ay[r][c], u, v, rxl[c], ryl[r], rxl[c], ryl[r ^ 1],
                                          rxl[cp], quad_patch, Bx, By, n_near, all_flagged, sm.near_list, k_term,
                                          h_f, tiny_r2);
            if (!valid) code = INT32_MIN;

            n_in += __builtin_popcountll(__ballot(code >= 0));
            n_out += __builtin_popcountll(__ballot(code == OUT));
            n_sing += __builtin_popcountll(__ballot(code == SINGULAR));

            if (PIX) {
                if (valid && code != FLAGGED) a.pix_out[(j - a.j0) * W + (i - a.i0)] = code;
            } else {
                aggregated_add(a.map, code);
            }
            if (MODE == 1) {
                const uint64_t fl = __ballot(code == FLAGGED);
                if (fl) sink.append(a, fl, lane, code == FLAGGED, i, j);
            }
        }
    if (lane == 0) {
        if (n_in) atomicAdd(a.counters + C_IN, n_in);
        if (n_out) atomicAdd(a.counters + C_OUT, n_out);
        if (n_sing) atomicAdd(a.counters + C_SING, n_sing);
    }
}

// Single map: one block per patch of this launch's rows.
template <int RX, int RY, int WX, int WY, bool UNIT, int MODE, bool PIX>
__global__ __launch_bounds__(64 * WX * WY, (RX * RY <= 8) ? 4 : 1) void shoot_kernel(const ShootArgs a) {
    __shared__ ShootSmem sm;
    shoot_patch<RX, RY, WX, WY, UNIT, MODE, PIX>(a, (int64_t)blockIdx.x, sm, SingleSink{});
}

// Batch: persistent blocks pull (map, patch) tiles from one counter until the
// work list is exhausted; every block exits when the counter passes the end.
template <int RX, int RY, int WX, int WY, bool UNIT, int MODE>
__global__ __launch_bounds__(64 * WX * WY, (RX * RY <= 8) ? 4 : 1) void shoot_batch_kernel(const BatchArgs b) {
    __shared__ ShootSmem sm;
    __shared__ long long s_tile;
    for (;;) {
        __syncthreads();  // s_tile of the previous round has been read by every thread
        if (threadIdx.x == 0) s_tile = (long long)atomicAdd(b.tile_counter, 1ull);
        __syncthreads();
        // The tile index is the same for the whole block; make that visible to the
        // compiler so per-map values live in scalar registers.
        const unsigned long long st = (unsigned long long)s_tile;
        const unsigned t_lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)st);
        const unsigned t_hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(st >> 32));
        const long long t = (long long)(((unsigned long long)t_hi << 32) | t_lo);
        if (t >= b.total_tiles) break;
        int lo = 0, hi = b.n_maps - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (b.maps[mid].tile_begin <= t) lo = mid;
            else hi = mid - 1;
        }
        const BatchMap &m = b.maps[lo];
        const ShootArgs a = make_uniform(shoot_args_of(m.p, m.lens_xy, m.lens_m, m.n_lens, m.map, m.counters));
        const int64_t tile_begin = make_uniform(m.tile_begin);
        uint32_t *const bits = make_uniform(m.flag_bits);
        const BatchSink sink{a.counters, bits};
        shoot_patch<RX, RY, WX, WY, UNIT, MODE, false>(a, t - tile_begin, sm, sink);
    }
}

// Zero each map of a batch (unless it accumulates), its counters, and the batch globals.
__global__ void fill_batch_kernel(const BatchArgs b, unsigned long long *globals) {
    const int mi = blockIdx.y;
    const BatchMap &m = b.maps[mi];
    if (blockIdx.x == 0 && threadIdx.x < N_COUNTERS) m.counters[threadIdx.x] = 0ull;
    if (mi == 0 && blockIdx.x == 0 && threadIdx.x < 4) globals[threadIdx.x] = 0ull;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < m.n_words; t += stride) {
        m.flag_bits[t] = 0u;
        m.unres_bits[t] = 0u;
    }
    if (m.accumulate) return;
    const int64_t n = m.p.npx * m.p.npy;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += stride) m.map[t] = 0u;
}

__global__ void fill_kernel(uint32_t *map, int64_t n_pix, uint32_t *ws_words, int64_t n_ws_words) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n_pix; t += stride) map[t] = 0u;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n_ws_words; t += stride)
        ws_words[t] = 0u;
}

}  // namespace


hipError_t launch_zero(uint32_t *p, int64_t n, hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    int blocks = (int)((n + 255) / 256);
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(fill_kernel, dim3(blocks), dim3(256), 0, stream, p, n, static_cast<uint32_t *>(nullptr),
                       (int64_t)0);
    return hipGetLastError();
}

hipError_t launch_fill(uint32_t *map, int64_t n_pix, void *workspace, int64_t n_qcount,
                       hipStream_t stream) {
    const int64_t n_ws_words = (int64_t)(WS_QCOUNT / 4) + n_qcount;
    const int64_t work = (map ? n_pix : 0) > n_ws_words ? (map ? n_pix : 0) : n_ws_words;
    int blocks = (int)((work + 255) / 256);
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(fill_kernel, dim3(blocks), dim3(256), 0, stream, map, map ? n_pix : 0,
                       static_cast<uint32_t *>(workspace), n_ws_words);
    return hipGetLastError();
}

template <int RX, int RY, int WX, int WY>
static void launch_shape(const ShootArgs &a, int mode, dim3 grid, hipStream_t stream) {
    const bool unit = a.lens_m == nullptr;
    const bool pix = a.pix_out != nullptr;
    const dim3 block(64 * WX * WY);
#define RS_LAUNCH(U, M, P) hipLaunchKernelGGL((shoot_kernel<RX, RY, WX, WY, U, M, P>), grid, block, 0, stream, a)
    if (mode == 0) {
        if (unit) { if (pix) RS_LAUNCH(true, 0, true); else RS_LAUNCH(true, 0, false); }
        else { if (pix) RS_LAUNCH(false, 0, true); else RS_LAUNCH(false, 0, false); }
    } else {
        if (unit) { if (pix) RS_LAUNCH(true, 1, true); else RS_LAUNCH(true, 1, false); }
        else { if (pix) RS_LAUNCH(false, 1, true); else RS_LAUNCH(false, 1, false); }
    }
#undef RS_LAUNCH
}
const ShapeInfo &shape_info(int shape) {
    static const ShapeInfo table[N_SHAPES] = {
        {4, 2, 2, 2}, {4, 4, 2, 1}, {8, 2, 1, 2}, {8, 4, 1, 1},
    };
    return table[(shape >= 0 && shape < N_SHAPES) ? shape : 0];
}

template <int RX, int RY, int WX, int WY, bool UNIT, int MODE>
static void launch_batch_variant(const BatchArgs &b, int blocks_per_cu, hipStream_t stream) {
    const int threads = 64 * WX * WY;
    auto k = shoot_batch_kernel<RX, RY, WX, WY, UNIT, MODE>;
    int grid_blocks = persistent_blocks(k, threads, blocks_per_cu);
    if ((int64_t)grid_blocks > b.total_tiles) grid_blocks = (int)b.total_tiles;
    hipLaunchKernelGGL(k, dim3((unsigned)grid_blocks), dim3(threads), 0, stream, b);
}

template <int RX, int RY, int WX, int WY>
static void launch_batch_shape(const BatchArgs &b, int blocks_per_cu, hipStream_t stream) {
    if (b.unit_masses) {
        if (b.mode == 0) launch_batch_variant<RX, RY, WX, WY, true, 0>(b, blocks_per_cu, stream);
        else launch_batch_variant<RX, RY, WX, WY, true, 1>(b, blocks_per_cu, stream);
    } else {
        if (b.mode == 0) launch_batch_variant<RX, RY, WX, WY, false, 0>(b, blocks_per_cu, stream);
        else launch_batch_variant<RX, RY, WX, WY, false, 1>(b, blocks_per_cu, stream);
    }
}

hipError_t launch_shoot_batch(const BatchArgs &b, int shape, int blocks_per_cu, hipStream_t stream) {
    if (b.total_tiles <= 0) return hipSuccess;
    switch (shape) {
        case 1: launch_batch_shape<4, 4, 2, 1>(b, blocks_per_cu, stream); break;
        case 2: launch_batch_shape<8, 2, 1, 2>(b, blocks_per_cu, stream); break;
        case 3: launch_batch_shape<8, 4, 1, 1>(b, blocks_per_cu, stream); break;
        default: launch_batch_shape<4, 2, 2, 2>(b, blocks_per_cu, stream); break;
    }
    return hipGetLastError();
}

hipError_t launch_batch_fill(const BatchArgs &b, void *workspace, int32_t n_maps, hipStream_t stream) {
    if (n_maps <= 0) return hipSuccess;
    const dim3 grid(64, (unsigned)n_maps), block(256);
    hipLaunchKernelGGL(fill_batch_kernel, grid, block, 0, stream, b,
                       static_cast<unsigned long long *>(workspace));
    return hipGetLastError();
}

hipError_t launch_shoot(const ShootArgs &a, int mode, int shape, hipStream_t stream) {
    const int64_t nby = (a.jc1 - a.jc0 + PATCH_Y - 1) / PATCH_Y;
    const int64_t blocks = a.nbx * nby;
    if (blocks <= 0) return hipSuccess;
    const dim3 grid((unsigned)blocks);
    switch (shape) {
        case 1: launch_shape<4, 4, 2, 1>(a, mode, grid, stream); break;
        case 2: launch_shape<8, 2, 1, 2>(a, mode, grid, stream); break;
        case 3: launch_shape<8, 4, 1, 1>(a, mode, grid, stream); break;
        default: launch_shape<4, 2, 2, 2>(a, mode, grid, stream); break;
    }
    return hipGetLastError();
}

}  // namespace rs
