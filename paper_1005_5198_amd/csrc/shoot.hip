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
//  * Each lane owns RX x RY rays (4x2, 4x4, 8x2 or 8x4: a tuned choice); per
//    lens it computes dx for RX columns and dy, dy^2 for RY rows, then
//    r^2 = fma(dx, dx, dy^2), v_rcp_f32, and two FMAs per ray. Every LDS read
//    is a 16-byte broadcast of two lenses.
//  * The sum runs in FP32 over GROUP lenses, then each partial is folded
//    exactly into an FP64 accumulator, so FP32 rounding never sees the large
//    running total.
//  * Mixed mode: while staging lenses the block also sums a rigorous bound on
//    the FP32 error of every ray in the patch (lenses close to the patch are
//    bounded per ray instead). A ray whose bound reaches a pixel edge goes to a
//    queue that an FP64 kernel re-evaluates with the plain definition.
//  * Binning uses wave-aggregated atomics: lanes that hit the same pixel add
//    their count with one atomic.
#include "recheck_ray.h"

namespace rs {
namespace {

constexpr double U32 = 5.9604644775390625e-08;  // 2^-24, FP32 unit roundoff

// Per-lens FP32 error constants (derivation in the design notes):
//   |t_hat - t| <= u m (K_TERM |dx| + K_H h) / r^2 for one term t = m dx / r^2,
//   the FP32 group sum adds u (GROUP - pos) |t_hat| for the lens at position pos.
// Unit masses: K_TERM covers dx (2.04u), r^2 (6.08u + 4.08u h/r) and rcp (2u, 1 ulp);
// with masses, the FP32 mass rounding and the extra multiply add 2u more.
constexpr double K_TERM_UNIT = 10.5;
constexpr double K_TERM_MASS = 13.0;
constexpr double K_GROUP = 1.01;
constexpr double K_H = 6.5;

constexpr int OUT = -1;
constexpr int SINGULAR = -2;
constexpr int FLAGGED = -3;

struct NearLens {
    float x, y, m;
    int pos;
};

__device__ __forceinline__ double ray_coord(double origin, int64_t idx, double spacing) {
    // The definition's own operations: origin + ((double)idx + 0.5) * spacing.
    // The library is built without floating-point contraction.
    return origin + ((double)idx + 0.5) * spacing;
}

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// Add one count per lane to map[p] for every lane with p >= 0, one atomic per distinct pixel.
__device__ __forceinline__ void aggregated_add(uint32_t *map, int p) {
    uint64_t pending = __ballot(p >= 0);
    while (pending) {
        const int leader = __builtin_ctzll(pending);
        const int lp = __builtin_amdgcn_readlane(p, leader);
        const uint64_t same = __ballot(p == lp) & pending;
        if (lane_id() == leader) atomicAdd(map + lp, (uint32_t)__builtin_popcountll(same));
        pending &= ~same;
    }
}

struct ShootSmem {
    float4 tile[LENS_TILE];        // UNIT: two (x,y) pairs per float4; else (x,y,m,0)
    NearLens near_list[NEAR_MAX];
    int near_count;
    double red_bx[16], red_by[16];
};

// Queue sink of a single-map launch: uint32 chunk-relative ray indices; the
// queue holds every ray of the launch, so it cannot overflow.
struct SingleSink {
    __device__ void append(const ShootArgs &a, uint64_t fl, int lane, bool mine, int64_t i, int64_t j) const {
        const int first = __builtin_ctzll(fl);
        uint32_t base = 0;
        if (lane == first) base = atomicAdd(a.qcount, (uint32_t)__builtin_popcountll(fl));
        base = __builtin_amdgcn_readlane(base, first);
        if (mine) {
            const uint32_t below = (uint32_t)__builtin_popcountll(fl & ((1ull << lane) - 1ull));
            a.queue[base + below] = (uint32_t)((j - a.jc0) * (a.i1 - a.i0) + (i - a.i0));
        }
    }
};

// Re-check sink of a batch launch: one bit per flagged ray in the map's flag
// bitmap (two bits per ray of workspace in all, whatever the flagged fraction).
struct BatchSink {
    unsigned long long *counters;
    uint32_t *flag_bits;
    __device__ void append(const ShootArgs &a, uint64_t fl, int lane, bool mine, int64_t i, int64_t j) const {
        if (lane == __builtin_ctzll(fl)) atomicAdd(counters + C_RECHECK, (unsigned long long)__builtin_popcountll(fl));
        if (mine) {
            const uint32_t ray = (uint32_t)((j - a.j0) * (a.i1 - a.i0) + (i - a.i0));
            atomicOr(flag_bits + (ray >> 5), 1u << (ray & 31u));
        }
    }
};

// Stage lenses t0 .. t0+cnt of the lens array into the LDS tile as FP32 offsets
// from the block origin (ox, oy), padded to whole groups with far massless
// lenses. Mixed mode: lenses within 2h of the block's box go to the near list
// (bounded per ray later); the others add their rigorous FP32 error weight for
// any ray in the box [ox +- hx] x [oy +- hy] to this thread's share (bx, by).
template <bool UNIT, int MODE, int BLOCK_THREADS>
__device__ __forceinline__ void stage_tile(const ShootArgs &a, int64_t t0, int cnt, int cnt_pad, double ox, double oy,
                                           double hx, double hy, double h, double near_r2, double k_term,
                                           ShootSmem &sm, int tid, double &bx, double &by) {
    float4 *tile = sm.tile;
        for (int s = tid; s < cnt_pad; s += BLOCK_THREADS) {
            float fx = 1.0e18f, fy = 0.0f, fm = 0.0f;  // padding lens: far away, massless
            if (s < cnt) {
                const int64_t k = t0 + s;
                const double X = a.lens_xy[2 * k];
                const double Y = a.lens_xy[2 * k + 1];
                const double m = (UNIT || a.lens_m == nullptr) ? 1.0 : a.lens_m[k];
                const double Lx = X - ox, Ly = Y - oy;
                fx = (float)Lx;
                fy = (float)Ly;
                fm = (float)m;
                if (MODE == 1) {
                    const double alx = fabs(Lx), aly = fabs(Ly);
                    const double ex = fmax(alx - hx, 0.0), ey = fmax(aly - hy, 0.0);
                    const double dmin2 = ex * ex + ey * ey;
                    const int pos = s % GROUP;
                    if (dmin2 < near_r2) {
                        const int q = atomicAdd(&sm.near_count, 1);
                        if (q < NEAR_MAX) sm.near_list[q] = NearLens{fx, fy, (float)fabs(m), pos};
                    } else {
                        const double wgt = k_term + K_GROUP * (double)(GROUP - pos);
                        const double im = fabs(m) / dmin2;
                        bx += im * (wgt * (alx + hx) + K_H * h);
                        by += im * (wgt * (aly + hy) + K_H * h);
                    }
                }
            }
            if (UNIT) {
                float *t2 = reinterpret_cast<float *>(tile);
                t2[2 * s] = fx;
                t2[2 * s + 1] = fy;
            } else {
                tile[s] = make_float4(fx, fy, fm, 0.0f);
            }
        }
}

// Pixel code of one ray from its FP64 position x, its folded deflection A and
// its source position (u, v) in pixel units. Mixed mode: the ray's error
// bound is the block's (Bx, By) plus the near lenses' per-ray terms, and a ray
// within it of a pixel edge is FLAGGED for the FP64 re-check.
template <int MODE>
__device__ __forceinline__ int classify_ray(const ShootArgs &a, double x1, double x2, double Axv, double Ayv, double u,
                                            double v, float rx, float ry, double Bx, double By, int n_near,
                                            bool all_flagged, const NearLens *near_list, double k_term, float h_f,
                                            float tiny_r2) {
    int code;
    if (MODE == 0) {
        if (!(isfinite(u) && isfinite(v))) code = SINGULAR;
        else if (u >= 0.0 && u < (double)a.npx && v >= 0.0 && v < (double)a.npy)
            code = (int)((int64_t)floor(v) * a.npx + (int64_t)floor(u));
        else code = OUT;
    } else {
        // Per-ray bound from the lenses next to the block.
        float cx = 0.0f, cy = 0.0f;
        for (int q = 0; q < n_near; ++q) {
            const NearLens nl = near_list[q];
            const float dxn = rx - nl.x, dyn = ry - nl.y;
            const float r2n = dxn * dxn + dyn * dyn;
            const float wgt = (float)(k_term + K_GROUP * (double)(GROUP - nl.pos));
            if (!(r2n > tiny_r2)) {
                cx = __builtin_inff();
                cy = __builtin_inff();
            } else {
                const float im = nl.m / (0.999f * r2n);
                cx += im * (wgt * (1.001f * fabsf(dxn) + 1e-6f * h_f) + (float)K_H * h_f);
                cy += im * (wgt * (1.001f * fabsf(dyn) + 1e-6f * h_f) + (float)K_H * h_f);
            }
        }
        const double ea = 1e-15 + 8.9e-16 * (fabs(a.c1 * x1) + fabs(Axv) + fabs(a.tx0));
        const double eb = 1e-15 + 8.9e-16 * (fabs(a.c2 * x2) + fabs(Ayv) + fabs(a.ty0));
        const double Eu = (U32 * (Bx + (double)cx) * a.bound_scale + ea) * a.inv_pixw * 1.000001;
        const double Ev = (U32 * (By + (double)cy) * a.bound_scale + eb) * a.inv_pixh * 1.000001;
        const double fu = floor(u), fv = floor(v);
        const bool ok_u = (fmin(u - fu, fu + 1.0 - u) > Eu) && (fu >= 0.0) && (fu < (double)a.npx);
        const bool ok_v = (fmin(v - fv, fv + 1.0 - v) > Ev) && (fv >= 0.0) && (fv < (double)a.npy);
        const bool out_u = (u < -Eu) || (u > (double)a.npx + Eu);
        const bool out_v = (v < -Ev) || (v > (double)a.npy + Ev);
        if (all_flagged) code = FLAGGED;
        else if (ok_u && ok_v) code = (int)((int64_t)fv * a.npx + (int64_t)fu);
        else if (out_u || out_v) code = OUT;
        else code = FLAGGED;
    }
    return code;
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

    // This lane's rays: column i = i_lane + c * STRIDE_X, row j = j_lane + r * STRIDE_Y,
    // held as FP32 offsets from the patch origin.
    const int64_t i_lane = ib + wx * LANES_X + lx;
    const int64_t j_lane = jb + wy * LANES_Y + ly;
    float rxl[RX], ryl[RY];
#pragma unroll
    for (int c = 0; c < RX; ++c) rxl[c] = (float)(ray_coord(a.sx0, i_lane + c * STRIDE_X, a.spx) - ox);
#pragma unroll
    for (int r = 0; r < RY; ++r) ryl[r] = (float)(ray_coord(a.sy0, j_lane + r * STRIDE_Y, a.spy) - oy);

    double Ax[RY][RX], Ay[RY][RX];
#pragma unroll
    for (int r = 0; r < RY; ++r)
#pragma unroll
        for (int c = 0; c < RX; ++c) {
            Ax[r][c] = 0.0;
            Ay[r][c] = 0.0;
        }

    if (tid == 0) near_count = 0;
    double bx = 0.0, by = 0.0;  // this thread's share of the block error bound (units of u)
    const double k_term = UNIT ? K_TERM_UNIT : K_TERM_MASS;

    for (int64_t t0 = 0; t0 < a.n_lens; t0 += LENS_TILE) {
        const int cnt = (int)((a.n_lens - t0) < LENS_TILE ? (a.n_lens - t0) : LENS_TILE);
        const int cnt_pad = (cnt + GROUP - 1) / GROUP * GROUP;
        __syncthreads();  // previous tile fully consumed (and near_count initialised)
        stage_tile<UNIT, MODE, BLOCK_THREADS>(a, t0, cnt, cnt_pad, ox, oy, hx, hy, h, near_r2, k_term, sm, tid, bx,
                                              by);
        __syncthreads();

        for (int g = 0; g < cnt_pad; g += GROUP) {
            float sx[RY][RX], sy[RY][RX];
#pragma unroll
            for (int r = 0; r < RY; ++r)
#pragma unroll
                for (int c = 0; c < RX; ++c) {
                    sx[r][c] = 0.0f;
                    sy[r][c] = 0.0f;
                }
            if (UNIT) {
#pragma unroll
                for (int kk = 0; kk < GROUP; kk += 2) {
                    const float4 q = tile[(g + kk) >> 1];
#pragma unroll
                    for (int half = 0; half < 2; ++half) {
                        const float LX = half ? q.z : q.x;
                        const float LY = half ? q.w : q.y;
                        float dy[RY], dy2[RY], dx[RX];
#pragma unroll
                        for (int r = 0; r < RY; ++r) {
                            dy[r] = ryl[r] - LY;
                            dy2[r] = dy[r] * dy[r];
                        }
#pragma unroll
                        for (int c = 0; c < RX; ++c) dx[c] = rxl[c] - LX;
#pragma unroll
                        for (int r = 0; r < RY; ++r)
#pragma unroll
                            for (int c = 0; c < RX; ++c) {
                                const float r2 = __builtin_fmaf(dx[c], dx[c], dy2[r]);
                                const float inv = __builtin_amdgcn_rcpf(r2);
                                sx[r][c] = __builtin_fmaf(dx[c], inv, sx[r][c]);
                                sy[r][c] = __builtin_fmaf(dy[r], inv, sy[r][c]);
                            }
                    }
                }
            } else {
#pragma unroll
                for (int kk = 0; kk < GROUP; ++kk) {
                    const float4 q = tile[g + kk];
                    float dy[RY], dy2[RY], dx[RX];
#pragma unroll
                    for (int r = 0; r < RY; ++r) {
                        dy[r] = ryl[r] - q.y;
                        dy2[r] = dy[r] * dy[r];
                    }
#pragma unroll
                    for (int c = 0; c < RX; ++c) dx[c] = rxl[c] - q.x;
#pragma unroll
                    for (int r = 0; r < RY; ++r)
#pragma unroll
                        for (int c = 0; c < RX; ++c) {
                            const float r2 = __builtin_fmaf(dx[c], dx[c], dy2[r]);
                            const float inv = q.z * __builtin_amdgcn_rcpf(r2);
                            sx[r][c] = __builtin_fmaf(dx[c], inv, sx[r][c]);
                            sy[r][c] = __builtin_fmaf(dy[r], inv, sy[r][c]);
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
        all_flagged = n_near > NEAR_MAX;
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
            const int64_t i = i_lane + c * STRIDE_X, j = j_lane + r * STRIDE_Y;
            const bool valid = (i < a.i1) && (j < a.jc1);
            const double x1 = ray_coord(a.sx0, i, a.spx);
            const double x2 = ray_coord(a.sy0, j, a.spy);
            const double y1 = a.c1 * x1 - Ax[r][c];
            const double y2 = a.c2 * x2 - Ay[r][c];
            const double u = (y1 - a.tx0) * a.inv_pixw;
            const double v = (y2 - a.ty0) * a.inv_pixh;
            int code = classify_ray<MODE>(a, x1, x2, Ax[r][c], Ay[r][c], u, v, rxl[c], ryl[r], Bx, By, n_near,
                                          all_flagged, sm.near_list, k_term, h_f, tiny_r2);
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

// ---------------------------------------------------------------------------
// Random rays (RS_RANDOM_RAYS). The launch's rays are counted into square bins
// of the shooting rectangle, the bins' offsets are scanned, and the rays are
// scattered into bin order (index and FP64 position); then one block deflects
// the rays of one bin, relative to the bin's centre, with the same lens tiles,
// FP32 sum, FP64 folding, error bound and binning as a grid patch. A ray's
// arithmetic depends only on its position and its bin, not on its slot.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int64_t bin_of(const ShootArgs &a, double x1, double x2) {
    int64_t bx = (int64_t)floor((x1 - a.sx0) * a.inv_bw);
    int64_t by = (int64_t)floor((x2 - a.sy0) * a.inv_bh);
    bx = bx < 0 ? 0 : (bx >= a.nbx_r ? a.nbx_r - 1 : bx);
    by = by < 0 ? 0 : (by >= a.nby_r ? a.nby_r - 1 : by);
    return by * a.nbx_r + bx;
}

__global__ __launch_bounds__(256) void rand_count_kernel(const ShootArgs a) {
    const int64_t W = a.i1 - a.i0;
    const int64_t n = (a.jc1 - a.jc0) * W;
    for (int64_t rel = blockIdx.x * (int64_t)256 + threadIdx.x; rel < n; rel += (int64_t)gridDim.x * 256) {
        const int64_t i = a.i0 + rel % W, j = a.jc0 + rel / W;
        double x1, x2;
        random_ray_xy(a.sx0, a.sy0, a.sw, a.sh, a.nx, a.seed, i, j, x1, x2);
        atomicAdd(a.bin_count + bin_of(a, x1, x2), 1u);
    }
}

// Exclusive prefix sums of the bin counts (one block): offset[0..nb], cursor = offset.
__global__ __launch_bounds__(1024) void rand_scan_kernel(const uint32_t *count, int64_t nb, uint32_t *offset,
                                                         uint32_t *cursor) {
    __shared__ uint32_t wsum[16];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t carry = 0;
    for (int64_t base = 0; base < nb; base += 1024) {
        const int64_t k = base + threadIdx.x;
        const uint32_t v = k < nb ? count[k] : 0u;
        uint32_t x = v;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t y = (uint32_t)__shfl_up((int)x, o);
            if (lane >= o) x += y;
        }
        if (lane == 63) wsum[wave] = x;
        __syncthreads();
        if (wave == 0) {
            uint32_t y = lane < 16 ? wsum[lane] : 0u;
#pragma unroll
            for (int o = 1; o < 16; o <<= 1) {
                const uint32_t z = (uint32_t)__shfl_up((int)y, o);
                if (lane >= o) y += z;
            }
            if (lane < 16) wsum[lane] = y;
        }
        __syncthreads();
        const uint32_t excl = carry + (wave ? wsum[wave - 1] : 0u) + x - v;
        if (k < nb) {
            offset[k] = excl;
            cursor[k] = excl;
        }
        carry += wsum[15];
        __syncthreads();
    }
    if (threadIdx.x == 0) offset[nb] = carry;
}

__global__ __launch_bounds__(256) void rand_scatter_kernel(const ShootArgs a) {
    const int64_t W = a.i1 - a.i0;
    const int64_t n = (a.jc1 - a.jc0) * W;
    for (int64_t rel = blockIdx.x * (int64_t)256 + threadIdx.x; rel < n; rel += (int64_t)gridDim.x * 256) {
        const int64_t i = a.i0 + rel % W, j = a.jc0 + rel / W;
        double x1, x2;
        random_ray_xy(a.sx0, a.sy0, a.sw, a.sh, a.nx, a.seed, i, j, x1, x2);
        const uint32_t slot = atomicAdd(a.bin_cursor + bin_of(a, x1, x2), 1u);
        a.ray_rel[slot] = (uint32_t)rel;
        a.ray_x[slot] = x1;
        a.ray_y[slot] = x2;
    }
}

// Up to 64 * WAVES * RR rays of one bin, slots [base, end) of the sorted list;
// (ox, oy) is the bin centre and [ox +- hx] x [oy +- hy] holds every ray of the bin.
template <int RR, int WAVES, bool UNIT, int MODE, bool PIX>
__device__ __forceinline__ void shoot_free_chunk(const ShootArgs &a, uint32_t base, uint32_t end, double ox,
                                                 double oy, double hx, double hy, ShootSmem &sm) {
    constexpr int BLOCK_THREADS = 64 * WAVES;
    const int tid = threadIdx.x;
    const int wave = tid >> 6;
    const int lane = tid & 63;
    __syncthreads();  // the previous chunk of this block is done with the shared buffers
    const double h = sqrt(hx * hx + hy * hy);
    const double near_r2 = 4.0 * h * h;

    float rx[RR], ry[RR];
    double Ax[RR], Ay[RR];
#pragma unroll
    for (int q = 0; q < RR; ++q) {
        const uint32_t slot = base + (uint32_t)(q * BLOCK_THREADS + tid);
        const bool ok = slot < end;
        rx[q] = ok ? (float)(a.ray_x[slot] - ox) : 0.0f;
        ry[q] = ok ? (float)(a.ray_y[slot] - oy) : 0.0f;
        Ax[q] = 0.0;
        Ay[q] = 0.0;
    }

    if (tid == 0) sm.near_count = 0;
    double bx = 0.0, by = 0.0;
    const double k_term = UNIT ? K_TERM_UNIT : K_TERM_MASS;
    float4 *tile = sm.tile;

    for (int64_t t0 = 0; t0 < a.n_lens; t0 += LENS_TILE) {
        const int cnt = (int)((a.n_lens - t0) < LENS_TILE ? (a.n_lens - t0) : LENS_TILE);
        const int cnt_pad = (cnt + GROUP - 1) / GROUP * GROUP;
        __syncthreads();
        stage_tile<UNIT, MODE, BLOCK_THREADS>(a, t0, cnt, cnt_pad, ox, oy, hx, hy, h, near_r2, k_term, sm, tid, bx,
                                              by);
        __syncthreads();
        for (int g = 0; g < cnt_pad; g += GROUP) {
            float sx[RR], sy[RR];
#pragma unroll
            for (int q = 0; q < RR; ++q) {
                sx[q] = 0.0f;
                sy[q] = 0.0f;
            }
            if (UNIT) {
#pragma unroll
                for (int kk = 0; kk < GROUP; kk += 2) {
                    const float4 l2 = tile[(g + kk) >> 1];
#pragma unroll
                    for (int half = 0; half < 2; ++half) {
                        const float LX = half ? l2.z : l2.x;
                        const float LY = half ? l2.w : l2.y;
#pragma unroll
                        for (int q = 0; q < RR; ++q) {
                            const float dx = rx[q] - LX;
                            const float dy = ry[q] - LY;
                            const float dy2 = dy * dy;
                            const float r2 = __builtin_fmaf(dx, dx, dy2);
                            const float inv = __builtin_amdgcn_rcpf(r2);
                            sx[q] = __builtin_fmaf(dx, inv, sx[q]);
                            sy[q] = __builtin_fmaf(dy, inv, sy[q]);
                        }
                    }
                }
            } else {
#pragma unroll
                for (int kk = 0; kk < GROUP; ++kk) {
                    const float4 l = tile[g + kk];
#pragma unroll
                    for (int q = 0; q < RR; ++q) {
                        const float dx = rx[q] - l.x;
                        const float dy = ry[q] - l.y;
                        const float dy2 = dy * dy;
                        const float r2 = __builtin_fmaf(dx, dx, dy2);
                        const float inv = l.z * __builtin_amdgcn_rcpf(r2);
                        sx[q] = __builtin_fmaf(dx, inv, sx[q]);
                        sy[q] = __builtin_fmaf(dy, inv, sy[q]);
                    }
                }
            }
#pragma unroll
            for (int q = 0; q < RR; ++q) {
                Ax[q] += (double)sx[q];
                Ay[q] += (double)sy[q];
            }
        }
    }

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
            sm.red_bx[wave] = bx;
            sm.red_by[wave] = by;
        }
        __syncthreads();
#pragma unroll
        for (int w = 0; w < WAVES; ++w) {
            Bx += sm.red_bx[w];
            By += sm.red_by[w];
        }
        n_near = sm.near_count;
        all_flagged = n_near > NEAR_MAX;
        if (all_flagged) n_near = 0;
    }

    const float h_f = (float)h;
    const float tiny_r2 = 1.0e-6f * h_f * h_f;
    unsigned long long n_in = 0, n_out = 0, n_sing = 0;
    const int64_t W = a.i1 - a.i0;
#pragma unroll
    for (int q = 0; q < RR; ++q) {
        const uint32_t slot = base + (uint32_t)(q * BLOCK_THREADS + tid);
        const bool valid = slot < end;
        const int64_t rel = valid ? (int64_t)a.ray_rel[slot] : 0;
        const int64_t i = a.i0 + rel % W, j = a.jc0 + rel / W;
        const double x1 = valid ? a.ray_x[slot] : ox;
        const double x2 = valid ? a.ray_y[slot] : oy;
        const double y1 = a.c1 * x1 - Ax[q];
        const double y2 = a.c2 * x2 - Ay[q];
        const double u = (y1 - a.tx0) * a.inv_pixw;
        const double v = (y2 - a.ty0) * a.inv_pixh;
        int code = classify_ray<MODE>(a, x1, x2, Ax[q], Ay[q], u, v, rx[q], ry[q], Bx, By, n_near, all_flagged,
                                      sm.near_list, k_term, h_f, tiny_r2);
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
            if (fl) SingleSink{}.append(a, fl, lane, code == FLAGGED, i, j);
        }
    }
    if (lane == 0) {
        if (n_in) atomicAdd(a.counters + C_IN, n_in);
        if (n_out) atomicAdd(a.counters + C_OUT, n_out);
        if (n_sing) atomicAdd(a.counters + C_SING, n_sing);
    }
}

constexpr int FREE_RR = 8;
constexpr int FREE_WAVES = 4;
constexpr int FREE_CAP = 64 * FREE_WAVES * FREE_RR;

// One block per bin; a bin with more rays than one chunk holds takes several passes.
template <bool UNIT, int MODE, bool PIX>
__global__ __launch_bounds__(64 * FREE_WAVES) void shoot_free_kernel(const ShootArgs a) {
    __shared__ ShootSmem sm;
    const int64_t bin = blockIdx.x;
    const uint32_t beg = a.bin_offset[bin], end = a.bin_offset[bin + 1];
    const int64_t bxi = bin % a.nbx_r, byi = bin / a.nbx_r;
    const double ox = a.sx0 + ((double)bxi + 0.5) * a.bw;
    const double oy = a.sy0 + ((double)byi + 0.5) * a.bh;
    // Half-extents with slack for the rounding of positions, bin indices and centres.
    const double hx = 0.5 * a.bw * (1.0 + 1e-6) + 1e-14 * (fabs(a.sx0) + a.sw);
    const double hy = 0.5 * a.bh * (1.0 + 1e-6) + 1e-14 * (fabs(a.sy0) + a.sh);
    for (uint32_t base = beg; base < end; base += (uint32_t)FREE_CAP)
        shoot_free_chunk<FREE_RR, FREE_WAVES, UNIT, MODE, PIX>(a, base, end, ox, oy, hx, hy, sm);
}

// ---------------------------------------------------------------------------
// Far-field expansion (RS_FARFIELD). The paper's tree codes group distant
// lenses into pseudo-lenses with higher multipoles (Section 2, Eq.
// (hierarchical)); here distant lenses enter local expansions of the
// deflection, to order FAR_P, on two levels:
//   * super-patch (FF_SP_X x FF_SP_Y patches, centre zS, half-diagonal H):
//     lenses farther than FAR_RATIO H give C_n = sum_k m_k tS_k^(n+1),
//     tS_k = 1 / (zS - z_k); nearer lenses go to the super-patch's list;
//   * patch (64 x 32 rays, centre z0, half-diagonal h): the super expansion
//     is re-centred exactly on z0 (a polynomial translation), and the listed
//     lenses farther than FAR_RATIO h from z0 add c_n = sum_k m_k t_k^(n+1),
//     t_k = 1 / (z0 - z_k); the rest are summed directly.
// With z = x1 + i x2 and w = z - z0, sum_k m_k / (z - z_k) = sum_n (-w)^n T_n,
// and the deflection (a1, a2) is (Re, -Im) of that sum. All of it is FP64; each
// ray carries a rigorous bound (series truncation on both levels, rounding of
// the coefficients, the translation and the evaluation, the near sum) plus the
// definition's own rounding, and rays within it of a pixel edge go to the FP64
// re-check, so the map equals the definition's.
// ---------------------------------------------------------------------------
constexpr int FAR_P = 16;
constexpr double FAR_RATIO = 4.0;
constexpr int FAR_THREADS = 256;
constexpr int FAR_ROWS = PATCH_X * PATCH_Y / FAR_THREADS;     // rays per thread (8)
static_assert(FAR_ROWS * (FAR_THREADS / 64) == (PATCH_X / 8) * (PATCH_Y / 8), "8 x 8 blocks cover the patch");
constexpr int NEAR_EXP = 512;
constexpr int FAR_EXTRA = 4;                                    // SFAR, TRUNC, SDEF, NFAR
constexpr int FAR_REC = 2 * FAR_P + FAR_EXTRA;
static_assert(FAR_REC == FF_REC_DOUBLES, "super-patch record size");

__device__ __forceinline__ double rcp64(double r2) {
    double rc = __builtin_amdgcn_rcp(r2);
    double e = __builtin_fma(-r2, rc, 1.0);
    rc = __builtin_fma(rc, e, rc);
    e = __builtin_fma(-r2, rc, 1.0);
    return __builtin_fma(rc, e, rc);
}

// One lens's contribution to an expansion about (ox, oy) with half-diagonal h
// (the lens is at least FAR_RATIO h away): the powers m t^(n+1) and the bound
// terms m/|d|, m/|d| rho^P / (1 - rho) and sqrt(2) m / (|d| - h).
struct FarAcc {
    double c1[FAR_P], c2[FAR_P];
    double sfar, trunc, sdef, nfar;
    __device__ void zero() {
#pragma unroll
        for (int n = 0; n < FAR_P; ++n) {
            c1[n] = 0.0;
            c2[n] = 0.0;
        }
        sfar = trunc = sdef = nfar = 0.0;
    }
    __device__ __forceinline__ void add(double d1, double d2, double r2, double m, double h) {
        const double inv = rcp64(r2);
        const double t1 = d1 * inv, t2 = -d2 * inv;   // t = 1 / d, d = centre - lens
        double p1 = m * t1, p2 = m * t2;
        c1[0] += p1;
        c2[0] += p2;
#pragma unroll
        for (int n = 1; n < FAR_P; ++n) {
            const double q1 = __builtin_fma(p1, t1, -p2 * t2);
            const double q2 = __builtin_fma(p1, t2, p2 * t1);
            p1 = q1;
            p2 = q2;
            c1[n] += p1;
            c2[n] += p2;
        }
        const double ad = sqrt(r2);
        const double am = fabs(m);
        const double rho = h / ad;
        const double rho2 = rho * rho, rho4 = rho2 * rho2, rho8 = rho4 * rho4, rho16 = rho8 * rho8;
        sfar += am / ad;
        trunc += am / ad * rho16 / (1.0 - rho);
        sdef += am * 1.4142135623730951 / (ad - h);
        nfar += 1.0;
    }
    // Block sum into out[FAR_REC] (shared); lanes by butterfly, then waves in index order.
    __device__ void reduce(double (*part)[FAR_REC], double *out) {
        const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
            for (int n = 0; n < FAR_P; ++n) {
                c1[n] += __shfl_xor(c1[n], off);
                c2[n] += __shfl_xor(c2[n], off);
            }
            sfar += __shfl_xor(sfar, off);
            trunc += __shfl_xor(trunc, off);
            sdef += __shfl_xor(sdef, off);
            nfar += __shfl_xor(nfar, off);
        }
        if (lane == 0) {
#pragma unroll
            for (int n = 0; n < FAR_P; ++n) {
                part[wave][n] = c1[n];
                part[wave][FAR_P + n] = c2[n];
            }
            part[wave][2 * FAR_P] = sfar;
            part[wave][2 * FAR_P + 1] = trunc;
            part[wave][2 * FAR_P + 2] = sdef;
            part[wave][2 * FAR_P + 3] = nfar;
        }
        __syncthreads();
        if (threadIdx.x < FAR_REC) {
            double v = 0.0;
            for (int w = 0; w < FAR_THREADS / 64; ++w) v += part[w][threadIdx.x];
            out[threadIdx.x] = v;
        }
        __syncthreads();
    }
};

// Geometry of super-patch sp of this launch: centre and half-diagonal (one ray
// spacing of slack on each side), of the full box even where the window clips it.
__device__ __forceinline__ void super_geometry(const ShootArgs &a, int64_t sp, double &cx, double &cy, double &H) {
    const int64_t sx = sp % a.ff_sbx, sy = sp / a.ff_sbx;
    const int64_t i_s = a.i0 + sx * (FF_SP_X * PATCH_X);
    const int64_t j_s = a.jc0 + sy * (FF_SP_Y * PATCH_Y);
    cx = a.sx0 + ((double)i_s + 0.5 * (FF_SP_X * PATCH_X)) * a.spx;
    cy = a.sy0 + ((double)j_s + 0.5 * (FF_SP_Y * PATCH_Y)) * a.spy;
    const double hx = (0.5 * (FF_SP_X * PATCH_X) + 1.0) * a.spx;
    const double hy = (0.5 * (FF_SP_Y * PATCH_Y) + 1.0) * a.spy;
    H = sqrt(hx * hx + hy * hy) * (1.0 + 1e-12);
}

struct FarSuperSmem {
    double part[FAR_THREADS / 64][FAR_REC];
    double out[FAR_REC];
    int count;
};

// Level 1: one block per super-patch. Far lenses -> coefficients C about zS;
// the others -> the super-patch's lens list (a count above FF_NEAR_CAP means
// the list is incomplete and the patches scan every lens instead).
template <bool UNIT>
__global__ __launch_bounds__(FAR_THREADS) void farfield_super_kernel(const ShootArgs a) {
    __shared__ FarSuperSmem sm;
    const int64_t sp = blockIdx.x;
    double cx, cy, H;
    super_geometry(a, sp, cx, cy, H);
    const double near_r2 = (FAR_RATIO * H) * (FAR_RATIO * H);
    int32_t *list = a.ff_near + sp * (int64_t)(1 + FF_NEAR_CAP);
    if (threadIdx.x == 0) sm.count = 0;
    __syncthreads();
    FarAcc acc;
    acc.zero();
    for (int64_t k = threadIdx.x; k < a.n_lens; k += FAR_THREADS) {
        const double X = a.lens_xy[2 * k], Y = a.lens_xy[2 * k + 1];
        const double d1 = cx - X, d2 = cy - Y;
        const double r2 = d1 * d1 + d2 * d2;
        if (!(r2 >= near_r2)) {
            const int q = atomicAdd(&sm.count, 1);
            if (q < FF_NEAR_CAP) list[1 + q] = (int32_t)k;
            continue;
        }
        const double m = (UNIT || a.lens_m == nullptr) ? 1.0 : a.lens_m[k];
        acc.add(d1, d2, r2, m, H);
    }
    acc.reduce(sm.part, sm.out);
    double *rec = a.ff_super + sp * (int64_t)FAR_REC;
    if (threadIdx.x < FAR_REC) rec[threadIdx.x] = sm.out[threadIdx.x];
    if (threadIdx.x == 0) list[0] = sm.count;
}

struct FarSmem {
    double near_x[NEAR_EXP], near_y[NEAR_EXP], near_m[NEAR_EXP];
    int near_count;
    double part[FAR_THREADS / 64][FAR_REC];
    double pc[FAR_REC];          // this patch's own expansion (listed lenses)
    double sc[FAR_REC];          // the super-patch's record
    double tc[2 * FAR_P];        // total coefficients about z0
};

// Level 2: one block per patch.
template <bool UNIT, bool PIX>
__global__ __launch_bounds__(FAR_THREADS) void farfield_kernel(const ShootArgs a) {
    __shared__ FarSmem sm;
    constexpr double U64 = 1.1102230246251565e-16;  // 2^-53
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int64_t patch = blockIdx.x;
    const int64_t pbx = patch % a.nbx, pby = patch / a.nbx;
    const int64_t ib = a.i0 + pbx * PATCH_X;
    const int64_t jb = a.jc0 + pby * PATCH_Y;
    const double ox = a.sx0 + ((double)ib + 0.5 * PATCH_X) * a.spx;
    const double oy = a.sy0 + ((double)jb + 0.5 * PATCH_Y) * a.spy;
    const double hx = (0.5 * PATCH_X + 1.0) * a.spx;
    const double hy = (0.5 * PATCH_Y + 1.0) * a.spy;
    const double h = sqrt(hx * hx + hy * hy) * (1.0 + 1e-12);
    const double near_r2 = (FAR_RATIO * h) * (FAR_RATIO * h);
    // This patch's super-patch.
    const int64_t sp = (pby / FF_SP_Y) * a.ff_sbx + pbx / FF_SP_X;
    double cx, cy, H;
    super_geometry(a, sp, cx, cy, H);
    const double super_r2 = (FAR_RATIO * H) * (FAR_RATIO * H);
    const int32_t *list = a.ff_near + sp * (int64_t)(1 + FF_NEAR_CAP);
    const int32_t listed = list[0];
    const bool scan_all = listed > FF_NEAR_CAP;
    if (tid == 0) sm.near_count = 0;
    if (tid < FAR_REC) sm.sc[tid] = a.ff_super[sp * (int64_t)FAR_REC + tid];
    __syncthreads();

    // The super-patch's nearer lenses: far from this patch -> its own expansion; else direct.
    FarAcc acc;
    acc.zero();
    const int64_t n_cand = scan_all ? a.n_lens : (int64_t)listed;
    for (int64_t q = tid; q < n_cand; q += FAR_THREADS) {
        const int64_t k = scan_all ? q : (int64_t)list[1 + q];
        const double X = a.lens_xy[2 * k], Y = a.lens_xy[2 * k + 1];
        if (scan_all) {   // the same test the super kernel made
            const double e1 = cx - X, e2 = cy - Y;
            if (e1 * e1 + e2 * e2 >= super_r2) continue;
        }
        const double m = (UNIT || a.lens_m == nullptr) ? 1.0 : a.lens_m[k];
        const double d1 = ox - X, d2 = oy - Y;
        const double r2 = d1 * d1 + d2 * d2;
        if (!(r2 >= near_r2)) {
            const int j = atomicAdd(&sm.near_count, 1);
            if (j < NEAR_EXP) {
                sm.near_x[j] = X;
                sm.near_y[j] = Y;
                sm.near_m[j] = m;
            }
            continue;
        }
        acc.add(d1, d2, r2, m, h);
    }
    acc.reduce(sm.part, sm.pc);

    // Re-centre the super expansion: sum_n C_n (e + v)^n = sum_m v^m sum_{n>=m} binom(n,m) e^(n-m) C_n,
    // v = -w = z0 - z, e = zS - z0; then add this patch's own coefficients.
    if (tid < FAR_P) {
        const int mm = tid;
        const double e1 = cx - ox, e2 = cy - oy;
        double s1 = 0.0, s2 = 0.0;
        double g1 = 1.0, g2 = 0.0;   // e^(n-m)
        double binom = 1.0;          // binom(n, m), exact in FP64 for n < 16
        for (int n = mm; n < FAR_P; ++n) {
            s1 = __builtin_fma(binom, g1 * sm.sc[n] - g2 * sm.sc[FAR_P + n], s1);
            s2 = __builtin_fma(binom, g1 * sm.sc[FAR_P + n] + g2 * sm.sc[n], s2);
            const double q1 = g1 * e1 - g2 * e2, q2 = g1 * e2 + g2 * e1;
            g1 = q1;
            g2 = q2;
            binom = binom * (double)(n + 1) / (double)(n + 1 - mm);
        }
        sm.tc[mm] = s1 + sm.pc[mm];
        sm.tc[FAR_P + mm] = s2 + sm.pc[FAR_P + mm];
    }
    __syncthreads();
    const double SFAR_S = sm.sc[2 * FAR_P], TRUNC_S = sm.sc[2 * FAR_P + 1], SDEF_S = sm.sc[2 * FAR_P + 2];
    const double NFAR_S = sm.sc[2 * FAR_P + 3];
    const double SFAR_P = sm.pc[2 * FAR_P], TRUNC_P = sm.pc[2 * FAR_P + 1], SDEF_P = sm.pc[2 * FAR_P + 2];
    const double NFAR_P = sm.pc[2 * FAR_P + 3];
    const int n_near_all = sm.near_count;
    const bool all_flagged = n_near_all > NEAR_EXP;
    const int n_near = all_flagged ? 0 : n_near_all;
    const double SFAR = SFAR_S + SFAR_P;
    // Our own far-field error: truncation on both levels; rounding of the coefficients,
    // the translation and the evaluation (per-level factors, generous constants).
    const double far_err = TRUNC_S + TRUNC_P + (NFAR_S + 24.0 * FAR_P + 64.0) * U64 * 1.34 * SFAR_S +
                           (NFAR_P + 16.0 * FAR_P + 64.0) * U64 * 1.34 * SFAR_P;
    const double kN = ((double)a.n_lens + 10.0) * U64 * 1.001;
    const double SDEF = SDEF_S + SDEF_P;

    unsigned long long n_in = 0, n_out = 0;
    const int64_t W = a.i1 - a.i0;
    // A wave takes 8 x 8-ray blocks of the patch (block wave + 4 r, r < 8), so the
    // rays of one wave land on few pixels and the binning atomics aggregate well.
    const int wave = tid >> 6;
#pragma unroll 1
    for (int r = 0; r < FAR_ROWS; ++r) {
        const int b = wave + (FAR_THREADS / 64) * r;
        const int64_t i = ib + 8 * (b % (PATCH_X / 8)) + (lane & 7);
        const int64_t j = jb + 8 * (b / (PATCH_X / 8)) + (lane >> 3);
        const bool valid = (i < a.i1) && (j < a.jc1);
        const double x1 = ray_coord(a.sx0, i, a.spx);
        const double x2 = ray_coord(a.sy0, j, a.spy);
        const double nw1 = ox - x1, nw2 = oy - x2;   // -w
        double S1 = sm.tc[FAR_P - 1], S2 = sm.tc[2 * FAR_P - 1];
#pragma unroll
        for (int n = FAR_P - 2; n >= 0; --n) {
            const double q1 = __builtin_fma(S1, nw1, __builtin_fma(-S2, nw2, sm.tc[n]));
            const double q2 = __builtin_fma(S1, nw2, __builtin_fma(S2, nw1, sm.tc[FAR_P + n]));
            S1 = q1;
            S2 = q2;
        }
        double a1 = S1, a2 = -S2;
        double snear = 0.0;
        bool tiny = false;
        for (int q = 0; q < n_near; ++q) {
            const double e1 = x1 - sm.near_x[q], e2 = x2 - sm.near_y[q];
            const double r2 = __builtin_fma(e1, e1, e2 * e2);
            tiny |= !(r2 > 1e-200);
            const double f = sm.near_m[q] * rcp64(r2);
            a1 = __builtin_fma(f, e1, a1);
            a2 = __builtin_fma(f, e2, a2);
            snear = __builtin_fma(fabs(e1) + fabs(e2), fabs(f), snear);
        }
        const double y1 = a.c1 * x1 - a1;
        const double y2 = a.c2 * x2 - a2;
        const double u = (y1 - a.tx0) * a.inv_pixw;
        const double v = (y2 - a.ty0) * a.inv_pixh;
        // Error bound in source units: ours (far field, near sum and its additions onto
        // the far sum, epilogue) and the definition's own lens-order rounding.
        const double near_err =
            ((double)n_near + 10.0) * U64 * 1.001 * snear + (double)n_near * U64 * 1.34 * SFAR;
        const double def_sum = kN * (snear + SDEF);
        const double eu = far_err + near_err + def_sum + 16.0 * U64 * (fabs(a.c1 * x1) + fabs(a1) + fabs(a.tx0));
        const double ev = far_err + near_err + def_sum + 16.0 * U64 * (fabs(a.c2 * x2) + fabs(a2) + fabs(a.ty0));
        const double Mu = 1.001 * eu * a.inv_pixw, Mv = 1.001 * ev * a.inv_pixh;
        const double fu = floor(u), fv = floor(v);
        const bool ok_u = (fmin(u - fu, fu + 1.0 - u) > Mu) && (fu >= 0.0) && (fu < (double)a.npx);
        const bool ok_v = (fmin(v - fv, fv + 1.0 - v) > Mv) && (fv >= 0.0) && (fv < (double)a.npy);
        const bool out_u = (u < -Mu) || (u > (double)a.npx + Mu);
        const bool out_v = (v < -Mv) || (v > (double)a.npy + Mv);
        const bool sane = !tiny && !all_flagged && isfinite(Mu) && isfinite(Mv) && isfinite(u) && isfinite(v);
        int code;
        if (sane && ok_u && ok_v) code = (int)((int64_t)fv * a.npx + (int64_t)fu);
        else if (sane && (out_u || out_v)) code = OUT;
        else code = FLAGGED;
        if (!valid) code = INT32_MIN;

        n_in += __builtin_popcountll(__ballot(code >= 0));
        n_out += __builtin_popcountll(__ballot(code == OUT));
        if (PIX) {
            if (valid && code != FLAGGED) a.pix_out[(j - a.j0) * W + (i - a.i0)] = code;
        } else {
            aggregated_add(a.map, code);
        }
        const uint64_t fl = __ballot(code == FLAGGED);
        if (fl) SingleSink{}.append(a, fl, lane, code == FLAGGED, i, j);
    }
    if (lane == 0) {
        if (n_in) atomicAdd(a.counters + C_IN, n_in);
        if (n_out) atomicAdd(a.counters + C_OUT, n_out);
    }
}

// Single map: one block per patch of this launch's rows.
template <int RX, int RY, int WX, int WY, bool UNIT, int MODE, bool PIX>
__global__ __launch_bounds__(64 * WX * WY) void shoot_kernel(const ShootArgs a) {
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

// Resident blocks of a persistent kernel: every CU times the blocks that fit on it.
template <class K>
static int resident_blocks(K kernel, int threads) {
    static int n_cu = 0;
    if (n_cu == 0) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n_cu <= 0)
            n_cu = 256;
    }
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0) != hipSuccess || per_cu <= 0)
        per_cu = 2;
    return n_cu * per_cu;
}

template <int RX, int RY, int WX, int WY, bool UNIT, int MODE>
static void launch_batch_variant(const BatchArgs &b, int grid_blocks, hipStream_t stream) {
    const int threads = 64 * WX * WY;
    auto k = shoot_batch_kernel<RX, RY, WX, WY, UNIT, MODE>;
    if (grid_blocks <= 0) grid_blocks = resident_blocks(k, threads);
    if ((int64_t)grid_blocks > b.total_tiles) grid_blocks = (int)b.total_tiles;
    hipLaunchKernelGGL(k, dim3((unsigned)grid_blocks), dim3(threads), 0, stream, b);
}

template <int RX, int RY, int WX, int WY>
static void launch_batch_shape(const BatchArgs &b, int grid_blocks, hipStream_t stream) {
    if (b.unit_masses) {
        if (b.mode == 0) launch_batch_variant<RX, RY, WX, WY, true, 0>(b, grid_blocks, stream);
        else launch_batch_variant<RX, RY, WX, WY, true, 1>(b, grid_blocks, stream);
    } else {
        if (b.mode == 0) launch_batch_variant<RX, RY, WX, WY, false, 0>(b, grid_blocks, stream);
        else launch_batch_variant<RX, RY, WX, WY, false, 1>(b, grid_blocks, stream);
    }
}

hipError_t launch_shoot_batch(const BatchArgs &b, int shape, int grid_blocks, hipStream_t stream) {
    if (b.total_tiles <= 0) return hipSuccess;
    switch (shape) {
        case 1: launch_batch_shape<4, 4, 2, 1>(b, grid_blocks, stream); break;
        case 2: launch_batch_shape<8, 2, 1, 2>(b, grid_blocks, stream); break;
        case 3: launch_batch_shape<8, 4, 1, 1>(b, grid_blocks, stream); break;
        default: launch_batch_shape<4, 2, 2, 2>(b, grid_blocks, stream); break;
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

hipError_t launch_farfield(const ShootArgs &a, hipStream_t stream) {
    const int64_t rows = a.jc1 - a.jc0;
    const int64_t nby = (rows + PATCH_Y - 1) / PATCH_Y;
    const int64_t patches = a.nbx * nby;
    if (patches <= 0) return hipSuccess;
    const int64_t n_super = a.ff_sbx * ((nby + FF_SP_Y - 1) / FF_SP_Y);
    const bool unit = a.lens_m == nullptr;
    const bool pix = a.pix_out != nullptr;
    const dim3 block(FAR_THREADS);
    if (unit) hipLaunchKernelGGL((farfield_super_kernel<true>), dim3((unsigned)n_super), block, 0, stream, a);
    else hipLaunchKernelGGL((farfield_super_kernel<false>), dim3((unsigned)n_super), block, 0, stream, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const dim3 grid((unsigned)patches);
    if (unit) {
        if (pix) hipLaunchKernelGGL((farfield_kernel<true, true>), grid, block, 0, stream, a);
        else hipLaunchKernelGGL((farfield_kernel<true, false>), grid, block, 0, stream, a);
    } else {
        if (pix) hipLaunchKernelGGL((farfield_kernel<false, true>), grid, block, 0, stream, a);
        else hipLaunchKernelGGL((farfield_kernel<false, false>), grid, block, 0, stream, a);
    }
    return hipGetLastError();
}

hipError_t launch_shoot_random(const ShootArgs &a, int mode, hipStream_t stream) {
    const int64_t n = (a.jc1 - a.jc0) * (a.i1 - a.i0);
    const int64_t nb = a.nbx_r * a.nby_r;
    if (n <= 0) return hipSuccess;
    hipError_t e = launch_zero(a.bin_count, nb, stream);
    if (e != hipSuccess) return e;
    const int64_t want = (n + 255) / 256;
    const int blocks = (int)(want < 8192 ? want : 8192);
    hipLaunchKernelGGL(rand_count_kernel, dim3(blocks), dim3(256), 0, stream, a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(rand_scan_kernel, dim3(1), dim3(1024), 0, stream, (const uint32_t *)a.bin_count, nb,
                       a.bin_offset, a.bin_cursor);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(rand_scatter_kernel, dim3(blocks), dim3(256), 0, stream, a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const bool unit = a.lens_m == nullptr;
    const bool pix = a.pix_out != nullptr;
    const dim3 grid((unsigned)nb), block(64 * FREE_WAVES);
#define RS_FREE(U, M, P) hipLaunchKernelGGL((shoot_free_kernel<U, M, P>), grid, block, 0, stream, a)
    if (mode == RS_MIXED) {
        if (unit) { if (pix) RS_FREE(true, 1, true); else RS_FREE(true, 1, false); }
        else { if (pix) RS_FREE(false, 1, true); else RS_FREE(false, 1, false); }
    } else {
        if (unit) { if (pix) RS_FREE(true, 0, true); else RS_FREE(true, 0, false); }
        else { if (pix) RS_FREE(false, 0, true); else RS_FREE(false, 0, false); }
    }
#undef RS_FREE
    return hipGetLastError();
}

}  // namespace rs
