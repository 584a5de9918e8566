// Random ray positions (RS_RANDOM_RAYS): count the launch's rays into square bins
// of the shooting rectangle, scan, scatter them into bin order, deflect bin by bin.
#include "shoot_common.h"

namespace rs {
namespace {

// ---------------------------------------------------------------------------
// Random rays (RS_RANDOM_RAYS). The launch's rays are counted into square bins
// of the shooting rectangle, the bins' offsets are scanned, and the rays are
// scattered into bin order (index and FP64 position); then one block deflects
// the rays of one bin, relative to the bin's centre, with the same lens tiles,
// FP32 sum, FP64 folding, error bound and binning as a grid patch (the shared
// reciprocal pairs two lenses of a ray rather than two rays). A ray's
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

// FP32 sums over the N lenses of tile entries g .. g+N-1 for RR rays with no
// shared rows or columns (per ray dx, dy, dy^2, r^2, reciprocal, two FMAs),
// folded into the FP64 accumulators. Unit masses: the two lenses of one LDS
// read share one v_rcp_f32 per ray, of the product of the ray's two r^2 (a
// ray's arithmetic must not depend on its slot, which the scatter's atomics set).
template <int N, int RR, bool UNIT>
__device__ __forceinline__ void free_group_sums(const float4 *tile, int g, const float (&rx)[RR],
                                                const float (&ry)[RR], double (&Ax)[RR], double (&Ay)[RR]) {
    float sx[RR], sy[RR];
#pragma unroll
    for (int q = 0; q < RR; ++q) {
        sx[q] = 0.0f;
        sy[q] = 0.0f;
    }
    if (UNIT) {
#pragma unroll
        for (int kk = 0; kk < N; kk += 2) {
            const float4 l2 = tile[(g + kk) >> 1];   // lenses g+kk (x, y) and g+kk+1 (z, w)
#pragma unroll
            for (int q = 0; q < RR; ++q) {
                const float dxa = rx[q] - l2.x, dya = ry[q] - l2.y;
                const float dxb = rx[q] - l2.z, dyb = ry[q] - l2.w;
                const float ra = __builtin_fmaf(dxa, dxa, dya * dya);
                const float rb = __builtin_fmaf(dxb, dxb, dyb * dyb);
                const float rab = __builtin_amdgcn_rcpf(ra * rb);
                const float ia = rb * rab, ib = ra * rab;
                sx[q] = __builtin_fmaf(dxa, ia, sx[q]);
                sy[q] = __builtin_fmaf(dya, ia, sy[q]);
                sx[q] = __builtin_fmaf(dxb, ib, sx[q]);
                sy[q] = __builtin_fmaf(dyb, ib, sy[q]);
            }
        }
    } else {
#pragma unroll
        for (int kk = 0; kk < N; kk += 2) {
            const float4 la = tile[g + kk], lb = tile[g + kk + 1];
#pragma unroll
            for (int q = 0; q < RR; ++q) {
                const float dxa = rx[q] - la.x, dya = ry[q] - la.y;
                const float dxb = rx[q] - lb.x, dyb = ry[q] - lb.y;
                const float ra = __builtin_fmaf(dxa, dxa, dya * dya);
                const float rb = __builtin_fmaf(dxb, dxb, dyb * dyb);
                const float rab = __builtin_amdgcn_rcpf(ra * rb);
                const float ia = la.z * (rb * rab), ib = lb.z * (ra * rab);
                sx[q] = __builtin_fmaf(dxa, ia, sx[q]);
                sy[q] = __builtin_fmaf(dya, ia, sy[q]);
                sx[q] = __builtin_fmaf(dxb, ib, sx[q]);
                sy[q] = __builtin_fmaf(dyb, ib, sy[q]);
            }
        }
    }
#pragma unroll
    for (int q = 0; q < RR; ++q) {
        Ax[q] += (double)sx[q];
        Ay[q] += (double)sy[q];
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
        const int cnt_pad = (cnt + GROUP / 2 - 1) / (GROUP / 2) * (GROUP / 2);
        __syncthreads();
        stage_tile<UNIT, MODE, BLOCK_THREADS>(a, t0, cnt, cnt_pad, ox, oy, hx, hy, h, near_r2, k_term, sm, tid, bx,
                                              by);
        __syncthreads();
        // Whole groups in the loop; the last tile may end with half a group, summed after it.
        const int full = cnt_pad / GROUP * GROUP;
        for (int g = 0; g < full; g += GROUP) free_group_sums<GROUP, RR, UNIT>(tile, g, rx, ry, Ax, Ay);
        if (full < cnt_pad) free_group_sums<GROUP / 2, RR, UNIT>(tile, full, rx, ry, Ax, Ay);
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
        // (a bin under 1e-6 across could underflow the paired products of r^2)
        all_flagged = n_near > NEAR_MAX || h < 1.0e-6;
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
        // reciprocals are shared between two lenses of one ray, not between rays
        int code = classify_ray<MODE>(a, x1, x2, Ax[q], Ay[q], u, v, rx[q], ry[q], rx[q], ry[q], rx[q], false, Bx, By,
                                      n_near, all_flagged, sm.near_list, k_term, h_f, tiny_r2);
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

}  // namespace

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
