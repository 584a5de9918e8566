// Device helpers shared by the deflection kernels (regular grid, random rays,
// far field): error-bound constants, ray positions, wave-aggregated binning,
// re-check sinks, lens staging with the per-lens FP32 bound, and the per-ray
// classification against a pixel edge.
#pragma once

#include "recheck_ray.h"

namespace rs {
namespace {


constexpr double U32 = 5.9604644775390625e-08;  // 2^-24, FP32 unit roundoff

// Per-lens FP32 error constants (derivation in the design notes):
//   |t_hat - t| <= u m (K_TERM |dx| + K_H h) / r^2 for one term t = m dx / r^2,
//   the FP32 group sum adds u (GROUP - pos) |t_hat| for the lens at position pos.
// Unit masses: K_TERM covers dx (2.04u), r^2 (6.08u + 4.08u h/r) and the reciprocal,
// shared by two terms (two rays of one lens on the grid, two lenses of one ray for
// random rays): b * rcp(a * b) is within 4u of 1/a (the product, v_rcp_f32's 1 ulp,
// the final multiply); with masses the FP32 mass rounding and the mass multiply
// add 2u.
constexpr double K_TERM_UNIT = 12.5;
constexpr double K_TERM_MASS = 15.0;
// Regular-grid unit-mass loop: one reciprocal for four rays (two rows of two
// columns) through the product of their r^2; b * (rcp(P) * cd) with
// P = (a b)(c d) is within 6u of 1/a (three products, the reciprocal, two
// multiplies; the rounding of c d cancels), so the term constant grows by 2.
constexpr double K_TERM_QUAD = 14.5;
constexpr double K_TERM_MASS_QUAD = 17.0;   // the same with masses (+2u)
// Range of the four-ray product P = r_a^2 r_b^2 r_c^2 r_d^2 in FP32: a tile whose
// lenses all lie within QUAD_RANGE of the patch centre on both axes, in a patch
// of half-diagonal h in [QUAD_H_MIN, QUAD_H_MAX], keeps P below 2^110 (no
// overflow); lenses outside the near list are at least 2h from every ray, so P
// stays above 256 h^8 >= 2^-100 (normal, with room); near lenses are checked per
// ray. Other tiles and patches use the two-ray form.
constexpr double QUAD_RANGE = 8192.0;
constexpr double QUAD_H_MIN = 1.0e-4;
constexpr double QUAD_H_MAX = 1024.0;
constexpr double QUAD_P_MIN = 7.888609052210118e-31;   // 2^-100
constexpr double K_GROUP = 1.01;
constexpr double K_H = 6.5;

constexpr double PAD_OFFSET = 1.0e9;   // exactly representable in FP32

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

// A block's counts per pixel in LDS (open addressing on the pixel index): rays add
// with LDS atomics, and the block then adds each distinct pixel's count to the map
// with one global atomic. A ray whose pixel finds no free slot within PT_PROBES
// probes adds to the map directly. Counts are integers, so the map does not depend
// on the order of the additions.
constexpr int PT_SLOTS = 2048;
constexpr int PT_PROBES = 8;
struct PixelTable {
    uint32_t key[PT_SLOTS];   // pixel + 1; 0 = empty
    uint32_t cnt[PT_SLOTS];
};

template <int THREADS>
__device__ __forceinline__ void table_clear(PixelTable &t, int tid) {
    for (int s = tid; s < PT_SLOTS; s += THREADS) {
        t.key[s] = 0u;
        t.cnt[s] = 0u;
    }
}

// Count one ray in pixel p (p < 0: nothing to count).
__device__ __forceinline__ void table_add(PixelTable &t, uint32_t *map, int p) {
    if (p < 0) return;
    const uint32_t k = (uint32_t)p + 1u;
    uint32_t s = (k * 2654435761u) >> 21;   // multiplicative hash onto 2^11 slots
    for (int probe = 0; probe < PT_PROBES; ++probe) {
        const uint32_t old = atomicCAS(&t.key[s], 0u, k);
        if (old == 0u || old == k) {
            atomicAdd(&t.cnt[s], 1u);
            return;
        }
        s = (s + 1u) & (PT_SLOTS - 1);
    }
    global_add(map + p, 1u);
}
static_assert(PT_SLOTS == 1 << 11, "the hash keeps 11 bits");

// Adds every used slot's count to the map and empties the slot (a slot holds a
// key exactly when its count is positive). All slots' counts and keys are read
// before the first global atomic is issued. The caller separates this from the
// table's last and next use by barriers.
template <int THREADS>
__device__ __forceinline__ void table_flush_clear(PixelTable &t, uint32_t *map, int tid) {
    static_assert(PT_SLOTS % THREADS == 0, "whole rounds of slots");
    constexpr int R = PT_SLOTS / THREADS;
    uint32_t c[R], k[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        c[r] = t.cnt[tid + r * THREADS];
        k[r] = t.key[tid + r * THREADS];
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if (c[r]) {
            t.cnt[tid + r * THREADS] = 0u;
            t.key[tid + r * THREADS] = 0u;
            global_add(map + (k[r] - 1u), c[r]);
        }
    }
}

struct ShootSmem {
    float4 tile[LENS_TILE];        // UNIT: two (x,y) pairs per float4; else (x,y,m,0)
    NearLens near_list[NEAR_MAX];
    int near_count;
    int far_tile;                  // last tile (index) with a lens beyond QUAD_RANGE of the patch centre
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
// from the block origin (ox, oy), padded to whole half groups with lenses at
// offset (PAD_OFFSET, 0): massless where masses are stored; with unit masses
// each adds at most 1/(PAD_OFFSET - hx) to a ray's deflection, which mixed mode
// adds to the bound (far enough to be negligible, near enough that a product
// of two r^2 stays finite). Mixed mode: lenses within 2h of the block's box go to the near list
// (bounded per ray later); the others add their rigorous FP32 error weight for
// any ray in the box [ox +- hx] x [oy +- hy] to this thread's share (bx, by).
template <bool UNIT, int MODE, int BLOCK_THREADS>
__device__ __forceinline__ void stage_tile(const ShootArgs &a, int64_t t0, int cnt, int cnt_pad, double ox, double oy,
                                           double hx, double hy, double h, double near_r2, double k_term,
                                           ShootSmem &sm, int tid, double &bx, double &by) {
    float4 *tile = sm.tile;
        for (int s = tid; s < cnt_pad; s += BLOCK_THREADS) {
            float fx = (float)PAD_OFFSET, fy = 0.0f, fm = 0.0f;  // padding lens
            if (s < cnt) {
                const int64_t k = t0 + s;
                // global-address-space reads (a batch descriptor's pointers are generic)
                const double X = ((global_double *)a.lens_xy)[2 * k];
                const double Y = ((global_double *)a.lens_xy)[2 * k + 1];
                const double m = (UNIT || a.lens_m == nullptr) ? 1.0 : ((global_double *)a.lens_m)[k];
                const double Lx = X - ox, Ly = Y - oy;
                fx = (float)Lx;
                fy = (float)Ly;
                fm = (float)m;
                // (every thread that finds one writes the same value)
                if (!(fmax(fabs(Lx), fabs(Ly)) <= QUAD_RANGE)) sm.far_tile = (int)(t0 / LENS_TILE);
                if (MODE == 1) {
                    const double alx = fabs(Lx), aly = fabs(Ly);
                    const double ex = fmax(alx - hx, 0.0), ey = fmax(aly - hy, 0.0);
                    const double dmin2 = ex * ex + ey * ey;
                    const int pos = s % GROUP;
                    // A lens beyond 1e9 could overflow the paired products of r^2: the
                    // block's rays all go to the FP64 re-check instead.
                    if (fmax(alx, aly) > 1.0e9) atomicAdd(&sm.near_count, NEAR_MAX + 1);
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
            } else if (MODE == 1 && UNIT) {
                // a unit-mass padding lens's whole term, in units of u
                const double d = PAD_OFFSET - hx;
                bx += 1.0 / (d * U32);
                by += hy / (d * d * U32);
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
// within it of a pixel edge is FLAGGED for the FP64 re-check. (rxp, ryp) is the
// ray whose reciprocals this one's share: a near lens almost on either of the
// two flags it (their product of r^2 could underflow). With quad set, the ray
// also shares reciprocals with the two rays of column rxq (rows ry and ryp), and
// a near lens whose four r^2, or either pair of them, multiply to less than
// QUAD_P_MIN flags it too. A ray with a non-finite position is never counted
// out, only flagged.
template <int MODE>
__device__ __forceinline__ int classify_ray(const ShootArgs &a, double x1, double x2, double Axv, double Ayv, double u,
                                            double v, float rx, float ry, float rxp, float ryp, float rxq, bool quad,
                                            double Bx, double By, int n_near,
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
            const float dxp = rxp - nl.x, dyp = ryp - nl.y;
            const float r2p = dxp * dxp + dyp * dyp;
            const float wgt = (float)(k_term + K_GROUP * (double)(GROUP - nl.pos));
            bool quad_ok = true;
            if (quad) {
                const float dxq = rxq - nl.x;
                const double r2q = (double)(dxq * dxq + dyn * dyn), r2qp = (double)(dxq * dxq + dyp * dyp);
                const double pa = (double)r2n * (double)r2p, pc = r2q * r2qp;
                quad_ok = pa > QUAD_P_MIN && pc > QUAD_P_MIN && pa * pc > QUAD_P_MIN;
            }
            if (!(r2n > tiny_r2) || !(r2p > tiny_r2) || !quad_ok) {
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
        const bool fin = isfinite(u) && isfinite(v);
        const bool out_u = (u < -Eu) || (u > (double)a.npx + Eu);
        const bool out_v = (v < -Ev) || (v > (double)a.npy + Ev);
        if (all_flagged) code = FLAGGED;
        else if (ok_u && ok_v) code = (int)((int64_t)fv * a.npx + (int64_t)fu);
        else if (fin && (out_u || out_v)) code = OUT;
        else code = FLAGGED;
    }
    return code;
}

}  // namespace
}  // namespace rs
