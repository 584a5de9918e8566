// FP64 far-field pieces shared by the far-field mode (farfield.hip) and the
// mixed mode's far-field re-check stage (single maps in farfield.hip, batches
// in recheck.hip): constants of the expansion, the super-patch geometry, the
// Newton-refined reciprocal, the per-ray decision against the rigorous bound,
// and the evaluation of one ray from its super-patch record and lens list.
#pragma once

#include "shoot_common.h"

namespace rs {
namespace {

constexpr int FAR_P = 16;                 // expansion order
constexpr double FAR_RATIO = 4.0;         // lenses beyond FAR_RATIO half-diagonals are expanded
constexpr int FAR_EXTRA = 4;              // SFAR, TRUNC, SDEF, NFAR
constexpr int FAR_REC = 2 * FAR_P + FAR_EXTRA;
static_assert(FAR_REC == FF_REC_DOUBLES, "super-patch record size");

__device__ __forceinline__ double rcp64(double r2) {
    double rc = __builtin_amdgcn_rcp(r2);
    double e = __builtin_fma(-r2, rc, 1.0);
    rc = __builtin_fma(rc, e, rc);
    e = __builtin_fma(-r2, rc, 1.0);
    return __builtin_fma(rc, e, rc);
}

// 1/sqrt(x) for normal positive x: v_rsq_f64 and two Newton steps
// y <- y + y (1/2 - (x/2) y^2).
__device__ __forceinline__ double rsq64(double x) {
    double y = __builtin_amdgcn_rsq(x);
    const double hx = 0.5 * x;
    double e = __builtin_fma(-hx * y, y, 0.5);
    y = __builtin_fma(y, e, y);
    e = __builtin_fma(-hx * y, y, 0.5);
    return __builtin_fma(y, e, y);
}

// Geometry of super-patch sp: centre and half-diagonal (one ray spacing of
// slack on each side), of the full box even where the window clips it.
__device__ __forceinline__ void super_geometry(const ShootArgs &a, int64_t sp, double &cx, double &cy, double &H) {
    const int64_t sx = sp % a.ff_sbx, sy = sp / a.ff_sbx;
    const int64_t i_s = a.ff_i0 + sx * (FF_SP_X * PATCH_X);
    const int64_t j_s = a.ff_j0 + sy * (FF_SP_Y * PATCH_Y);
    cx = a.sx0 + ((double)i_s + 0.5 * (FF_SP_X * PATCH_X)) * a.spx;
    cy = a.sy0 + ((double)j_s + 0.5 * (FF_SP_Y * PATCH_Y)) * a.spy;
    const double hx = (0.5 * (FF_SP_X * PATCH_X) + 1.0) * a.spx;
    const double hy = (0.5 * (FF_SP_Y * PATCH_Y) + 1.0) * a.spy;
    H = sqrt(hx * hx + hy * hy) * (1.0 + 1e-12);
}

// Pixel decision of one ray from its FP64 deflection (a1, a2) = expansion +
// directly summed lenses. Bound terms in source units: far_err (truncation and
// rounding of the expansion), SFAR (sum of |m|/|d| over the expanded lenses,
// which bounds the far sum by 1.34 SFAR), SDEF (the definition's rounding
// weight of those lenses), snear and n_near (the direct sum, with its additions
// onto the far sum), plus the definition's own lens-order rounding and the
// epilogue. Returns the pixel, OUT, or FLAGGED.
__device__ __forceinline__ int far_decide(const ShootArgs &a, double x1, double x2, double a1, double a2,
                                          double far_err, double SFAR, double SDEF, double snear, int n_near,
                                          bool sane_in) {
    constexpr double U64 = 1.1102230246251565e-16;  // 2^-53
    const double kN = ((double)a.n_lens + 10.0) * U64 * 1.001;
    const double y1 = a.c1 * x1 - a1;
    const double y2 = a.c2 * x2 - a2;
    const double u = (y1 - a.tx0) * a.inv_pixw;
    const double v = (y2 - a.ty0) * a.inv_pixh;
    const double near_err = ((double)n_near + 10.0) * U64 * 1.001 * snear + (double)n_near * U64 * 1.34 * SFAR;
    const double def_sum = kN * (snear + SDEF);
    const double eu = far_err + near_err + def_sum + 16.0 * U64 * (fabs(a.c1 * x1) + fabs(a1) + fabs(a.tx0));
    const double ev = far_err + near_err + def_sum + 16.0 * U64 * (fabs(a.c2 * x2) + fabs(a2) + fabs(a.ty0));
    const double Mu = 1.001 * eu * a.inv_pixw, Mv = 1.001 * ev * a.inv_pixh;
    const double fu = floor(u), fv = floor(v);
    const bool ok_u = (fmin(u - fu, fu + 1.0 - u) > Mu) && (fu >= 0.0) && (fu < (double)a.npx);
    const bool ok_v = (fmin(v - fv, fv + 1.0 - v) > Mv) && (fv >= 0.0) && (fv < (double)a.npy);
    const bool out_u = (u < -Mu) || (u > (double)a.npx + Mu);
    const bool out_v = (v < -Mv) || (v > (double)a.npy + Mv);
    const bool sane = sane_in && isfinite(Mu) && isfinite(Mv) && isfinite(u) && isfinite(v);
    if (sane && ok_u && ok_v) return (int)((int64_t)fv * a.npx + (int64_t)fu);
    if (sane && (out_u || out_v)) return OUT;
    return FLAGGED;
}

// Far-field arguments of one map of a batch: the whole window is one launch.
__device__ inline ShootArgs batch_far_args(const BatchMap &m) {
    ShootArgs a = shoot_args_of(m.p, m.lens_xy, m.lens_m, m.n_lens, m.map, m.counters);
    a.ff_sbx = m.ff_sbx;
    a.ff_i0 = m.p.i0;
    a.ff_j0 = m.p.j0;
    a.ff_super = m.ff_super;
    a.ff_near = m.ff_near;
    a.ff_cap = FF_BATCH_CAP;
    return a;
}

// Re-check stage F for one ray at (x1, x2) inside super-patch sp: the
// super-patch's series (Horner in -w = zS - z, the series the patch kernel
// re-centres) plus its listed lenses summed directly in FP64, under the patch
// kernel's bound with no patch level. Returns the definition's pixel or OUT,
// or FLAGGED when the bound reaches a pixel edge, the ray sits on a listed
// lens, or the list overflowed.
template <bool UNIT>
__device__ inline int far_eval(const ShootArgs &a, int64_t sp, double x1, double x2) {
    constexpr double U64 = 1.1102230246251565e-16;  // 2^-53
    const int32_t *list = a.ff_near + sp * (int64_t)(1 + a.ff_cap);
    const int32_t listed = list[0];
    if (listed > a.ff_cap) return FLAGGED;
    const double *rec = a.ff_super + sp * (int64_t)FAR_REC;
    double cx, cy, H;
    super_geometry(a, sp, cx, cy, H);
    const double nw1 = cx - x1, nw2 = cy - x2;   // -w
    double S1 = rec[FAR_P - 1], S2 = rec[2 * FAR_P - 1];
#pragma unroll
    for (int nn = FAR_P - 2; nn >= 0; --nn) {
        const double q1 = __builtin_fma(S1, nw1, __builtin_fma(-S2, nw2, rec[nn]));
        const double q2 = __builtin_fma(S1, nw2, __builtin_fma(S2, nw1, rec[FAR_P + nn]));
        S1 = q1;
        S2 = q2;
    }
    double a1 = S1, a2 = -S2;
    double snear = 0.0;
    bool tiny = false;
    for (int l = 0; l < listed; ++l) {
        const int64_t k = list[1 + l];
        const double e1 = x1 - ((global_double *)a.lens_xy)[2 * k];
        const double e2 = x2 - ((global_double *)a.lens_xy)[2 * k + 1];
        const double r2 = __builtin_fma(e1, e1, e2 * e2);
        tiny |= !(r2 > 1e-200);
        const double m = (UNIT || a.lens_m == nullptr) ? 1.0 : ((global_double *)a.lens_m)[k];
        const double f = m * rcp64(r2);
        a1 = __builtin_fma(f, e1, a1);
        a2 = __builtin_fma(f, e2, a2);
        snear = __builtin_fma(fabs(e1) + fabs(e2), fabs(f), snear);
    }
    const double SFAR = rec[2 * FAR_P], TRUNC = rec[2 * FAR_P + 1], SDEF = rec[2 * FAR_P + 2];
    const double NFAR = rec[2 * FAR_P + 3];
    const double far_err = TRUNC + (NFAR + 24.0 * FAR_P + 64.0) * U64 * 1.34 * SFAR;
    return far_decide(a, x1, x2, a1, a2, far_err, SFAR, SDEF, snear, listed, !tiny);
}

// Stage F for ray (i, j): on the grid its super-patch follows from its indices;
// a random ray's from its position (the cell of the whole rectangle's
// super-patch grid that holds it, clamped: a ray within rounding of a cell
// edge is still inside the neighbouring box's one-spacing slack).
template <bool UNIT>
__device__ inline int far_recheck_ray(const ShootArgs &a, int64_t i, int64_t j) {
    double x1, x2;
    int64_t sp;
    if (a.random) {
        random_ray_xy(a.sx0, a.sy0, a.sw, a.sh, a.nx, a.seed, i, j, x1, x2);
        int64_t sx = (int64_t)floor((x1 - a.sx0) / ((double)(FF_SP_X * PATCH_X) * a.spx));
        int64_t sy = (int64_t)floor((x2 - a.sy0) / ((double)(FF_SP_Y * PATCH_Y) * a.spy));
        sx = sx < 0 ? 0 : (sx >= a.ff_sbx ? a.ff_sbx - 1 : sx);
        sy = sy < 0 ? 0 : (sy >= a.ff_sby ? a.ff_sby - 1 : sy);
        sp = sy * a.ff_sbx + sx;
    } else {
        x1 = ray_coord(a.sx0, i, a.spx);
        x2 = ray_coord(a.sy0, j, a.spy);
        sp = ((j - a.ff_j0) / (PATCH_Y * FF_SP_Y)) * a.ff_sbx + (i - a.ff_i0) / (PATCH_X * FF_SP_X);
    }
    return far_eval<UNIT>(a, sp, x1, x2);
}

}  // namespace
}  // namespace rs
