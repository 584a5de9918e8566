// Launch planning of single maps (declarations and contracts in rs_plan.h).
#include "rs_plan.h"

#include <cmath>

namespace rs {

static size_t a256(size_t v) { return (v + 255) / 256 * 256; }

// (never more bins than the target plus one row)
void random_bins(int64_t rays, double sw, double sh, int64_t &nbx, int64_t &nby) {
    int64_t target = (rays + RAND_BIN_RAYS - 1) / RAND_BIN_RAYS;
    if (target < 1) target = 1;
    const double side = std::sqrt(sw * sh / (double)target);
    double fx = std::floor(sw / side + 0.5);
    if (!(fx >= 1.0)) fx = 1.0;
    if (fx > (double)target) fx = (double)target;
    nbx = (int64_t)fx;
    nby = (target + nbx - 1) / nbx;
}

static bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

int validate(const rs_map_params *p, int64_t n_lens) {
    if (!p) return fail(RS_EINVAL, "params is NULL");
    if (p->nx <= 0 || p->ny <= 0) return fail(RS_EINVAL, "ray grid must be positive (nx=%lld ny=%lld)", (long long)p->nx, (long long)p->ny);
    if (p->npx <= 0 || p->npy <= 0) return fail(RS_EINVAL, "source grid must be positive");
    // each side below 2^31 first, so that the product cannot overflow
    if (p->npx >= (int64_t(1) << 31) || p->npy >= (int64_t(1) << 31) || p->npx * p->npy >= (int64_t(1) << 31))
        return fail(RS_EINVAL, "source map must have fewer than 2^31 pixels");
    if (!finite_pos(p->sw) || !finite_pos(p->sh)) return fail(RS_EINVAL, "shooting extents must be finite and > 0");
    if (!finite_pos(p->tw) || !finite_pos(p->th)) return fail(RS_EINVAL, "source extents must be finite and > 0");
    if (!std::isfinite(p->sx0) || !std::isfinite(p->sy0) || !std::isfinite(p->tx0) || !std::isfinite(p->ty0))
        return fail(RS_EINVAL, "grid origins must be finite");
    if (!std::isfinite(p->gamma) || !std::isfinite(p->sigma_c) || !std::isfinite(p->sigma_star))
        return fail(RS_EINVAL, "gamma, sigma_c and sigma_star must be finite");
    if (p->i0 < 0 || p->i1 > p->nx || p->i0 > p->i1 || p->j0 < 0 || p->j1 > p->ny || p->j0 > p->j1)
        return fail(RS_EINVAL, "ray window [%lld,%lld)x[%lld,%lld) outside the %lldx%lld grid", (long long)p->i0,
                    (long long)p->i1, (long long)p->j0, (long long)p->j1, (long long)p->nx, (long long)p->ny);
    if (p->nx >= (int64_t(1) << 52) || p->ny >= (int64_t(1) << 52)) return fail(RS_EINVAL, "ray grid too large");
    // A launch holds at least one 32-row band, and the re-check queue keeps a launch's
    // ray index below bit 30 (its two top bits mark entries): 32 * 2^22 = 2^27.
    if (p->i1 - p->i0 > (int64_t(1) << 22)) return fail(RS_EINVAL, "window wider than 2^22 rays");
    if (p->mode != RS_FP32 && p->mode != RS_MIXED && p->mode != RS_FARFIELD)
        return fail(RS_EINVAL, "mode must be RS_FP32, RS_MIXED or RS_FARFIELD");
    if (p->mode == RS_FARFIELD && (p->flags & RS_RANDOM_RAYS))
        return fail(RS_EINVAL, "RS_FARFIELD works on the regular grid only");
    if (p->flags & ~(RS_ACCUMULATE | RS_EXACT_RECHECK | RS_RANDOM_RAYS))
        return fail(RS_EINVAL, "unknown flags 0x%x", p->flags);
    if (n_lens < 0) return fail(RS_EINVAL, "n_lens < 0");
    return RS_OK;
}

Plan make_plan(const rs_map_params *p, int64_t n_lens, int64_t rows_override) {
    Plan pl;
    pl.W = p->i1 - p->i0;
    pl.H = p->j1 - p->j0;
    pl.random = (p->flags & RS_RANDOM_RAYS) != 0;
    const int64_t chunk_rays = pl.random ? RAND_CHUNK_RAYS : CHUNK_RAYS;
    int64_t rows = pl.W > 0 ? chunk_rays / pl.W : PATCH_Y;
    rows = rows / PATCH_Y * PATCH_Y;
    if (rows < PATCH_Y) rows = PATCH_Y;
    if (rows_override > 0) rows = rows_override;
    pl.rows_per_chunk = rows;
    pl.n_chunks = (pl.W > 0 && pl.H > 0) ? (pl.H + rows - 1) / rows : 0;
    const int64_t rows_cap = pl.H < rows ? pl.H : rows;
    pl.queue_cap = (p->mode != RS_FP32) ? rows_cap * pl.W : 0;
    pl.qcount_bytes = (WS_QCOUNT + 16 * (size_t)pl.n_chunks + 8 + 255) / 256 * 256;
    pl.bytes = pl.qcount_bytes + 4 * (size_t)pl.queue_cap;
    pl.far_recheck = p->mode == RS_MIXED && !(p->flags & RS_EXACT_RECHECK);
    if (pl.far_recheck && pl.random) {
        // Random rays land anywhere in the shooting rectangle, so the records cover all
        // of it, built once per map; used unless the window holds few of its rays.
        pl.rand_sbx = (p->nx + FF_SP_X * PATCH_X - 1) / (FF_SP_X * PATCH_X);
        pl.rand_sby = (p->ny + FF_SP_Y * PATCH_Y - 1) / (FF_SP_Y * PATCH_Y);
        const int64_t own = (pl.W * pl.H + FF_SP_X * PATCH_X * FF_SP_Y * PATCH_Y - 1) / (FF_SP_X * PATCH_X * FF_SP_Y * PATCH_Y);
        if (pl.rand_sbx * pl.rand_sby > 4 * own + 64) pl.far_recheck = false;
    }
    if ((p->mode == RS_FARFIELD || pl.far_recheck) && pl.n_chunks > 0) {
        const int64_t nbx = (pl.W + PATCH_X - 1) / PATCH_X;
        const int64_t nby = (rows_cap + PATCH_Y - 1) / PATCH_Y;
        pl.super_cap = pl.random ? pl.rand_sbx * pl.rand_sby
                                 : ((nbx + FF_SP_X - 1) / FF_SP_X) * ((nby + FF_SP_Y - 1) / FF_SP_Y);
        size_t off = a256(pl.bytes);
        pl.ff_super_off = off;
        off += a256(sizeof(double) * FF_REC_DOUBLES * (size_t)pl.super_cap);
        pl.ff_near_off = off;
        off += a256(sizeof(int32_t) * (1 + (size_t)FF_NEAR_CAP) * (size_t)pl.super_cap);
        if (p->mode == RS_FARFIELD) {
            pl.patch_cap = nbx * nby;
            pl.ff_patch_off = off;
            off += a256(sizeof(double) * FF_PATCH_DOUBLES * (size_t)pl.patch_cap);
            pl.ff_work_off = off;
            off += 256;
            const int64_t sbx = (nbx + FF_SP_X - 1) / FF_SP_X, sby = (nby + FF_SP_Y - 1) / FF_SP_Y;
            pl.group_cap = ((sbx + FF_GROUP - 1) / FF_GROUP) * ((sby + FF_GROUP - 1) / FF_GROUP);
            pl.ff_group_off = off;
            off += a256(sizeof(double) * FF_REC_DOUBLES * FF_GROUP_PARTS * (size_t)pl.group_cap);
            pl.ff_glist_off = off;
            off += a256(sizeof(int32_t) * (1 + (size_t)FF_PART_CAP) * FF_GROUP_PARTS * (size_t)pl.group_cap);
            if (n_lens >= FF_TOP_MIN_LENSES) {
                const int64_t gbx = (sbx + FF_GROUP - 1) / FF_GROUP, gby = (sby + FF_GROUP - 1) / FF_GROUP;
                pl.top_cap = ((gbx + FF_TOP - 1) / FF_TOP) * ((gby + FF_TOP - 1) / FF_TOP);
                pl.ff_top_off = off;
                off += a256(sizeof(double) * FF_REC_DOUBLES * FF_TOP_PARTS * (size_t)pl.top_cap);
                pl.ff_tlist_off = off;
                off += a256(sizeof(int32_t) * (1 + (size_t)FF_TOP_PART_CAP) * FF_TOP_PARTS * (size_t)pl.top_cap);
            }
        }
        pl.bytes = off;
    }
    if (p->mode != RS_FP32 && !(p->flags & RS_EXACT_RECHECK) && pl.n_chunks > 1) {
        pl.defer = true;
        pl.defer_off = a256(pl.bytes);
        pl.bytes = pl.defer_off + 2 * sizeof(int64_t) * 2 * (size_t)DEFER_CAP;
    }
    if (pl.random && pl.n_chunks > 0) {
        pl.rays_cap = rows_cap * pl.W;
        const int64_t last_rows = pl.H - (pl.n_chunks - 1) * rows;
        int64_t bx, by;
        random_bins(pl.rays_cap, p->sw, p->sh, bx, by);
        pl.bins_cap = bx * by;
        random_bins(last_rows * pl.W, p->sw, p->sh, bx, by);
        if (bx * by > pl.bins_cap) pl.bins_cap = bx * by;
        size_t off = a256(pl.bytes);
        pl.bin_count_off = off;
        off += a256(4 * (size_t)pl.bins_cap);
        pl.bin_offset_off = off;
        off += a256(4 * ((size_t)pl.bins_cap + 1));
        pl.bin_cursor_off = off;
        off += a256(4 * (size_t)pl.bins_cap);
        pl.rel_off = off;
        off += a256(4 * (size_t)pl.rays_cap);
        pl.x_off = off;
        off += a256(8 * (size_t)pl.rays_cap);
        pl.y_off = off;
        off += a256(8 * (size_t)pl.rays_cap);
        pl.bytes = off;
    }
    return pl;
}

// (the workspace grows with the rows per launch: a binary search over bands)
bool plan_within(const rs_map_params *p, int64_t n_lens, size_t max_bytes, Plan &out) {
    out = make_plan(p, n_lens);
    if (out.bytes <= max_bytes) return true;
    int64_t lo = 1, hi = out.rows_per_chunk / PATCH_Y - 1;   // bands per launch
    Plan best = make_plan(p, n_lens, PATCH_Y);
    if (best.bytes > max_bytes) return false;
    while (lo < hi) {
        const int64_t mid = lo + (hi - lo + 1) / 2;
        Plan t = make_plan(p, n_lens, mid * PATCH_Y);
        if (t.bytes <= max_bytes) {
            lo = mid;
            best = t;
        } else {
            hi = mid - 1;
        }
    }
    if (best.rows_per_chunk != lo * PATCH_Y) best = make_plan(p, n_lens, lo * PATCH_Y);
    out = best;
    return true;
}

}  // namespace rs
