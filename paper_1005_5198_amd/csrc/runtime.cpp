// Host runtime of the C ABI declared in include/rayshoot.h: argument
// validation, planning of ray chunks and workspace, and the launch sequence
// (zero map and counters -> per chunk: deflection kernel, FP64 re-check).
#include "rs_internal.h"
#include "rayshoot.h"
#include "rs_debug.h"
#include "rs_plan.h"

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

namespace rs {

static thread_local std::string g_last_error;

int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

int hip_fail(hipError_t e, const char *what) {
    return fail(RS_EHIP, "%s: %s", what, hipGetErrorString(e));
}

struct Profile {
    std::mutex mu;
    bool on = false;
    struct Rec { hipEvent_t a, b; double inter; };
    std::vector<Rec> pending;
    double ms = 0.0, inter = 0.0;
    int64_t launches = 0;
};
static Profile g_prof;

// Kernel timing hooks: when profiling is on, record an event pair around a launch.
void profile_begin(hipStream_t stream, void **token) {
    *token = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_prof.mu);
        if (!g_prof.on) return;
    }
    hipEvent_t a = nullptr;
    if (hipEventCreate(&a) != hipSuccess) return;
    if (hipEventRecord(a, stream) != hipSuccess) {
        (void)hipEventDestroy(a);
        return;
    }
    *token = a;
}

// Takes ownership of token (the event profile_begin recorded), also on failure.
int profile_end(hipStream_t stream, void *token, double interactions) {
    if (!token) return RS_OK;
    hipEvent_t a = static_cast<hipEvent_t>(token), b = nullptr;
    if (hipEventCreate(&b) != hipSuccess) {
        (void)hipEventDestroy(a);
        return fail(RS_EHIP, "hipEventCreate failed");
    }
    if (hipEventRecord(b, stream) != hipSuccess) {
        (void)hipEventDestroy(a);
        (void)hipEventDestroy(b);
        return fail(RS_EHIP, "hipEventRecord failed");
    }
    std::lock_guard<std::mutex> lk(g_prof.mu);
    g_prof.pending.push_back({a, b, interactions});
    return RS_OK;
}

// A profile_begin event that an early return would otherwise leak.
struct ProfileToken {
    void *tok = nullptr;
    ProfileToken() = default;
    ProfileToken(const ProfileToken &) = delete;
    ProfileToken &operator=(const ProfileToken &) = delete;
    ~ProfileToken() {
        if (tok) (void)hipEventDestroy(static_cast<hipEvent_t>(tok));
    }
    void *release() {
        void *t = tok;
        tok = nullptr;
        return t;
    }
};

// The deflection launches' timing events, destroyed on every return.
struct EventPair {
    hipEvent_t first = nullptr, last = nullptr;
    EventPair() = default;
    EventPair(const EventPair &) = delete;
    EventPair &operator=(const EventPair &) = delete;
    ~EventPair() {
        if (first) (void)hipEventDestroy(first);
        if (last) (void)hipEventDestroy(last);
    }
};

int choose_shape(int mode, bool unit, int64_t n_lens, int64_t patches);

// Enqueue the whole map (or pixel) computation. map may be null when pix is set.
// shape < 0 picks the tuned or default thread shape. When kernel_ms is given,
// the deflection launches are timed with events and the call synchronises.
static int check_inputs(const rs_map_params *p, const double *lens_xy, const double *lens_m, int64_t n_lens,
                        const uint32_t *map, const int32_t *pix) {
    int rc = validate(p, n_lens);
    if (rc) return rc;
    if (n_lens > 0 && !lens_xy) return fail(RS_EINVAL, "lens_xy is NULL");
    if (!map && !pix) return fail(RS_EINVAL, "output is NULL");
    if ((reinterpret_cast<uintptr_t>(lens_xy) | reinterpret_cast<uintptr_t>(lens_m)) & 7)
        return fail(RS_EINVAL, "lens arrays must be 8-byte aligned");
    return RS_OK;
}

static int enqueue_planned(const rs_map_params *p, const double *lens_xy, const double *lens_m, int64_t n_lens,
                           uint32_t *map, int32_t *pix, void *workspace, hipStream_t stream, int shape,
                           float *kernel_ms, const Plan &pl, bool profile);

int enqueue_map(const rs_map_params *p, const double *lens_xy, const double *lens_m, int64_t n_lens,
                uint32_t *map, int32_t *pix, void *workspace, size_t workspace_bytes, hipStream_t stream,
                int shape, float *kernel_ms) {
    int rc = check_inputs(p, lens_xy, lens_m, n_lens, map, pix);
    if (rc) return rc;
    if (!workspace) return fail(RS_EINVAL, "workspace is NULL");
    const Plan pl = make_plan(p, n_lens);
    if (workspace_bytes < pl.bytes)
        return fail(RS_ENOMEM, "workspace has %zu bytes, needs %zu", workspace_bytes, pl.bytes);
    return enqueue_planned(p, lens_xy, lens_m, n_lens, map, pix, workspace, stream, shape, kernel_ms, pl, true);
}

// The map in launches small enough for a fixed scratch buffer of scratch_bytes (the
// entry point without allocation). The arguments are checked and the launches planned
// before scratch_of_device gives the buffer's device address. Profiling events are never
// created here.
int enqueue_map_fixed(const rs_map_params *p, const double *lens_xy, const double *lens_m, int64_t n_lens,
                      uint32_t *map, int (*scratch_of_device)(void **), size_t scratch_bytes,
                      hipStream_t stream, void **scratch_used) {
    int rc = check_inputs(p, lens_xy, lens_m, n_lens, map, nullptr);
    if (rc) return rc;
    if (!map) return fail(RS_EINVAL, "map is NULL");
    Plan pl;
    if (!plan_within(p, n_lens, scratch_bytes, pl))
        return fail(RS_ENOMEM, "one band of %d rows of this window needs %zu bytes of scratch; the static "
                    "scratch holds %zu", PATCH_Y, make_plan(p, n_lens, PATCH_Y).bytes, scratch_bytes);
    void *scratch = nullptr;
    rc = scratch_of_device(&scratch);
    if (rc) return rc;
    *scratch_used = scratch;
    return enqueue_planned(p, lens_xy, lens_m, n_lens, map, nullptr, scratch, stream, -1, nullptr, pl, false);
}

static int enqueue_planned(const rs_map_params *p, const double *lens_xy, const double *lens_m, int64_t n_lens,
                           uint32_t *map, int32_t *pix, void *workspace, hipStream_t stream, int shape,
                           float *kernel_ms, const Plan &pl, bool profile) {
    int rc = RS_OK;
    Range range(pix ? "rs_ray_pixels" : "rs_make_map");

    const bool accumulate = (p->flags & RS_ACCUMULATE) != 0;
    hipError_t e =
        launch_fill((map && !accumulate) ? map : nullptr, p->npx * p->npy, workspace, 4 * pl.n_chunks + 2, stream);
    if (e != hipSuccess) return hip_fail(e, "fill kernel");

    char *ws = static_cast<char *>(workspace);
    ShootArgs a{};
    a.sx0 = p->sx0;
    a.sy0 = p->sy0;
    a.spx = p->sw / (double)p->nx;
    a.spy = p->sh / (double)p->ny;
    a.i0 = p->i0;
    a.i1 = p->i1;
    a.j0 = p->j0;
    a.nbx = (pl.W + PATCH_X - 1) / PATCH_X;
    a.c1 = (1.0 - p->gamma) - p->sigma_c;
    a.c2 = (1.0 + p->gamma) - p->sigma_c;
    a.tx0 = p->tx0;
    a.ty0 = p->ty0;
    a.inv_pixw = (double)p->npx / p->tw;
    a.inv_pixh = (double)p->npy / p->th;
    a.npx = p->npx;
    a.npy = p->npy;
    a.lens_xy = lens_xy;
    a.lens_m = lens_m;
    a.n_lens = n_lens;
    a.bound_scale = 1.0 + (double)(n_lens + 64) * 4.7e-10;
    a.map = map;
    a.pix_out = pix;
    a.counters = reinterpret_cast<unsigned long long *>(ws + WS_COUNTERS);
    a.queue = reinterpret_cast<uint32_t *>(ws + pl.qcount_bytes);

    RecheckArgs r{};
    r.sx0 = p->sx0;
    r.sy0 = p->sy0;
    r.sw = p->sw;
    r.sh = p->sh;
    r.nx = p->nx;
    r.ny = p->ny;
    r.i0 = p->i0;
    r.i1 = p->i1;
    r.j0 = p->j0;
    r.gamma = p->gamma;
    r.sigma_c = p->sigma_c;
    r.tx0 = p->tx0;
    r.ty0 = p->ty0;
    r.tw = p->tw;
    r.th = p->th;
    r.npx = p->npx;
    r.npy = p->npy;
    r.lens_xy = lens_xy;
    r.lens_m = lens_m;
    r.n_lens = n_lens;
    r.map = map;
    r.pix_out = pix;
    r.counters = a.counters;
    r.queue = a.queue;
    r.random = pl.random ? 1 : 0;
    r.seed = p->seed;
    if (pl.defer) {
        r.defer = reinterpret_cast<int64_t *>(ws + pl.defer_off);
        r.dcount = reinterpret_cast<uint32_t *>(ws + WS_QCOUNT) + 4 * pl.n_chunks;
        r.udefer = r.defer + 2 * DEFER_CAP;
        r.ucount = r.dcount + 1;
    }
    if (pl.random) {
        a.random = 1;
        a.seed = p->seed;
        a.nx = p->nx;
        a.sw = p->sw;
        a.sh = p->sh;
        a.bin_count = reinterpret_cast<uint32_t *>(ws + pl.bin_count_off);
        a.bin_offset = reinterpret_cast<uint32_t *>(ws + pl.bin_offset_off);
        a.bin_cursor = reinterpret_cast<uint32_t *>(ws + pl.bin_cursor_off);
        a.ray_rel = reinterpret_cast<uint32_t *>(ws + pl.rel_off);
        a.ray_x = reinterpret_cast<double *>(ws + pl.x_off);
        a.ray_y = reinterpret_cast<double *>(ws + pl.y_off);
    }

    if ((p->mode == RS_FARFIELD || pl.far_recheck) && pl.n_chunks > 0) {
        a.ff_sbx = pl.random ? pl.rand_sbx : (a.nbx + FF_SP_X - 1) / FF_SP_X;
        a.ff_sby = pl.rand_sby;
        a.ff_super = reinterpret_cast<double *>(ws + pl.ff_super_off);
        a.ff_near = reinterpret_cast<int32_t *>(ws + pl.ff_near_off);
        a.ff_cap = FF_NEAR_CAP;
        if (p->mode == RS_FARFIELD) {
            a.ff_patch = reinterpret_cast<double *>(ws + pl.ff_patch_off);
            a.ff_work = reinterpret_cast<uint32_t *>(ws + pl.ff_work_off);
            a.ff_gbx = (a.ff_sbx + FF_GROUP - 1) / FF_GROUP;
            a.ff_group = reinterpret_cast<double *>(ws + pl.ff_group_off);
            a.ff_glist = reinterpret_cast<int32_t *>(ws + pl.ff_glist_off);
            if (pl.top_cap > 0) {
                a.ff_tbx = (a.ff_gbx + FF_TOP - 1) / FF_TOP;
                a.ff_top = reinterpret_cast<double *>(ws + pl.ff_top_off);
                a.ff_tlist = reinterpret_cast<int32_t *>(ws + pl.ff_tlist_off);
            }
        }
        if (pl.random) {
            a.ff_i0 = 0;
            a.ff_j0 = 0;
            e = launch_super_records(a, pl.super_cap, stream);
            if (e != hipSuccess) return hip_fail(e, "super-patch records");
        }
    }
    if (shape < 0 && !pl.random && p->mode != RS_FARFIELD)
        shape = choose_shape(p->mode, lens_m == nullptr, n_lens, (pl.W + PATCH_X - 1) / PATCH_X * ((pl.H + PATCH_Y - 1) / PATCH_Y));
    debug_print(1, "map %lldx%lld rays, %lld lenses%s, mode %d%s: %lld launch(es) of %lld rows, workspace %zu B, shape %d",
                (long long)pl.W, (long long)pl.H, (long long)n_lens, lens_m ? " with masses" : "", p->mode,
                pl.random ? ", random rays" : "", (long long)pl.n_chunks, (long long)pl.rows_per_chunk, pl.bytes,
                shape);
    EventPair ev;
    if (kernel_ms) {
        *kernel_ms = 0.0f;
        if (hipEventCreate(&ev.first) != hipSuccess || hipEventCreate(&ev.last) != hipSuccess)
            return fail(RS_EHIP, "hipEventCreate failed");
    }
    float timed_ms = 0.0f;
    for (int64_t c = 0; c < pl.n_chunks; ++c) {
        a.jc0 = p->j0 + c * pl.rows_per_chunk;
        a.jc1 = a.jc0 + pl.rows_per_chunk < p->j1 ? a.jc0 + pl.rows_per_chunk : p->j1;
        a.qcount = reinterpret_cast<uint32_t *>(ws + WS_QCOUNT) + c;
        if (!pl.random) {   // grid super-patches start at this launch's first patch
            a.ff_i0 = a.i0;
            a.ff_j0 = a.jc0;
        }
        ProfileToken tok;
        if (profile) profile_begin(stream, &tok.tok);
        if (kernel_ms && hipEventRecord(ev.first, stream) != hipSuccess) return fail(RS_EHIP, "hipEventRecord failed");
        if (pl.random) {
            random_bins((a.jc1 - a.jc0) * pl.W, p->sw, p->sh, a.nbx_r, a.nby_r);
            a.bw = p->sw / (double)a.nbx_r;
            a.bh = p->sh / (double)a.nby_r;
            a.inv_bw = (double)a.nbx_r / p->sw;
            a.inv_bh = (double)a.nby_r / p->sh;
            e = launch_shoot_random(a, p->mode, stream);
        } else if (p->mode == RS_FARFIELD) {
            e = launch_farfield(a, stream);
        } else {
            e = launch_shoot(a, p->mode, shape, stream);
        }
        if (e != hipSuccess) return hip_fail(e, "deflection kernel");
        if (kernel_ms) {
            float ms = 0.0f;
            if (hipEventRecord(ev.last, stream) != hipSuccess || hipEventSynchronize(ev.last) != hipSuccess ||
                hipEventElapsedTime(&ms, ev.first, ev.last) != hipSuccess)
                return fail(RS_EHIP, "timing the deflection kernel failed");
            timed_ms += ms;
        }
        rc = profile_end(stream, tok.release(), (double)(a.jc1 - a.jc0) * (double)pl.W * (double)n_lens);
        if (rc) return rc;
        if (p->mode != RS_FP32) {
            r.jc0 = a.jc0;
            r.qcount = a.qcount;
            r.qlive = nullptr;
            r.qunres = reinterpret_cast<uint32_t *>(ws + WS_QCOUNT) + 2 * pl.n_chunks + c;
            if (pl.defer) r.qleft = reinterpret_cast<uint32_t *>(ws + WS_QCOUNT) + 3 * pl.n_chunks + c;
            if (pl.far_recheck) {
                uint32_t *qlive = reinterpret_cast<uint32_t *>(ws + WS_QCOUNT) + pl.n_chunks + c;
                e = launch_recheck_far(a, qlive, (a.jc1 - a.jc0) * pl.W, stream);
                if (e != hipSuccess) return hip_fail(e, "far-field re-check kernel");
                r.qlive = qlive;
            }
            e = launch_recheck(r, (a.jc1 - a.jc0) * pl.W, (p->flags & RS_EXACT_RECHECK) != 0, stream);
            if (e != hipSuccess) return hip_fail(e, "re-check kernel");
        }
    }
    if (pl.defer) {
        e = launch_recheck_deferred(r, stream);
        if (e != hipSuccess) return hip_fail(e, "deferred exact re-check kernel");
    }
    if (kernel_ms) {
        *kernel_ms = timed_ms;
        if (hipStreamSynchronize(stream) != hipSuccess) return fail(RS_EHIP, "hipStreamSynchronize failed");
    }
    return RS_OK;
}

}  // namespace rs

using namespace rs;

extern "C" {

const char *rs_version(void) { return "rayshoot-mi355x 0.1 (gfx950)"; }

const char *rs_last_error(void) { return g_last_error.c_str(); }

size_t rs_workspace_bytes(const rs_map_params *params, int64_t n_lens) {
    if (validate(params, n_lens) != RS_OK) return 0;
    return make_plan(params, n_lens).bytes;
}

int rs_make_map(const rs_map_params *params, const double *lens_xy, const double *lens_m, int64_t n_lens,
                uint32_t *map, void *workspace, size_t workspace_bytes, void *stream) {
    if (!map) return fail(RS_EINVAL, "map is NULL");
    return enqueue_map(params, lens_xy, lens_m, n_lens, map, nullptr, workspace, workspace_bytes,
                       static_cast<hipStream_t>(stream), -1, nullptr);
}

int rs_ray_pixels(const rs_map_params *params, const double *lens_xy, const double *lens_m, int64_t n_lens,
                  int32_t *pix, void *workspace, size_t workspace_bytes, void *stream) {
    if (!pix) return fail(RS_EINVAL, "pix is NULL");
    return enqueue_map(params, lens_xy, lens_m, n_lens, nullptr, pix, workspace, workspace_bytes,
                       static_cast<hipStream_t>(stream), -1, nullptr);
}

int rs_read_stats(const void *workspace, rs_map_stats *stats_host, void *stream) {
    if (!workspace || !stats_host) return fail(RS_EINVAL, "NULL argument");
    unsigned long long c[8];
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = hipMemcpyAsync(c, static_cast<const char *>(workspace) + WS_COUNTERS, sizeof(c),
                                  hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "reading stats");
    stats_host->rays_in_map = c[C_IN];
    stats_host->rays_out = c[C_OUT];
    stats_host->rays_singular = c[C_SING];
    stats_host->rays_rechecked = c[C_RECHECK];
    stats_host->rays_rechecked_direct = c[C_DIRECT];
    stats_host->rays_shot = c[C_IN] + c[C_OUT] + c[C_SING];
    return RS_OK;
}

int rs_profile_enable(int on) {
    std::lock_guard<std::mutex> lk(g_prof.mu);
    g_prof.on = on != 0;
    return RS_OK;
}

int rs_profile_read(double *kernel_ms, int64_t *launches, double *interactions) {
    std::vector<Profile::Rec> recs;
    {
        std::lock_guard<std::mutex> lk(g_prof.mu);
        recs.swap(g_prof.pending);
    }
    double ms_sum = 0.0, inter = 0.0;
    int64_t n = 0;
    int rc = RS_OK;
    for (auto &r : recs) {
        float ms = 0.0f;
        hipError_t e = hipEventSynchronize(r.b);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, r.a, r.b);
        if (e != hipSuccess) rc = hip_fail(e, "reading kernel timing");
        ms_sum += ms;
        inter += r.inter;
        ++n;
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    if (kernel_ms) *kernel_ms = ms_sum;
    if (launches) *launches = n;
    if (interactions) *interactions = inter;
    return rc;
}

}  // extern "C"
