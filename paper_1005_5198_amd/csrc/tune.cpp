// Autotuner for the deflection kernel's thread shape (rays per lane and waves
// per block). Shapes all cover the same ray patch, so the choice affects speed
// only. The cache maps a map signature (mode, unit masses, N* bucket) to the
// fastest shape measured on the device.
#include "rs_internal.h"
#include "rayshoot.h"

#include <cstdio>
#include <map>
#include <mutex>
#include <tuple>

namespace rs {

int fail(int code, const char *fmt, ...);
int hip_fail(hipError_t e, const char *what);
int enqueue_map(const rs_map_params *p, const double *lens_xy, const double *lens_m, int64_t n_lens,
                uint32_t *map, int32_t *pix, void *workspace, size_t workspace_bytes, hipStream_t stream,
                int shape, float *kernel_ms);

namespace {
using Key = std::tuple<int, int, int>;  // mode, unit masses, floor(log2(n_lens + 1))
std::mutex g_mu;
std::map<Key, int> g_cache;
int g_forced = -1;
// Built-in choice when nothing was tuned (measured on MI355X for the 1024-lens-tile kernel).
int g_default_shape = 0;

Key key_of(int mode, bool unit, int64_t n_lens) {
    int b = 0;
    for (int64_t v = n_lens + 1; v > 1; v >>= 1) ++b;
    return Key{mode, unit ? 1 : 0, b};
}
}  // namespace

int choose_shape(int mode, bool unit, int64_t n_lens) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_forced >= 0) return g_forced;
    auto it = g_cache.find(key_of(mode, unit, n_lens));
    return it == g_cache.end() ? g_default_shape : it->second;
}

}  // namespace rs

using namespace rs;

extern "C" {

int rs_set_shape(int shape, int *previous) {
    if (shape < -1 || shape >= N_SHAPES) return fail(RS_EINVAL, "shape %d out of range [-1, %d)", shape, N_SHAPES);
    std::lock_guard<std::mutex> lk(g_mu);
    if (previous) *previous = g_forced;
    g_forced = shape;
    return RS_OK;
}

int rs_tune(const rs_map_params *params, const double *lens_xy, const double *lens_m, int64_t n_lens,
            uint32_t *scratch_map, void *workspace, size_t workspace_bytes, int64_t sample_rays, void *stream,
            rs_tune_result *result_host) {
    if (!params || !result_host || !scratch_map) return fail(RS_EINVAL, "NULL argument");
    if (params->flags & RS_RANDOM_RAYS) return fail(RS_EINVAL, "the tuner times regular-grid maps only");
    if (params->mode == RS_FARFIELD) return fail(RS_EINVAL, "the tuner times the direct kernels only");
    rs_map_params p = *params;
    p.flags &= ~RS_ACCUMULATE;
    const int64_t W = p.i1 - p.i0, H = p.j1 - p.j0;
    if (W <= 0 || H <= 0) return fail(RS_EINVAL, "empty window");
    if (sample_rays <= 0) sample_rays = int64_t(1) << 22;
    int64_t rows = sample_rays / W;
    rows = rows / PATCH_Y * PATCH_Y;
    if (rows < PATCH_Y) rows = PATCH_Y;
    if (rows > H) rows = H;
    p.j0 = params->j0 + (H - rows) / 2;
    p.j1 = p.j0 + rows;
    hipStream_t s = static_cast<hipStream_t>(stream);
    rs_tune_result r{};
    r.n_shapes = N_SHAPES;
    r.sample_interactions = (double)W * (double)rows * (double)n_lens;
    int best = -1;
    for (int shape = 0; shape < N_SHAPES; ++shape) {
        const ShapeInfo &si = shape_info(shape);
        r.rays_per_lane[shape][0] = si.rx;
        r.rays_per_lane[shape][1] = si.ry;
        r.threads[shape] = 64 * si.wx * si.wy;
        float ms = 0.0f, best_ms = 1e30f;
        for (int rep = 0; rep < 3; ++rep) {  // first run warms up; keep the fastest of the rest
            int rc = enqueue_map(&p, lens_xy, lens_m, n_lens, scratch_map, nullptr, workspace, workspace_bytes, s,
                                 shape, &ms);
            if (rc) return rc;
            if (rep > 0 && ms < best_ms) best_ms = ms;
        }
        r.ms[shape] = best_ms;
        if (best < 0 || best_ms < r.ms[best]) best = shape;
    }
    r.shape = best;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        g_cache[key_of(params->mode, lens_m == nullptr, n_lens)] = best;
    }
    *result_host = r;
    return RS_OK;
}

int rs_tune_save(const char *path) {
    if (!path) return fail(RS_EINVAL, "NULL path");
    FILE *f = fopen(path, "w");
    if (!f) return fail(RS_EINVAL, "cannot write %s", path);
    std::lock_guard<std::mutex> lk(g_mu);
    for (const auto &kv : g_cache)
        fprintf(f, "%d %d %d %d\n", std::get<0>(kv.first), std::get<1>(kv.first), std::get<2>(kv.first), kv.second);
    fclose(f);
    return RS_OK;
}

int rs_tune_load(const char *path) {
    if (!path) return fail(RS_EINVAL, "NULL path");
    FILE *f = fopen(path, "r");
    if (!f) return fail(RS_EINVAL, "cannot read %s", path);
    int mode, unit, bucket, shape, n = 0;
    std::map<Key, int> loaded;
    while (fscanf(f, "%d %d %d %d", &mode, &unit, &bucket, &shape) == 4) {
        if (shape < 0 || shape >= N_SHAPES || (mode != RS_FP32 && mode != RS_MIXED)) {
            fclose(f);
            return fail(RS_EINVAL, "bad line %d in %s", n + 1, path);
        }
        loaded[Key{mode, unit, bucket}] = shape;
        ++n;
    }
    fclose(f);
    std::lock_guard<std::mutex> lk(g_mu);
    for (const auto &kv : loaded) g_cache[kv.first] = kv.second;
    return RS_OK;
}

}  // extern "C"
