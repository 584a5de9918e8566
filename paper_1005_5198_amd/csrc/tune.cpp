// Autotuner of the deflection kernel's launch configuration. The paper notes that
// the direct GPU code's batch and thread-group sizes depend on the hardware
// (Section 2, GPU-D); here they are measured. Every candidate covers the same
// 64 x 32-ray patch with the same per-ray arithmetic, so the choice affects
// speed only:
//  * single maps: the thread shape (rays per lane, waves per block), timed on a
//    band of the map;
//  * batches: the thread shape and the persistent grid (blocks per CU), timed
//    on a band of every map of the batch.
// The cache maps a signature to the fastest choice: (mode, unit masses, N*
// rounded down to a power of two, the number of 64 x 32-ray patches rounded down
// to a power of two) for single maps; the same with the heaviest map's N* and
// the batch's patch count for batches. RAYSHOOT_TUNE_CACHE names a file that is
// loaded on first use and rewritten after every tuning run.
#include "rs_internal.h"
#include "rayshoot.h"
#include "rs_debug.h"

#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <string>
#include <tuple>

namespace rs {

int fail(int code, const char *fmt, ...);
int hip_fail(hipError_t e, const char *what);
int enqueue_map(const rs_map_params *p, const double *lens_xy, const double *lens_m, int64_t n_lens,
                uint32_t *map, int32_t *pix, void *workspace, size_t workspace_bytes, hipStream_t stream,
                int shape, float *kernel_ms);

namespace {
// kind (0 single map, 1 batch), mode, unit masses, log2 bucket of N*, log2 bucket of patches
using Key = std::tuple<int, int, int, int, int>;
std::mutex g_mu;
std::map<Key, int> g_cache;   // single maps: shape; batches: shape + 16 * blocks per CU
int g_forced = -1;
bool g_env_loaded = false;
// Built-in choice when nothing was tuned (measured on MI355X: 4 x 2 rays per lane, 2 x 2 waves).
constexpr int DEFAULT_SHAPE = 0;

int log2_bucket(int64_t v) {
    int b = 0;
    for (int64_t x = v + 1; x > 1; x >>= 1) ++b;
    return b;
}

Key key_of(int kind, int mode, bool unit, int64_t n_lens, int64_t patches) {
    return Key{kind, mode, unit ? 1 : 0, log2_bucket(n_lens), log2_bucket(patches)};
}

const char *env_path() { return std::getenv("RAYSHOOT_TUNE_CACHE"); }

int load_locked(const char *path, bool quiet);
int save_locked(const char *path);

// Load RAYSHOOT_TUNE_CACHE once (a missing file is not an error). Called with g_mu held.
void load_env_locked() {
    if (g_env_loaded) return;
    g_env_loaded = true;
    const char *p = env_path();
    if (p && *p) {
        const int rc = load_locked(p, true);
        debug_print(1, "tune cache %s: %s (%zu entries)", p, rc == RS_OK ? "loaded" : "not loaded", g_cache.size());
    }
}

void remember_locked(const Key &k, int choice) {
    g_cache[k] = choice;
    const char *p = env_path();
    if (p && *p) (void)save_locked(p);
}

int save_locked(const char *path) {
    FILE *f = fopen(path, "w");
    if (!f) return fail(RS_EINVAL, "cannot write %s", path);
    for (const auto &kv : g_cache)
        fprintf(f, "%d %d %d %d %d %d\n", std::get<0>(kv.first), std::get<1>(kv.first), std::get<2>(kv.first),
                std::get<3>(kv.first), std::get<4>(kv.first), kv.second);
    fclose(f);
    return RS_OK;
}

int load_locked(const char *path, bool quiet) {
    FILE *f = fopen(path, "r");
    if (!f) return quiet ? RS_EINVAL : fail(RS_EINVAL, "cannot read %s", path);
    int kind, mode, unit, nb, pb, choice, n = 0, got;
    std::map<Key, int> loaded;
    while ((got = fscanf(f, "%d %d %d %d %d %d", &kind, &mode, &unit, &nb, &pb, &choice)) != EOF) {
        if (got != 6) {
            fclose(f);
            return fail(RS_EINVAL, "line %d of %s: expected six integers", n + 1, path);
        }
        const int shape = choice % 16, bpc = choice / 16;
        if ((kind != 0 && kind != 1) || shape < 0 || shape >= N_SHAPES || bpc < 0 || (kind == 0 && bpc != 0) ||
            (mode != RS_FP32 && mode != RS_MIXED) || (unit != 0 && unit != 1)) {
            fclose(f);
            return fail(RS_EINVAL, "bad line %d in %s", n + 1, path);
        }
        loaded[Key{kind, mode, unit, nb, pb}] = choice;
        ++n;
    }
    fclose(f);
    for (const auto &kv : loaded) g_cache[kv.first] = kv.second;
    return RS_OK;
}
}  // namespace

int choose_shape(int mode, bool unit, int64_t n_lens, int64_t patches) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_forced >= 0) return g_forced;
    load_env_locked();
    auto it = g_cache.find(key_of(0, mode, unit, n_lens, patches));
    return it == g_cache.end() ? DEFAULT_SHAPE : it->second;
}

// A batch's choice (shape + 16 * blocks per CU; 0 blocks = as many as fit).
int choose_batch(int mode, bool unit, int64_t n_lens, int64_t tiles) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_forced >= 0) return g_forced;
    load_env_locked();
    auto it = g_cache.find(key_of(1, mode, unit, n_lens, tiles));
    if (it != g_cache.end()) return it->second;
    // untuned batch: the single-map choice for its heaviest map, every CU filled
    auto single = g_cache.lower_bound(key_of(0, mode, unit, n_lens, 0));
    if (single != g_cache.end() && std::get<0>(single->first) == 0 && std::get<1>(single->first) == mode &&
        std::get<2>(single->first) == (unit ? 1 : 0) && std::get<3>(single->first) == log2_bucket(n_lens))
        return single->second;
    return DEFAULT_SHAPE;
}

void remember_batch(int mode, bool unit, int64_t n_lens, int64_t tiles, int choice) {
    std::lock_guard<std::mutex> lk(g_mu);
    load_env_locked();
    remember_locked(key_of(1, mode, unit, n_lens, tiles), choice);
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
    const int64_t patches = ((W + PATCH_X - 1) / PATCH_X) * ((H + PATCH_Y - 1) / PATCH_Y);
    {
        std::lock_guard<std::mutex> lk(g_mu);
        load_env_locked();
        remember_locked(key_of(0, params->mode, lens_m == nullptr, n_lens, patches), best);
    }
    debug_print(1, "tuned %lldx%lld-ray map, %lld lenses: shape %d (%.3f ms on the sample)", (long long)W, (long long)H,
                (long long)n_lens, best, r.ms[best]);
    *result_host = r;
    return RS_OK;
}

int rs_tune_save(const char *path) {
    if (!path) return fail(RS_EINVAL, "NULL path");
    std::lock_guard<std::mutex> lk(g_mu);
    load_env_locked();
    return save_locked(path);
}

int rs_tune_load(const char *path) {
    if (!path) return fail(RS_EINVAL, "NULL path");
    std::lock_guard<std::mutex> lk(g_mu);
    return load_locked(path, false);
}

}  // extern "C"
