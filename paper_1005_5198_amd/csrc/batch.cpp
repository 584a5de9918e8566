// Host side of the batched path: validate the requests, order the work list
// (most expensive maps first, so the tail of the persistent launch is made of
// cheap tiles), upload the descriptors into the workspace, and enqueue
// fill -> persistent deflection -> batched FP64 re-check.
#include "rs_internal.h"
#include "rayshoot.h"
#include "rs_debug.h"

#include <algorithm>
#include <numeric>
#include <vector>

namespace rs {

int fail(int code, const char *fmt, ...);
int hip_fail(hipError_t e, const char *what);
int validate(const rs_map_params *p, int64_t n_lens);
int choose_batch(int mode, bool unit, int64_t n_lens, int64_t tiles);
void remember_batch(int mode, bool unit, int64_t n_lens, int64_t tiles, int choice);
void profile_begin(hipStream_t stream, void **token);
int profile_end(hipStream_t stream, void *token, double interactions);

}  // namespace rs

using namespace rs;

extern "C" {

// Per-map workspace after the counters: two bitmaps; in mixed mode also the
// far-field re-check stage's super-patch records and lens lists.
static size_t map_bytes(const rs_map_params &p) {
    size_t b = 2 * 4 * (size_t)bitmap_words_of(p);
    if (p.mode == RS_MIXED) {
        const size_t ns = (size_t)super_patches_of(p);
        b += align256(sizeof(double) * FF_REC_DOUBLES * ns) + align256(sizeof(int32_t) * (1 + FF_BATCH_CAP) * ns);
    }
    return b;
}

// Workspace bytes: globals, descriptors, counters, and the per-map parts.
static size_t batch_bytes(const rs_map_request *reqs, int32_t n) {
    size_t off = batch_bitmaps_offset(n);
    for (int32_t k = 0; k < n; ++k) off += map_bytes(reqs[k].params);
    return off;
}

size_t rs_batch_workspace_bytes(const rs_map_request *reqs, int32_t n) {
    if (!reqs || n < 1 || n > 65536) return 0;
    for (int32_t k = 0; k < n; ++k)
        if (validate(&reqs[k].params, reqs[k].n_lens) != RS_OK) return 0;
    return batch_bytes(reqs, n);
}

// The batch's launches. choice < 0: the tuned (or default) kernel configuration;
// otherwise shape = choice % 16, blocks per CU = choice / 16 (0 = as many as fit).
// deflection_only: no re-check (the tuner's timing runs); kernel_ms: time the
// persistent deflection launch with events and synchronise.
static int enqueue_batch(const rs_map_request *reqs, int32_t n, void *workspace, size_t workspace_bytes,
                         hipStream_t s, int choice, bool deflection_only, float *kernel_ms) {
    if (!reqs || n < 1 || n > 65536) return fail(RS_EINVAL, "need 1..65536 requests");
    if (!workspace) return fail(RS_EINVAL, "workspace is NULL");
    const int mode = reqs[0].params.mode;
    for (int32_t k = 0; k < n; ++k) {
        const rs_map_request &r = reqs[k];
        int rc = validate(&r.params, r.n_lens);
        if (rc) return fail(rc, "request %d: %s", k, rs_last_error());
        if (r.params.mode != mode) return fail(RS_EINVAL, "request %d: every request of a batch needs the same mode", k);
        if (r.params.mode == RS_FARFIELD)
            return fail(RS_EINVAL, "request %d: RS_FARFIELD maps are made by rs_make_map only, not in batches", k);
        if (r.params.flags & RS_RANDOM_RAYS)
            return fail(RS_EINVAL, "request %d: random rays are made by rs_make_map only, not in batches", k);
        if (!r.map) return fail(RS_EINVAL, "request %d: map is NULL", k);
        if (r.n_lens > 0 && !r.lens_xy) return fail(RS_EINVAL, "request %d: lens_xy is NULL", k);
        if ((reinterpret_cast<uintptr_t>(r.lens_xy) | reinterpret_cast<uintptr_t>(r.lens_m)) & 7)
            return fail(RS_EINVAL, "request %d: lens arrays must be 8-byte aligned", k);
        const double rays = (double)(r.params.i1 - r.params.i0) * (double)(r.params.j1 - r.params.j0);
        if (rays >= 4294967296.0) return fail(RS_EINVAL, "request %d: window holds 2^32 rays or more", k);
    }
    const size_t need = batch_bytes(reqs, n);
    if (workspace_bytes < need) return fail(RS_ENOMEM, "workspace has %zu bytes, needs %zu", workspace_bytes, need);
    std::vector<int32_t> order(n);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(),
                     [&](int32_t x, int32_t y) { return reqs[x].n_lens > reqs[y].n_lens; });

    char *ws = static_cast<char *>(workspace);
    auto *counters = reinterpret_cast<unsigned long long *>(ws + batch_counters_offset(n));
    std::vector<char *> parts(n);
    {
        size_t off = batch_bitmaps_offset(n);
        for (int32_t k = 0; k < n; ++k) {
            parts[k] = ws + off;
            off += map_bytes(reqs[k].params);
        }
    }
    std::vector<BatchMap> maps(n);
    int64_t tiles = 0, words = 0, supers = 0;
    double interactions = 0.0;
    bool unit = true;
    for (int32_t w = 0; w < n; ++w) {
        const int32_t k = order[w];
        const rs_map_request &r = reqs[k];
        BatchMap &m = maps[w];
        m = BatchMap{};
        m.p = r.params;
        m.lens_xy = r.lens_xy;
        m.lens_m = r.lens_m;
        m.n_lens = r.n_lens;
        m.map = r.map;
        m.counters = counters + (size_t)k * N_COUNTERS;
        const int64_t W = r.params.i1 - r.params.i0, H = r.params.j1 - r.params.j0;
        m.n_tiles = (W > 0 && H > 0) ? ((W + PATCH_X - 1) / PATCH_X) * ((H + PATCH_Y - 1) / PATCH_Y) : 0;
        m.tile_begin = tiles;
        m.n_words = bitmap_words_of(r.params);
        m.word_begin = words;
        m.flag_bits = reinterpret_cast<uint32_t *>(parts[k]);
        m.unres_bits = m.flag_bits + m.n_words;
        if (mode == RS_MIXED) {
            m.n_super = super_patches_of(r.params);
            m.ff_sbx = (((W + PATCH_X - 1) / PATCH_X) + FF_SP_X - 1) / FF_SP_X;
            m.super_begin = supers;
            char *rec = parts[k] + 2 * 4 * (size_t)m.n_words;
            m.ff_super = reinterpret_cast<double *>(rec);
            m.ff_near = reinterpret_cast<int32_t *>(rec + align256(sizeof(double) * FF_REC_DOUBLES * (size_t)m.n_super));
            supers += m.n_super;
        }
        m.request = k;
        m.accumulate = (r.params.flags & RS_ACCUMULATE) ? 1 : 0;
        if (r.lens_m != nullptr) unit = false;
        tiles += m.n_tiles;
        words += m.n_words;
        interactions += (double)W * (double)H * (double)r.n_lens;
    }
    Range range("rs_make_maps");
    hipError_t e = hipMemcpyAsync(ws + batch_maps_offset(), maps.data(), sizeof(BatchMap) * (size_t)n,
                                  hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(e, "uploading batch descriptors");

    BatchArgs b{};
    b.maps = reinterpret_cast<const BatchMap *>(ws + batch_maps_offset());
    b.n_maps = n;
    b.mode = mode;
    b.unit_masses = unit ? 1 : 0;
    b.total_tiles = tiles;
    b.total_words = words;
    b.total_super = supers;
    b.tile_counter = reinterpret_cast<unsigned long long *>(ws);
    b.unresolved = reinterpret_cast<unsigned int *>(ws + 8);

    e = launch_batch_fill(b, workspace, n, s);
    if (e != hipSuccess) return hip_fail(e, "batch fill kernel");
    const rs_map_request &heavy = reqs[order[0]];
    if (choice < 0) choice = choose_batch(mode, heavy.lens_m == nullptr, heavy.n_lens, tiles);
    const int shape = choice % 16, blocks_per_cu = choice / 16;
    debug_print(1, "batch of %d maps, %lld tiles, %.3e interactions, mode %d: shape %d, %d blocks per CU%s", n,
                (long long)tiles, interactions, mode, shape, blocks_per_cu, blocks_per_cu ? "" : " (as many as fit)");
    void *tok = nullptr;
    hipEvent_t ev[2] = {nullptr, nullptr};
    if (kernel_ms) {
        if (hipEventCreate(&ev[0]) != hipSuccess || hipEventCreate(&ev[1]) != hipSuccess ||
            hipEventRecord(ev[0], s) != hipSuccess) {
            for (hipEvent_t x : ev)
                if (x) (void)hipEventDestroy(x);
            return fail(RS_EHIP, "timing events");
        }
    } else {
        profile_begin(s, &tok);
    }
    e = launch_shoot_batch(b, shape, blocks_per_cu, s);
    // profile_end takes the event in every case, also after a failed launch
    int rc = kernel_ms ? RS_OK : profile_end(s, tok, interactions);
    if (kernel_ms) {
        *kernel_ms = 0.0f;
        hipError_t t = hipEventRecord(ev[1], s);
        if (t == hipSuccess) t = hipEventSynchronize(ev[1]);
        if (t == hipSuccess) t = hipEventElapsedTime(kernel_ms, ev[0], ev[1]);
        for (hipEvent_t x : ev) (void)hipEventDestroy(x);
        if (e == hipSuccess && t != hipSuccess) return hip_fail(t, "timing the batched kernel");
    }
    if (e != hipSuccess) return hip_fail(e, "batched deflection kernel");
    if (rc) return rc;
    if (mode == RS_MIXED && !deflection_only) {
        e = launch_batch_super(b, s);
        if (e != hipSuccess) return hip_fail(e, "batched super-patch kernel");
        e = launch_recheck_batch(b, s);
        if (e != hipSuccess) return hip_fail(e, "batched re-check kernels");
    }
    return RS_OK;
}

int rs_make_maps(const rs_map_request *reqs, int32_t n, void *workspace, size_t workspace_bytes, void *stream) {
    return enqueue_batch(reqs, n, workspace, workspace_bytes, static_cast<hipStream_t>(stream), -1, false, nullptr);
}

int rs_tune_batch(const rs_map_request *requests, int32_t n, void *workspace, size_t workspace_bytes,
                  int64_t sample_rays, void *stream, rs_tune_batch_result *result_host) {
    if (!requests || !result_host || n < 1 || n > 65536) return fail(RS_EINVAL, "bad arguments");
    if (sample_rays <= 0) sample_rays = int64_t(1) << 20;
    // The sample: a band of whole 32-row patch rows from the middle of each window.
    std::vector<rs_map_request> sample(requests, requests + n);
    double inter = 0.0;
    int64_t full_tiles = 0;
    for (rs_map_request &r : sample) {
        rs_map_params &p = r.params;
        const int64_t W = p.i1 - p.i0, H = p.j1 - p.j0;
        if (W > 0 && H > 0) full_tiles += ((W + PATCH_X - 1) / PATCH_X) * ((H + PATCH_Y - 1) / PATCH_Y);
        if (W <= 0 || H <= 0) continue;
        int64_t rows = std::max<int64_t>(PATCH_Y, sample_rays / W / PATCH_Y * PATCH_Y);
        rows = std::min(rows, H);
        p.j0 += (H - rows) / 2 / PATCH_Y * PATCH_Y;
        p.j1 = p.j0 + rows;
        p.flags &= ~RS_ACCUMULATE;
        inter += (double)W * (double)rows * (double)r.n_lens;
    }
    if (batch_bytes(sample.data(), n) > workspace_bytes) return fail(RS_ENOMEM, "workspace too small for the sample");
    hipStream_t s = static_cast<hipStream_t>(stream);
    rs_tune_batch_result res{};
    res.sample_interactions = inter;
    const int bpcs[3] = {0, 3, 2};   // as many blocks per CU as fit, then fewer
    int best = -1;
    for (int shape = 0; shape < N_SHAPES; ++shape)
        for (int bpc : bpcs) {
            if (res.n >= RS_MAX_BATCH_CHOICES) break;
            const int choice = shape + 16 * bpc;
            float ms = 0.0f, best_ms = 1e30f;
            for (int rep = 0; rep < 3; ++rep) {   // first run warms up; keep the fastest of the rest
                const int rc = enqueue_batch(sample.data(), n, workspace, workspace_bytes, s, choice, true, &ms);
                if (rc) return rc;
                if (rep > 0 && ms < best_ms) best_ms = ms;
            }
            const int k = res.n++;
            res.shape[k] = shape;
            res.blocks_per_cu[k] = bpc;
            res.ms[k] = best_ms;
            if (best < 0 || best_ms < res.ms[best]) best = k;
        }
    res.best = best;
    const rs_map_request *heavy = &requests[0];
    for (int32_t k = 1; k < n; ++k)
        if (requests[k].n_lens > heavy->n_lens) heavy = &requests[k];
    remember_batch(requests[0].params.mode, heavy->lens_m == nullptr, heavy->n_lens, full_tiles,
                   res.shape[best] + 16 * res.blocks_per_cu[best]);
    *result_host = res;
    return RS_OK;
}

int rs_batch_read_stats(const void *workspace, int32_t n, rs_map_stats *stats_host, void *stream) {
    if (!workspace || !stats_host || n < 1 || n > 65536) return fail(RS_EINVAL, "bad arguments");
    std::vector<unsigned long long> c((size_t)n * N_COUNTERS);
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = hipMemcpyAsync(c.data(), static_cast<const char *>(workspace) + batch_counters_offset(n),
                                  c.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "reading batch stats");
    for (int32_t k = 0; k < n; ++k) {
        const unsigned long long *q = &c[(size_t)k * N_COUNTERS];
        stats_host[k].rays_in_map = q[C_IN];
        stats_host[k].rays_out = q[C_OUT];
        stats_host[k].rays_singular = q[C_SING];
        stats_host[k].rays_rechecked = q[C_RECHECK];
        stats_host[k].rays_rechecked_direct = q[C_DIRECT];
        stats_host[k].rays_shot = q[C_IN] + q[C_OUT] + q[C_SING];
    }
    return RS_OK;
}

}  // extern "C"
