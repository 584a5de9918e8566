// Request loop with continuous batching (iteration-level): a scheduler thread
// admits requests by HBM footprint and slot count, and keeps the GPU busy with
// launch steps; each step gives every active request one slice (a band of ray
// rows) and runs all slices as one batched launch (rs_make_maps: persistent
// deflection kernel + FP64 re-check). Requests that arrive while a step runs
// join the next one. The threads and bookkeeping are in rs_server_core.h; this
// file is its device side:
//  * two launch steps in flight, alternating between two streams and two
//    workspaces, so the next step's blocks fill the GPU while the previous one
//    drains; each step's counters are copied to pinned host memory on its own
//    stream, so retiring a step reads host memory only;
//  * lens sets are uploaded and maps zeroed at admission on a third stream
//    (steps wait on its event); every slice adds into its map with integer
//    atomics, so slices of one map may overlap in time;
//  * finished maps are copied out on a fourth stream, without the server's lock.
// A map is the integer sum of its slices, so every result is bit-identical to the
// same map made alone.
#include "rs_internal.h"
#include "rayshoot.h"
#include "rs_debug.h"
#include "rs_server_core.h"

#include <cstring>
#include <new>
#include <vector>

namespace rs {
int fail(int code, const char *fmt, ...);
}  // namespace rs

using namespace rs;
using rs::serve::Request;
using rs::serve::StepItem;

namespace {

class HipExecutor final : public serve::Executor {
  public:
    ~HipExecutor() override { release(); }

    int create(size_t pool_bytes) {
        if (hipGetDevice(&device_) != hipSuccess) return fail(RS_EHIP, "no current device");
        if (hipMalloc(reinterpret_cast<void **>(&pool_), pool_bytes) != hipSuccess) {
            pool_ = nullptr;
            return fail(RS_ENOMEM, "cannot allocate a %zu-byte device pool", pool_bytes);
        }
        if (hipStreamCreateWithFlags(&step_stream_[0], hipStreamNonBlocking) != hipSuccess ||
            hipStreamCreateWithFlags(&step_stream_[1], hipStreamNonBlocking) != hipSuccess ||
            hipStreamCreateWithFlags(&admit_, hipStreamNonBlocking) != hipSuccess ||
            hipStreamCreateWithFlags(&copy_, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&admitted_ev_, hipEventDisableTiming) != hipSuccess ||
            hipEventCreate(&origin_) != hipSuccess || hipEventRecord(origin_, admit_) != hipSuccess)
            return fail(RS_EHIP, "cannot create streams and events");
        return RS_OK;
    }

    // Synchronise and free everything (idempotent).
    void release() {
        for (hipStream_t s : {step_stream_[0], step_stream_[1], admit_, copy_})
            if (s) (void)hipStreamSynchronize(s);
        for (int k = 0; k < 2; ++k) {
            if (ws_[k]) (void)hipFree(ws_[k]);
            if (stats_host_[k]) (void)hipHostFree(stats_host_[k]);
            ws_[k] = nullptr;
            stats_host_[k] = nullptr;
        }
        if (pool_) (void)hipFree(pool_);
        pool_ = nullptr;
        for (hipStream_t *s : {&step_stream_[0], &step_stream_[1], &admit_, &copy_}) {
            if (*s) (void)hipStreamDestroy(*s);
            *s = nullptr;
        }
        for (hipEvent_t *e : {&admitted_ev_, &origin_}) {
            if (*e) (void)hipEventDestroy(*e);
            *e = nullptr;
        }
    }

    int bind_thread() override { return hipSetDevice(device_) == hipSuccess ? RS_OK : RS_EHIP; }

    int admit(const Request &r) override {
        Range range("serve:admit");
        debug_print(2, "server: admit request %llu (%lld lenses, %lldx%lld px)", (unsigned long long)r.ticket,
                    (long long)r.n_lens, (long long)r.p.npx, (long long)r.p.npy);
        hipError_t e = launch_zero(reinterpret_cast<uint32_t *>(pool_ + r.off_map), r.p.npx * r.p.npy, admit_);
        if (e == hipSuccess && r.has_lens)
            e = hipMemcpyAsync(pool_ + r.off_lens, r.lens_xy.data(), 16 * (size_t)r.n_lens, hipMemcpyHostToDevice,
                               admit_);
        if (e == hipSuccess && r.has_m)
            e = hipMemcpyAsync(pool_ + r.off_m, r.lens_m.data(), 8 * (size_t)r.n_lens, hipMemcpyHostToDevice,
                               admit_);
        admit_pending_ = true;
        return e == hipSuccess ? RS_OK : RS_EHIP;
    }

    int launch(const std::vector<StepItem> &items, int slot, void **out) override {
        Range range("serve:launch_step");
        std::vector<rs_map_request> batch;
        batch.reserve(items.size());
        for (const StepItem &it : items) {
            const Request &r = *it.req;
            rs_map_request q{};
            q.params = r.p;
            q.params.j0 = r.p.j0 + it.row0;
            q.params.j1 = r.p.j0 + it.row1;
            q.params.flags = (r.p.flags & RS_EXACT_RECHECK) | RS_ACCUMULATE;  // zeroed at admission
            q.lens_xy = r.n_lens ? reinterpret_cast<const double *>(pool_ + r.off_lens) : nullptr;
            q.lens_m = r.has_m ? reinterpret_cast<const double *>(pool_ + r.off_m) : nullptr;
            q.n_lens = r.n_lens;
            q.map = reinterpret_cast<uint32_t *>(pool_ + r.off_map);
            batch.push_back(q);
        }
        const int32_t n = (int32_t)batch.size();
        if (debug_level() >= 2) {
            double inter = 0.0;
            for (const rs_map_request &q : batch)
                inter += (double)(q.params.i1 - q.params.i0) * (double)(q.params.j1 - q.params.j0) * (double)q.n_lens;
            debug_print(2, "server: step on slot %d, %d slices, %.3e interactions", slot, n, inter);
        }
        const size_t need = rs_batch_workspace_bytes(batch.data(), n);
        if (!need) return fail(RS_EINVAL, "invalid step");
        if (need > ws_bytes_[slot]) {
            // the other slot's step may still run; this slot's last step has retired
            if (ws_[slot]) (void)hipFree(ws_[slot]);
            ws_[slot] = nullptr;
            ws_bytes_[slot] = 0;
            const size_t bytes = need + need / 4;
            if (hipMalloc(&ws_[slot], bytes) != hipSuccess) return fail(RS_EHIP, "step workspace");
            ws_bytes_[slot] = bytes;
        }
        const size_t stats_bytes = sizeof(unsigned long long) * N_COUNTERS * (size_t)n;
        if (stats_bytes > stats_cap_[slot]) {
            if (stats_host_[slot]) (void)hipHostFree(stats_host_[slot]);
            stats_host_[slot] = nullptr;
            stats_cap_[slot] = 0;
            const size_t bytes = stats_bytes * 2;
            if (hipHostMalloc(reinterpret_cast<void **>(&stats_host_[slot]), bytes, hipHostMallocDefault) != hipSuccess) {
                stats_host_[slot] = nullptr;
                return fail(RS_EHIP, "pinned step counters");
            }
            stats_cap_[slot] = bytes;
        }
        hipStream_t stream = step_stream_[slot];
        if (admit_pending_) {
            // the maps and lenses this step uses were prepared on the admission stream
            if (hipEventRecord(admitted_ev_, admit_) != hipSuccess ||
                hipStreamWaitEvent(step_stream_[0], admitted_ev_, 0) != hipSuccess ||
                hipStreamWaitEvent(step_stream_[1], admitted_ev_, 0) != hipSuccess)
                return fail(RS_EHIP, "ordering a step after admission");
            admit_pending_ = false;
        }
        Step *st = new (std::nothrow) Step();
        if (!st) return fail(RS_ENOMEM, "out of host memory");
        st->slot = slot;
        st->n = n;
        int rc = RS_OK;
        if (hipEventCreate(&st->ev_start) != hipSuccess || hipEventCreate(&st->ev_end) != hipSuccess ||
            hipEventRecord(st->ev_start, stream) != hipSuccess)
            rc = fail(RS_EHIP, "step events");
        if (rc == RS_OK) rc = rs_make_maps(batch.data(), n, ws_[slot], ws_bytes_[slot], stream);
        if (rc == RS_OK &&
            hipMemcpyAsync(stats_host_[slot], static_cast<const char *>(ws_[slot]) + batch_counters_offset(n),
                           stats_bytes, hipMemcpyDeviceToHost, stream) != hipSuccess)
            rc = fail(RS_EHIP, "step counters");
        if (rc == RS_OK && hipEventRecord(st->ev_end, stream) != hipSuccess) rc = fail(RS_EHIP, "step events");
        if (rc != RS_OK) {
            drop(st);
            return rc;
        }
        *out = st;
        return RS_OK;
    }

    int poll(void *h, bool block) override {
        Step *st = static_cast<Step *>(h);
        const hipError_t q = block ? hipEventSynchronize(st->ev_end) : hipEventQuery(st->ev_end);
        if (q == hipSuccess) return RS_OK;
        if (q == hipErrorNotReady) return 1;
        return RS_EHIP;
    }

    void retire(void *h, double *own_ms, double *end_ms, std::vector<rs_map_stats> *stats) override {
        Range range("serve:retire");
        Step *st = static_cast<Step *>(h);
        float own = 0.0f, end = 0.0f;
        *own_ms = hipEventElapsedTime(&own, st->ev_start, st->ev_end) == hipSuccess ? own : 0.0;
        *end_ms = hipEventElapsedTime(&end, origin_, st->ev_end) == hipSuccess ? end : 0.0;
        // the counters reached pinned memory before the step's end event
        const unsigned long long *c = stats_host_[st->slot];
        stats->assign(st->n, rs_map_stats{});
        for (int32_t k = 0; k < st->n; ++k) {
            const unsigned long long *ck = c + (size_t)k * N_COUNTERS;
            rs_map_stats &s = (*stats)[k];
            s.rays_in_map = ck[C_IN];
            s.rays_out = ck[C_OUT];
            s.rays_singular = ck[C_SING];
            s.rays_rechecked = ck[C_RECHECK];
            s.rays_rechecked_direct = ck[C_DIRECT];
            s.rays_shot = ck[C_IN] + ck[C_OUT] + ck[C_SING];
        }
        drop(st);
    }

    void drop(void *h) override {
        Step *st = static_cast<Step *>(h);
        if (!st) return;
        if (st->ev_start) (void)hipEventDestroy(st->ev_start);
        if (st->ev_end) (void)hipEventDestroy(st->ev_end);
        delete st;
    }

    int copy_map(const Request &r, uint32_t *host) override {
        Range range("serve:copy_map");
        const size_t bytes = 4 * (size_t)(r.p.npx * r.p.npy);
        // every step that touched the map has retired (its end event completed)
        if (hipMemcpyAsync(host, pool_ + r.off_map, bytes, hipMemcpyDeviceToHost, copy_) != hipSuccess ||
            hipStreamSynchronize(copy_) != hipSuccess)
            return RS_EHIP;
        return RS_OK;
    }

  private:
    struct Step {
        hipEvent_t ev_start = nullptr, ev_end = nullptr;
        int slot = 0;
        int32_t n = 0;
    };

    int device_ = 0;
    char *pool_ = nullptr;
    hipStream_t step_stream_[2] = {nullptr, nullptr};
    hipStream_t admit_ = nullptr, copy_ = nullptr;
    hipEvent_t admitted_ev_ = nullptr, origin_ = nullptr;
    bool admit_pending_ = false;
    void *ws_[2] = {nullptr, nullptr};
    size_t ws_bytes_[2] = {0, 0};
    unsigned long long *stats_host_[2] = {nullptr, nullptr};
    size_t stats_cap_[2] = {0, 0};
};

}  // namespace

struct rs_server {
    HipExecutor ex;
    serve::Server core;
    explicit rs_server(const rs_server_cfg &cfg) : core(cfg, &ex) {}
};

extern "C" {

int rs_server_create(const rs_server_cfg *cfg, rs_server **out) {
    if (!cfg || !out) return fail(RS_EINVAL, "NULL argument");
    if (cfg->hbm_budget_bytes < 4096 || cfg->max_inflight < 1 || (cfg->mode != RS_FP32 && cfg->mode != RS_MIXED))
        return fail(RS_EINVAL, "bad server configuration");
    rs_server *s = new (std::nothrow) rs_server(*cfg);
    if (!s) return fail(RS_ENOMEM, "out of host memory");
    const int rc = s->ex.create(cfg->hbm_budget_bytes);
    if (rc != RS_OK) {
        delete s;
        return rc;
    }
    s->core.start();
    *out = s;
    return RS_OK;
}

int rs_server_submit(rs_server *s, const rs_map_params *params, const double *lens_xy_host,
                     const double *lens_m_host, int64_t n_lens, uint32_t *map_host, uint64_t *ticket) {
    if (!s) return fail(RS_EINVAL, "NULL argument");
    return s->core.submit(params, lens_xy_host, lens_m_host, n_lens, map_host, ticket);
}

int rs_server_poll(rs_server *s, uint64_t ticket, int *done) {
    if (!s) return fail(RS_EINVAL, "NULL argument");
    return s->core.poll(ticket, done);
}

int rs_server_wait(rs_server *s, uint64_t ticket, rs_map_stats *stats, double *latency_s) {
    if (!s) return fail(RS_EINVAL, "NULL argument");
    return s->core.wait(ticket, stats, latency_s);
}

int rs_server_cancel(rs_server *s, uint64_t ticket) {
    if (!s) return fail(RS_EINVAL, "NULL argument");
    return s->core.cancel(ticket);
}

int rs_server_get_stats(rs_server *s, rs_server_stats *out) {
    if (!s || !out) return fail(RS_EINVAL, "NULL argument");
    s->core.get_stats(out);
    return RS_OK;
}

void rs_server_destroy(rs_server *s) {
    if (!s) return;
    s->core.stop();
    s->ex.release();
    delete s;
}

}  // extern "C"
