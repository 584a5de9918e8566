// Request loop with continuous batching (iteration-level): a scheduler thread
// admits requests by HBM footprint and slot count, and keeps the GPU busy with
// launch steps; each step gives every active request one slice (a band of ray
// rows) and runs all slices as one batched launch (rs_make_maps: persistent
// deflection kernel + FP64 re-check). Requests that arrive while a step runs
// join the next one. Two steps are kept in flight, on two streams, so the next
// step's blocks fill the GPU while the previous one drains. Lens sets are
// uploaded and maps zeroed at admission on a third stream; every slice then
// adds into its map with integer atomics, so slices of one map may overlap in
// time. Finished maps are copied out on a fourth stream. A map is the integer
// sum of its slices, so every result is bit-identical to the same map made alone.
#include "rs_internal.h"
#include "rayshoot.h"
#include "rs_sched.h"

#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

namespace rs {
int fail(int code, const char *fmt, ...);
int validate(const rs_map_params *p, int64_t n_lens);
}  // namespace rs

using namespace rs;
using rs::sched::Arena;
using rs::sched::Job;
using rs::sched::Policy;
using rs::sched::Slice;

namespace {

double now_s() {
    using clk = std::chrono::steady_clock;
    static const clk::time_point t0 = clk::now();
    return std::chrono::duration<double>(clk::now() - t0).count();
}

enum State { WAITING = 0, ACTIVE = 1, DONE = 2, CANCELED = 3, FAILED = 4 };

struct Request {
    uint64_t ticket = 0;
    rs_map_params p{};
    std::vector<double> lens_xy, lens_m;
    int64_t n_lens = 0;
    uint32_t *map_host = nullptr;
    size_t off_lens = 0, off_m = 0, off_map = 0;
    bool has_lens = false, has_m = false, has_map = false;
    rs_map_stats stats{};
    int state = WAITING;
    int error = RS_OK;
    double t_submit = 0, t_done = 0;
};

struct Step {
    std::vector<Slice> slices;
    hipEvent_t ev_start = nullptr, ev_end = nullptr;
    int ws_index = 0;
    double interactions = 0;
};

size_t footprint_of(const rs_map_params &p, int64_t n_lens, bool masses) {
    const size_t a = 256;
    return Arena::round_up(16 * (size_t)n_lens, a) + (masses ? Arena::round_up(8 * (size_t)n_lens, a) : 0) +
           Arena::round_up(4 * (size_t)(p.npx * p.npy), a);
}

}  // namespace

struct rs_server {
    rs_server_cfg cfg{};
    Policy policy;
    Arena arena;
    char *pool = nullptr;
    hipStream_t step_stream[2] = {nullptr, nullptr};  // alternate launch steps
    hipStream_t admit = nullptr;                       // lens uploads, map zeroing
    hipStream_t copy = nullptr;                        // stats and maps back to the host
    hipEvent_t admitted_ev = nullptr;                  // last admission work
    struct Retired {
        hipEvent_t ev;
        double interactions;
    };
    std::deque<Retired> recent;                        // ends of the last retired steps
    bool admit_pending = false;
    int device = 0;

    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::map<uint64_t, Request> reqs;
    uint64_t next_ticket = 1;
    bool stop = false;
    bool dead = false;   // the scheduler thread stopped (no device, or a device error)
    std::thread thread;

    std::deque<Step> inflight;
    void *ws[2] = {nullptr, nullptr};
    size_t ws_bytes[2] = {0, 0};
    int ws_next = 0;
    double rate = 6e12;   // ray-lens interactions per second, refined from measured steps

    // statistics
    std::vector<double> latencies;
    uint64_t completed = 0, canceled = 0, failed = 0, steps = 0;
    double interactions = 0, t_first_submit = -1, t_last_done = 0, gpu_busy_s = 0;
    size_t max_waiting = 0;

    rs_server(const rs_server_cfg &c) : cfg(c), policy(c.hbm_budget_bytes, c.max_inflight), arena(c.hbm_budget_bytes) {}

    void run();
    bool launch_step();
    void retire_step(Step &s);
    void finish(Request &r, int state, int error);
    void fail_all(int error);
};

// The scheduler thread cannot go on (no device, or a device error): every request
// not yet finished fails with error, the steps in flight are dropped, and the
// server refuses new submissions. Called with mu held.
void rs_server::fail_all(int error) {
    dead = true;
    for (Step &st : inflight) {
        if (st.ev_start) (void)hipEventDestroy(st.ev_start);
        if (st.ev_end) (void)hipEventDestroy(st.ev_end);
    }
    inflight.clear();
    for (auto &kv : reqs)
        if (kv.second.state < DONE) finish(kv.second, FAILED, error);
}

void rs_server::finish(Request &r, int state, int error) {
    if (r.has_lens) arena.release(r.off_lens);
    if (r.has_m) arena.release(r.off_m);
    if (r.has_map) arena.release(r.off_map);
    r.has_lens = r.has_m = r.has_map = false;
    r.state = state;
    r.error = error;
    r.t_done = now_s();
    std::vector<double>().swap(r.lens_xy);
    std::vector<double>().swap(r.lens_m);
    if (state == DONE) {
        ++completed;
        latencies.push_back(r.t_done - r.t_submit);
        t_last_done = r.t_done;
    } else if (state == CANCELED) {
        ++canceled;
    } else {
        ++failed;
    }
    cv_done.notify_all();
}

// Plan and enqueue one step (called with the lock held). Returns false if there was nothing to run.
bool rs_server::launch_step() {
    // Requests waiting for admission mean the GPU is the bottleneck: longer steps then
    // trade a little responsiveness for less per-step overhead.
    const double slice_s = (cfg.slice_ms > 0 ? cfg.slice_ms : 10.0) * 1e-3 * (policy.waiting() > 0 ? 4.0 : 1.0);
    const double target = rate * slice_s;
    std::vector<Slice> slices = policy.plan(target, now_s(), 0.25, cfg.starve_s > 0 ? cfg.starve_s : 0.5);
    if (slices.empty()) return false;
    std::vector<rs_map_request> batch;
    batch.reserve(slices.size());
    double inter = 0;
    for (const Slice &s : slices) {
        Request &r = reqs.at(s.ticket);
        rs_map_request q{};
        q.params = r.p;
        q.params.j0 = r.p.j0 + s.row0;
        q.params.j1 = r.p.j0 + s.row1;
        q.params.flags = (r.p.flags & RS_EXACT_RECHECK) | RS_ACCUMULATE;  // zeroed at admission
        q.params.mode = cfg.mode;
        q.lens_xy = r.n_lens ? reinterpret_cast<const double *>(pool + r.off_lens) : nullptr;
        q.lens_m = r.has_m ? reinterpret_cast<const double *>(pool + r.off_m) : nullptr;
        q.n_lens = r.n_lens;
        q.map = reinterpret_cast<uint32_t *>(pool + r.off_map);
        inter += (double)(q.params.i1 - q.params.i0) * (double)(s.row1 - s.row0) * (double)r.n_lens;
        batch.push_back(q);
    }
    Step st;
    st.slices = slices;
    st.ws_index = ws_next;
    st.interactions = inter;
    ws_next ^= 1;
    const size_t need = rs_batch_workspace_bytes(batch.data(), (int32_t)batch.size());
    int rc = need ? RS_OK : RS_EINVAL;
    if (rc == RS_OK && need > ws_bytes[st.ws_index]) {
        if (ws[st.ws_index]) (void)hipFree(ws[st.ws_index]);
        ws[st.ws_index] = nullptr;
        ws_bytes[st.ws_index] = 0;
        const size_t bytes = need + need / 4;
        if (hipMalloc(&ws[st.ws_index], bytes) != hipSuccess) rc = RS_EHIP;
        else ws_bytes[st.ws_index] = bytes;
    }
    hipStream_t stream = step_stream[st.ws_index];
    if (rc == RS_OK && admit_pending) {
        // the maps and lenses this step uses were prepared on the admission stream
        if (hipEventRecord(admitted_ev, admit) != hipSuccess ||
            hipStreamWaitEvent(step_stream[0], admitted_ev, 0) != hipSuccess ||
            hipStreamWaitEvent(step_stream[1], admitted_ev, 0) != hipSuccess)
            rc = RS_EHIP;
        admit_pending = false;
    }
    if (rc == RS_OK && (hipEventCreate(&st.ev_start) != hipSuccess || hipEventCreate(&st.ev_end) != hipSuccess ||
                        hipEventRecord(st.ev_start, stream) != hipSuccess))
        rc = RS_EHIP;
    if (rc == RS_OK)
        rc = rs_make_maps(batch.data(), (int32_t)batch.size(), ws[st.ws_index], ws_bytes[st.ws_index], stream);
    if (rc == RS_OK && hipEventRecord(st.ev_end, stream) != hipSuccess) rc = RS_EHIP;
    if (rc != RS_OK) {
        // the step could not run: fail its requests
        for (const Slice &s : slices) {
            policy.cancel(s.ticket);
            Request &r = reqs.at(s.ticket);
            r.error = rc;
        }
        std::vector<Job> done = policy.step_done(slices, now_s());
        for (Job &j : done) finish(reqs.at(j.ticket), FAILED, rc);
        if (st.ev_start) (void)hipEventDestroy(st.ev_start);
        if (st.ev_end) (void)hipEventDestroy(st.ev_end);
        return true;
    }
    ++steps;
    inflight.push_back(std::move(st));
    return true;
}

void rs_server::retire_step(Step &s) {
    // Device throughput from retirements: interactions of the last steps over the
    // GPU time between their ends (exact while the pipeline is busy; low when it
    // idles, which only makes the next steps smaller).
    float own = 0.0f;
    if (hipEventElapsedTime(&own, s.ev_start, s.ev_end) == hipSuccess && own > 0.0f) gpu_busy_s += own * 1e-3;
    const hipEvent_t end_ev = s.ev_end;  // kept in `recent`, destroyed when it leaves
    recent.push_back({end_ev, s.interactions});
    s.ev_end = nullptr;
    while (recent.size() > 8) {
        (void)hipEventDestroy(recent.front().ev);
        recent.pop_front();
    }
    if (recent.size() >= 3) {
        float span = 0.0f;
        double work = 0.0;
        for (size_t k = 1; k < recent.size(); ++k) work += recent[k].interactions;
        if (hipEventElapsedTime(&span, recent.front().ev, recent.back().ev) == hipSuccess && span > 0.0f &&
            work > 1e9) {
            const double r = work / (span * 1e-3);
            rate = std::min(2e13, std::max(1e12, r));
        }
    }
    interactions += s.interactions;
    // per-slice counters of this step, in slice order
    std::vector<rs_map_stats> st(s.slices.size());
    const bool have_stats =
        rs_batch_read_stats(ws[s.ws_index], (int32_t)s.slices.size(), st.data(), copy) == RS_OK;
    for (size_t k = 0; k < s.slices.size(); ++k) {
        Request &r = reqs.at(s.slices[k].ticket);
        if (!have_stats) r.error = RS_EHIP;
        r.stats.rays_shot += st[k].rays_shot;
        r.stats.rays_in_map += st[k].rays_in_map;
        r.stats.rays_out += st[k].rays_out;
        r.stats.rays_singular += st[k].rays_singular;
        r.stats.rays_rechecked += st[k].rays_rechecked;
        r.stats.rays_rechecked_direct += st[k].rays_rechecked_direct;
    }
    std::vector<Job> done = policy.step_done(s.slices, now_s());
    for (Job &j : done) {
        Request &r = reqs.at(j.ticket);
        if (j.cancel) {
            finish(r, CANCELED, RS_ECANCELED);
            continue;
        }
        int err = r.error;
        if (err == RS_OK && r.map_host) {
            const size_t bytes = 4 * (size_t)(r.p.npx * r.p.npy);
            if (hipStreamWaitEvent(copy, end_ev, 0) != hipSuccess ||
                hipMemcpyAsync(r.map_host, pool + r.off_map, bytes, hipMemcpyDeviceToHost, copy) != hipSuccess ||
                hipStreamSynchronize(copy) != hipSuccess)
                err = RS_EHIP;
        }
        finish(r, err == RS_OK ? DONE : FAILED, err);
    }
    (void)hipEventDestroy(s.ev_start);
}

void rs_server::run() {
    std::unique_lock<std::mutex> lk(mu);
    if (hipSetDevice(device) != hipSuccess) {
        // no device for this thread: nothing can run, so fail everything now and later
        fail_all(RS_EHIP);
        return;
    }
    for (;;) {
        // 1. admission (FIFO, by slot and arena space)
        std::vector<uint64_t> dropped;
        std::vector<uint64_t> admitted = policy.admit(
            now_s(),
            [&](Job &j) {
                Request &r = reqs.at(j.ticket);
                size_t a = 0, b = 0, c = 0;
                const bool masses = !r.lens_m.empty();
                if (r.n_lens > 0 && !arena.alloc(16 * (size_t)r.n_lens, &a)) return false;
                if (masses && !arena.alloc(8 * (size_t)r.n_lens, &b)) {
                    if (r.n_lens > 0) arena.release(a);
                    return false;
                }
                if (!arena.alloc(4 * (size_t)(r.p.npx * r.p.npy), &c)) {
                    if (r.n_lens > 0) arena.release(a);
                    if (masses) arena.release(b);
                    return false;
                }
                r.off_lens = a;
                r.off_m = b;
                r.off_map = c;
                r.has_lens = r.n_lens > 0;
                r.has_m = masses;
                r.has_map = true;
                return true;
            },
            &dropped);
        for (uint64_t t : dropped) {
            Request &r = reqs.at(t);
            const bool too_big = footprint_of(r.p, r.n_lens, !r.lens_m.empty()) > cfg.hbm_budget_bytes;
            finish(r, too_big ? FAILED : CANCELED, too_big ? RS_ENOMEM : RS_ECANCELED);
        }
        for (uint64_t t : admitted) {
            Request &r = reqs.at(t);
            r.state = ACTIVE;
            hipError_t e = launch_zero(reinterpret_cast<uint32_t *>(pool + r.off_map), r.p.npx * r.p.npy, admit);
            if (e == hipSuccess && r.has_lens)
                e = hipMemcpyAsync(pool + r.off_lens, r.lens_xy.data(), 16 * (size_t)r.n_lens, hipMemcpyHostToDevice,
                                   admit);
            if (e == hipSuccess && r.has_m)
                e = hipMemcpyAsync(pool + r.off_m, r.lens_m.data(), 8 * (size_t)r.n_lens, hipMemcpyHostToDevice,
                                   admit);
            admit_pending = true;
            if (e != hipSuccess) {
                policy.cancel(t);
                r.error = RS_EHIP;
            }
        }
        {
            std::vector<Job> done = policy.reap(now_s());  // cancelled before any slice ran, or empty windows
            for (Job &j : done) {
                Request &r = reqs.at(j.ticket);
                if (j.cancel) finish(r, r.error ? FAILED : CANCELED, r.error ? r.error : RS_ECANCELED);
                else finish(r, DONE, RS_OK);
            }
        }
        max_waiting = std::max(max_waiting, policy.waiting());

        // 2. keep two steps in flight
        bool launched = false;
        if (inflight.size() < 2) launched = launch_step();

        // 3. retire the oldest step when it is done, or block on it when the pipeline is full
        if (!inflight.empty()) {
            Step &s = inflight.front();
            const bool full = inflight.size() >= 2 || !launched;
            hipError_t q = hipEventQuery(s.ev_end);
            if (q == hipErrorNotReady && full) {
                hipEvent_t ev = s.ev_end;
                lk.unlock();
                q = hipEventSynchronize(ev);
                lk.lock();
            }
            if (q == hipSuccess) {
                Step done = std::move(inflight.front());
                inflight.pop_front();
                retire_step(done);
            } else if (q != hipErrorNotReady) {
                // the device reported an error: nothing more can run, so fail every
                // unfinished request and stop (submissions are refused from now on)
                fail_all(RS_EHIP);
                return;
            }
            continue;
        }
        if (stop && policy.waiting() == 0 && policy.active() == 0) break;
        if (!launched) cv_work.wait_for(lk, std::chrono::milliseconds(20));
    }
}

extern "C" {

int rs_server_create(const rs_server_cfg *cfg, rs_server **out) {
    if (!cfg || !out) return fail(RS_EINVAL, "NULL argument");
    if (cfg->hbm_budget_bytes < 4096 || cfg->max_inflight < 1 || (cfg->mode != RS_FP32 && cfg->mode != RS_MIXED))
        return fail(RS_EINVAL, "bad server configuration");
    rs_server *s = new (std::nothrow) rs_server(*cfg);
    if (!s) return fail(RS_ENOMEM, "out of host memory");
    if (hipGetDevice(&s->device) != hipSuccess ||
        hipMalloc(reinterpret_cast<void **>(&s->pool), cfg->hbm_budget_bytes) != hipSuccess) {
        delete s;
        return fail(RS_ENOMEM, "cannot allocate a %zu-byte device pool", cfg->hbm_budget_bytes);
    }
    if (hipStreamCreateWithFlags(&s->step_stream[0], hipStreamNonBlocking) != hipSuccess ||
        hipStreamCreateWithFlags(&s->step_stream[1], hipStreamNonBlocking) != hipSuccess ||
        hipStreamCreateWithFlags(&s->admit, hipStreamNonBlocking) != hipSuccess ||
        hipStreamCreateWithFlags(&s->copy, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&s->admitted_ev, hipEventDisableTiming) != hipSuccess) {
        for (hipStream_t st : {s->step_stream[0], s->step_stream[1], s->admit, s->copy})
            if (st) (void)hipStreamDestroy(st);
        if (s->admitted_ev) (void)hipEventDestroy(s->admitted_ev);
        (void)hipFree(s->pool);
        delete s;
        return fail(RS_EHIP, "cannot create streams");
    }
    s->thread = std::thread([s] { s->run(); });
    *out = s;
    return RS_OK;
}

int rs_server_submit(rs_server *s, const rs_map_params *params, const double *lens_xy_host,
                     const double *lens_m_host, int64_t n_lens, uint32_t *map_host, uint64_t *ticket) {
    if (!s || !params || !ticket) return fail(RS_EINVAL, "NULL argument");
    int rc = validate(params, n_lens);
    if (rc) return rc;
    if (params->flags & RS_RANDOM_RAYS) return fail(RS_EINVAL, "the server makes regular-grid maps only");
    if (n_lens > 0 && !lens_xy_host) return fail(RS_EINVAL, "lens_xy is NULL");
    const double rays = (double)(params->i1 - params->i0) * (double)(params->j1 - params->j0);
    if (rays >= 4294967296.0) return fail(RS_EINVAL, "window holds 2^32 rays or more");
    Request r;
    r.p = *params;
    r.p.mode = s->cfg.mode;
    r.n_lens = n_lens;
    r.lens_xy.assign(lens_xy_host, lens_xy_host + 2 * n_lens);
    if (lens_m_host) r.lens_m.assign(lens_m_host, lens_m_host + n_lens);
    r.map_host = map_host;
    r.t_submit = now_s();
    Job j;
    j.width = params->i1 - params->i0;
    j.rows = params->j1 - params->j0;
    j.n_lens = n_lens;
    j.footprint = footprint_of(r.p, n_lens, lens_m_host != nullptr);
    j.t_submit = r.t_submit;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stop) return fail(RS_ECANCELED, "server is stopping");
        if (s->dead) return fail(RS_EHIP, "server stopped: no device or a device error");
        r.ticket = j.ticket = s->next_ticket++;
        if (s->t_first_submit < 0) s->t_first_submit = r.t_submit;
        s->reqs.emplace(r.ticket, std::move(r));
        s->policy.submit(j);
        *ticket = j.ticket;
    }
    s->cv_work.notify_all();
    return RS_OK;
}

int rs_server_poll(rs_server *s, uint64_t ticket, int *done) {
    if (!s || !done) return fail(RS_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return fail(RS_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
    *done = it->second.state >= DONE ? 1 : 0;
    return RS_OK;
}

int rs_server_wait(rs_server *s, uint64_t ticket, rs_map_stats *stats, double *latency_s) {
    if (!s) return fail(RS_EINVAL, "NULL argument");
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return fail(RS_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
    s->cv_done.wait(lk, [&] { return it->second.state >= DONE; });
    const Request &r = it->second;
    const int err = r.error;
    if (stats) *stats = r.stats;
    if (latency_s) *latency_s = r.t_done - r.t_submit;
    const int state = r.state;
    s->reqs.erase(it);
    if (state == CANCELED) return fail(RS_ECANCELED, "request %llu was cancelled", (unsigned long long)ticket);
    if (err != RS_OK) return fail(err, "request %llu failed", (unsigned long long)ticket);
    return RS_OK;
}

int rs_server_cancel(rs_server *s, uint64_t ticket) {
    if (!s) return fail(RS_EINVAL, "NULL argument");
    {
        std::lock_guard<std::mutex> lk(s->mu);
        auto it = s->reqs.find(ticket);
        if (it == s->reqs.end() || it->second.state >= DONE) return fail(RS_EINVAL, "ticket not pending");
        s->policy.cancel(ticket);
    }
    s->cv_work.notify_all();
    return RS_OK;
}

int rs_server_get_stats(rs_server *s, rs_server_stats *out) {
    if (!s || !out) return fail(RS_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    rs_server_stats st{};
    st.completed = s->completed;
    st.canceled = s->canceled;
    st.failed = s->failed;
    st.steps = s->steps;
    st.waiting = s->policy.waiting();
    st.active = s->policy.active();
    st.max_waiting = s->max_waiting;
    st.hbm_in_use_bytes = s->arena.in_use();
    st.hbm_peak_bytes = s->arena.peak();
    st.interactions = s->interactions;
    st.gpu_busy_s = s->gpu_busy_s;
    const double span = s->t_last_done - s->t_first_submit;
    st.maps_per_s = (s->completed && span > 0) ? (double)s->completed / span : 0.0;
    st.latency_p50_s = sched::percentile(s->latencies, 50.0);
    st.latency_p99_s = sched::percentile(s->latencies, 99.0);
    double mean = 0;
    for (double v : s->latencies) mean += v;
    st.latency_mean_s = s->latencies.empty() ? 0.0 : mean / (double)s->latencies.size();
    st.latency_max_s = s->latencies.empty() ? 0.0 : *std::max_element(s->latencies.begin(), s->latencies.end());
    *out = st;
    return RS_OK;
}

void rs_server_destroy(rs_server *s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        // drop what has not been admitted yet; running requests finish
        for (auto &kv : s->reqs)
            if (kv.second.state == WAITING) s->policy.cancel(kv.first);
    }
    s->cv_work.notify_all();
    if (s->thread.joinable()) s->thread.join();
    for (hipStream_t st : {s->step_stream[0], s->step_stream[1], s->admit, s->copy})
        if (st) (void)hipStreamSynchronize(st);
    for (void *w : s->ws)
        if (w) (void)hipFree(w);
    (void)hipFree(s->pool);
    for (hipStream_t st : {s->step_stream[0], s->step_stream[1], s->admit, s->copy})
        if (st) (void)hipStreamDestroy(st);
    if (s->admitted_ev) (void)hipEventDestroy(s->admitted_ev);
    for (auto &r : s->recent) (void)hipEventDestroy(r.ev);
    delete s;
}

}  // extern "C"
