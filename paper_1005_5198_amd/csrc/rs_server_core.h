// The request loop's threads and bookkeeping (continuous batching), free of
// device calls: a scheduler thread admits requests (Policy, Arena), plans launch
// steps, keeps two in flight, retires them and hands finished maps back. Every
// device operation goes through an Executor (serve.cpp: HIP streams, events and
// rs_make_maps; tests: a simulated device), so the threading can be checked on
// the CPU under a thread sanitizer.
//
// Locking: one mutex guards the request table, the policy, the arena and the
// statistics. The scheduler thread releases it while it waits for a step and
// while it copies finished maps to host memory, so submissions, polls and
// waits never stall behind a device copy.
#pragma once

#include "rayshoot.h"
#include "rs_sched.h"

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdint>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

namespace rs {
int fail(int code, const char *fmt, ...);
int validate(const rs_map_params *p, int64_t n_lens);

namespace serve {

enum State { WAITING = 0, ACTIVE = 1, COPYING = 2, DONE = 3, CANCELED = 4, FAILED = 5 };

struct Request {
    uint64_t ticket = 0;
    rs_map_params p{};
    std::vector<double> lens_xy, lens_m;
    int64_t n_lens = 0;
    uint32_t *map_host = nullptr;
    size_t off_lens = 0, off_m = 0, off_map = 0;   // offsets in the device pool
    bool has_lens = false, has_m = false, has_map = false;
    rs_map_stats stats{};
    int state = WAITING;
    int error = RS_OK;
    double t_submit = 0, t_done = 0;
};

// One band of rows of a request in a launch step.
struct StepItem {
    const Request *req;
    int64_t row0, row1;   // relative to the request window's first row
};

// Device side of the loop. Calls come from the scheduler thread only, with the
// server's mutex held except for copy_map.
class Executor {
  public:
    virtual ~Executor() = default;
    // Once, on the scheduler thread, before anything else.
    virtual int bind_thread() = 0;
    // Zero the request's map and upload its lenses into the pool (asynchronous;
    // later launches are ordered after it).
    virtual int admit(const Request &r) = 0;
    // Enqueue one step on workspace/stream slot `slot` (0 or 1, never the slot of
    // the step still in flight). On success *step identifies it.
    virtual int launch(const std::vector<StepItem> &items, int slot, void **step) = 0;
    // RS_OK when the step has finished, 1 while it runs, an RS_E* code on a device
    // error. block: wait for it (called without the mutex).
    virtual int poll(void *step, bool block) = 0;
    // A finished step: its device time, the time of its end since the executor's
    // start (ms), the counters of each item in launch order; releases it.
    virtual void retire(void *step, double *own_ms, double *end_ms, std::vector<rs_map_stats> *stats) = 0;
    // Release a step without reading it (device error).
    virtual void drop(void *step) = 0;
    // Blocking copy of a finished map to host memory (called without the mutex).
    virtual int copy_map(const Request &r, uint32_t *host) = 0;
};

inline double now_s() {
    using clk = std::chrono::steady_clock;
    static const clk::time_point t0 = clk::now();
    return std::chrono::duration<double>(clk::now() - t0).count();
}

inline size_t footprint_of(const rs_map_params &p, int64_t n_lens, bool masses) {
    const size_t a = 256;
    return sched::Arena::round_up(16 * (size_t)n_lens, a) + (masses ? sched::Arena::round_up(8 * (size_t)n_lens, a) : 0) +
           sched::Arena::round_up(4 * (size_t)(p.npx * p.npy), a);
}

class Server {
  public:
    Server(const rs_server_cfg &cfg, Executor *ex)
        : cfg_(cfg), ex_(ex), policy_(cfg.hbm_budget_bytes, cfg.max_inflight), arena_(cfg.hbm_budget_bytes) {}
    Server(const Server &) = delete;
    Server &operator=(const Server &) = delete;

    void start() { thread_ = std::thread([this] { run(); }); }

    int submit(const rs_map_params *params, const double *lens_xy, const double *lens_m, int64_t n_lens,
               uint32_t *map_host, uint64_t *ticket) {
        if (!params || !ticket) return fail(RS_EINVAL, "NULL argument");
        int rc = validate(params, n_lens);
        if (rc) return rc;
        if (params->flags & RS_RANDOM_RAYS) return fail(RS_EINVAL, "the server makes regular-grid maps only");
        if (n_lens > 0 && !lens_xy) return fail(RS_EINVAL, "lens_xy is NULL");
        const double rays = (double)(params->i1 - params->i0) * (double)(params->j1 - params->j0);
        if (rays >= 4294967296.0) return fail(RS_EINVAL, "window holds 2^32 rays or more");
        {
            // refuse early, before copying the lenses, when the queue is full
            std::lock_guard<std::mutex> lk(mu_);
            if (rc = refusal(); rc) return rc;
        }
        Request r;
        r.p = *params;
        r.p.mode = cfg_.mode;
        r.n_lens = n_lens;
        r.lens_xy.assign(lens_xy, lens_xy + 2 * n_lens);
        if (lens_m) r.lens_m.assign(lens_m, lens_m + n_lens);
        r.map_host = map_host;
        r.t_submit = now_s();
        sched::Job j;
        j.width = params->i1 - params->i0;
        j.rows = params->j1 - params->j0;
        j.n_lens = n_lens;
        j.footprint = footprint_of(r.p, n_lens, lens_m != nullptr);
        j.t_submit = r.t_submit;
        {
            std::lock_guard<std::mutex> lk(mu_);
            if (rc = refusal(); rc) return rc;
            r.ticket = j.ticket = next_ticket_++;
            if (t_first_submit_ < 0) t_first_submit_ = r.t_submit;
            reqs_.emplace(r.ticket, std::move(r));
            policy_.submit(j);
            *ticket = j.ticket;
        }
        cv_work_.notify_all();
        return RS_OK;
    }

    int poll(uint64_t ticket, int *done) {
        if (!done) return fail(RS_EINVAL, "NULL argument");
        std::lock_guard<std::mutex> lk(mu_);
        auto it = reqs_.find(ticket);
        if (it == reqs_.end()) return fail(RS_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
        *done = it->second.state >= DONE ? 1 : 0;
        return RS_OK;
    }

    int wait(uint64_t ticket, rs_map_stats *stats, double *latency_s) {
        std::unique_lock<std::mutex> lk(mu_);
        auto it = reqs_.find(ticket);
        if (it == reqs_.end()) return fail(RS_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
        cv_done_.wait(lk, [&] { return it->second.state >= DONE; });
        const Request &r = it->second;
        const int err = r.error;
        if (stats) *stats = r.stats;
        if (latency_s) *latency_s = r.t_done - r.t_submit;
        const int state = r.state;
        reqs_.erase(it);
        if (state == CANCELED) return fail(RS_ECANCELED, "request %llu was cancelled", (unsigned long long)ticket);
        if (err != RS_OK) return fail(err, "request %llu failed", (unsigned long long)ticket);
        return RS_OK;
    }

    int cancel(uint64_t ticket) {
        {
            std::lock_guard<std::mutex> lk(mu_);
            auto it = reqs_.find(ticket);
            if (it == reqs_.end() || it->second.state >= COPYING) return fail(RS_EINVAL, "ticket not pending");
            policy_.cancel(ticket);
        }
        cv_work_.notify_all();
        return RS_OK;
    }

    void get_stats(rs_server_stats *out) {
        std::lock_guard<std::mutex> lk(mu_);
        rs_server_stats st{};
        st.completed = completed_;
        st.canceled = canceled_;
        st.failed = failed_;
        st.steps = steps_;
        st.waiting = policy_.waiting();
        st.active = policy_.active();
        st.max_waiting = max_waiting_;
        st.hbm_in_use_bytes = arena_.in_use();
        st.hbm_peak_bytes = arena_.peak();
        st.interactions = interactions_;
        st.gpu_busy_s = gpu_busy_s_;
        const double span = t_last_done_ - t_first_submit_;
        st.maps_per_s = (completed_ && span > 0) ? (double)completed_ / span : 0.0;
        st.latency_p50_s = sched::percentile(latencies_, 50.0);
        st.latency_p99_s = sched::percentile(latencies_, 99.0);
        double mean = 0;
        for (double v : latencies_) mean += v;
        st.latency_mean_s = latencies_.empty() ? 0.0 : mean / (double)latencies_.size();
        st.latency_max_s = latencies_.empty() ? 0.0 : *std::max_element(latencies_.begin(), latencies_.end());
        st.rejected_busy = rejected_busy_;
        *out = st;
    }

    // Stop admitting, drop waiting requests, finish running ones, join the thread.
    void stop() {
        {
            std::lock_guard<std::mutex> lk(mu_);
            stop_ = true;
            for (auto &kv : reqs_)
                if (kv.second.state == WAITING) policy_.cancel(kv.first);
        }
        cv_work_.notify_all();
        if (thread_.joinable()) thread_.join();
    }

    size_t max_waiting_queue() const { return cfg_.max_waiting > 0 ? (size_t)cfg_.max_waiting : 4096; }

  private:
    struct Step {
        void *h = nullptr;
        std::vector<sched::Slice> slices;
        int slot = 0;
        double interactions = 0;
    };
    struct EndMark {
        double end_ms, interactions;
    };

    // Why a submission is refused now (with the mutex held), or RS_OK.
    int refusal() {
        if (stop_) return fail(RS_ECANCELED, "server is stopping");
        if (dead_) return fail(RS_EHIP, "server stopped: no device or a device error");
        if (policy_.waiting() >= max_waiting_queue()) {
            ++rejected_busy_;
            return fail(RS_EBUSY, "%zu requests are waiting for admission (the server's limit)", policy_.waiting());
        }
        return RS_OK;
    }

    void finish(Request &r, int state, int error) {
        if (r.has_lens) arena_.release(r.off_lens);
        if (r.has_m) arena_.release(r.off_m);
        if (r.has_map) arena_.release(r.off_map);
        r.has_lens = r.has_m = r.has_map = false;
        r.state = state;
        r.error = error;
        r.t_done = now_s();
        std::vector<double>().swap(r.lens_xy);
        std::vector<double>().swap(r.lens_m);
        if (state == DONE) {
            ++completed_;
            latencies_.push_back(r.t_done - r.t_submit);
            t_last_done_ = r.t_done;
        } else if (state == CANCELED) {
            ++canceled_;
        } else {
            ++failed_;
        }
        cv_done_.notify_all();
    }

    // No device, or a device error: every unfinished request fails, the steps in
    // flight are dropped, and submissions are refused from now on.
    void fail_all(int error) {
        dead_ = true;
        for (Step &st : inflight_) ex_->drop(st.h);
        inflight_.clear();
        for (auto &kv : reqs_)
            if (kv.second.state < DONE) finish(kv.second, FAILED, error);
    }

    bool launch_step() {
        // Requests waiting for admission mean the GPU is the bottleneck: longer steps then
        // trade a little responsiveness for less per-step overhead.
        const double slice_s =
            (cfg_.slice_ms > 0 ? cfg_.slice_ms : 10.0) * 1e-3 * (policy_.waiting() > 0 ? 4.0 : 1.0);
        std::vector<sched::Slice> slices =
            policy_.plan(rate_ * slice_s, now_s(), 0.25, cfg_.starve_s > 0 ? cfg_.starve_s : 0.5);
        if (slices.empty()) return false;
        std::vector<StepItem> items;
        items.reserve(slices.size());
        double inter = 0;
        for (const sched::Slice &s : slices) {
            const Request &r = reqs_.at(s.ticket);
            items.push_back(StepItem{&r, s.row0, s.row1});
            inter += (double)(r.p.i1 - r.p.i0) * (double)(s.row1 - s.row0) * (double)r.n_lens;
        }
        Step st;
        st.slices = slices;
        st.interactions = inter;
        // the workspace and stream of the step still in flight are never reused
        st.slot = inflight_.empty() ? 0 : 1 - inflight_.front().slot;
        const int rc = ex_->launch(items, st.slot, &st.h);
        if (rc != RS_OK) {
            // the step could not run: fail its requests
            for (const sched::Slice &s : slices) {
                policy_.cancel(s.ticket);
                reqs_.at(s.ticket).error = rc;
            }
            for (sched::Job &j : policy_.step_done(slices, now_s())) finish(reqs_.at(j.ticket), FAILED, rc);
            return true;
        }
        ++steps_;
        inflight_.push_back(std::move(st));
        return true;
    }

    // A finished step: statistics, throughput, and the requests it completed
    // (maps to copy are returned in *to_copy, marked COPYING).
    void retire_step(Step &s, std::vector<uint64_t> *to_copy) {
        double own_ms = 0, end_ms = 0;
        std::vector<rs_map_stats> st;
        ex_->retire(s.h, &own_ms, &end_ms, &st);
        s.h = nullptr;
        if (own_ms > 0) gpu_busy_s_ += own_ms * 1e-3;
        // Device throughput from the ends of the last retired steps: exact while the
        // pipeline is busy; low when it idles, which only makes the next steps smaller.
        recent_.push_back({end_ms, s.interactions});
        while (recent_.size() > 8) recent_.pop_front();
        if (recent_.size() >= 3) {
            double work = 0.0;
            for (size_t k = 1; k < recent_.size(); ++k) work += recent_[k].interactions;
            const double span = recent_.back().end_ms - recent_.front().end_ms;
            if (span > 0 && work > 1e9) rate_ = std::min(2e13, std::max(1e12, work / (span * 1e-3)));
        }
        interactions_ += s.interactions;
        const bool have_stats = st.size() == s.slices.size();
        for (size_t k = 0; k < s.slices.size(); ++k) {
            Request &r = reqs_.at(s.slices[k].ticket);
            if (!have_stats) {
                r.error = RS_EHIP;
                continue;
            }
            r.stats.rays_shot += st[k].rays_shot;
            r.stats.rays_in_map += st[k].rays_in_map;
            r.stats.rays_out += st[k].rays_out;
            r.stats.rays_singular += st[k].rays_singular;
            r.stats.rays_rechecked += st[k].rays_rechecked;
            r.stats.rays_rechecked_direct += st[k].rays_rechecked_direct;
        }
        for (sched::Job &j : policy_.step_done(s.slices, now_s())) {
            Request &r = reqs_.at(j.ticket);
            if (j.cancel) {
                finish(r, CANCELED, RS_ECANCELED);
            } else if (r.error != RS_OK) {
                finish(r, FAILED, r.error);
            } else if (r.map_host) {
                r.state = COPYING;
                to_copy->push_back(j.ticket);
            } else {
                finish(r, DONE, RS_OK);
            }
        }
    }

    // Copy finished maps out with the mutex released, then finish them.
    void copy_out(std::unique_lock<std::mutex> &lk, const std::vector<uint64_t> &tickets) {
        if (tickets.empty()) return;
        std::vector<std::pair<Request *, int>> done;
        for (uint64_t t : tickets) done.push_back({&reqs_.at(t), RS_OK});
        lk.unlock();
        // COPYING requests are not erased, cancelled or changed by other threads, and
        // references into the request table stay valid while others are inserted.
        for (auto &d : done) d.second = ex_->copy_map(*d.first, d.first->map_host);
        lk.lock();
        for (auto &d : done) finish(*d.first, d.second == RS_OK ? DONE : FAILED, d.second);
    }

    bool admit_fits(sched::Job &j) {
        Request &r = reqs_.at(j.ticket);
        size_t a = 0, b = 0, c = 0;
        const bool masses = !r.lens_m.empty();
        if (r.n_lens > 0 && !arena_.alloc(16 * (size_t)r.n_lens, &a)) return false;
        if (masses && !arena_.alloc(8 * (size_t)r.n_lens, &b)) {
            if (r.n_lens > 0) arena_.release(a);
            return false;
        }
        if (!arena_.alloc(4 * (size_t)(r.p.npx * r.p.npy), &c)) {
            if (r.n_lens > 0) arena_.release(a);
            if (masses) arena_.release(b);
            return false;
        }
        r.off_lens = a;
        r.off_m = b;
        r.off_map = c;
        r.has_lens = r.n_lens > 0;
        r.has_m = masses;
        r.has_map = true;
        return true;
    }

    void run() {
        std::unique_lock<std::mutex> lk(mu_);
        if (ex_->bind_thread() != RS_OK) {
            // no device for this thread: nothing can run, so fail everything now and later
            fail_all(RS_EHIP);
            return;
        }
        for (;;) {
            // 1. admission (FIFO, by slot and arena space)
            std::vector<uint64_t> dropped;
            std::vector<uint64_t> admitted =
                policy_.admit(now_s(), [&](sched::Job &j) { return admit_fits(j); }, &dropped);
            for (uint64_t t : dropped) {
                Request &r = reqs_.at(t);
                const bool too_big = footprint_of(r.p, r.n_lens, !r.lens_m.empty()) > cfg_.hbm_budget_bytes;
                finish(r, too_big ? FAILED : CANCELED, too_big ? RS_ENOMEM : RS_ECANCELED);
            }
            for (uint64_t t : admitted) {
                Request &r = reqs_.at(t);
                r.state = ACTIVE;
                if (ex_->admit(r) != RS_OK) {
                    policy_.cancel(t);
                    r.error = RS_EHIP;
                }
            }
            for (sched::Job &j : policy_.reap(now_s())) {   // cancelled before any slice ran, or empty windows
                Request &r = reqs_.at(j.ticket);
                if (j.cancel) finish(r, r.error ? FAILED : CANCELED, r.error ? r.error : RS_ECANCELED);
                else finish(r, DONE, RS_OK);
            }
            max_waiting_ = std::max(max_waiting_, policy_.waiting());

            // 2. keep two steps in flight
            bool launched = false;
            if (inflight_.size() < 2) launched = launch_step();

            // 3. retire the oldest step when it is done, or block on it when the pipeline is full
            if (!inflight_.empty()) {
                const bool full = inflight_.size() >= 2 || !launched;
                void *h = inflight_.front().h;
                int q = ex_->poll(h, false);
                if (q == 1 && full) {
                    lk.unlock();
                    q = ex_->poll(h, true);
                    lk.lock();
                }
                if (q == RS_OK) {
                    Step done = std::move(inflight_.front());
                    inflight_.pop_front();
                    std::vector<uint64_t> to_copy;
                    retire_step(done, &to_copy);
                    copy_out(lk, to_copy);
                } else if (q != 1) {
                    fail_all(RS_EHIP);
                    return;
                }
                continue;
            }
            if (stop_ && policy_.waiting() == 0 && policy_.active() == 0) break;
            if (!launched) cv_work_.wait_for(lk, std::chrono::milliseconds(20));
        }
    }

    rs_server_cfg cfg_;
    Executor *ex_;
    sched::Policy policy_;
    sched::Arena arena_;

    std::mutex mu_;
    std::condition_variable cv_work_, cv_done_;
    std::map<uint64_t, Request> reqs_;
    uint64_t next_ticket_ = 1;
    bool stop_ = false;
    bool dead_ = false;
    std::thread thread_;

    std::deque<Step> inflight_;
    std::deque<EndMark> recent_;
    double rate_ = 6e12;   // ray-lens interactions per second, refined from retired steps

    std::vector<double> latencies_;
    uint64_t completed_ = 0, canceled_ = 0, failed_ = 0, steps_ = 0, rejected_busy_ = 0;
    double interactions_ = 0, t_first_submit_ = -1, t_last_done_ = 0, gpu_busy_s_ = 0;
    size_t max_waiting_ = 0;
};

}  // namespace serve
}  // namespace rs
