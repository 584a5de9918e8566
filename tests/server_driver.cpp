// CPU driver of the request loop's threads (rs_server_core.h) over a simulated
// device, built with a thread sanitizer by tests/test_server_threads.py.
//
// The simulated device runs launch steps in order on a thread of its own, each
// for a time proportional to its ray-lens pairs, and "maps" ray (i, j) of a
// request to pixel (i + 3 j + k0) mod npix, k0 from the request's first lens, so
// a map is right only if every row of the window was handed out exactly once.
// Several client threads submit, poll, wait and cancel at once. Prints one JSON
// object of results.
#include "rs_server_core.h"

#include <atomic>
#include <cinttypes>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <random>
#include <string>

namespace rs {
static thread_local std::string g_err;
int fail(int code, const char *fmt, ...) {
    char buf[256];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}
int validate(const rs_map_params *p, int64_t n_lens) {
    if (!p || p->npx <= 0 || p->npy <= 0 || p->i0 < 0 || p->i1 > p->nx || p->i0 > p->i1 || p->j0 < 0 ||
        p->j1 > p->ny || p->j0 > p->j1 || n_lens < 0)
        return fail(RS_EINVAL, "bad parameters");
    return RS_OK;
}
}  // namespace rs

using namespace rs;
using rs::serve::Request;
using rs::serve::StepItem;

namespace {

struct Work {
    uint32_t *map;
    int64_t npix, i0, i1, j0, j1, k0;
};

class FakeDevice final : public serve::Executor {
  public:
    FakeDevice(size_t pool_bytes, double pairs_per_s, int fail_at_step)
        : pool_(pool_bytes / 4 + 1, 0u), rate_(pairs_per_s), fail_at_(fail_at_step) {
        worker_ = std::thread([this] { loop(); });
    }
    ~FakeDevice() override {
        {
            std::lock_guard<std::mutex> lk(mu_);
            quit_ = true;
        }
        cv_.notify_all();
        worker_.join();
        for (Step *s : all_) delete s;
    }
    int bind_thread() override { return RS_OK; }
    int admit(const Request &r) override {
        // the map is zeroed before any step that uses it (steps run after admission, in order)
        std::lock_guard<std::mutex> lk(mu_);
        queue_.push_back(new Step{});
        Step *z = queue_.back();
        all_.push_back(z);
        z->zero = &pool_[r.off_map / 4];
        z->zero_n = r.p.npx * r.p.npy;
        z->internal = true;
        cv_.notify_all();
        return RS_OK;
    }
    int launch(const std::vector<StepItem> &items, int slot, void **out) override {
        if (slot != 0 && slot != 1) return fail(RS_EINVAL, "slot");
        Step *st = new Step{};
        st->slot = slot;
        double pairs = 0;
        for (const StepItem &it : items) {
            const Request &r = *it.req;
            Work w{&pool_[r.off_map / 4], r.p.npx * r.p.npy, r.p.i0, r.p.i1, r.p.j0 + it.row0, r.p.j0 + it.row1,
                   r.n_lens ? (int64_t)r.lens_xy[0] : 0};
            st->work.push_back(w);
            pairs += (double)(w.i1 - w.i0) * (double)(w.j1 - w.j0) * (double)(r.n_lens ? r.n_lens : 1);
        }
        st->seconds = pairs / rate_;
        {
            std::lock_guard<std::mutex> lk(mu_);
            if (in_flight_[slot]) return fail(RS_EINVAL, "slot %d reused while its step runs", slot);
            in_flight_[slot] = true;
            st->index = launched_++;
            all_.push_back(st);
            queue_.push_back(st);
        }
        cv_.notify_all();
        *out = st;
        return RS_OK;
    }
    int poll(void *h, bool block) override {
        Step *st = static_cast<Step *>(h);
        std::unique_lock<std::mutex> lk(mu_);
        if (block) cv_.wait(lk, [&] { return st->done; });
        if (!st->done) return 1;
        return st->error ? RS_EHIP : RS_OK;
    }
    void retire(void *h, double *own_ms, double *end_ms, std::vector<rs_map_stats> *stats) override {
        Step *st = static_cast<Step *>(h);
        std::lock_guard<std::mutex> lk(mu_);
        *own_ms = st->seconds * 1e3;
        *end_ms = st->end_s * 1e3;
        stats->clear();
        for (const Work &w : st->work) {
            rs_map_stats s{};
            s.rays_shot = s.rays_in_map = (uint64_t)((w.i1 - w.i0) * (w.j1 - w.j0));
            stats->push_back(s);
        }
        in_flight_[st->slot] = false;
        ++retired_;
    }
    void drop(void *h) override {
        Step *st = static_cast<Step *>(h);
        std::lock_guard<std::mutex> lk(mu_);
        in_flight_[st->slot] = false;
    }
    int copy_map(const Request &r, uint32_t *host) override {
        std::lock_guard<std::mutex> lk(mu_);   // the device thread may be writing other maps
        std::memcpy(host, &pool_[r.off_map / 4], 4 * (size_t)(r.p.npx * r.p.npy));
        ++copies_;
        return RS_OK;
    }
    int64_t launched() {
        std::lock_guard<std::mutex> lk(mu_);
        return launched_;
    }

  private:
    struct Step {
        std::vector<Work> work;
        uint32_t *zero = nullptr;
        int64_t zero_n = 0;
        bool internal = false;
        double seconds = 0, end_s = 0;
        int slot = 0;
        int64_t index = 0;
        bool done = false, error = false;
    };
    void loop() {
        std::unique_lock<std::mutex> lk(mu_);
        for (;;) {
            cv_.wait(lk, [&] { return quit_ || !queue_.empty(); });
            if (queue_.empty()) return;
            Step *st = queue_.front();
            queue_.pop_front();
            lk.unlock();
            if (st->internal) {
                std::lock_guard<std::mutex> g(mu_);
                for (int64_t k = 0; k < st->zero_n; ++k) st->zero[k] = 0u;
            } else {
                std::this_thread::sleep_for(std::chrono::duration<double>(st->seconds));
                std::lock_guard<std::mutex> g(mu_);
                for (const Work &w : st->work)
                    for (int64_t j = w.j0; j < w.j1; ++j)
                        for (int64_t i = w.i0; i < w.i1; ++i) w.map[(i + 3 * j + w.k0) % w.npix] += 1u;
            }
            lk.lock();
            st->end_s = serve::now_s();
            st->error = !st->internal && fail_at_ >= 0 && st->index >= fail_at_;
            st->done = true;
            cv_.notify_all();
        }
    }

    std::vector<uint32_t> pool_;
    double rate_;
    int fail_at_;
    std::mutex mu_;
    std::condition_variable cv_;
    std::deque<Step *> queue_;
    std::vector<Step *> all_;
    bool in_flight_[2] = {false, false};
    bool quit_ = false;
    int64_t launched_ = 0, retired_ = 0, copies_ = 0;
    std::thread worker_;
};

rs_map_params params(int64_t w, int64_t h, int64_t npx, int64_t npy) {
    rs_map_params p{};
    p.sw = p.sh = p.tw = p.th = 1.0;
    p.nx = w;
    p.ny = h;
    p.i0 = 0;
    p.i1 = w;
    p.j0 = 0;
    p.j1 = h;
    p.npx = npx;
    p.npy = npy;
    p.mode = RS_MIXED;
    return p;
}

std::vector<uint32_t> expected(const rs_map_params &p, int64_t k0) {
    const int64_t npix = p.npx * p.npy;
    std::vector<uint32_t> m((size_t)npix, 0u);
    for (int64_t j = p.j0; j < p.j1; ++j)
        for (int64_t i = p.i0; i < p.i1; ++i) m[(size_t)((i + 3 * j + k0) % npix)] += 1u;
    return m;
}

}  // namespace

int main() {
    std::string out = "{";
    auto put = [&](const char *k, const std::string &v) {
        if (out.size() > 1) out += ",";
        out += "\"";
        out += k;
        out += "\":";
        out += v;
    };

    // 1. Four clients submit 30 requests each (sizes mixed, a few too large for the pool),
    //    wait for them and check every map; one client cancels every fifth request; a
    //    fifth thread reads the statistics meanwhile.
    {
        rs_server_cfg cfg{};
        cfg.hbm_budget_bytes = 1 << 20;
        cfg.max_inflight = 6;
        cfg.mode = RS_MIXED;
        cfg.slice_ms = 2.0;
        cfg.starve_s = 0.05;
        FakeDevice dev(cfg.hbm_budget_bytes, 2e9, -1);
        serve::Server srv(cfg, &dev);
        srv.start();
        std::atomic<int> ok{0}, bad{0}, canceled{0}, nomem{0}, other{0};
        std::atomic<bool> stats_run{true};
        std::thread reader([&] {
            while (stats_run.load()) {
                rs_server_stats st{};
                srv.get_stats(&st);
                std::this_thread::sleep_for(std::chrono::microseconds(300));
            }
        });
        std::vector<std::thread> clients;
        for (int c = 0; c < 4; ++c) {
            clients.emplace_back([&, c] {
                std::mt19937_64 rng(100 + c);
                for (int k = 0; k < 30; ++k) {
                    const int64_t w = 64 + (int64_t)(rng() % 400), h = 32 + (int64_t)(rng() % 300);
                    const bool huge = k % 13 == 12;
                    const int64_t npx = huge ? 1024 : 16 + (int64_t)(rng() % 48), npy = huge ? 1024 : 16 + (int64_t)(rng() % 48);
                    rs_map_params p = params(w, h, npx, npy);
                    std::vector<double> lens(2 * 10);
                    for (auto &v : lens) v = (double)(rng() % 1000);
                    std::vector<uint32_t> map((size_t)(npx * npy), 7u);
                    uint64_t t = 0;
                    int rc = srv.submit(&p, lens.data(), nullptr, 10, map.data(), &t);
                    if (rc != RS_OK) {
                        ++other;
                        continue;
                    }
                    const bool do_cancel = c == 0 && k % 5 == 4;
                    if (do_cancel) (void)srv.cancel(t);
                    int done = 0;
                    (void)srv.poll(t, &done);
                    rs_map_stats st{};
                    double lat = 0;
                    rc = srv.wait(t, &st, &lat);
                    if (rc == RS_OK) {
                        if (map == expected(p, (int64_t)lens[0]) && st.rays_shot == (uint64_t)(w * h)) ++ok;
                        else ++bad;
                    } else if (rc == RS_ECANCELED) {
                        ++canceled;
                    } else if (rc == RS_ENOMEM) {
                        ++nomem;
                    } else {
                        ++other;
                    }
                }
            });
        }
        for (auto &t : clients) t.join();
        stats_run = false;
        reader.join();
        rs_server_stats st{};
        srv.get_stats(&st);
        srv.stop();
        put("mix_ok", std::to_string(ok.load()));
        put("mix_bad", std::to_string(bad.load()));
        put("mix_canceled", std::to_string(canceled.load()));
        put("mix_nomem", std::to_string(nomem.load()));
        put("mix_other", std::to_string(other.load()));
        put("mix_completed", std::to_string(st.completed));
        put("mix_steps", std::to_string(st.steps));
        put("mix_in_use_after", std::to_string(st.hbm_in_use_bytes));
    }

    // 2. A bounded waiting queue: one slot, a slow device, max_waiting 3; a burst of 12
    //    submissions gets RS_EBUSY for those beyond the queue, and the rest complete.
    {
        rs_server_cfg cfg{};
        cfg.hbm_budget_bytes = 1 << 20;
        cfg.max_inflight = 1;
        cfg.mode = RS_MIXED;
        cfg.max_waiting = 3;
        FakeDevice dev(cfg.hbm_budget_bytes, 2e7, -1);
        serve::Server srv(cfg, &dev);
        srv.start();
        std::vector<uint64_t> tickets;
        std::vector<std::vector<uint32_t>> maps(12, std::vector<uint32_t>(256, 0u));
        int busy = 0;
        double lens[2] = {5.0, 1.0};
        for (int k = 0; k < 12; ++k) {
            rs_map_params p = params(256, 64, 16, 16);
            uint64_t t = 0;
            const int rc = srv.submit(&p, lens, nullptr, 1, maps[k].data(), &t);
            if (rc == RS_EBUSY) ++busy;
            else if (rc == RS_OK) tickets.push_back(t);
        }
        int ok = 0;
        for (uint64_t t : tickets) ok += srv.wait(t, nullptr, nullptr) == RS_OK;
        rs_server_stats st{};
        srv.get_stats(&st);
        srv.stop();
        put("busy_refused", std::to_string(busy));
        put("busy_accepted_ok", std::to_string(ok));
        put("busy_accepted", std::to_string(tickets.size()));
        put("busy_counter", std::to_string(st.rejected_busy));
    }

    // 3. A device error from the second step on: the first request completes, every
    //    later unfinished request fails with RS_EHIP, and later submissions are refused.
    {
        rs_server_cfg cfg{};
        cfg.hbm_budget_bytes = 1 << 20;
        cfg.max_inflight = 4;
        cfg.mode = RS_MIXED;
        cfg.slice_ms = 1.0;
        FakeDevice dev(cfg.hbm_budget_bytes, 1e8, 1);
        serve::Server srv(cfg, &dev);
        srv.start();
        std::vector<uint64_t> tickets;
        std::vector<std::vector<uint32_t>> maps(7, std::vector<uint32_t>(256, 0u));
        double lens[2] = {5.0, 1.0};
        rs_map_params p0 = params(64, 64, 16, 16);
        uint64_t t0 = 0;
        const int first = srv.submit(&p0, lens, nullptr, 1, maps[6].data(), &t0) == RS_OK
                              ? srv.wait(t0, nullptr, nullptr) : -100;
        put("err_first", std::to_string(first));
        for (int k = 0; k < 6; ++k) {
            rs_map_params p = params(512, 512, 16, 16);
            uint64_t t = 0;
            if (srv.submit(&p, lens, nullptr, 1, maps[k].data(), &t) == RS_OK) tickets.push_back(t);
        }
        int ehip = 0;
        for (uint64_t t : tickets) ehip += srv.wait(t, nullptr, nullptr) == RS_EHIP;
        rs_map_params p = params(64, 64, 16, 16);
        uint64_t t = 0;
        const int after = srv.submit(&p, lens, nullptr, 1, maps[0].data(), &t);
        srv.stop();
        put("err_failed", std::to_string(ehip));
        put("err_submitted", std::to_string(tickets.size()));
        put("err_after", std::to_string(after));
    }
    out += "}";
    std::printf("%s\n", out.c_str());
    return 0;
}
