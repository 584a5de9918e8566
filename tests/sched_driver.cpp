// CPU driver for the request-loop policy (admission, slicing, cancellation,
// arena, percentiles) with simulated time; prints one JSON object of results.
#include "rs_sched.h"

#include <cstdio>
#include <string>
#include <vector>

using namespace rs::sched;

static Job job(uint64_t t, size_t fp, int64_t width = 1000, int64_t rows = 100, int64_t n_lens = 10) {
    Job j;
    j.ticket = t;
    j.footprint = fp;
    j.width = width;
    j.rows = rows;
    j.n_lens = n_lens;
    return j;
}

int main() {
    std::string out = "{";
    auto put = [&](const char *k, const std::string &v) {
        if (out.size() > 1) out += ",";
        out += "\"";
        out += k;
        out += "\":";
        out += v;
    };
    auto list = [](const std::vector<uint64_t> &v) {
        std::string s = "[";
        for (size_t i = 0; i < v.size(); ++i) s += (i ? "," : "") + std::to_string(v[i]);
        return s + "]";
    };
    // 1. admission by footprint and slots, FIFO without overtaking, oversize rejection
    {
        Policy p(1000, 3);
        p.submit(job(1, 600));
        p.submit(job(2, 300));
        p.submit(job(3, 200));   // fits the slot count but not the memory left (100)
        p.submit(job(4, 50));    // would fit, but must not overtake 3
        p.submit(job(5, 5000));  // larger than the whole budget
        size_t used = 0;
        auto fits = [&](Job &j) { if (used + j.footprint > 1000) return false; used += j.footprint; return true; };
        std::vector<uint64_t> rej;
        put("admit1", list(p.admit(0.0, fits, &rej)));
        // finish job 1: plan and complete its rows
        std::vector<Slice> s = p.plan(1e12);
        put("plan1_n", std::to_string(s.size()));
        bool rows_ok = true;
        for (const Slice &x : s) rows_ok = rows_ok && ((x.row1 - x.row0) % ROW_QUANTUM == 0 || x.row1 == 100);
        put("plan1_rows_quantum", rows_ok ? "true" : "false");
        std::vector<Job> done = p.step_done(s, 1.0);
        std::vector<uint64_t> dt;
        for (Job &j : done) { dt.push_back(j.ticket); used -= j.footprint; }
        put("done1", list(dt));
        put("admit2", list(p.admit(1.0, fits, &rej)));
        put("rejected", list(rej));
    }
    // 2. slot limit
    {
        Policy p(1 << 30, 2);
        for (uint64_t t = 1; t <= 5; ++t) p.submit(job(t, 10));
        auto fits = [](Job &) { return true; };
        put("slots_admit", list(p.admit(0.0, fits, nullptr)));
        put("slots_waiting", std::to_string(p.waiting()));
    }
    // 3. slicing: least remaining work first, 32-row quanta, one band minimum per job
    {
        Policy p(1 << 30, 8);
        p.submit(job(1, 1, 1000, 1000, 100));   // 1e5 interactions per row, 1e8 in all
        p.submit(job(2, 1, 1000, 70, 100));     // 7e6 in all: the smaller one
        auto fits = [](Job &) { return true; };
        p.admit(0.0, fits, nullptr);
        std::vector<Slice> s = p.plan(128 * 1e5);  // budget of 128 rows
        std::string sl = "[";
        for (size_t i = 0; i < s.size(); ++i)
            sl += (i ? "," : "") + std::string("[") + std::to_string(s[i].ticket) + "," + std::to_string(s[i].row0) +
                  "," + std::to_string(s[i].row1) + "," + (s[i].first ? "1" : "0") + "]";
        put("srpt_step1", sl + "]");
        std::vector<Job> d1 = p.step_done(s, 1.0);
        std::vector<uint64_t> t1;
        for (Job &j : d1) t1.push_back(j.ticket);
        put("srpt_done1", list(t1));
        int steps = 1;
        while (p.active()) { p.step_done(p.plan(128 * 1e5), 1.0 + steps); ++steps; if (steps > 100) break; }
        put("srpt_total_steps", std::to_string(steps));
    }
    // 3b. starvation guard: a large job older than starve_s goes before a small new one
    {
        Policy p(1 << 30, 8);
        Job big = job(1, 1, 1000, 1000, 100);
        big.t_submit = 0.0;
        Job small = job(2, 1, 1000, 70, 100);
        small.t_submit = 0.9;
        p.submit(big);
        p.submit(small);
        auto fits = [](Job &) { return true; };
        p.admit(0.0, fits, nullptr);
        auto show = [](const std::vector<Slice> &s) {
            std::string sl = "[";
            for (size_t i = 0; i < s.size(); ++i)
                sl += (i ? "," : "") + std::string("[") + std::to_string(s[i].ticket) + "," +
                      std::to_string(s[i].row0) + "," + std::to_string(s[i].row1) + "]";
            return sl + "]";
        };
        std::vector<Slice> a = p.plan(128 * 1e5, 1.0, 0.25, 0.5);   // big has waited 1.0 s > 0.5 s
        put("starve_step1", show(a));
        p.step_done(a, 1.0);
        Policy q(1 << 30, 8);
        big.t_submit = 0.8;
        q.submit(big);
        q.submit(small);
        q.admit(0.0, fits, nullptr);
        put("starve_none", show(q.plan(128 * 1e5, 1.0, 0.25, 0.5)));  // neither has waited 0.5 s
    }
    // 4. cancellation of a waiting and of a running job
    {
        Policy p(1 << 30, 1);
        p.submit(job(1, 10));
        p.submit(job(2, 10));
        auto fits = [](Job &) { return true; };
        p.admit(0.0, fits, nullptr);
        std::vector<Slice> s = p.plan(1e5 * 10 * 32);  // one 32-row slice of job 1
        p.cancel(1);
        p.cancel(2);
        std::vector<uint64_t> rej;
        p.admit(0.0, fits, &rej);  // job 2 dropped from the queue
        put("cancel_dropped", list(rej));
        put("cancel_plan_after", std::to_string(p.plan(1e12).size()));
        std::vector<Job> d = p.step_done(s, 1.0);
        put("cancel_reaped", std::to_string(d.size()));
        put("cancel_reaped_flag", d.size() == 1 && d[0].cancel ? "true" : "false");
        put("cancel_active_left", std::to_string(p.active()));
    }
    // 5. arena: first fit, coalescing, peak
    {
        Arena a(4096, 256);
        size_t o1, o2, o3, o4;
        bool ok = a.alloc(1000, &o1) && a.alloc(1000, &o2) && a.alloc(1000, &o3);
        put("arena_three", ok ? "true" : "false");
        put("arena_full", a.alloc(2000, &o4) ? "true" : "false");
        a.release(o2);
        put("arena_hole", std::to_string(a.largest_free()));
        a.release(o1);
        put("arena_coalesced", std::to_string(a.largest_free()));
        a.release(o3);
        put("arena_empty", std::to_string(a.largest_free()));
        put("arena_peak", std::to_string(a.peak()));
        put("arena_in_use", std::to_string(a.in_use()));
    }
    // 6. percentiles (nearest rank)
    {
        std::vector<double> v;
        for (int i = 1; i <= 100; ++i) v.push_back(i);
        put("p50", std::to_string(percentile(v, 50)));
        put("p99", std::to_string(percentile(v, 99)));
        put("p100", std::to_string(percentile(v, 100)));
    }
    out += "}";
    std::printf("%s\n", out.c_str());
    return 0;
}
