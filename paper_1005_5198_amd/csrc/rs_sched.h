// Scheduling policy of the request loop: admission by HBM footprint and slot
// count, fair slicing of active requests into launch steps, a first-fit device
// arena, and latency bookkeeping. Pure host logic (no HIP calls), so it can be
// exercised on the CPU with simulated time.
#pragma once

#include <algorithm>
#include <cstddef>
#include <cstdint>
#include <deque>
#include <map>
#include <vector>

namespace rs {
namespace sched {

// First-fit allocator over [0, size) with coalescing free list; offsets are
// aligned to `align` bytes. Used for the server's device arena.
class Arena {
  public:
    explicit Arena(size_t size = 0, size_t align = 256) : size_(size), align_(align) {
        if (size) free_[0] = size;
    }
    size_t size() const { return size_; }
    size_t in_use() const { return in_use_; }
    size_t peak() const { return peak_; }
    static size_t round_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

    // Returns true and the offset, or false when no free range is large enough.
    bool alloc(size_t bytes, size_t *offset) {
        bytes = round_up(bytes ? bytes : 1, align_);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *offset = it->first;
                const size_t rest = it->second - bytes;
                const size_t at = it->first + bytes;
                free_.erase(it);
                if (rest) free_[at] = rest;
                used_[*offset] = bytes;
                in_use_ += bytes;
                peak_ = std::max(peak_, in_use_);
                return true;
            }
        }
        return false;
    }

    void release(size_t offset) {
        auto u = used_.find(offset);
        if (u == used_.end()) return;
        size_t at = offset, len = u->second;
        in_use_ -= len;
        used_.erase(u);
        auto next = free_.lower_bound(at);
        if (next != free_.end() && at + len == next->first) {
            len += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == at) {
                prev->second += len;
                return;
            }
        }
        free_[at] = len;
    }

    size_t largest_free() const {
        size_t m = 0;
        for (const auto &kv : free_) m = std::max(m, kv.second);
        return m;
    }

  private:
    size_t size_, align_;
    size_t in_use_ = 0, peak_ = 0;
    std::map<size_t, size_t> free_;  // offset -> length
    std::map<size_t, size_t> used_;  // offset -> length
};

// One request as the policy sees it.
struct Job {
    uint64_t ticket = 0;
    int64_t width = 0;           // rays per row of the window
    int64_t rows = 0;            // rows of the window
    int64_t n_lens = 0;
    size_t footprint = 0;        // device bytes held while active (lenses, masses, map)
    int64_t next_row = 0;        // rows already handed to steps
    int64_t rows_done = 0;       // rows whose step has completed
    int64_t steps_in_flight = 0;
    bool cancel = false;
    double t_submit = 0, t_admit = 0, t_done = 0;
};

// A slice of a job: rows [row0, row1) of its window, relative to the window's first row.
struct Slice {
    uint64_t ticket;
    int64_t row0, row1;
    bool first;                  // the job's first slice (zeroes the map)
};

constexpr int64_t ROW_QUANTUM = 32;  // slices are whole 32-row bands (the kernel's patch height)

class Policy {
  public:
    Policy(size_t budget_bytes, int max_inflight) : budget_(budget_bytes), max_inflight_(max_inflight) {}

    void submit(const Job &j) { waiting_.push_back(j); }

    // FIFO admission: the head waits until a slot is free and its footprint fits;
    // later requests do not overtake it. `fits` decides whether memory can be had
    // (e.g. an arena allocation); jobs whose footprint exceeds the whole budget are
    // returned in `rejected`.
    template <class Fits>
    std::vector<uint64_t> admit(double now, Fits fits, std::vector<uint64_t> *rejected) {
        std::vector<uint64_t> out;
        while (!waiting_.empty()) {
            Job &j = waiting_.front();
            if (j.cancel) {
                if (rejected) rejected->push_back(j.ticket);
                waiting_.pop_front();
                continue;
            }
            if (j.footprint > budget_) {
                if (rejected) rejected->push_back(j.ticket);
                waiting_.pop_front();
                continue;
            }
            if ((int)active_.size() >= max_inflight_) break;
            if (!fits(j)) break;
            j.t_admit = now;
            active_.push_back(j);
            out.push_back(j.ticket);
            waiting_.pop_front();
        }
        return out;
    }

    // Next step, holding about `target_interactions` ray-lens pairs. The budget
    // goes first to jobs that have waited longer than starve_s since submission
    // (oldest first), then to the others in order of least remaining work,
    // discounted by age: remaining / (1 + waited / aging_s). A small request
    // finishes in the next step instead of queueing behind a large one, and a
    // large one cannot be postponed past starve_s. Bands are whole multiples of
    // 32 rows; the first job in that order always gets one, the others only
    // while the budget lasts.
    std::vector<Slice> plan(double target_interactions, double now = 0.0, double aging_s = 0.25,
                            double starve_s = 0.5) {
        std::vector<Slice> step;
        std::vector<Job *> open;
        for (Job &j : active_)
            if (!j.cancel && j.next_row < j.rows) open.push_back(&j);
        if (open.empty()) return step;
        auto per_row = [](const Job *j) { return (double)j->width * (double)std::max<int64_t>(j->n_lens, 1); };
        auto key = [&](const Job *j) {
            const double waited = now > j->t_submit ? now - j->t_submit : 0.0;
            return per_row(j) * (double)(j->rows - j->next_row) / (1.0 + waited / aging_s);
        };
        auto starved = [&](const Job *j) { return now - j->t_submit > starve_s; };
        std::stable_sort(open.begin(), open.end(), [&](const Job *a, const Job *b) {
            const bool sa = starved(a), sb = starved(b);
            if (sa != sb) return sa;
            if (sa) return a->t_submit < b->t_submit;
            return key(a) < key(b);
        });
        double left = target_interactions;
        for (Job *j : open) {
            // The first job in priority order always gets at least one band (progress);
            // the others share what is left of the budget, in whole bands.
            if (!step.empty() && left < per_row(j) * (double)ROW_QUANTUM) continue;
            int64_t rows = left > 0 ? (int64_t)(left / per_row(j)) : 0;
            rows = std::max<int64_t>(ROW_QUANTUM, rows / ROW_QUANTUM * ROW_QUANTUM);
            const int64_t row1 = std::min(j->rows, j->next_row + rows);
            left -= per_row(j) * (double)(row1 - j->next_row);
            step.push_back(Slice{j->ticket, j->next_row, row1, j->next_row == 0});
            j->next_row = row1;
            ++j->steps_in_flight;
        }
        return step;
    }

    // A step finished. Returns the jobs that are now complete (all rows done)
    // or cancelled with nothing in flight; they leave the active set.
    std::vector<Job> step_done(const std::vector<Slice> &step, double now) {
        for (const Slice &s : step) {
            for (Job &j : active_) {
                if (j.ticket != s.ticket) continue;
                j.rows_done += s.row1 - s.row0;
                --j.steps_in_flight;
            }
        }
        return reap(now);
    }

    std::vector<Job> reap(double now) {
        std::vector<Job> finished;
        for (auto it = active_.begin(); it != active_.end();) {
            const bool complete = it->rows_done >= it->rows;
            const bool dropped = it->cancel && it->steps_in_flight == 0;
            if ((complete || dropped) && it->steps_in_flight == 0) {
                it->t_done = now;
                finished.push_back(*it);
                it = active_.erase(it);
            } else {
                ++it;
            }
        }
        return finished;
    }

    // Mark a job cancelled; returns false if it is unknown (already finished).
    bool cancel(uint64_t ticket) {
        for (Job &j : waiting_)
            if (j.ticket == ticket) return j.cancel = true;
        for (Job &j : active_)
            if (j.ticket == ticket) return j.cancel = true;
        return false;
    }

    size_t waiting() const { return waiting_.size(); }
    size_t active() const { return active_.size(); }
    const std::vector<Job> &active_jobs() const { return active_; }

  private:
    size_t budget_;
    int max_inflight_;
    std::deque<Job> waiting_;
    std::vector<Job> active_;
};

// Latency percentiles (nearest-rank).
inline double percentile(std::vector<double> v, double p) {
    if (v.empty()) return 0.0;
    std::sort(v.begin(), v.end());
    size_t rank = (size_t)(p / 100.0 * (double)v.size() + 0.999999999);
    if (rank < 1) rank = 1;
    if (rank > v.size()) rank = v.size();
    return v[rank - 1];
}

}  // namespace sched
}  // namespace rs
