// Host-side observability: RAYSHOOT_DEBUG=1 prints each map's launch plan and
// each batch's shape to stderr (=2 also the request loop's steps), and named
// roctx ranges mark the library's phases in rocprofv3 traces (--marker-trace).
#pragma once

#include <rocprofiler-sdk-roctx/roctx.h>

#include <cstdarg>
#include <cstdio>
#include <cstdlib>

namespace rs {

// RAYSHOOT_DEBUG as an integer (0 when unset), read once.
inline int debug_level() {
    static const int level = [] {
        const char *v = std::getenv("RAYSHOOT_DEBUG");
        return v ? std::atoi(v) : 0;
    }();
    return level;
}

inline void debug_print(int level, const char *fmt, ...) {
    if (debug_level() < level) return;
    va_list ap;
    va_start(ap, fmt);
    std::fputs("[rayshoot] ", stderr);
    std::vfprintf(stderr, fmt, ap);
    std::fputc('\n', stderr);
    va_end(ap);
}

// A roctx range for the lifetime of the object (a no-op unless a tool listens).
class Range {
  public:
    explicit Range(const char *name) { roctxRangePushA(name); }
    ~Range() { roctxRangePop(); }
    Range(const Range &) = delete;
    Range &operator=(const Range &) = delete;
};

}  // namespace rs
