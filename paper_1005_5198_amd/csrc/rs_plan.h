// Launch planning of single maps, host only (no device calls): argument
// validation, and how a ray window is cut into launches and laid out in the
// workspace. Shared by the runtime (runtime.cpp) and its CPU tests.
#pragma once

#include <cstddef>
#include <cstdint>

#include "rayshoot.h"
#include "rs_layout.h"

namespace rs {

int fail(int code, const char *fmt, ...);

struct Plan {
    int64_t W = 0, H = 0;
    int64_t rows_per_chunk = 0, n_chunks = 0;
    int64_t queue_cap = 0;   // uint32 entries (mixed only)
    size_t qcount_bytes = 0; // WS_QCOUNT + 16 * n_chunks + 8 (per launch: queue length, live, unresolved and
                             // left-after-gathering counts; the gathered and gathered-unresolved counts),
                             // 256-aligned
    bool defer = false;      // several launches: rays for the stages over every lens gathered, run after the last
    size_t defer_off = 0;    // int64 [2][DEFER_CAP][2]: (i, j) of the gathered rays, then of those stage A left
    bool far_recheck = false; // mixed mode: far-field re-check stage first
    int64_t rand_sbx = 0, rand_sby = 0; // random rays: super-patch grid of the whole rectangle
    // Random rays: bin arrays for the largest number of bins of a launch, and
    // the sorted ray list (index, x, y) of the largest launch.
    bool random = false;
    int64_t bins_cap = 0, rays_cap = 0;
    size_t bin_count_off = 0, bin_offset_off = 0, bin_cursor_off = 0;
    size_t rel_off = 0, x_off = 0, y_off = 0;
    // Far-field expansion: super-patch records and lens lists for the largest launch.
    int64_t super_cap = 0;
    size_t ff_super_off = 0, ff_near_off = 0;
    // Far-field mode: the patch records of the largest launch, and the counter
    // from which the ray kernel's blocks take patches.
    int64_t patch_cap = 0;
    size_t ff_patch_off = 0, ff_work_off = 0;
    // Far-field mode: group records and lists of the largest launch.
    int64_t group_cap = 0;
    size_t ff_group_off = 0, ff_glist_off = 0;
    int64_t top_cap = 0;      // far-field mode with at least FF_TOP_MIN_LENSES lenses: tops per launch
    size_t ff_top_off = 0, ff_tlist_off = 0;
    size_t bytes = 0;
};

// RS_OK, or RS_EINVAL with rs_last_error's message set.
int validate(const rs_map_params *p, int64_t n_lens);

// Square-ish bins of the shooting rectangle holding about RAND_BIN_RAYS of a
// launch's rays each.
void random_bins(int64_t rays, double sw, double sh, int64_t &nbx, int64_t &nby);

// The plan of a valid window; rows_override > 0 (a multiple of PATCH_Y) replaces
// the default rows per launch.
Plan make_plan(const rs_map_params *p, int64_t n_lens, int64_t rows_override = 0);

// The plan with the most rows per launch (a multiple of PATCH_Y, at most the default)
// whose workspace fits max_bytes; false when a single band of PATCH_Y rows does not fit.
bool plan_within(const rs_map_params *p, int64_t n_lens, size_t max_bytes, Plan &out);

}  // namespace rs
