// CPU driver of the host-side launch planning (paper_1005_5198_amd/csrc/plan.cpp:
// validation, launch plans, plans within a fixed scratch), built with
// AddressSanitizer and UndefinedBehaviorSanitizer by tests/test_plan_host.py.
// For a table of windows (every mode, random rays, exact re-check, widths up to
// the 2^22 limit, a single ray, empty windows) it checks the plan's invariants and
// prints one JSON object of results.
#include "rs_plan.h"

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <string>
#include <vector>

namespace rs {
static std::string g_err;
int fail(int code, const char *fmt, ...) {
    char buf[256];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}
}  // namespace rs

using namespace rs;

namespace {

rs_map_params base(int64_t nx, int64_t ny) {
    rs_map_params p{};
    p.sigma_star = 0.4;
    p.sx0 = -20.0;
    p.sy0 = -10.0;
    p.sw = 40.0;
    p.sh = 20.0;
    p.nx = nx;
    p.ny = ny;
    p.i1 = nx;
    p.j1 = ny;
    p.tx0 = p.ty0 = -10.0;
    p.tw = p.th = 20.0;
    p.npx = p.npy = 1024;
    p.mode = RS_MIXED;
    return p;
}

// Every invariant of a plan that the launch code relies on; returns the first broken one.
std::string check(const rs_map_params &p, int64_t n_lens, const Plan &pl) {
    const int64_t W = p.i1 - p.i0, H = p.j1 - p.j0;
    if (pl.W != W || pl.H != H) return "window";
    if (pl.rows_per_chunk <= 0 || pl.rows_per_chunk % PATCH_Y) return "rows not whole bands";
    if (W > 0 && H > 0 && pl.n_chunks != (H + pl.rows_per_chunk - 1) / pl.rows_per_chunk) return "chunk count";
    const int64_t rows_cap = H < pl.rows_per_chunk ? H : pl.rows_per_chunk;
    // queue entries are launch-relative ray indices; bits 30 and 31 mark them
    if (p.mode != RS_FP32 && W > 0 && H > 0) {
        if (pl.queue_cap < rows_cap * W) return "queue below a launch's rays";
        if (rows_cap * W - 1 >= (int64_t(1) << 30)) return "queue index reaches the mark bits";
    }
    // per launch: queue length, live, unresolved and left counts; then the gathered counts
    if (pl.qcount_bytes < WS_QCOUNT + 16 * (size_t)pl.n_chunks + 8 || pl.qcount_bytes % 256) return "qcount area";
    size_t end = pl.qcount_bytes + 4 * (size_t)pl.queue_cap;
    if (end > pl.bytes) return "queue beyond the workspace";
    if (pl.super_cap > 0) {
        if (pl.ff_super_off % 256 || pl.ff_near_off % 256 || pl.ff_super_off < end) return "record offsets";
        if (pl.ff_near_off < pl.ff_super_off + sizeof(double) * FF_REC_DOUBLES * (size_t)pl.super_cap)
            return "records overlap the lists";
        end = pl.ff_near_off + sizeof(int32_t) * (1 + (size_t)FF_NEAR_CAP) * (size_t)pl.super_cap;
        if (end > pl.bytes) return "lists beyond the workspace";
        // every patch row of the largest launch has its super-patch record
        const int64_t nbx = (W + PATCH_X - 1) / PATCH_X, nby = (rows_cap + PATCH_Y - 1) / PATCH_Y;
        const int64_t sbx = (nbx + FF_SP_X - 1) / FF_SP_X, sby = (nby + FF_SP_Y - 1) / FF_SP_Y;
        if (!pl.random && pl.super_cap < sbx * sby) return "too few records";
        if (p.mode == RS_FARFIELD) {
            // patch records, the patch counter, group records and group lists, in that order
            if (pl.patch_cap < nbx * nby) return "too few patch records";
            if (pl.ff_patch_off % 256 || pl.ff_patch_off < end) return "patch record offset";
            end = pl.ff_patch_off + sizeof(double) * FF_PATCH_DOUBLES * (size_t)pl.patch_cap;
            if (pl.ff_work_off % 256 || pl.ff_work_off < end) return "patch counter offset";
            end = pl.ff_work_off + 4;
            const int64_t groups = ((sbx + FF_GROUP - 1) / FF_GROUP) * ((sby + FF_GROUP - 1) / FF_GROUP);
            if (pl.group_cap < groups) return "too few group records";
            if (pl.ff_group_off % 256 || pl.ff_group_off < end) return "group record offset";
            end = pl.ff_group_off + sizeof(double) * FF_REC_DOUBLES * FF_GROUP_PARTS * (size_t)pl.group_cap;
            if (pl.ff_glist_off % 256 || pl.ff_glist_off < end) return "group list offset";
            end = pl.ff_glist_off + sizeof(int32_t) * (1 + (size_t)FF_PART_CAP) * FF_GROUP_PARTS * (size_t)pl.group_cap;
            if (end > pl.bytes) return "group lists beyond the workspace";
            // tops above the groups from FF_TOP_MIN_LENSES lenses on: records, then lists
            const int64_t gbx = (sbx + FF_GROUP - 1) / FF_GROUP, gby = (sby + FF_GROUP - 1) / FF_GROUP;
            const int64_t tops = ((gbx + FF_TOP - 1) / FF_TOP) * ((gby + FF_TOP - 1) / FF_TOP);
            if ((n_lens >= FF_TOP_MIN_LENSES) != (pl.top_cap > 0)) return "tops";
            if (pl.top_cap > 0) {
                if (pl.top_cap < tops) return "too few top records";
                if (pl.ff_top_off % 256 || pl.ff_top_off < end) return "top record offset";
                end = pl.ff_top_off + sizeof(double) * FF_REC_DOUBLES * FF_TOP_PARTS * (size_t)pl.top_cap;
                if (pl.ff_tlist_off % 256 || pl.ff_tlist_off < end) return "top list offset";
                end = pl.ff_tlist_off + sizeof(int32_t) * (1 + (size_t)FF_TOP_PART_CAP) * FF_TOP_PARTS * (size_t)pl.top_cap;
                if (end > pl.bytes) return "top lists beyond the workspace";
            }
        } else if (pl.top_cap != 0) {
            return "tops outside the far-field mode";
        }
    }
    // several launches of a mode with re-checks gather their exact-stage rays
    const bool want_defer = p.mode != RS_FP32 && !(p.flags & RS_EXACT_RECHECK) && pl.n_chunks > 1;
    if (pl.defer != want_defer) return "deferred list";
    if (pl.defer) {
        if (pl.defer_off % 256 || pl.defer_off < end) return "deferred list offset";
        end = pl.defer_off + 2 * sizeof(int64_t) * 2 * (size_t)DEFER_CAP;
        if (end > pl.bytes) return "deferred list beyond the workspace";
    }
    if (pl.random && pl.n_chunks > 0) {
        if (pl.rays_cap < rows_cap * W) return "sorted-ray list below a launch";
        int64_t bx, by;
        for (int64_t c = 0; c < pl.n_chunks; ++c) {
            const int64_t r0 = c * pl.rows_per_chunk, r1 = std::min(H, r0 + pl.rows_per_chunk);
            random_bins((r1 - r0) * W, p.sw, p.sh, bx, by);
            if (bx * by > pl.bins_cap || bx < 1 || by < 1) return "bins of a launch";
        }
        const size_t offs[] = {pl.bin_count_off, pl.bin_offset_off, pl.bin_cursor_off, pl.rel_off, pl.x_off, pl.y_off};
        for (size_t o : offs)
            if (o % 256 || o < end) return "random-ray offsets";
        if (pl.y_off + 8 * (size_t)pl.rays_cap > pl.bytes) return "random rays beyond the workspace";
    }
    return "";
}

}  // namespace

int main() {
    std::string out = "{";
    auto put = [&](const std::string &k, const std::string &v) {
        if (out.size() > 1) out += ",";
        out += "\"" + k + "\":" + v;
    };

    // 1. Validation: each bad field is refused, each good edge accepted.
    {
        struct Case {
            const char *name;
            bool ok;
            rs_map_params p;
        };
        std::vector<Case> cases;
        auto add = [&](const char *name, bool ok, auto edit) {
            rs_map_params p = base(1024, 512);
            edit(p);
            cases.push_back({name, ok, p});
        };
        add("good", true, [](rs_map_params &) {});
        add("nx0", false, [](rs_map_params &p) { p.nx = 0; });
        add("npy_neg", false, [](rs_map_params &p) { p.npy = -1; });
        add("pixels_2p31", false, [](rs_map_params &p) { p.npx = 65536; p.npy = 32768; });
        add("pixels_below_2p31", true, [](rs_map_params &p) { p.npx = 65536; p.npy = 32767; });
        add("sw_nan", false, [](rs_map_params &p) { p.sw = NAN; });
        add("th_zero", false, [](rs_map_params &p) { p.th = 0.0; });
        add("tx0_inf", false, [](rs_map_params &p) { p.tx0 = INFINITY; });
        add("gamma_nan", false, [](rs_map_params &p) { p.gamma = NAN; });
        add("window_past_grid", false, [](rs_map_params &p) { p.i1 = p.nx + 1; });
        add("window_reversed", false, [](rs_map_params &p) { p.j0 = 5; p.j1 = 4; });
        add("window_empty", true, [](rs_map_params &p) { p.i0 = p.i1 = 7; });
        add("width_2p22", true, [](rs_map_params &p) { p.nx = int64_t(1) << 22; p.i1 = p.nx; });
        add("width_over_2p22", false, [](rs_map_params &p) { p.nx = (int64_t(1) << 22) + 1; p.i1 = p.nx; });
        add("mode_bad", false, [](rs_map_params &p) { p.mode = 9; });
        add("farfield_random", false, [](rs_map_params &p) { p.mode = RS_FARFIELD; p.flags = RS_RANDOM_RAYS; });
        add("flags_bad", false, [](rs_map_params &p) { p.flags = 64; });
        std::string bad;
        for (const Case &c : cases) {
            const bool ok = validate(&c.p, 10) == RS_OK;
            if (ok != c.ok) bad += std::string(bad.empty() ? "" : ",") + "\"" + c.name + "\"";
        }
        if (validate(nullptr, 0) != RS_EINVAL) bad += std::string(bad.empty() ? "" : ",") + "\"null\"";
        rs_map_params p = base(64, 64);
        if (validate(&p, -1) != RS_EINVAL) bad += std::string(bad.empty() ? "" : ",") + "\"n_lens\"";
        put("validate_cases", std::to_string(cases.size() + 2));
        put("validate_wrong", "[" + bad + "]");
    }

    // 2. Plans: invariants over modes, flags and window shapes; plans within a scratch.
    {
        const int64_t widths[] = {1, 63, 64, 65, 1000, 19200, 32768, 1 << 20, 1 << 22};
        const int64_t heights[] = {1, 31, 32, 33, 640, 3840, 32768};
        const int modes[] = {RS_FP32, RS_MIXED, RS_FARFIELD};
        const int flag_sets[] = {0, RS_RANDOM_RAYS, RS_EXACT_RECHECK};
        const int64_t lens_counts[] = {100, FF_TOP_MIN_LENSES};
        const size_t caps[] = {size_t(64) << 20, size_t(8) << 20, size_t(1) << 20};
        int plans = 0, within = 0, refused = 0;
        std::string broken;
        for (int64_t W : widths)
            for (int64_t H : heights)
                for (int m : modes)
                    for (int f : flag_sets)
                    for (int64_t n_lens : lens_counts) {
                        if (m == RS_FARFIELD && (f & RS_RANDOM_RAYS)) continue;
                        if (m != RS_FARFIELD && n_lens != 100) continue;   // only the far-field plan depends on it
                        if ((double)W * (double)H > 3e9) continue;   // keep the table quick
                        rs_map_params p = base(W, H + 5);
                        p.j0 = 5;
                        p.j1 = H + 5;
                        p.mode = m;
                        p.flags = f;
                        if (validate(&p, n_lens) != RS_OK) {
                            broken += "\"invalid " + std::to_string(W) + "x" + std::to_string(H) + "\",";
                            continue;
                        }
                        const Plan pl = make_plan(&p, n_lens);
                        ++plans;
                        std::string e = check(p, n_lens, pl);
                        if (!e.empty())
                            broken += "\"" + e + " " + std::to_string(W) + "x" + std::to_string(H) + " m" +
                                      std::to_string(m) + " f" + std::to_string(f) + "\",";
                        for (size_t cap : caps) {
                            Plan pc;
                            if (!plan_within(&p, n_lens, cap, pc)) {
                                ++refused;
                                // refused only when one band does not fit
                                if (make_plan(&p, n_lens, PATCH_Y).bytes <= cap) broken += "\"refused a fitting window\",";
                                continue;
                            }
                            ++within;
                            e = check(p, n_lens, pc);
                            if (!e.empty() || pc.bytes > cap || pc.rows_per_chunk > pl.rows_per_chunk)
                                broken += "\"within " + e + " " + std::to_string(W) + "x" + std::to_string(H) + "\",";
                            // the most rows that fit: one more band would not (unless the whole window fits)
                            if (pc.rows_per_chunk < pl.rows_per_chunk && pc.rows_per_chunk < H &&
                                make_plan(&p, n_lens, pc.rows_per_chunk + PATCH_Y).bytes <= cap)
                                broken += "\"not the largest fitting band count\",";
                        }
                    }
        if (!broken.empty()) broken.pop_back();
        put("plans", std::to_string(plans));
        put("plans_within", std::to_string(within));
        put("plans_refused", std::to_string(refused));
        put("plan_broken", "[" + broken + "]");
    }

    // 3. The config-2 plan (19200 x 3840 rays, mixed): one launch, 4 bytes of queue per ray.
    {
        rs_map_params p = base(19200, 3840);
        p.sx0 = -120.0;
        p.sw = 240.0;
        p.sy0 = -24.0;
        p.sh = 48.0;
        const Plan pl = make_plan(&p, 17240);
        put("c2_chunks", std::to_string(pl.n_chunks));
        put("c2_bytes", std::to_string(pl.bytes));
        Plan pc;
        const bool ok = plan_within(&p, 17240, size_t(64) << 20, pc);
        put("c2_scratch_chunks", std::to_string(ok ? pc.n_chunks : -1));
        put("c2_scratch_rows", std::to_string(ok ? pc.rows_per_chunk : -1));
    }
    out += "}";
    std::printf("%s\n", out.c_str());
    return 0;
}
