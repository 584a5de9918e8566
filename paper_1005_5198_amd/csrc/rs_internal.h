// Internal declarations shared by the HIP kernels and the host runtime.
// Not part of the public ABI (include/rayshoot.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

#include "rayshoot.h"
#include "rs_layout.h"

namespace rs {

// The deflection kernel's thread shape (rays per lane, waves per block) is a
// tunable choice among N_SHAPES that all cover the same PATCH_X x PATCH_Y patch.
struct ShapeInfo {
    int rx, ry, wx, wy;   // rays per lane along x, y; waves per block along x, y
};
const ShapeInfo &shape_info(int shape);


struct ShootArgs {
    // Ray grid: x1 = sx0 + ((double)i + 0.5) * spx (the same FP64 operations
    // as the definition), spx = sw / nx, spy = sh / ny.
    double sx0, sy0, spx, spy;
    int64_t i0, i1;      // window columns
    int64_t jc0, jc1;    // rows of this launch (a chunk of the window)
    int64_t j0;          // first row of the window (pix_out row offset)
    int64_t nbx;         // patches along x
    // Macro model and source grid.
    double c1, c2;       // (1 - gamma) - sigma_c, (1 + gamma) - sigma_c
    double tx0, ty0, inv_pixw, inv_pixh;  // u = (y1 - tx0) * inv_pixw
    int64_t npx, npy;
    // Lenses.
    const double *lens_xy;
    const double *lens_m;  // nullptr = unit masses
    int64_t n_lens;
    double bound_scale;    // covers FP64 fold and reference rounding, >= 1
    // Outputs.
    uint32_t *map;         // may be nullptr when pix_out is used
    int32_t *pix_out;      // per-ray output (window row-major) or nullptr
    unsigned long long *counters;
    uint32_t *queue;       // chunk-relative ray indices to re-check (mixed)
    uint32_t *qcount;
    // Random rays (RS_RANDOM_RAYS): the launch's rays are counted into square
    // bins of the shooting rectangle, sorted by bin, and a block deflects the
    // rays of one bin relative to the bin's centre.
    int32_t random;
    uint64_t seed;
    int64_t nx;            // ray grid width: the generator counter is j * nx + i
    double sw, sh;
    int64_t nbx_r, nby_r;  // bins of this launch
    double bw, bh;         // bin width and height
    double inv_bw, inv_bh; // nbx_r / sw, nby_r / sh
    uint32_t *bin_count;   // [n_bins]
    uint32_t *bin_offset;  // [n_bins + 1] exclusive prefix sums of bin_count
    uint32_t *bin_cursor;  // [n_bins] scatter cursors
    uint32_t *ray_rel;     // [rays] chunk-relative index (j - jc0) * (i1 - i0) + (i - i0), by bin
    double *ray_x, *ray_y; // [rays] FP64 positions, same order
    // Far-field expansion (RS_FARFIELD): super-patches of FF_SP_X x FF_SP_Y patches.
    int64_t ff_sbx;        // super-patches along x in this launch
    int64_t ff_sby;        // super-patches along y (random rays: a ray's cell is clamped to it)
    int64_t ff_i0, ff_j0;  // ray-grid origin of super-patch 0: the launch's (i0, jc0), or (0, 0)
                           // for random rays, whose records cover the whole shooting rectangle
    double *ff_super;      // [n_super][2 * 16 + 4] coefficients and bound terms
    int32_t *ff_near;      // [n_super][1 + ff_cap] count, then indices of the nearer lenses
    int32_t ff_cap;        // list capacity per super-patch
    double *ff_patch;      // far-field mode: [patches of the launch][FF_PATCH_DOUBLES] patch records
    uint32_t *ff_work;     // far-field mode: next patch to take (reset by the record kernel)
    int64_t ff_gbx;        // far-field mode: groups (FF_GROUP x FF_GROUP super-patches) along x
    double *ff_group;      // far-field mode: [groups][FF_GROUP_PARTS][FF_REC_DOUBLES] group records, per part
    int32_t *ff_glist;     // far-field mode: [groups][FF_GROUP_PARTS][1 + FF_PART_CAP] count, then the nearer lenses
                           // (with tops: one list of FF_GROUP_ONE_CAP per group in the same place)
    int64_t ff_tbx;        // far-field mode with tops: tops (FF_TOP x FF_TOP groups) along x
    double *ff_top;        // [tops][FF_TOP_PARTS][FF_REC_DOUBLES] top records, per part, or nullptr (no tops)
    int32_t *ff_tlist;     // [tops][FF_TOP_PARTS][1 + FF_TOP_PART_CAP] count, then the nearer lenses
};


struct RecheckArgs {
    double sx0, sy0, sw, sh;
    int64_t nx, ny;
    int64_t i0, i1, jc0, j0;
    double gamma, sigma_c;
    double tx0, ty0, tw, th;
    int64_t npx, npy;
    const double *lens_xy;
    const double *lens_m;
    int64_t n_lens;
    uint32_t *map;
    int32_t *pix_out;
    unsigned long long *counters;
    uint32_t *queue;       // stage A marks unresolved entries in place
    const uint32_t *qcount;
    const uint32_t *qlive; // entries the far-field stage left undecided, or nullptr (no such stage)
    uint32_t *qunres;      // entries stage A left to the exact stage (counted by stage A), or nullptr
    int32_t random;        // Philox-random ray positions (RS_RANDOM_RAYS)
    uint64_t seed;
    int64_t *defer;        // (i, j) pairs gathered for the stages over every lens after the last launch, or nullptr
    uint32_t *dcount;      // their count (may exceed DEFER_CAP: the rest stayed with their launch)
    int64_t *udefer;       // (i, j) pairs of the gathered rays stage A left to the exact stage (DEFER_CAP)
    uint32_t *ucount;      // their count
    uint32_t *qleft;       // this launch's live entries that were not gathered
};

// Shoot arguments of a whole window (no chunking): the same values the host
// computes for a single map, by the same IEEE operations, on host or device.
__host__ __device__ inline ShootArgs shoot_args_of(const rs_map_params &p, const double *lens_xy,
                                                   const double *lens_m, int64_t n_lens, uint32_t *map,
                                                   unsigned long long *counters) {
    ShootArgs a{};
    a.sx0 = p.sx0;
    a.sy0 = p.sy0;
    a.spx = p.sw / (double)p.nx;
    a.spy = p.sh / (double)p.ny;
    a.i0 = p.i0;
    a.i1 = p.i1;
    a.jc0 = p.j0;
    a.jc1 = p.j1;
    a.j0 = p.j0;
    a.nbx = (p.i1 - p.i0 + PATCH_X - 1) / PATCH_X;
    a.c1 = (1.0 - p.gamma) - p.sigma_c;
    a.c2 = (1.0 + p.gamma) - p.sigma_c;
    a.tx0 = p.tx0;
    a.ty0 = p.ty0;
    a.inv_pixw = (double)p.npx / p.tw;
    a.inv_pixh = (double)p.npy / p.th;
    a.npx = p.npx;
    a.npy = p.npy;
    a.lens_xy = lens_xy;
    a.lens_m = lens_m;
    a.n_lens = n_lens;
    a.bound_scale = 1.0 + (double)(n_lens + 64) * 4.7e-10;
    a.map = map;
    a.pix_out = nullptr;
    a.counters = counters;
    a.queue = nullptr;
    a.qcount = nullptr;
    return a;
}

__host__ __device__ inline RecheckArgs recheck_args_of(const rs_map_params &p, const double *lens_xy,
                                                       const double *lens_m, int64_t n_lens, uint32_t *map,
                                                       unsigned long long *counters) {
    RecheckArgs r{};
    r.sx0 = p.sx0;
    r.sy0 = p.sy0;
    r.sw = p.sw;
    r.sh = p.sh;
    r.nx = p.nx;
    r.ny = p.ny;
    r.i0 = p.i0;
    r.i1 = p.i1;
    r.jc0 = p.j0;
    r.j0 = p.j0;
    r.gamma = p.gamma;
    r.sigma_c = p.sigma_c;
    r.tx0 = p.tx0;
    r.ty0 = p.ty0;
    r.tw = p.tw;
    r.th = p.th;
    r.npx = p.npx;
    r.npy = p.npy;
    r.lens_xy = lens_xy;
    r.lens_m = lens_m;
    r.n_lens = n_lens;
    r.map = map;
    r.pix_out = nullptr;
    r.counters = counters;
    r.queue = nullptr;
    r.qcount = nullptr;
    r.random = (p.flags & RS_RANDOM_RAYS) ? 1 : 0;
    r.seed = p.seed;
    return r;
}

// ---------------------------------------------------------------------------
// Batched maps: one persistent launch over the patches of many maps.
// ---------------------------------------------------------------------------

// Per-map descriptor in device memory (work order: most expensive maps first).
struct BatchMap {
    rs_map_params p;
    const double *lens_xy;
    const double *lens_m;
    int64_t n_lens;
    uint32_t *map;
    unsigned long long *counters;  // N_COUNTERS per map, in the workspace (request order)
    int64_t tile_begin;            // first tile of this map in the work list
    int64_t n_tiles;
    uint32_t *flag_bits;           // one bit per ray of the window: re-check this ray
    uint32_t *unres_bits;          // one bit per ray: stage A could not place it
    int64_t word_begin;            // first bitmap word of this map in the batch's word space
    int64_t n_words;               // bitmap words, a multiple of 64
    int32_t request;               // index of the request this map came from
    int32_t accumulate;            // keep the map's contents (RS_ACCUMULATE)
    // Mixed mode: the far-field re-check stage's super-patch records of the window.
    int64_t ff_sbx;                // super-patches along x
    int64_t super_begin;           // first record of this map in the batch's record space
    int64_t n_super;
    double *ff_super;              // [n_super][FF_REC_DOUBLES]
    int32_t *ff_near;              // [n_super][1 + FF_BATCH_CAP]
};

struct QueueEntry {
    uint32_t map;   // index into the BatchMap array
    uint32_t ray;   // (j - j0) * (i1 - i0) + (i - i0)
};

struct BatchArgs {
    const BatchMap *maps;
    int32_t n_maps;
    int32_t mode;
    int32_t unit_masses;           // every map of the batch has unit masses
    int32_t pad;
    int64_t total_tiles;
    int64_t total_words;
    int64_t total_super;           // super-patch records of every map (mixed mode)
    unsigned long long *tile_counter;
    unsigned int *unresolved;          // set when stage A left a ray to the exact stage
};

// Batch workspace layout (bytes):
//   [globals 256: uint64 tile counter, uint32 unresolved flag]
//   [BatchMap x n][counters 64 x n][per map: flag bitmap, unresolved bitmap;
//    mixed mode: super-patch records, lens lists]
constexpr size_t BWS_GLOBALS = 256;
constexpr int64_t BITMAP_WORD_ALIGN = 64;   // a 64-word scan block never straddles two maps
inline size_t align256(size_t v) { return (v + 255) / 256 * 256; }
inline size_t batch_maps_offset() { return BWS_GLOBALS; }
inline size_t batch_counters_offset(int32_t n) { return align256(BWS_GLOBALS + sizeof(BatchMap) * (size_t)n); }
inline size_t batch_bitmaps_offset(int32_t n) {
    return align256(batch_counters_offset(n) + sizeof(unsigned long long) * N_COUNTERS * (size_t)n);
}
inline int64_t super_patches_of(const rs_map_params &p) {
    const int64_t nbx = (p.i1 - p.i0 + PATCH_X - 1) / PATCH_X, nby = (p.j1 - p.j0 + PATCH_Y - 1) / PATCH_Y;
    return ((nbx + FF_SP_X - 1) / FF_SP_X) * ((nby + FF_SP_Y - 1) / FF_SP_Y);
}
inline int64_t bitmap_words_of(const rs_map_params &p) {
    const int64_t rays = (p.i1 - p.i0) * (p.j1 - p.j0);
    const int64_t words = (rays + 31) / 32;
    return (words + BITMAP_WORD_ALIGN - 1) / BITMAP_WORD_ALIGN * BITMAP_WORD_ALIGN;
}

// Blocks of a persistent kernel on the current device: every CU times
// min(blocks_per_cu, the blocks that fit on it); blocks_per_cu <= 0 takes all that fit.
template <class K>
inline int persistent_blocks(K kernel, int threads, int blocks_per_cu) {
    int dev = 0, n_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n_cu <= 0)
        n_cu = 256;
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0) != hipSuccess || per_cu <= 0)
        per_cu = 2;
    if (blocks_per_cu > 0 && blocks_per_cu < per_cu) per_cu = blocks_per_cu;
    return n_cu * per_cu;
}

hipError_t launch_fill(uint32_t *map, int64_t n_pix, void *workspace, int64_t n_qcount,
                       hipStream_t stream);
hipError_t launch_zero(uint32_t *p, int64_t n, hipStream_t stream);
hipError_t launch_shoot(const ShootArgs &a, int mode, int shape, hipStream_t stream);
// Far-field expansion (RS_FARFIELD): one block per patch, FP64 local expansion plus near lenses.
hipError_t launch_farfield(const ShootArgs &a, hipStream_t stream);
// Random rays: count into bins, scan, scatter, then deflect bin by bin.
hipError_t launch_shoot_random(const ShootArgs &a, int mode, hipStream_t stream);
hipError_t launch_recheck(const RecheckArgs &a, int64_t max_rays, bool exact_only, hipStream_t stream);
// The exact stage of the rays a map's launches gathered in a.defer.
hipError_t launch_recheck_deferred(const RecheckArgs &a, hipStream_t stream);
// Mixed mode on the regular grid: the super-patch expansions of the launch, then
// the far-field re-check stage over the queue (a.queue, a.qcount); it counts the
// entries it leaves undecided in *qlive.
hipError_t launch_recheck_far(const ShootArgs &a, uint32_t *qlive, int64_t max_rays, hipStream_t stream);
// Records of n_super super-patches from origin (a.ff_i0, a.ff_j0), unconditionally
// (random rays: the whole rectangle, once per map).
hipError_t launch_super_records(const ShootArgs &a, int64_t n_super, hipStream_t stream);

hipError_t launch_batch_fill(const BatchArgs &b, void *workspace, int32_t n_maps, hipStream_t stream);
// Persistent launch: blocks_per_cu <= 0 fills every CU with as many blocks as fit.
hipError_t launch_shoot_batch(const BatchArgs &b, int shape, int blocks_per_cu, hipStream_t stream);
hipError_t launch_recheck_batch(const BatchArgs &b, hipStream_t stream);
// Mixed batches: super-patch records of every map that flagged rays.
hipError_t launch_batch_super(const BatchArgs &b, hipStream_t stream);

}  // namespace rs
