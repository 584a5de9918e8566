// Internal declarations shared by the HIP kernels and the host runtime.
// Not part of the public ABI (include/rayshoot.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace rs {

// Ray patch of one block of the deflection kernel: PATCH_X x PATCH_Y rays,
// lanes laid out 8 x 8 per wave. The thread shape (rays per lane, waves per
// block) is a tunable choice among N_SHAPES that all cover the same patch.
constexpr int LANES_X = 8;
constexpr int LANES_Y = 8;
constexpr int PATCH_X = 64;
constexpr int PATCH_Y = 32;
constexpr int N_SHAPES = 4;
struct ShapeInfo {
    int rx, ry, wx, wy;   // rays per lane along x, y; waves per block along x, y
};
const ShapeInfo &shape_info(int shape);

// Lenses staged into LDS per tile, and lenses per FP32 partial sum before it
// is folded into the FP64 accumulator.
constexpr int LENS_TILE = 1024;
constexpr int GROUP = 16;
constexpr int NEAR_MAX = 64;                  // per-block list of lenses close to the patch

// Workspace layout (bytes).
constexpr size_t WS_COUNTERS = 0;             // uint64 [8]: in, out, singular, rechecked, spare
constexpr size_t WS_QCOUNT = 64;              // uint32 [n_chunks] queue lengths
constexpr int64_t CHUNK_RAYS = int64_t(1) << 27;  // rays per launch (queue capacity)

enum Counter { C_IN = 0, C_OUT = 1, C_SING = 2, C_RECHECK = 3 };

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
};

hipError_t launch_fill(uint32_t *map, int64_t n_pix, void *workspace, int64_t n_qcount,
                       hipStream_t stream);
hipError_t launch_shoot(const ShootArgs &a, int mode, int shape, hipStream_t stream);
hipError_t launch_recheck(const RecheckArgs &a, int64_t max_rays, bool exact_only, hipStream_t stream);

}  // namespace rs
