// Sizes and workspace layout of the library's launches: plain constants, shared
// by the HIP kernels, the host runtime and the host-only planning code.
#pragma once

#include <cstddef>
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

// Lenses staged into LDS per tile, and lenses per FP32 partial sum before it
// is folded into the FP64 accumulator.
constexpr int LENS_TILE = 1024;
constexpr int GROUP = 32;
constexpr int NEAR_MAX = 64;                  // per-block list of lenses close to the patch

// Workspace layout (bytes).
constexpr size_t WS_COUNTERS = 0;             // uint64 [8]: in, out, singular, rechecked, spare
constexpr size_t WS_QCOUNT = 64;              // uint32 [n_chunks] each: queue lengths, live counts, unresolved counts
constexpr int64_t CHUNK_RAYS = int64_t(1) << 27;  // rays per launch (queue capacity)
// Maps of several launches: the rays a launch's first re-check stage leaves are
// gathered (as (i, j) pairs) into one list of this capacity, and the stages over
// every lens run on it once, after the last launch; beyond it, rays stay with
// their own launch's stages.
constexpr int64_t DEFER_CAP = 65536;

enum Counter { C_IN = 0, C_OUT = 1, C_SING = 2, C_RECHECK = 3, C_DIRECT = 4 };
constexpr int N_COUNTERS = 8;

constexpr int FF_SP_X = 4;
constexpr int FF_SP_Y = 4;
constexpr int FF_NEAR_CAP = 4096;    // single maps (the far-field mode rescans all lenses beyond it)
constexpr int FF_BATCH_CAP = 1024;   // batches (the re-check stage only; beyond it, the stage over every lens)
constexpr int FF_REC_DOUBLES = 36;
// Far-field mode: groups of FF_GROUP x FF_GROUP super-patches above the
// super-patches (their lists hold the candidates of their super-patches).
constexpr int FF_GROUP = 4;
// A group's lenses are scanned by FF_GROUP_PARTS blocks, each over a contiguous range of lens
// indices with a record and a list (of capacity FF_GROUP_CAP / FF_GROUP_PARTS) of its own.
constexpr int FF_GROUP_PARTS = 4;
constexpr int FF_GROUP_CAP = 16384;
constexpr int FF_PART_CAP = FF_GROUP_CAP / FF_GROUP_PARTS;
// Far-field mode with at least FF_TOP_MIN_LENSES lenses: tops of FF_TOP x FF_TOP groups above
// the groups. A top's lenses are scanned as a group's were, by FF_TOP_PARTS blocks (a launch
// holds few tops), each with a record and a list of capacity FF_TOP_PART_CAP; a group then
// scans its top's lists instead of every lens and keeps one list of capacity FF_GROUP_ONE_CAP
// in its lists' place.
constexpr int FF_TOP = 4;
constexpr int64_t FF_TOP_MIN_LENSES = 131072;
constexpr int FF_TOP_PARTS = 8;
constexpr int FF_TOP_PART_CAP = 16384;
constexpr int FF_GROUP_ONE_CAP = FF_GROUP_PARTS * (1 + FF_PART_CAP) - 1;
// Far-field mode, per 64 x 32-ray patch: the local expansion about the patch
// centre (16 real, 16 imaginary coefficients), the bound terms SFAR, far_err and
// SDEF, the number of near lenses (summed directly), three spare doubles, then
// the first FF_PATCH_NEAR near lenses' x, y and mass (when there are more, the
// ray kernel finds them itself).
constexpr int FF_PATCH_HEAD = 40;
constexpr int FF_PATCH_NEAR = 24;
constexpr int FF_PATCH_DOUBLES = FF_PATCH_HEAD + 3 * FF_PATCH_NEAR;

// Random rays: expected rays per bin (a block's capacity is 2048, so a bin
// overflows it only beyond three standard deviations, about one bin in 3000,
// and then takes a second pass), and the largest launch.
constexpr int64_t RAND_BIN_RAYS = 1900;
constexpr int64_t RAND_CHUNK_RAYS = int64_t(1) << 26;

}  // namespace rs
