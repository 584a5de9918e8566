// FP64 re-evaluation of rays whose FP32 source position is within its error
// bound of a pixel edge (the arithmetic lives in recheck_ray.h).
//
// Three stages keep the work per queued ray small and the exact evaluation rare:
//   stage F (far_ray.h, farfield.hip): the ray's super-patch FP64 expansion
//     plus the lenses listed near the super-patch, under a rigorous bound; it
//     places all but a few queued rays;
//   stage A (fast_ray): FP64 over every lens with fused multiply-adds and a
//     bound that also covers the definition's own FP64 rounding; it decides
//     almost every ray stage F left, identically to the definition, and marks
//     the rest;
//   stage B (exact_ray_wave): the marked rays, one wave per ray, with the
//     definition's exact operation sequence.
// RS_EXACT_RECHECK runs the exact sequence for every queued ray instead (one
// thread per ray).
//
// Single map: the queue holds uint32 chunk-relative ray indices. Unless the
// caller asked for the exact sequence only (or a random-ray window holds few of
// its map's rays), the far-field stage (farfield.hip) runs first and marks the entries it decided RESOLVED; stage A skips them and
// picks its form from the number left (*qlive).
// Batch: the deflection kernel sets one bit per flagged ray in each map's
// bitmap; a persistent scan compacts the set bits per wave and the map's
// descriptor supplies its parameters and its super-patch records (stage F).
#include "far_ray.h"

namespace rs {
namespace {

__device__ inline void count_wave(unsigned long long *counters, unsigned long long n_in,
                                  unsigned long long n_out, unsigned long long n_sing) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        n_in += __shfl_xor(n_in, off);
        n_out += __shfl_xor(n_out, off);
        n_sing += __shfl_xor(n_sing, off);
    }
    if (__lane_id() == 0) {
        if (n_in) atomicAdd(counters + C_IN, n_in);
        if (n_out) atomicAdd(counters + C_OUT, n_out);
        if (n_sing) atomicAdd(counters + C_SING, n_sing);
    }
}

__device__ inline void tally(int code, unsigned long long &n_in, unsigned long long &n_out,
                             unsigned long long &n_sing) {
    if (code >= 0) ++n_in;
    else if (code == CODE_OUT) ++n_out;
    else ++n_sing;
}

__device__ inline void place(const RecheckArgs &a, int64_t i, int64_t j, int code) {
    if (a.pix_out) a.pix_out[(j - a.j0) * (a.i1 - a.i0) + (i - a.i0)] = code;
    else if (code >= 0) atomicAdd(a.map + code, 1u);
}

// ----------------------------- single map ---------------------------------

// Below this many queued rays stage A runs one wave per ray (latency: a few
// rays must not each take a thread through every lens); above it, one thread
// per ray (throughput). Each of the two kernels checks the count on the device.
constexpr uint32_t WAVE_STAGE_MAX = 32768;

template <bool UNIT>
__global__ __launch_bounds__(256) void recheck_exact_kernel(const RecheckArgs a) {
    const uint32_t n = *a.qcount;
    const int64_t W = a.i1 - a.i0;
    unsigned long long n_in = 0, n_out = 0, n_sing = 0;
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t idx = blockIdx.x * blockDim.x + threadIdx.x; idx < n; idx += stride) {
        const uint32_t q = a.queue[idx];
        const int64_t i = a.i0 + (int64_t)(q % (uint64_t)W);
        const int64_t j = a.jc0 + (int64_t)(q / (uint64_t)W);
        const int code = exact_ray_thread<UNIT>(a, i, j);
        tally(code, n_in, n_out, n_sing);
        place(a, i, j, code);
    }
    count_wave(a.counters, n_in, n_out, n_sing);
    if (blockIdx.x == 0 && threadIdx.x == 0 && n) {
        atomicAdd(a.counters + C_RECHECK, (unsigned long long)n);
        atomicAdd(a.counters + C_DIRECT, (unsigned long long)n);
    }
}

template <bool UNIT>
__global__ __launch_bounds__(256) void recheck_fast_kernel(const RecheckArgs a) {
    const uint32_t n = *a.qcount;
    const uint32_t live = a.qlive ? *a.qlive : n;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        if (n) atomicAdd(a.counters + C_RECHECK, (unsigned long long)n);
        if (live) atomicAdd(a.counters + C_DIRECT, (unsigned long long)live);
    }
    if (live < WAVE_STAGE_MAX) return;   // recheck_fast_wave_kernel takes short queues
    const int64_t W = a.i1 - a.i0;
    unsigned long long n_in = 0, n_out = 0, n_sing = 0;
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t idx = blockIdx.x * blockDim.x + threadIdx.x; idx < n; idx += stride) {
        const uint32_t q = a.queue[idx];
        if (q & RESOLVED) continue;
        const int64_t i = a.i0 + (int64_t)(q % (uint64_t)W);
        const int64_t j = a.jc0 + (int64_t)(q / (uint64_t)W);
        int code;
        if (fast_ray<UNIT>(a, i, j, code)) {
            tally(code, n_in, n_out, n_sing);
            place(a, i, j, code);
        } else {
            a.queue[idx] = q | UNRESOLVED;
            if (a.qunres) atomicAdd(a.qunres, 1u);
        }
    }
    count_wave(a.counters, n_in, n_out, n_sing);
}

// Stage A for few live entries: one wave per ray. Entries are dealt to the
// waves 64 at a time (lane l of wave k reads entry k + (t + l) n_waves), so a
// long queue whose entries the far-field stage mostly decided costs each wave
// a few vector loads, and neighbouring live rays go to different waves.
template <bool UNIT>
__global__ __launch_bounds__(256) void recheck_fast_wave_kernel(const RecheckArgs a) {
    const uint32_t n = *a.qcount;
    const uint32_t live = a.qlive ? *a.qlive : n;
    if (live >= WAVE_STAGE_MAX || live == 0) return;
    const int64_t W = a.i1 - a.i0;
    const int lane = __lane_id();
    const uint32_t wave_id = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint32_t n_waves = (gridDim.x * blockDim.x) >> 6;
    unsigned long long n_in = 0, n_out = 0, n_sing = 0;
    for (uint64_t t0 = 0; (uint64_t)wave_id + t0 * n_waves < n; t0 += 64) {
        const uint64_t idx64 = (uint64_t)wave_id + (t0 + (uint64_t)lane) * n_waves;
        const uint32_t q_lane = idx64 < n ? a.queue[idx64] : RESOLVED;
        uint64_t todo = __ballot(!(q_lane & RESOLVED));
        while (todo) {
            const int src = __builtin_ctzll(todo);
            todo &= todo - 1;
            const uint32_t q = (uint32_t)__builtin_amdgcn_readlane((int)q_lane, src);
            const int64_t i = a.i0 + (int64_t)(q % (uint64_t)W);
            const int64_t j = a.jc0 + (int64_t)(q / (uint64_t)W);
            int code = 0;
            const bool decided = fast_ray_wave<UNIT>(a, i, j, code);
            if (lane == src) {
                if (decided) {
                    tally(code, n_in, n_out, n_sing);
                    place(a, i, j, code);
                } else {
                    a.queue[idx64] = q | UNRESOLVED;
                    if (a.qunres) atomicAdd(a.qunres, 1u);
                }
            }
        }
    }
    count_wave(a.counters, n_in, n_out, n_sing);
}

template <bool UNIT>
__global__ __launch_bounds__(256) void recheck_exact_wave_kernel(const RecheckArgs a) {
    if (a.qunres && *a.qunres == 0u) return;   // stage A decided every entry
    const uint32_t n = *a.qcount;
    const int64_t W = a.i1 - a.i0;
    const int lane = __lane_id();
    const uint32_t wave_id = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint32_t n_waves = (gridDim.x * blockDim.x) >> 6;
    // Entries are dealt to the waves one at a time (entry wave_id + t * n_waves), so
    // neighbouring marked rays go to different waves instead of queueing in one.
    for (uint64_t t0 = 0; (uint64_t)wave_id + t0 * n_waves < n; t0 += 64) {
        const uint64_t idx64 = (uint64_t)wave_id + (t0 + (uint64_t)lane) * n_waves;
        const uint32_t idx = (uint32_t)(idx64 < n ? idx64 : 0);
        const uint32_t q_lane = idx64 < n ? a.queue[idx] : 0u;
        uint64_t todo = __ballot(idx64 < n && (q_lane & UNRESOLVED));
        while (todo) {
            const int src = __builtin_ctzll(todo);
            todo &= todo - 1;
            const uint32_t q = (uint32_t)__builtin_amdgcn_readlane((int)q_lane, src) & ~UNRESOLVED;
            const int64_t i = a.i0 + (int64_t)(q % (uint64_t)W);
            const int64_t j = a.jc0 + (int64_t)(q / (uint64_t)W);
            const int code = exact_ray_wave<UNIT>(a, i, j);
            if (lane == 0) emit_ray(a, i, j, code);
        }
    }
}

// Maps of several launches: before stage A, the entries the far-field stage left
// (every entry, in the far-field mode) go to the map's gathered list and are
// marked placed in the launch's queue; the rest (past the list's capacity) are
// counted in *qleft, which stage A of this launch then reads as its live count.
// The stages over every lens cost about one pass over the lenses per wave whatever
// the number of rays, so running them once per map instead of once per launch
// saves a pass per launch.
__global__ __launch_bounds__(256) void recheck_defer_kernel(const RecheckArgs a) {
    const uint32_t n = *a.qcount;
    const int64_t W = a.i1 - a.i0;
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t idx = blockIdx.x * blockDim.x + threadIdx.x; idx < n; idx += stride) {
        const uint32_t q = a.queue[idx];
        if (q & RESOLVED) continue;
        // Once the list is full the count stops growing (by more than a grid's
        // worth), so it cannot wrap however many launches feed it.
        const uint32_t d = __hip_atomic_load(a.dcount, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >=
                                   (uint32_t)DEFER_CAP
                               ? (uint32_t)DEFER_CAP
                               : atomicAdd(a.dcount, 1u);
        if (d >= (uint32_t)DEFER_CAP) {
            atomicAdd(a.qleft, 1u);
            continue;
        }
        a.defer[2 * (int64_t)d] = a.i0 + (int64_t)(q % (uint64_t)W);
        a.defer[2 * (int64_t)d + 1] = a.jc0 + (int64_t)(q / (uint64_t)W);
        a.queue[idx] = q | RESOLVED;
    }
}

// Stage A over a map's gathered list, one wave per ray; the rays it cannot place
// go to a list of their own, so that the exact stage deals them out one per wave
// (marked in place, two of them could fall to one wave and its time would double).
template <bool UNIT>
__global__ __launch_bounds__(256) void recheck_fast_deferred_kernel(const RecheckArgs a) {
    const uint32_t total = *a.dcount;
    const uint32_t n = total < (uint32_t)DEFER_CAP ? total : (uint32_t)DEFER_CAP;
    if (blockIdx.x == 0 && threadIdx.x == 0 && n) atomicAdd(a.counters + C_DIRECT, (unsigned long long)n);
    const int lane = __lane_id();
    const uint32_t wave_id = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint32_t n_waves = (gridDim.x * blockDim.x) >> 6;
    for (uint32_t e = wave_id; e < n; e += n_waves) {
        const int64_t i = a.defer[2 * (int64_t)e], j = a.defer[2 * (int64_t)e + 1];
        int code = 0;
        const bool decided = fast_ray_wave<UNIT>(a, i, j, code);
        if (lane == 0) {
            if (decided) {
                emit_ray(a, i, j, code);
            } else {
                const uint32_t u = atomicAdd(a.ucount, 1u);   // u < n <= DEFER_CAP
                a.udefer[2 * (int64_t)u] = i;
                a.udefer[2 * (int64_t)u + 1] = j;
            }
        }
    }
}

// The exact stage over the gathered rays stage A left, one wave per ray.
template <bool UNIT>
__global__ __launch_bounds__(256) void recheck_exact_deferred_kernel(const RecheckArgs a) {
    const uint32_t n = *a.ucount;
    const int lane = __lane_id();
    const uint32_t wave_id = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint32_t n_waves = (gridDim.x * blockDim.x) >> 6;
    for (uint32_t e = wave_id; e < n; e += n_waves) {
        const int64_t i = a.udefer[2 * (int64_t)e], j = a.udefer[2 * (int64_t)e + 1];
        const int code = exact_ray_wave<UNIT>(a, i, j);
        if (lane == 0) emit_ray(a, i, j, code);
    }
}

// ------------------------------- batch -------------------------------------

__device__ inline RecheckArgs batch_recheck_args(const BatchMap &m) {
    return recheck_args_of(m.p, m.lens_xy, m.lens_m, m.n_lens, m.map, m.counters);
}

__device__ __forceinline__ void wave_sync() {
    // LDS operations of one wave execute in order; keep the compiler from moving
    // them across this point.
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Stage A for the entries held one per lane (valid lanes only): lanes are
// grouped by map, and each group runs with its map's parameters in scalar
// registers. Rays are decided, or marked for the exact stage.
template <bool ALL_UNIT>
__device__ inline void batch_stage_a(const BatchArgs &b, QueueEntry e, bool valid) {
    uint64_t pending = __ballot(valid);
    while (pending) {
        const int leader = __builtin_ctzll(pending);
        const uint32_t mi = (uint32_t)__builtin_amdgcn_readlane((int)e.map, leader);
        const bool mine = valid && e.map == mi;
        pending &= ~__ballot(mine);
        const BatchMap &m = b.maps[mi];
        const RecheckArgs a = make_uniform(batch_recheck_args(m));
        uint32_t *const unres = make_uniform(m.unres_bits);
        int code = CODE_OUT;
        bool ok = false;
        if (mine) {
            const int64_t W = a.i1 - a.i0;
            const int64_t i = a.i0 + (int64_t)(e.ray % (uint64_t)W);
            const int64_t j = a.j0 + (int64_t)(e.ray / (uint64_t)W);
            if (ALL_UNIT || a.lens_m == nullptr) ok = fast_ray<true>(a, i, j, code);
            else ok = fast_ray<false>(a, i, j, code);
            if (ok) {
                if (code >= 0) atomicAdd(a.map + code, 1u);
            } else {
                atomicOr(unres + (e.ray >> 5), 1u << (e.ray & 31u));
            }
        }
        // one counter update per group (stage A never yields a singular ray)
        const unsigned n_in = (unsigned)__builtin_popcountll(__ballot(mine && ok && code >= 0));
        const unsigned n_out = (unsigned)__builtin_popcountll(__ballot(mine && ok && code < 0));
        const bool any_unres = __ballot(mine && !ok) != 0;
        if (__lane_id() == leader) {
            if (n_in) atomicAdd(a.counters + C_IN, (unsigned long long)n_in);
            if (n_out) atomicAdd(a.counters + C_OUT, (unsigned long long)n_out);
            if (any_unres) atomicOr(b.unresolved, 1u);
        }
    }
}

// Stage F for the entries held one per lane (valid lanes only), lanes grouped
// by map as in stage A: each ray from its map's super-patch record and lens
// list. Returns true in the lanes whose ray it placed; the others are counted
// in their map's C_DIRECT and go on to stage A.
template <bool ALL_UNIT>
__device__ inline bool batch_stage_f(const BatchArgs &b, QueueEntry e, bool valid) {
    bool placed = false;
    uint64_t pending = __ballot(valid);
    while (pending) {
        const int leader = __builtin_ctzll(pending);
        const uint32_t mi = (uint32_t)__builtin_amdgcn_readlane((int)e.map, leader);
        const bool mine = valid && e.map == mi;
        pending &= ~__ballot(mine);
        const ShootArgs a = make_uniform(batch_far_args(b.maps[mi]));
        int code = FLAGGED;
        if (mine) {
            const int64_t W = a.i1 - a.i0;
            const int64_t i = a.i0 + (int64_t)(e.ray % (uint64_t)W);
            const int64_t j = a.j0 + (int64_t)(e.ray / (uint64_t)W);
            code = (ALL_UNIT || a.lens_m == nullptr) ? far_recheck_ray<true>(a, i, j) : far_recheck_ray<false>(a, i, j);
            if (code >= 0) atomicAdd(a.map + code, 1u);
            placed = code != FLAGGED;
        }
        const unsigned n_in = (unsigned)__builtin_popcountll(__ballot(mine && code >= 0));
        const unsigned n_out = (unsigned)__builtin_popcountll(__ballot(mine && code == OUT));
        const unsigned n_left = (unsigned)__builtin_popcountll(__ballot(mine && code == FLAGGED));
        if (__lane_id() == leader) {
            if (n_in) atomicAdd(a.counters + C_IN, (unsigned long long)n_in);
            if (n_out) atomicAdd(a.counters + C_OUT, (unsigned long long)n_out);
            if (n_left) atomicAdd(a.counters + C_DIRECT, (unsigned long long)n_left);
        }
    }
    return placed;
}

// Exact stage for up to 64 entries held one per lane: one wave per ray.
// Stage A of one queued ray (wave-uniform entry) by the whole wave: lanes split the
// lenses. Used for a wave's last few rays, where one ray per lane would leave the
// GPU mostly idle while each lane walks every lens.
__device__ inline void batch_stage_a_wave(const BatchArgs &b, QueueEntry e) {
    const BatchMap &m = b.maps[e.map];
    const RecheckArgs a = make_uniform(batch_recheck_args(m));
    const int64_t W = a.i1 - a.i0;
    const int64_t i = a.i0 + (int64_t)(e.ray % (uint64_t)W);
    const int64_t j = a.j0 + (int64_t)(e.ray / (uint64_t)W);
    int code = CODE_OUT;
    const bool ok = a.lens_m == nullptr ? fast_ray_wave<true>(a, i, j, code) : fast_ray_wave<false>(a, i, j, code);
    if (__lane_id() == 0) {
        if (ok) {
            if (code >= 0) atomicAdd(a.map + code, 1u);
            atomicAdd(a.counters + (code >= 0 ? C_IN : C_OUT), 1ull);
        } else {
            uint32_t *const unres = m.unres_bits;
            atomicOr(unres + (e.ray >> 5), 1u << (e.ray & 31u));
            atomicOr(b.unresolved, 1u);
        }
    }
}

__device__ inline void batch_stage_b(const BatchArgs &b, QueueEntry e, int n_valid) {
    const int lane = __lane_id();
    for (int s = 0; s < n_valid; ++s) {
        const uint32_t mi = (uint32_t)__builtin_amdgcn_readlane((int)e.map, s);
        const uint32_t ray = (uint32_t)__builtin_amdgcn_readlane((int)e.ray, s);
        const BatchMap &m = b.maps[mi];
        const RecheckArgs a = make_uniform(batch_recheck_args(m));
        const int64_t W = a.i1 - a.i0;
        const int64_t i = a.i0 + (int64_t)(ray % (uint64_t)W);
        const int64_t j = a.j0 + (int64_t)(ray / (uint64_t)W);
        const int code = a.lens_m == nullptr ? exact_ray_wave<true>(a, i, j) : exact_ray_wave<false>(a, i, j);
        if (lane == 0) emit_ray(a, i, j, code);
    }
}

// Persistent scan of the batch's bitmaps (STAGE 0: flag bits -> stage F, then
// stage A for the rays it leaves; STAGE 1: unresolved bits -> exact stage). The batch's words are dealt to the
// waves one at a time (lane l of wave k reads word k + (t + l) n_waves), so a
// dense run of flagged rays - a crowded lens region fills whole rows of them -
// is spread over many waves instead of queueing in one. Each wave compacts its
// set bits into its own ring buffer in LDS and evaluates them 64 at a time, one
// per lane. A wave leaves when its words are done and its buffer is empty.
template <int STAGE, bool ALL_UNIT>
__global__ __launch_bounds__(256) void recheck_scan_batch_kernel(const BatchArgs b) {
    if (STAGE == 1 && *b.unresolved == 0u) return;
    constexpr int RING = 128;
    __shared__ QueueEntry ring_all[4][RING];
    const int lane = __lane_id();
    QueueEntry *ring = ring_all[threadIdx.x >> 6];
    const uint64_t below = (1ull << lane) - 1ull;
    int head = 0, tail = 0;  // wave-uniform; tail - head < 64 between evaluations
    const int64_t wave_id = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int64_t n_waves = (int64_t)gridDim.x * (blockDim.x >> 6);
    for (int64_t t0 = 0; wave_id + t0 * n_waves < b.total_words; t0 += 64) {
        const int64_t word = wave_id + (t0 + lane) * n_waves;
        uint32_t bits = 0u;
        int lo = 0;
        int64_t w = 0;
        if (word < b.total_words) {
            int hi = b.n_maps - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (b.maps[mid].word_begin <= word) lo = mid;
                else hi = mid - 1;
            }
            const BatchMap &m = b.maps[lo];
            w = word - m.word_begin;
            bits = (STAGE == 0 ? m.flag_bits : m.unres_bits)[w];
        }
        for (;;) {
            const uint64_t hm = __ballot(bits != 0u);
            if (!hm) break;
            if (bits) {
                const int bit = __builtin_ctz(bits);
                bits &= bits - 1u;
                const int pos = (tail + __builtin_popcountll(hm & below)) % RING;
                ring[pos] = QueueEntry{(uint32_t)lo, (uint32_t)(w * 32 + bit)};
            }
            tail += __builtin_popcountll(hm);
            wave_sync();
            if (tail - head >= 64) {
                const QueueEntry e = ring[(head + lane) % RING];
                head += 64;
                wave_sync();
                if (STAGE == 0) {
                    const bool placed = batch_stage_f<ALL_UNIT>(b, e, true);
                    batch_stage_a<ALL_UNIT>(b, e, !placed);
                }
                else batch_stage_b(b, e, 64);
            }
        }
    }
    const int left = tail - head;
    if (left > 0) {
        QueueEntry e{0u, 0u};
        if (lane < left) e = ring[(head + lane) % RING];
        if (STAGE == 0) {
            // the last few rays: stage F one per lane, then stage A one wave per ray
            // (lenses split over the lanes) for those it could not place
            const bool placed = batch_stage_f<ALL_UNIT>(b, e, lane < left);
            uint64_t rest = __ballot(lane < left && !placed);
            while (rest) {
                const int s = __builtin_ctzll(rest);
                rest &= rest - 1;
                QueueEntry es;
                es.map = (uint32_t)__builtin_amdgcn_readlane((int)e.map, s);
                es.ray = (uint32_t)__builtin_amdgcn_readlane((int)e.ray, s);
                batch_stage_a_wave(b, es);
            }
        } else {
            batch_stage_b(b, e, left);
        }
    }
}

}  // namespace

hipError_t launch_recheck(const RecheckArgs &a, int64_t max_rays, bool exact_only, hipStream_t stream) {
    int64_t blocks = (max_rays + 255) / 256;
    if (blocks > 2048) blocks = 2048;
    if (blocks < 1) blocks = 1;
    const dim3 grid((unsigned)blocks), block(256);
    const bool unit = a.lens_m == nullptr;
    if (exact_only) {
        if (unit) hipLaunchKernelGGL(recheck_exact_kernel<true>, grid, block, 0, stream, a);
        else hipLaunchKernelGGL(recheck_exact_kernel<false>, grid, block, 0, stream, a);
    } else {
        RecheckArgs b = a;
        if (a.defer) {
            hipLaunchKernelGGL(recheck_defer_kernel, grid, block, 0, stream, a);
            b.qlive = a.qleft;   // stage A of this launch takes what was not gathered
        }
        if (unit) {
            hipLaunchKernelGGL(recheck_fast_kernel<true>, grid, block, 0, stream, b);
            hipLaunchKernelGGL(recheck_fast_wave_kernel<true>, grid, block, 0, stream, b);
            hipLaunchKernelGGL(recheck_exact_wave_kernel<true>, grid, block, 0, stream, b);
        } else {
            hipLaunchKernelGGL(recheck_fast_kernel<false>, grid, block, 0, stream, b);
            hipLaunchKernelGGL(recheck_fast_wave_kernel<false>, grid, block, 0, stream, b);
            hipLaunchKernelGGL(recheck_exact_wave_kernel<false>, grid, block, 0, stream, b);
        }
    }
    return hipGetLastError();
}

hipError_t launch_recheck_deferred(const RecheckArgs &a, hipStream_t stream) {
    const dim3 grid(1024), block(256);
    if (a.lens_m == nullptr) {
        hipLaunchKernelGGL(recheck_fast_deferred_kernel<true>, grid, block, 0, stream, a);
        hipLaunchKernelGGL(recheck_exact_deferred_kernel<true>, grid, block, 0, stream, a);
    } else {
        hipLaunchKernelGGL(recheck_fast_deferred_kernel<false>, grid, block, 0, stream, a);
        hipLaunchKernelGGL(recheck_exact_deferred_kernel<false>, grid, block, 0, stream, a);
    }
    return hipGetLastError();
}

hipError_t launch_recheck_batch(const BatchArgs &b, hipStream_t stream) {
    if (b.total_words <= 0) return hipSuccess;
    const dim3 grid(2048), block(256);
    // stage A in a kernel of its own for batches of unit-mass maps only (fewer registers)
    if (b.unit_masses) hipLaunchKernelGGL((recheck_scan_batch_kernel<0, true>), grid, block, 0, stream, b);
    else hipLaunchKernelGGL((recheck_scan_batch_kernel<0, false>), grid, block, 0, stream, b);
    hipLaunchKernelGGL((recheck_scan_batch_kernel<1, false>), grid, block, 0, stream, b);
    return hipGetLastError();
}

}  // namespace rs
