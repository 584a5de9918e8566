// Per-ray FP64 re-evaluation, shared by the re-check kernels (single map and
// batch) and by the deflection kernel's in-place fallback when a batch queue
// is full.
//
// exact_ray_*: the plain definition, operation for operation —
//   ray position (Section 3.1 regular grid, cell-centred, or the ray's random point):
//       x1 = sx0 + ((double)i + 0.5) * (sw / nx)   or   x1 = sx0 + U1 * sw
//   Section 2, Eq. (sigma): a1 = sum_k (m_k / r2) * d1 in lens order,
//       d1 = x1 - X_k, r2 = d1*d1 + d2*d2; a ray with r2 == 0 is singular;
//   y1 = ((1 - gamma) - sigma_c) * x1 - a1, u = (y1 - tx0) / (tw / npx);
//   pixel floor(u), floor(v) if 0 <= u < npx and 0 <= v < npy, else out.
// Every operation is one IEEE-754 binary64 operation (no contraction: the
// library is compiled with -ffp-contract=off), so the result is the
// definition's, bit for bit.
//
// fast_ray: FP64 with fused multiply-adds and a Newton-refined v_rcp_f64,
// plus S = sum (|d1|+|d2|) |m|/r2. Its deviation from the exact real value,
// and the definition's own, are each at most (N+10) 2^-53 S + 8 2^-53
// (|c1 x1| + |a1| + |tx0|) in source units; a ray farther than twice that
// from every pixel edge is decided identically to the definition.
#pragma once

#include "rs_internal.h"
#include "philox.h"

namespace rs {

constexpr uint32_t UNRESOLVED = 0x80000000u;  // queue mark: stage A could not place the ray
constexpr uint32_t RESOLVED = 0x40000000u;    // queue mark: the far-field stage placed the ray

// A copy of a wave-uniform struct whose every 32-bit word goes through
// readfirstlane, so the compiler keeps it in scalar registers.
template <class T>
__device__ __forceinline__ T make_uniform(const T &v) {
    static_assert(sizeof(T) % 4 == 0, "word-sized struct");
    T out;
    const int *src = reinterpret_cast<const int *>(&v);
    int *dst = reinterpret_cast<int *>(&out);
#pragma unroll
    for (int k = 0; k < (int)(sizeof(T) / 4); ++k) dst[k] = __builtin_amdgcn_readfirstlane(src[k]);
    return out;
}
constexpr int CODE_OUT = -1;
constexpr int CODE_SINGULAR = -2;

// Lens reads through a global-address-space pointer. A batch's descriptors hold
// plain (generic) pointers; read through those, the lens loop compiles to flat
// loads that wait on every memory counter each iteration.
typedef __attribute__((address_space(1))) const double global_double;
typedef __attribute__((address_space(1))) const int32_t global_i32;

// Relaxed device-scope atomic adds through global (not flat) addressing, so a
// later wait on LDS results does not also wait for these to complete.
__device__ __forceinline__ void global_add(uint32_t *p, uint32_t v) {
    __hip_atomic_fetch_add((__attribute__((address_space(1))) uint32_t *)p, v, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void global_add(unsigned long long *p, unsigned long long v) {
    __hip_atomic_fetch_add((__attribute__((address_space(1))) unsigned long long *)p, v, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double lens_x(const RecheckArgs &a, int64_t k) {
    return ((global_double *)a.lens_xy)[2 * k];
}
__device__ __forceinline__ double lens_y(const RecheckArgs &a, int64_t k) {
    return ((global_double *)a.lens_xy)[2 * k + 1];
}
__device__ __forceinline__ double lens_mass(const RecheckArgs &a, int64_t k) {
    return ((global_double *)a.lens_m)[k];
}

// Image-plane position of ray (i, j): the regular grid's cell centre, or the
// ray's Philox-random point of the shooting rectangle.
__device__ __forceinline__ void ray_xy(const RecheckArgs &a, int64_t i, int64_t j, double &x1, double &x2) {
    if (a.random) {
        random_ray_xy(a.sx0, a.sy0, a.sw, a.sh, a.nx, a.seed, i, j, x1, x2);
    } else {
        x1 = a.sx0 + ((double)i + 0.5) * (a.sw / (double)a.nx);
        x2 = a.sy0 + ((double)j + 0.5) * (a.sh / (double)a.ny);
    }
}

template <bool UNIT>
__device__ inline int exact_ray_thread(const RecheckArgs &a, int64_t i, int64_t j) {
    double x1, x2;
    ray_xy(a, i, j, x1, x2);
    double a1 = 0.0, a2 = 0.0;
    for (int64_t k = 0; k < a.n_lens; ++k) {
        const double d1 = x1 - lens_x(a, k);
        const double d2 = x2 - lens_y(a, k);
        const double r2 = d1 * d1 + d2 * d2;
        if (r2 == 0.0) return CODE_SINGULAR;
        const double m = UNIT ? 1.0 : lens_mass(a, k);
        const double f = m / r2;
        a1 += f * d1;
        a2 += f * d2;
    }
    const double y1 = ((1.0 - a.gamma) - a.sigma_c) * x1 - a1;
    const double y2 = ((1.0 + a.gamma) - a.sigma_c) * x2 - a2;
    const double u = (y1 - a.tx0) / (a.tw / (double)a.npx);
    const double v = (y2 - a.ty0) / (a.th / (double)a.npy);
    if (isfinite(u) && isfinite(v) && u >= 0.0 && u < (double)a.npx && v >= 0.0 && v < (double)a.npy)
        return (int)((int64_t)floor(v) * a.npx + (int64_t)floor(u));
    return CODE_OUT;
}

// The same definition evaluated by a whole wave for one ray (i, j wave-uniform):
// lanes form the per-lens terms (m/r2)*d1, (m/r2)*d2 of 64 lenses at a time and
// stage them in LDS; every lane then adds them in lens order (the same sum in
// every lane, so no lane-to-scalar moves sit on the dependent chain). Callers
// are blocks of at most 256 threads.
__device__ __forceinline__ void wave_lds_fence() {
    // LDS accesses of one wave complete in order; keep the compiler from moving them across.
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

template <bool UNIT>
__device__ inline int exact_ray_wave(const RecheckArgs &a, int64_t i, int64_t j) {
    __shared__ double2 terms[4][2][64];   // [wave][buffer][lens of the chunk]: (m/r2 d1, m/r2 d2)
    const int lane = __lane_id();
    const int w = (threadIdx.x >> 6) & 3;
    double x1, x2;
    ray_xy(a, i, j, x1, x2);
    double a1 = 0.0, a2 = 0.0;
    bool zero = false;
    if (a.n_lens > 0) {
        // Loads and terms have no branches (indices past the last lens read the last
        // lens, and their terms are replaced by zero, which adds nothing: the running
        // sums start at +0 and never become -0), so the compiler can count the loads
        // in flight and wait for the oldest only.
        const int64_t last = a.n_lens - 1;
        auto load = [&](int64_t k, double &X, double &Y, double &M) {
            const int64_t kc = k < a.n_lens ? k : last;
            X = lens_x(a, kc);
            Y = lens_y(a, kc);
            M = UNIT ? 1.0 : lens_mass(a, kc);
        };
        auto term = [&](int64_t k, double X, double Y, double M) {
            const double d1 = x1 - X;
            const double d2 = x2 - Y;
            const double r2 = d1 * d1 + d2 * d2;
            const bool real = k < a.n_lens;
            zero |= real && (r2 == 0.0);
            const double m = UNIT ? 1.0 : M;
            const double f = m / r2;
            return make_double2(real ? f * d1 : 0.0, real ? f * d2 : 0.0);
        };
        const int64_t n_chunks = (a.n_lens + 63) / 64;
        {
            double X, Y, M;
            load(lane, X, Y, M);
            terms[w][0][lane] = term(lane, X, Y, M);
        }
        // Lens positions are loaded P chunks ahead of their terms (slot s of the ring
        // holds chunk c + 1 while chunk c is summed, c = s mod P), and a chunk's terms
        // are formed while the previous chunk is summed, so neither the memory latency
        // nor the division sits on the dependent chain of additions.
        constexpr int P = 4;
        double SX[P], SY[P], SM[P];
#pragma unroll
        for (int s = 0; s < P; ++s) load(64 * (s + 1) + lane, SX[s], SY[s], SM[s]);
        wave_lds_fence();
        // Whole rounds of P chunks: the chunks past the last one hold zero terms.
        for (int64_t c0 = 0; c0 < n_chunks; c0 += P) {
#pragma unroll
            for (int s = 0; s < P; ++s) {
                const int64_t c = c0 + s;
                const double2 tn = term(64 * (c + 1) + lane, SX[s], SY[s], SM[s]);
                load(64 * (c + 1 + P) + lane, SX[s], SY[s], SM[s]);
                const double2 *T = terms[w][c & 1];
                // in lens order, eight terms read ahead of their additions (LDS latency
                // is several times one addition's)
                constexpr int B = 8;
                double2 cur[B];
#pragma unroll
                for (int l = 0; l < B; ++l) cur[l] = T[l];
#pragma unroll
                for (int g = 0; g < 64 / B; ++g) {
                    double2 nxt[B];
#pragma unroll
                    for (int l = 0; l < B; ++l) nxt[l] = T[(B * (g + 1) + l) & 63];
#pragma unroll
                    for (int l = 0; l < B; ++l) {
                        a1 += cur[l].x;
                        a2 += cur[l].y;
                    }
#pragma unroll
                    for (int l = 0; l < B; ++l) cur[l] = nxt[l];
                }
                terms[w][(c + 1) & 1][lane] = tn;
                wave_lds_fence();   // every lane has read chunk c, and chunk c + 1 is written
            }
        }
    }
    if (__ballot(zero)) return CODE_SINGULAR;
    const double y1 = ((1.0 - a.gamma) - a.sigma_c) * x1 - a1;
    const double y2 = ((1.0 + a.gamma) - a.sigma_c) * x2 - a2;
    const double u = (y1 - a.tx0) / (a.tw / (double)a.npx);
    const double v = (y2 - a.ty0) / (a.th / (double)a.npy);
    if (isfinite(u) && isfinite(v) && u >= 0.0 && u < (double)a.npx && v >= 0.0 && v < (double)a.npy)
        return (int)((int64_t)floor(v) * a.npx + (int64_t)floor(u));
    return CODE_OUT;
}

// Stage A's pixel decision. (a1, a2) is this stage's FP64 sum, S = sum (|d1| + |d2|) |m| / r^2
// over every lens, and t1, t2 bound |definition's a_i - this a_i| (both roundings added); the
// ray is decided when its position is farther than that, plus both epilogues' rounding, from
// every pixel edge.
__device__ inline bool stage_a_decide(const RecheckArgs &a, double x1, double x2, double a1, double a2, double S,
                                      double t1, double t2, bool tiny, int &code) {
    const double U64 = 1.1102230246251565e-16;  // 2^-53
    const double c1 = (1.0 - a.gamma) - a.sigma_c;
    const double c2 = (1.0 + a.gamma) - a.sigma_c;
    const double inv_pixw = (double)a.npx / a.tw;
    const double inv_pixh = (double)a.npy / a.th;
    const double u = (c1 * x1 - a1 - a.tx0) * inv_pixw;
    const double v = (c2 * x2 - a2 - a.ty0) * inv_pixh;
    const double Mu = (t1 + 2.002 * 8.0 * U64 * (fabs(c1 * x1) + fabs(a1) + fabs(a.tx0))) * inv_pixw;
    const double Mv = (t2 + 2.002 * 8.0 * U64 * (fabs(c2 * x2) + fabs(a2) + fabs(a.ty0))) * inv_pixh;
    const double fu = floor(u), fv = floor(v);
    const bool ok_u = (fmin(u - fu, fu + 1.0 - u) > Mu) && (fu >= 0.0) && (fu < (double)a.npx);
    const bool ok_v = (fmin(v - fv, fv + 1.0 - v) > Mv) && (fv >= 0.0) && (fv < (double)a.npy);
    const bool out_u = (u < -Mu) || (u > (double)a.npx + Mu);
    const bool out_v = (v < -Mv) || (v > (double)a.npy + Mv);
    const bool sane = !tiny && isfinite(S) && isfinite(Mu) && isfinite(Mv);
    if (sane && ok_u && ok_v) {
        code = (int)((int64_t)fv * a.npx + (int64_t)fu);
        return true;
    }
    if (sane && (out_u || out_v)) {
        code = CODE_OUT;
        return true;
    }
    return false;
}

// The bound t of stage_a_decide. Any summation order of N terms stays within (N + 10) 2^-53 S
// of the exact sum, so 2 (N + 10) 2^-53 S covers both evaluations (any_order). Tighter, from the
// partial sums: the definition adds its terms in lens order and the k-th addition's rounding is
// at most 2^-53 |s_k| (s_k its partial sum), so its sum is within 2^-53 sum_k |s_k| of its own
// terms' exact sum, and that within 8 2^-53 S of the exact one (per-term rounding). This stage
// estimates sum_k |s_k|; the two functions below add its error and this stage's own. Constants
// are rounded up; N 2^-53 < 1e-3 for every map the library takes.
__device__ inline double any_order_bound(int64_t n_lens, double S) {
    const double U64 = 1.1102230246251565e-16;  // 2^-53
    return 2.002 * ((double)n_lens + 10.0) * U64 * 1.001 * S;
}

// This stage summing in lens order itself (one thread per ray): Q = sum_k |running sum after
// lens k|. Its own sum is within 8 2^-53 S + 2^-53 Q, its partial sums within that of the
// definition's terms' partial sums, so sum_k |s_k| <= Q (1 + N 2^-53) + 16 N 2^-53 S.
__device__ inline double sequential_bound(int64_t n_lens, double S, double Q) {
    const double U64 = 1.1102230246251565e-16;  // 2^-53
    const double N = (double)n_lens;
    const double partial = 1.001 * (16.0 * U64 * S + 2.2 * U64 * Q + 17.0 * N * U64 * U64 * S);
    return fmin(any_order_bound(n_lens, S), partial);
}

// This stage summing lenses in blocks of B in lens order (one wave per ray, the lanes' sums
// combined at every block's end): Q = sum over block starts of |partial sum|. For lens k of a
// block, |s_k| <= |s at the block's start| + the block's sum of |terms|, so sum_k |s_k| <=
// B Q + B S plus each block start's error (its sum depth e: e 2^-53 S, plus 16 2^-53 S for the
// two term evaluations); this stage's own sum is within (e + 8) 2^-53 S.
__device__ inline double block_bound(int64_t n_lens, double S, double Q, double B, double e) {
    const double U64 = 1.1102230246251565e-16;  // 2^-53
    const double N = (double)n_lens;
    const double partial = 1.001 * ((e + 32.0 + 1.05 * B) * U64 * S + 1.05 * B * U64 * Q +
                                    1.05 * (N + B) * (e + 32.0) * U64 * U64 * S);
    return fmin(any_order_bound(n_lens, S), partial);
}

// Stage A. Returns true (and the definition's code) when the ray is decided.
template <bool UNIT>
__device__ inline bool fast_ray(const RecheckArgs &a, int64_t i, int64_t j, int &code) {
    double x1, x2;
    ray_xy(a, i, j, x1, x2);
    double a1 = 0.0, a2 = 0.0, S = 0.0, Q1 = 0.0, Q2 = 0.0;
    bool tiny = false;
#pragma unroll 4
    for (int64_t k = 0; k < a.n_lens; ++k) {
        const double d1 = x1 - lens_x(a, k);
        const double d2 = x2 - lens_y(a, k);
        const double r2 = __builtin_fma(d1, d1, d2 * d2);
        tiny |= !(r2 > 1e-200);
        double rc = __builtin_amdgcn_rcp(r2);
        double e = __builtin_fma(-r2, rc, 1.0);
        rc = __builtin_fma(rc, e, rc);
        e = __builtin_fma(-r2, rc, 1.0);
        rc = __builtin_fma(rc, e, rc);
        if (!UNIT) rc = rc * lens_mass(a, k);
        a1 = __builtin_fma(d1, rc, a1);
        a2 = __builtin_fma(d2, rc, a2);
        S = __builtin_fma(fabs(d1) + fabs(d2), fabs(rc), S);
        Q1 += fabs(a1);
        Q2 += fabs(a2);
    }
    return stage_a_decide(a, x1, x2, a1, a2, S, sequential_bound(a.n_lens, S, Q1),
                          sequential_bound(a.n_lens, S, Q2), tiny, code);
}

// Stage A by a whole wave for one ray (i, j wave-uniform): lanes take every 64th lens, U of
// them per step; every L steps (blocks of B = 64 U L lenses in lens order) the lanes' running
// sums are added over the wave to give the partial sum at the block's end, whose magnitudes
// feed block_bound; the totals meet in the same butterfly. Every lane returns the same result.
template <bool UNIT>
__device__ inline bool fast_ray_wave(const RecheckArgs &a, int64_t i, int64_t j, int &code) {
    double x1, x2;
    ray_xy(a, i, j, x1, x2);
    double a1 = 0.0, a2 = 0.0, S = 0.0, Q1 = 0.0, Q2 = 0.0;
    int tiny = 0;
    // Lane l takes lenses l, l + 64, ...; U of them per step, whose positions were
    // loaded during the previous step, so the memory latency is not waited for.
    // Loads past the last lens read the last lens and their terms are dropped, so
    // the loop has no branches and the compiler can count the loads in flight.
    constexpr int U = 4, L = 4;
    constexpr double B = 64.0 * U * L;
    double LX[U], LY[U], LM[U];
    const int64_t last = a.n_lens - 1;
    auto load = [&](int64_t k0) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t k = k0 + 64 * u < a.n_lens ? k0 + 64 * u : last;
            LX[u] = lens_x(a, k);
            LY[u] = lens_y(a, k);
            LM[u] = UNIT ? 1.0 : lens_mass(a, k);
        }
    };
    auto wave_sum = [](double v) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
        return v;
    };
    const int64_t steps = (a.n_lens + 64 * U - 1) / (64 * U);   // the same for every lane
    if (a.n_lens > 0) load(__lane_id());
    for (int64_t it = 0; it < steps; ++it) {
        const int64_t k0 = __lane_id() + 64 * U * it;
        double X[U], Y[U], M[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            X[u] = LX[u];
            Y[u] = LY[u];
            M[u] = LM[u];
        }
        load(k0 + 64 * U);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const bool real = k0 + 64 * u < a.n_lens;
            const double d1 = x1 - X[u];
            const double d2 = x2 - Y[u];
            const double r2 = __builtin_fma(d1, d1, d2 * d2);
            tiny |= real && !(r2 > 1e-200);
            double rc = __builtin_amdgcn_rcp(r2);
            double e = __builtin_fma(-r2, rc, 1.0);
            rc = __builtin_fma(rc, e, rc);
            e = __builtin_fma(-r2, rc, 1.0);
            rc = __builtin_fma(rc, e, rc);
            if (!UNIT) rc = rc * M[u];
            rc = real ? rc : 0.0;
            a1 = __builtin_fma(d1, rc, a1);
            a2 = __builtin_fma(d2, rc, a2);
            S = __builtin_fma(fabs(d1) + fabs(d2), fabs(rc), S);
        }
        if (it % L == L - 1 || it == steps - 1) {   // a block's end: its partial sums
            Q1 += fabs(wave_sum(a1));
            Q2 += fabs(wave_sum(a2));
        }
    }
    a1 = wave_sum(a1);
    a2 = wave_sum(a2);
    S = wave_sum(S);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) tiny |= __shfl_xor(tiny, off);
    // a partial sum's depth: a lane's running sum plus the six butterfly levels
    const double depth = (double)steps * U + 6.0;
    return stage_a_decide(a, x1, x2, a1, a2, S, block_bound(a.n_lens, S, Q1, B, depth),
                          block_bound(a.n_lens, S, Q2, B, depth), tiny != 0, code);
}

// Bin one re-checked ray (or write its pixel) and count it in the map's counters.
__device__ inline void emit_ray(const RecheckArgs &a, int64_t i, int64_t j, int code) {
    if (a.pix_out) {
        a.pix_out[(j - a.j0) * (a.i1 - a.i0) + (i - a.i0)] = code;
    } else if (code >= 0) {
        atomicAdd(a.map + code, 1u);
    }
    atomicAdd(a.counters + (code >= 0 ? C_IN : (code == CODE_OUT ? C_OUT : C_SING)), 1ull);
}

// Full re-check of one ray by one thread: stage A, then the exact sequence.
__device__ inline int recheck_ray_thread(const RecheckArgs &a, int64_t i, int64_t j) {
    int code = 0;
    if (a.lens_m == nullptr) {
        if (!fast_ray<true>(a, i, j, code)) code = exact_ray_thread<true>(a, i, j);
    } else {
        if (!fast_ray<false>(a, i, j, code)) code = exact_ray_thread<false>(a, i, j);
    }
    return code;
}

}  // namespace rs
