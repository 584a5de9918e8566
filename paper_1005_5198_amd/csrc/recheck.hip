// FP64 re-evaluation of rays whose FP32 source position is within its error
// bound of a pixel edge.
//
// The arithmetic is the plain definition, operation for operation:
//   - ray position, Section 3.1 regular grid, cell-centred:
//       x1 = sx0 + ((double)i + 0.5) * (sw / nx)
//   - Section 2, Eq. (sigma): a1 = sum_k (m_k / r2) * d1 in lens order k = 0..N-1,
//     d1 = x1 - X_k, r2 = d1*d1 + d2*d2, sequential, no fused multiply-add
//     (the library is compiled with -ffp-contract=off), IEEE division; a ray
//     with r2 == 0 is singular;
//   - y1 = ((1 - gamma) - sigma_c) * x1 - a1, u = (y1 - tx0) / (tw / npx);
//   - pixel floor(u), floor(v) if 0 <= u < npx and 0 <= v < npy, else out.
// Because every operation is an IEEE-754 binary64 operation in the same
// order, the result of a re-checked ray is the definition's result bit for bit.
//
// Two stages keep the exact evaluation rare:
//   stage A (recheck_fast_kernel): FP64 with fused multiply-adds and a
//     Newton-refined v_rcp_f64, plus a running sum S = sum (|d1|+|d2|) m/r^2
//     that bounds the error of both this evaluation and the definition's own
//     FP64 rounding by 2 [(N + 10) 2^-53 S + 2^-50 (|c1 x1| + |a1| + |tx0|)]
//     (in source-plane units). A ray whose position is farther than that from
//     every pixel edge is decided here, identically to the definition.
//   stage B (recheck_exact_wave_kernel): the remaining rays (marked in the
//     queue) are evaluated with the definition's exact operation sequence, one
//     wave per ray: the 64 lanes compute the per-lens terms (m/r^2) d1 and
//     (m/r^2) d2 for 64 lenses at a time, and the lens-order sum then adds
//     them one by one, so every rounding step is the definition's.
// Stage A and the exact-only path run one thread per queued ray; every lane of
// a wave walks the lens list in the same order, so lens loads are wave-uniform.
#include "rs_internal.h"

namespace rs {
namespace {

constexpr uint32_t UNRESOLVED = 0x80000000u;  // queue-entry mark set by stage A

template <bool UNIT, bool PIX>
__global__ __launch_bounds__(256) void recheck_kernel(const RecheckArgs a) {
    const uint32_t n = *a.qcount;
    const int64_t W = a.i1 - a.i0;
    unsigned long long n_in = 0, n_out = 0, n_sing = 0;
    const double spx = a.sw / (double)a.nx;
    const double spy = a.sh / (double)a.ny;
    const double c1 = (1.0 - a.gamma) - a.sigma_c;
    const double c2 = (1.0 + a.gamma) - a.sigma_c;
    const double pixw = a.tw / (double)a.npx;
    const double pixh = a.th / (double)a.npy;
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t idx = blockIdx.x * blockDim.x + threadIdx.x; idx < n; idx += stride) {
        const uint32_t q = a.queue[idx];
        const int64_t i = a.i0 + (int64_t)(q % (uint64_t)W);
        const int64_t j = a.jc0 + (int64_t)(q / (uint64_t)W);
        const double x1 = a.sx0 + ((double)i + 0.5) * spx;
        const double x2 = a.sy0 + ((double)j + 0.5) * spy;
        double a1 = 0.0, a2 = 0.0;
        bool singular = false;
        for (int64_t k = 0; k < a.n_lens; ++k) {
            const double d1 = x1 - a.lens_xy[2 * k];
            const double d2 = x2 - a.lens_xy[2 * k + 1];
            const double r2 = d1 * d1 + d2 * d2;
            if (r2 == 0.0) {
                singular = true;
                break;
            }
            const double m = UNIT ? 1.0 : a.lens_m[k];
            const double f = m / r2;
            a1 += f * d1;
            a2 += f * d2;
        }
        int code;
        if (singular) {
            code = -2;
            ++n_sing;
        } else {
            const double y1 = c1 * x1 - a1;
            const double y2 = c2 * x2 - a2;
            const double u = (y1 - a.tx0) / pixw;
            const double v = (y2 - a.ty0) / pixh;
            if (isfinite(u) && isfinite(v) && u >= 0.0 && u < (double)a.npx && v >= 0.0 &&
                v < (double)a.npy) {
                code = (int)((int64_t)floor(v) * a.npx + (int64_t)floor(u));
                ++n_in;
            } else {
                code = -1;
                ++n_out;
            }
        }
        if (PIX) {
            a.pix_out[(j - a.j0) * W + (i - a.i0)] = code;
        } else if (code >= 0) {
            atomicAdd(a.map + code, 1u);
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        n_in += __shfl_xor(n_in, off);
        n_out += __shfl_xor(n_out, off);
        n_sing += __shfl_xor(n_sing, off);
    }
    if (__lane_id() == 0) {
        if (n_in) atomicAdd(a.counters + C_IN, n_in);
        if (n_out) atomicAdd(a.counters + C_OUT, n_out);
        if (n_sing) atomicAdd(a.counters + C_SING, n_sing);
    }
    if (blockIdx.x == 0 && threadIdx.x == 0 && n) atomicAdd(a.counters + C_RECHECK, (unsigned long long)n);
}

__device__ __forceinline__ double readlane_f64(double v, int l) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, l);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), l);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Stage B: rays marked UNRESOLVED by stage A, one wave per ray.
template <bool UNIT, bool PIX>
__global__ __launch_bounds__(256) void recheck_exact_wave_kernel(const RecheckArgs a) {
    const uint32_t n = *a.qcount;
    const int64_t W = a.i1 - a.i0;
    const int lane = __lane_id();
    const uint32_t wave_id = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint32_t n_waves = (gridDim.x * blockDim.x) >> 6;
    const double spx = a.sw / (double)a.nx;
    const double spy = a.sh / (double)a.ny;
    const double c1 = (1.0 - a.gamma) - a.sigma_c;
    const double c2 = (1.0 + a.gamma) - a.sigma_c;
    const double pixw = a.tw / (double)a.npx;
    const double pixh = a.th / (double)a.npy;
    unsigned long long n_in = 0, n_out = 0, n_sing = 0;
    for (uint32_t base = wave_id * 64u; base < n; base += n_waves * 64u) {
        const uint32_t idx = base + (uint32_t)lane;
        const uint32_t q_lane = idx < n ? a.queue[idx] : 0u;
        uint64_t todo = __ballot(idx < n && (q_lane & UNRESOLVED));
        while (todo) {
            const int src = __builtin_ctzll(todo);
            todo &= todo - 1;
            const uint32_t q = (uint32_t)__builtin_amdgcn_readlane((int)q_lane, src) & ~UNRESOLVED;
            const int64_t i = a.i0 + (int64_t)(q % (uint64_t)W);
            const int64_t j = a.jc0 + (int64_t)(q / (uint64_t)W);
            const double x1 = a.sx0 + ((double)i + 0.5) * spx;
            const double x2 = a.sy0 + ((double)j + 0.5) * spy;
            double a1 = 0.0, a2 = 0.0;
            bool singular = false;
            for (int64_t k0 = 0; k0 < a.n_lens; k0 += 64) {
                const int64_t k = k0 + lane;
                double t1 = 0.0, t2 = 0.0;
                bool zero = false;
                if (k < a.n_lens) {
                    const double d1 = x1 - a.lens_xy[2 * k];
                    const double d2 = x2 - a.lens_xy[2 * k + 1];
                    const double r2 = d1 * d1 + d2 * d2;
                    zero = (r2 == 0.0);
                    const double m = UNIT ? 1.0 : a.lens_m[k];
                    const double f = m / r2;
                    t1 = f * d1;
                    t2 = f * d2;
                }
                if (__ballot(zero)) {
                    singular = true;
                    break;
                }
                const int cnt = (a.n_lens - k0) < 64 ? (int)(a.n_lens - k0) : 64;
                for (int l = 0; l < cnt; ++l) {
                    a1 += readlane_f64(t1, l);
                    a2 += readlane_f64(t2, l);
                }
            }
            int code;
            if (singular) {
                code = -2;
                ++n_sing;
            } else {
                const double y1 = c1 * x1 - a1;
                const double y2 = c2 * x2 - a2;
                const double u = (y1 - a.tx0) / pixw;
                const double v = (y2 - a.ty0) / pixh;
                if (isfinite(u) && isfinite(v) && u >= 0.0 && u < (double)a.npx && v >= 0.0 &&
                    v < (double)a.npy) {
                    code = (int)((int64_t)floor(v) * a.npx + (int64_t)floor(u));
                    ++n_in;
                } else {
                    code = -1;
                    ++n_out;
                }
            }
            if (lane == 0) {
                if (PIX) a.pix_out[(j - a.j0) * W + (i - a.i0)] = code;
                else if (code >= 0) atomicAdd(a.map + code, 1u);
            }
        }
    }
    if (lane == 0) {
        if (n_in) atomicAdd(a.counters + C_IN, n_in);
        if (n_out) atomicAdd(a.counters + C_OUT, n_out);
        if (n_sing) atomicAdd(a.counters + C_SING, n_sing);
    }
}

// Stage A. Decides every queued ray whose FP64 position is provably on the
// same side of every pixel edge as the definition's; marks the others.
template <bool UNIT, bool PIX>
__global__ __launch_bounds__(256) void recheck_fast_kernel(const RecheckArgs a) {
    const uint32_t n = *a.qcount;
    const int64_t W = a.i1 - a.i0;
    unsigned long long n_in = 0, n_out = 0;
    const double spx = a.sw / (double)a.nx;
    const double spy = a.sh / (double)a.ny;
    const double c1 = (1.0 - a.gamma) - a.sigma_c;
    const double c2 = (1.0 + a.gamma) - a.sigma_c;
    const double inv_pixw = (double)a.npx / a.tw;
    const double inv_pixh = (double)a.npy / a.th;
    const double U64 = 1.1102230246251565e-16;  // 2^-53
    const double kN = ((double)a.n_lens + 10.0) * U64 * 1.001;
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t idx = blockIdx.x * blockDim.x + threadIdx.x; idx < n; idx += stride) {
        const uint32_t q = a.queue[idx];
        const int64_t i = a.i0 + (int64_t)(q % (uint64_t)W);
        const int64_t j = a.jc0 + (int64_t)(q / (uint64_t)W);
        const double x1 = a.sx0 + ((double)i + 0.5) * spx;
        const double x2 = a.sy0 + ((double)j + 0.5) * spy;
        double a1 = 0.0, a2 = 0.0, S = 0.0;
        bool tiny = false;
#pragma unroll 4
        for (int64_t k = 0; k < a.n_lens; ++k) {
            const double d1 = x1 - a.lens_xy[2 * k];
            const double d2 = x2 - a.lens_xy[2 * k + 1];
            const double r2 = __builtin_fma(d1, d1, d2 * d2);
            tiny |= !(r2 > 1e-200);
            double rc = __builtin_amdgcn_rcp(r2);
            double e = __builtin_fma(-r2, rc, 1.0);
            rc = __builtin_fma(rc, e, rc);
            e = __builtin_fma(-r2, rc, 1.0);
            rc = __builtin_fma(rc, e, rc);
            if (!UNIT) rc = rc * a.lens_m[k];
            a1 = __builtin_fma(d1, rc, a1);
            a2 = __builtin_fma(d2, rc, a2);
            S = __builtin_fma(fabs(d1) + fabs(d2), fabs(rc), S);
        }
        const double y1 = c1 * x1 - a1;
        const double y2 = c2 * x2 - a2;
        const double u = (y1 - a.tx0) * inv_pixw;
        const double v = (y2 - a.ty0) * inv_pixh;
        const double Mu = 2.002 * (kN * S + 8.0 * U64 * (fabs(c1 * x1) + fabs(a1) + fabs(a.tx0))) * inv_pixw;
        const double Mv = 2.002 * (kN * S + 8.0 * U64 * (fabs(c2 * x2) + fabs(a2) + fabs(a.ty0))) * inv_pixh;
        const double fu = floor(u), fv = floor(v);
        const bool ok_u = (fmin(u - fu, fu + 1.0 - u) > Mu) && (fu >= 0.0) && (fu < (double)a.npx);
        const bool ok_v = (fmin(v - fv, fv + 1.0 - v) > Mv) && (fv >= 0.0) && (fv < (double)a.npy);
        const bool out_u = (u < -Mu) || (u > (double)a.npx + Mu);
        const bool out_v = (v < -Mv) || (v > (double)a.npy + Mv);
        const bool sane = !tiny && isfinite(S) && isfinite(Mu) && isfinite(Mv);
        int code;
        if (sane && ok_u && ok_v) {
            code = (int)((int64_t)fv * a.npx + (int64_t)fu);
            ++n_in;
        } else if (sane && (out_u || out_v)) {
            code = -1;
            ++n_out;
        } else {
            a.queue[idx] = q | UNRESOLVED;
            continue;
        }
        if (PIX) {
            a.pix_out[(j - a.j0) * W + (i - a.i0)] = code;
        } else if (code >= 0) {
            atomicAdd(a.map + code, 1u);
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        n_in += __shfl_xor(n_in, off);
        n_out += __shfl_xor(n_out, off);
    }
    if (__lane_id() == 0) {
        if (n_in) atomicAdd(a.counters + C_IN, n_in);
        if (n_out) atomicAdd(a.counters + C_OUT, n_out);
    }
    if (blockIdx.x == 0 && threadIdx.x == 0 && n) atomicAdd(a.counters + C_RECHECK, (unsigned long long)n);
}

}  // namespace

hipError_t launch_recheck(const RecheckArgs &a, int64_t max_rays, bool exact_only, hipStream_t stream) {
    int64_t blocks = (max_rays + 255) / 256;
    if (blocks > 2048) blocks = 2048;
    if (blocks < 1) blocks = 1;
    const bool unit = a.lens_m == nullptr;
    const bool pix = a.pix_out != nullptr;
    const dim3 grid((unsigned)blocks), block(256);
#define RS_PAIR(U, P)                                                                        \
    do {                                                                                     \
        if (exact_only) {                                                                    \
            hipLaunchKernelGGL((recheck_kernel<U, P>), grid, block, 0, stream, a);           \
        } else {                                                                             \
            hipLaunchKernelGGL((recheck_fast_kernel<U, P>), grid, block, 0, stream, a);      \
            hipLaunchKernelGGL((recheck_exact_wave_kernel<U, P>), grid, block, 0, stream, a); \
        }                                                                                    \
    } while (0)
    if (unit) {
        if (pix) RS_PAIR(true, true);
        else RS_PAIR(true, false);
    } else {
        if (pix) RS_PAIR(false, true);
        else RS_PAIR(false, false);
    }
#undef RS_PAIR
    return hipGetLastError();
}

}  // namespace rs
