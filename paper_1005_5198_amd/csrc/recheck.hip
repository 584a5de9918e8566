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
// One thread per queued ray; every lane of a wave walks the lens list in the
// same order, so lens loads are wave-uniform.
#include "rs_internal.h"

namespace rs {
namespace {

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

}  // namespace

hipError_t launch_recheck(const RecheckArgs &a, int64_t max_rays, hipStream_t stream) {
    int64_t blocks = (max_rays + 255) / 256;
    if (blocks > 2048) blocks = 2048;
    if (blocks < 1) blocks = 1;
    const bool unit = a.lens_m == nullptr;
    const bool pix = a.pix_out != nullptr;
    const dim3 grid((unsigned)blocks), block(256);
    if (unit) {
        if (pix) hipLaunchKernelGGL((recheck_kernel<true, true>), grid, block, 0, stream, a);
        else hipLaunchKernelGGL((recheck_kernel<true, false>), grid, block, 0, stream, a);
    } else {
        if (pix) hipLaunchKernelGGL((recheck_kernel<false, true>), grid, block, 0, stream, a);
        else hipLaunchKernelGGL((recheck_kernel<false, false>), grid, block, 0, stream, a);
    }
    return hipGetLastError();
}

}  // namespace rs
