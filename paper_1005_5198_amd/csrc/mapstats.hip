// Map statistics of the accuracy assessment (Section 3.1, Accuracy; Eq. deltam; Eq. mu):
// per-pixel change in magnitude, the RMS of its difference between two maps,
// the two-sample Kolmogorov-Smirnov statistic of the two dm distributions and
// its probability, and the histogram of ray counts.
//
// Plan for a pair of maps (one stream, five launches):
//   zero      clear the globals and both histograms (no hipMemsetAsync, so the
//             sequence stays valid under stream capture);
//   pass      one streaming read of both maps (16-byte loads): per-block LDS
//             histograms of the counts (counts >= LDS_BINS go straight to the
//             global histogram), FP64 sums for the RMS and the means, maxima;
//             per-block partial sums are stored, not atomically added, so the
//             result does not depend on block timing;
//   scan      inclusive prefix sums of each histogram (one block per map);
//   ks        one thread per histogram bin of either map: D is the largest
//             |G_a(x) - G_b(x)| over the sample values x, G the empirical CDF
//             of mu (dm is a decreasing function of mu, so the statistic is the
//             same); the other map's CDF comes from a binary search of its bins;
//   final     one block: fixed-order sum of the partials, P(KS), the result.
// The pass is bound by HBM (8 bytes read per pixel pair); the rest touches
// only the histograms, a few KiB to MiB.
#include "rs_internal.h"
#include "rayshoot.h"

#include <cmath>

namespace rs {
int fail(int code, const char *fmt, ...);
int hip_fail(hipError_t e, const char *what);
int validate(const rs_map_params *p, int64_t n_lens);
}  // namespace rs

using namespace rs;

namespace {

constexpr int PASS_THREADS = 256;
constexpr int LDS_BINS = 4096;          // per map
constexpr int DM_TBL = 1536;            // per map: dm of counts below this, from an LDS table
constexpr int MAX_PASS_BLOCKS = 1024;
constexpr int SCAN_THREADS = 1024;
constexpr int SCAN_ITEMS = 4;
constexpr int KS_THREADS = 256;
constexpr int FINAL_THREADS = 256;
constexpr int64_t MAX_PIX = int64_t(1) << 31;

struct Partial {               // one block's sums over its pixels
    double rms_sum;
    unsigned long long n_both, sum_a, sum_b, zero_a, zero_b, pad0, pad1;
};
static_assert(sizeof(Partial) == 64, "partial record is one 64-byte line");

struct Globals {               // head of the compare workspace
    unsigned long long d_bits; // D as the bit pattern of a non-negative double (ordered like the value)
    unsigned int max_a, max_b; // largest count seen in each map
    unsigned long long overflow;
    unsigned long long pad[5];
    rs_compare_result result;
};
static_assert(sizeof(Globals) <= 256, "globals fit the 256-byte head");

constexpr size_t WS_PARTIALS = 256;
constexpr size_t WS_HIST = WS_PARTIALS + sizeof(Partial) * MAX_PASS_BLOCKS;

size_t hist_bytes(uint32_t max_count) { return align256(((size_t)max_count + 2) * sizeof(unsigned long long)); }

struct PassArgs {
    const uint32_t *map_a, *map_b;   // map_b == nullptr: histogram of map_a only
    int64_t npix;
    double nr_a, nr_b;
    uint32_t max_a, max_b;           // histogram bounds; larger counts go to bin max + 1
    unsigned long long *hist_a, *hist_b;
    Partial *partials;               // nullptr: no sums
    Globals *g;                      // nullptr: no maxima
    int vec4;                        // both maps 16-byte aligned
};

__global__ void zero_u64_kernel(unsigned long long *p, int64_t n) {
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x)
        p[k] = 0ull;
}

__global__ void zero_u32_kernel(uint32_t *p) { *p = 0u; }

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}
__device__ __forceinline__ unsigned long long wave_sum(unsigned long long v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}
__device__ __forceinline__ unsigned int wave_max(unsigned int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = max(v, (unsigned int)__shfl_xor((int)v, o));
    return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    return v;
}

// dm of one pixel, the definition's operations: mu = N / N_rays, dm = -2.5 log10(mu).
__device__ __forceinline__ double delta_m_of(uint32_t c, double n_rays) {
    const double mu = (double)c / n_rays;
    return -2.5 * log10(mu);
}

template <bool PAIR>
struct PassState {
    double rms = 0.0;
    unsigned long long n_both = 0, sum_a = 0, sum_b = 0, zero_a = 0, zero_b = 0;
    unsigned int mx_a = 0, mx_b = 0;
};

__device__ __forceinline__ void bin_count(uint32_t c, uint32_t max_c, uint32_t *lds, unsigned long long *hist) {
    if (c < (uint32_t)LDS_BINS && c <= max_c)
        atomicAdd(&lds[c], 1u);
    else
        atomicAdd(&hist[c <= max_c ? (size_t)c : (size_t)max_c + 1], 1ull);
}

template <bool PAIR>
__device__ __forceinline__ void visit(const PassArgs &a, PassState<PAIR> &s, uint32_t ca, uint32_t cb,
                                      uint32_t *lds_a, uint32_t *lds_b, const double *tbl) {
    bin_count(ca, a.max_a, lds_a, a.hist_a);
    s.mx_a = max(s.mx_a, ca);
    s.sum_a += ca;
    s.zero_a += (ca == 0u);
    if (PAIR) {
        bin_count(cb, a.max_b, lds_b, a.hist_b);
        s.mx_b = max(s.mx_b, cb);
        s.sum_b += cb;
        s.zero_b += (cb == 0u);
        if (ca != 0u && cb != 0u) {
            // the table holds delta_m_of(c, N_rays) itself, so both branches give the same value
            const double da = ca < (uint32_t)DM_TBL ? tbl[ca] : delta_m_of(ca, a.nr_a);
            const double db = cb < (uint32_t)DM_TBL ? tbl[DM_TBL + cb] : delta_m_of(cb, a.nr_b);
            const double d = da - db;
            s.rms += d * d;
            s.n_both += 1;
        }
    }
}

template <bool PAIR>
__global__ __launch_bounds__(PASS_THREADS) void pass_kernel(const PassArgs a) {
    __shared__ uint32_t lds[PAIR ? 2 * LDS_BINS : LDS_BINS];
    __shared__ double tbl[PAIR ? 2 * DM_TBL : 1];
    __shared__ double red_d[PASS_THREADS / 64];
    __shared__ unsigned long long red_u[5][PASS_THREADS / 64];
    __shared__ unsigned int red_m[2][PASS_THREADS / 64];
    uint32_t *lds_a = lds;
    uint32_t *lds_b = PAIR ? lds + LDS_BINS : lds;
    for (int k = threadIdx.x; k < (PAIR ? 2 : 1) * LDS_BINS; k += PASS_THREADS) lds[k] = 0u;
    if (PAIR)
        for (int k = threadIdx.x; k < 2 * DM_TBL; k += PASS_THREADS)
            tbl[k] = delta_m_of((uint32_t)(k % DM_TBL), k < DM_TBL ? a.nr_a : a.nr_b);
    __syncthreads();

    PassState<PAIR> s;
    const int64_t gid = blockIdx.x * (int64_t)PASS_THREADS + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * PASS_THREADS;
    int64_t tail = 0;
    if (a.vec4) {
        const int64_t n4 = a.npix / 4;
        const uint4 *va = reinterpret_cast<const uint4 *>(a.map_a);
        const uint4 *vb = reinterpret_cast<const uint4 *>(a.map_b);
        for (int64_t q = gid; q < n4; q += stride) {
            const uint4 x = va[q];
            const uint4 y = PAIR ? vb[q] : make_uint4(0u, 0u, 0u, 0u);
            visit<PAIR>(a, s, x.x, y.x, lds_a, lds_b, tbl);
            visit<PAIR>(a, s, x.y, y.y, lds_a, lds_b, tbl);
            visit<PAIR>(a, s, x.z, y.z, lds_a, lds_b, tbl);
            visit<PAIR>(a, s, x.w, y.w, lds_a, lds_b, tbl);
        }
        tail = n4 * 4;
    }
    for (int64_t p = tail + gid; p < a.npix; p += stride)
        visit<PAIR>(a, s, a.map_a[p], PAIR ? a.map_b[p] : 0u, lds_a, lds_b, tbl);

    // Block sums in a fixed order: lanes (butterfly), then waves in index order.
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const double r = wave_sum(s.rms);
    const unsigned long long u0 = wave_sum(s.n_both), u1 = wave_sum(s.sum_a), u2 = wave_sum(s.sum_b),
                             u3 = wave_sum(s.zero_a), u4 = wave_sum(s.zero_b);
    const unsigned int m0 = wave_max(s.mx_a), m1 = wave_max(s.mx_b);
    if (lane == 0) {
        red_d[wave] = r;
        red_u[0][wave] = u0;
        red_u[1][wave] = u1;
        red_u[2][wave] = u2;
        red_u[3][wave] = u3;
        red_u[4][wave] = u4;
        red_m[0][wave] = m0;
        red_m[1][wave] = m1;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        Partial pt{};
        unsigned int ma = 0, mb = 0;
        for (int w = 0; w < PASS_THREADS / 64; ++w) {
            pt.rms_sum += red_d[w];
            pt.n_both += red_u[0][w];
            pt.sum_a += red_u[1][w];
            pt.sum_b += red_u[2][w];
            pt.zero_a += red_u[3][w];
            pt.zero_b += red_u[4][w];
            ma = max(ma, red_m[0][w]);
            mb = max(mb, red_m[1][w]);
        }
        if (a.partials) a.partials[blockIdx.x] = pt;
        if (a.g) {
            atomicMax(&a.g->max_a, ma);
            if (PAIR) atomicMax(&a.g->max_b, mb);
        }
    }
    // Flush the LDS histograms: only bins that can hold counts, only non-zero ones.
    const int lim_a = (int)min((uint32_t)LDS_BINS, a.max_a + 1u);   // max < 2^32 - 1
    for (int k = threadIdx.x; k < lim_a; k += PASS_THREADS)
        if (lds_a[k]) atomicAdd(&a.hist_a[k], (unsigned long long)lds_a[k]);
    if (PAIR) {
        const int lim_b = (int)min((uint32_t)LDS_BINS, a.max_b + 1u);
        for (int k = threadIdx.x; k < lim_b; k += PASS_THREADS)
            if (lds_b[k]) atomicAdd(&a.hist_b[k], (unsigned long long)lds_b[k]);
    }
}

constexpr int SCAN_TILE = SCAN_THREADS * SCAN_ITEMS;   // histogram bins per block of the tiled scan

int64_t scan_tiles(uint32_t max_count) { return ((int64_t)max_count + 1 + SCAN_TILE - 1) / SCAN_TILE; }

// Inclusive scan of one tile h[i0 .. min(i0 + SCAN_TILE, n)) in place, plus carry;
// returns the tile's total to every thread.
__device__ unsigned long long scan_tile(unsigned long long *h, int64_t base, int64_t n, unsigned long long carry,
                                        unsigned long long *wsum) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t i0 = base + (int64_t)threadIdx.x * SCAN_ITEMS;
    unsigned long long v[SCAN_ITEMS];
    unsigned long long run = 0;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        run += (i0 + k < n) ? h[i0 + k] : 0ull;
        v[k] = run;
    }
    unsigned long long x = run;   // inclusive scan of the thread totals within the wave
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const unsigned long long y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    if (lane == 63) wsum[wave] = x;
    __syncthreads();
    if (wave == 0) {
        unsigned long long y = lane < SCAN_THREADS / 64 ? wsum[lane] : 0ull;
#pragma unroll
        for (int o = 1; o < SCAN_THREADS / 64; o <<= 1) {
            const unsigned long long z = __shfl_up(y, o);
            if (lane >= o) y += z;
        }
        if (lane < SCAN_THREADS / 64) wsum[lane] = y;
    }
    __syncthreads();
    const unsigned long long before = carry + (wave ? wsum[wave - 1] : 0ull) + (x - run);
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k)
        if (i0 + k < n) h[i0 + k] = v[k] + before;
    const unsigned long long total = wsum[SCAN_THREADS / 64 - 1];
    __syncthreads();
    return total;
}

// Tiled scan, phase 1: each block sums one tile of one histogram (blocks [0, ta)
// are map a's tiles, [ta, ta + tb) map b's) into sums[block].
__global__ __launch_bounds__(SCAN_THREADS) void tile_sum_kernel(const unsigned long long *ha, int64_t na, int64_t ta,
                                                                const unsigned long long *hb, int64_t nb,
                                                                unsigned long long *sums) {
    __shared__ unsigned long long wsum[SCAN_THREADS / 64];
    const bool side_a = (int64_t)blockIdx.x < ta;
    const unsigned long long *h = side_a ? ha : hb;
    const int64_t n = side_a ? na : nb;
    const int64_t base = (side_a ? (int64_t)blockIdx.x : (int64_t)blockIdx.x - ta) * SCAN_TILE;
    unsigned long long t = 0;
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        const int64_t i = base + (int64_t)k * SCAN_THREADS + threadIdx.x;
        if (i < n) t += h[i];
    }
    t = wave_sum(t);
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = t;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long total = 0;
        for (int w = 0; w < SCAN_THREADS / 64; ++w) total += wsum[w];
        sums[blockIdx.x] = total;
    }
}

// Tiled scan, phase 3: each tile scanned in place, offset by the inclusive scan of
// the tile sums before it (phase 2 is scan_kernel over the sums).
__global__ __launch_bounds__(SCAN_THREADS) void tile_scan_kernel(unsigned long long *ha, int64_t na, int64_t ta,
                                                                 unsigned long long *hb, int64_t nb,
                                                                 const unsigned long long *sums) {
    __shared__ unsigned long long wsum[SCAN_THREADS / 64];
    const bool side_a = (int64_t)blockIdx.x < ta;
    unsigned long long *h = side_a ? ha : hb;
    const int64_t n = side_a ? na : nb;
    const int64_t tile = side_a ? (int64_t)blockIdx.x : (int64_t)blockIdx.x - ta;
    const unsigned long long carry = tile ? sums[blockIdx.x - 1] : 0ull;
    scan_tile(h, tile * SCAN_TILE, n, carry, wsum);
}

// In-place inclusive prefix sum of h[0..n), one block per array.
__global__ __launch_bounds__(SCAN_THREADS) void scan_kernel(unsigned long long *ha, int64_t na,
                                                            unsigned long long *hb, int64_t nb) {
    unsigned long long *h = blockIdx.x ? hb : ha;
    const int64_t n = blockIdx.x ? nb : na;
    __shared__ unsigned long long wsum[SCAN_THREADS / 64];
    unsigned long long carry = 0;
    for (int64_t base = 0; base < n; base += SCAN_TILE) carry += scan_tile(h, base, n, carry, wsum);
}

struct KsArgs {
    const unsigned long long *cum_a, *cum_b;   // inclusive prefix sums of the histograms
    uint32_t max_a, max_b;
    double nr_a, nr_b;
    double npix;
    Globals *g;
};

// One thread per bin of either histogram. A bin with pixels is a sample value
// x = c / N_rays of its map; both CDFs are evaluated there, the other map's by
// the largest of its bins whose value does not exceed x.
__global__ __launch_bounds__(KS_THREADS) void ks_kernel(const KsArgs a) {
    const int64_t t = blockIdx.x * (int64_t)KS_THREADS + threadIdx.x;
    const int64_t n_a = (int64_t)a.max_a + 1, total = n_a + (int64_t)a.max_b + 1;
    double diff = 0.0;
    if (t < total) {
        const bool own_a = t < n_a;
        const unsigned long long *own = own_a ? a.cum_a : a.cum_b;
        const unsigned long long *oth = own_a ? a.cum_b : a.cum_a;
        const uint32_t c = (uint32_t)(own_a ? t : t - n_a);
        const uint32_t m_oth = own_a ? a.max_b : a.max_a;
        const double nr_own = own_a ? a.nr_a : a.nr_b, nr_oth = own_a ? a.nr_b : a.nr_a;
        const unsigned long long here = own[c], below = c ? own[c - 1] : 0ull;
        if (here != below) {
            const double x = (double)c / nr_own;
            uint32_t lo = 0, hi = m_oth;   // 0 / nr_oth <= x always holds
            while (lo < hi) {
                const uint32_t mid = lo + (uint32_t)(((uint64_t)hi - lo + 1) / 2);
                if ((double)mid / nr_oth <= x) lo = mid; else hi = mid - 1;
            }
            const double f_own = (double)here / a.npix;
            const double f_oth = (double)oth[lo] / a.npix;
            diff = fabs(f_own - f_oth);
        }
    }
    const double m = wave_max(diff);
    if ((threadIdx.x & 63) == 0 && m > 0.0)
        atomicMax(&a.g->d_bits, (unsigned long long)__double_as_longlong(m));
}

// Kolmogorov survival function Q(l) = P(K > l): the alternating series for
// l >= 1.18, else one minus the theta-transformed series of the CDF,
// sqrt(2 pi)/l sum_j exp(-(2j-1)^2 pi^2 / (8 l^2)).
__device__ double kolmogorov_q(double l) {
    if (!(l > 0.0)) return 1.0;
    const double pi = 3.14159265358979323846;
    double s = 0.0;
    if (l < 1.18) {
        for (int j = 1; j <= 7; ++j) {
            const double k = 2.0 * j - 1.0;
            s += exp(-(k * k) * (pi * pi) / (8.0 * l * l));
        }
        return 1.0 - sqrt(2.0 * pi) / l * s;
    }
    for (int j = 1; j <= 11; ++j) {
        const double t = exp(-2.0 * j * j * l * l);
        s += (j & 1) ? t : -t;
    }
    return 2.0 * s;
}

struct FinalArgs {
    const Partial *partials;
    int n_blocks;
    int64_t npix;
    double nr_a, nr_b;
    const unsigned long long *hist_a, *hist_b;   // after the scan: overflow bins are untouched
    uint32_t max_a, max_b;
    Globals *g;
};

__global__ __launch_bounds__(FINAL_THREADS) void final_kernel(const FinalArgs a) {
    __shared__ double sd[FINAL_THREADS];
    __shared__ unsigned long long su[5][FINAL_THREADS];
    double r = 0.0;
    unsigned long long u[5] = {0, 0, 0, 0, 0};
    for (int b = threadIdx.x; b < a.n_blocks; b += FINAL_THREADS) {
        const Partial &p = a.partials[b];
        r += p.rms_sum;
        u[0] += p.n_both;
        u[1] += p.sum_a;
        u[2] += p.sum_b;
        u[3] += p.zero_a;
        u[4] += p.zero_b;
    }
    sd[threadIdx.x] = r;
    for (int k = 0; k < 5; ++k) su[k][threadIdx.x] = u[k];
    __syncthreads();
    for (int h = FINAL_THREADS / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            sd[threadIdx.x] += sd[threadIdx.x + h];
            for (int k = 0; k < 5; ++k) su[k][threadIdx.x] += su[k][threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    rs_compare_result &res = a.g->result;
    const double npix = (double)a.npix;
    res.n_pix = a.npix;
    res.n_both = (int64_t)su[0][0];
    res.n_zero_a = (int64_t)su[3][0];
    res.n_zero_b = (int64_t)su[4][0];
    res.mean_mu_a = (double)su[1][0] / (npix * a.nr_a);
    res.mean_mu_b = (double)su[2][0] / (npix * a.nr_b);
    res.rms_dm = su[0][0] ? sqrt(sd[0] / (double)su[0][0]) : __longlong_as_double(0x7ff8000000000000ll);
    const double d = __longlong_as_double((long long)a.g->d_bits);
    const double ne = 0.5 * npix;                 // n_a n_b / (n_a + n_b) with n_a = n_b = npix
    const double sq = sqrt(ne);
    res.ks_d = d;
    res.ks_p = kolmogorov_q((sq + 0.12 + 0.11 / sq) * d);
    res.max_a = a.g->max_a;
    res.max_b = a.g->max_b;
    a.g->overflow = a.hist_a[(size_t)a.max_a + 1] + a.hist_b[(size_t)a.max_b + 1];
}

__global__ void max_kernel(const uint32_t *map, int64_t npix, int vec4, uint32_t *out) {
    const int64_t gid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    unsigned int m = 0;
    int64_t tail = 0;
    if (vec4) {
        const int64_t n4 = npix / 4;
        const uint4 *v = reinterpret_cast<const uint4 *>(map);
        for (int64_t q = gid; q < n4; q += stride) {
            const uint4 x = v[q];
            m = max(m, max(max(x.x, x.y), max(x.z, x.w)));
        }
        tail = n4 * 4;
    }
    for (int64_t p = tail + gid; p < npix; p += stride) m = max(m, map[p]);
    __shared__ unsigned int wmax[4];
    m = wave_max(m);
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned int b = max(max(wmax[0], wmax[1]), max(wmax[2], wmax[3]));
        if (b) atomicMax(out, b);
    }
}

__global__ void delta_m_kernel(const uint32_t *map, int64_t npix, double n_rays, double *dm) {
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < npix; p += (int64_t)gridDim.x * blockDim.x)
        dm[p] = delta_m_of(map[p], n_rays);
}

int pass_blocks(int64_t npix) {
    const int64_t b = (npix + (int64_t)PASS_THREADS * 16 - 1) / ((int64_t)PASS_THREADS * 16);
    return (int)(b < 1 ? 1 : (b > MAX_PASS_BLOCKS ? MAX_PASS_BLOCKS : b));
}

int stream_blocks(int64_t n, int threads, int cap) {
    const int64_t b = (n + threads - 1) / threads;
    return (int)(b < 1 ? 1 : (b > cap ? cap : b));
}

bool aligned(const void *p, size_t k) { return (reinterpret_cast<uintptr_t>(p) % k) == 0; }

int check_map(const uint32_t *map, int64_t npix, const char *name) {
    if (!map) return fail(RS_EINVAL, "%s is NULL", name);
    if (!aligned(map, 4)) return fail(RS_EINVAL, "%s must be 4-byte aligned", name);
    if (npix < 1 || npix >= MAX_PIX) return fail(RS_EINVAL, "npix must be in [1, 2^31), got %lld", (long long)npix);
    return RS_OK;
}

int check_n_rays(double n, const char *name) {
    if (!std::isfinite(n) || !(n > 0.0)) return fail(RS_EINVAL, "%s must be finite and > 0", name);
    return RS_OK;
}

}  // namespace

extern "C" {

double rs_rays_per_pixel(const rs_map_params *params) {
    if (validate(params, 0) != RS_OK) return NAN;
    const double density = ((double)params->nx / params->sw) * ((double)params->ny / params->sh);
    const double pixel_area = (params->tw / (double)params->npx) * (params->th / (double)params->npy);
    return density * pixel_area;
}

size_t rs_compare_workspace_bytes(uint32_t max_a, uint32_t max_b) {
    return WS_HIST + hist_bytes(max_a) + hist_bytes(max_b) +
           align256(sizeof(unsigned long long) * (size_t)(scan_tiles(max_a) + scan_tiles(max_b)));
}

int rs_map_max(const uint32_t *map, int64_t npix, uint32_t *max_dev, void *stream) {
    int rc = check_map(map, npix, "map");
    if (rc) return rc;
    if (!max_dev || !aligned(max_dev, 4)) return fail(RS_EINVAL, "max_dev must be a 4-byte aligned device pointer");
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(zero_u32_kernel, dim3(1), dim3(1), 0, s, max_dev);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "zeroing the maximum");
    hipLaunchKernelGGL(max_kernel, dim3(stream_blocks(npix, 256 * 16, 1024)), dim3(256), 0, s, map, npix,
                       aligned(map, 16) ? 1 : 0, max_dev);
    e = hipGetLastError();
    return e == hipSuccess ? RS_OK : hip_fail(e, "map maximum kernel");
}

int rs_map_histogram(const uint32_t *map, int64_t npix, uint32_t max_count, uint64_t *hist, void *stream) {
    int rc = check_map(map, npix, "map");
    if (rc) return rc;
    if (!hist || !aligned(hist, 8)) return fail(RS_EINVAL, "hist must be an 8-byte aligned device pointer");
    if (max_count == 0xffffffffu) return fail(RS_EINVAL, "max_count must be below 2^32 - 1");
    hipStream_t s = static_cast<hipStream_t>(stream);
    auto *h = reinterpret_cast<unsigned long long *>(hist);
    const int64_t n = (int64_t)max_count + 2;
    hipLaunchKernelGGL(zero_u64_kernel, dim3(stream_blocks(n, 256, 1024)), dim3(256), 0, s, h, n);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "zeroing the histogram");
    PassArgs a{};
    a.map_a = map;
    a.npix = npix;
    a.max_a = max_count;
    a.hist_a = h;
    a.vec4 = aligned(map, 16) ? 1 : 0;
    hipLaunchKernelGGL(pass_kernel<false>, dim3(pass_blocks(npix)), dim3(PASS_THREADS), 0, s, a);
    e = hipGetLastError();
    return e == hipSuccess ? RS_OK : hip_fail(e, "histogram kernel");
}

int rs_delta_m(const uint32_t *map, int64_t npix, double n_rays, double *dm, void *stream) {
    int rc = check_map(map, npix, "map");
    if (rc) return rc;
    if ((rc = check_n_rays(n_rays, "n_rays"))) return rc;
    if (!dm || !aligned(dm, 8)) return fail(RS_EINVAL, "dm must be an 8-byte aligned device pointer");
    hipLaunchKernelGGL(delta_m_kernel, dim3(stream_blocks(npix, 256 * 8, 4096)), dim3(256), 0,
                       static_cast<hipStream_t>(stream), map, npix, n_rays, dm);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? RS_OK : hip_fail(e, "dm kernel");
}

int rs_compare_maps(const uint32_t *map_a, const uint32_t *map_b, int64_t npix, double n_rays_a, double n_rays_b,
                    uint32_t max_a, uint32_t max_b, void *workspace, size_t workspace_bytes,
                    rs_compare_result *result_host, void *stream) {
    int rc = check_map(map_a, npix, "map_a");
    if (rc) return rc;
    if ((rc = check_map(map_b, npix, "map_b"))) return rc;
    if ((rc = check_n_rays(n_rays_a, "n_rays_a"))) return rc;
    if ((rc = check_n_rays(n_rays_b, "n_rays_b"))) return rc;
    if (!result_host) return fail(RS_EINVAL, "result_host is NULL");
    if (max_a == 0xffffffffu || max_b == 0xffffffffu) return fail(RS_EINVAL, "count bounds must be below 2^32 - 1");
    if (!workspace || !aligned(workspace, 256)) return fail(RS_EINVAL, "workspace must be a 256-byte aligned device pointer");
    const size_t need = rs_compare_workspace_bytes(max_a, max_b);
    if (workspace_bytes < need) return fail(RS_ENOMEM, "workspace has %zu bytes, needs %zu", workspace_bytes, need);

    char *ws = static_cast<char *>(workspace);
    auto *g = reinterpret_cast<Globals *>(ws);
    auto *partials = reinterpret_cast<Partial *>(ws + WS_PARTIALS);
    auto *hist_a = reinterpret_cast<unsigned long long *>(ws + WS_HIST);
    auto *hist_b = reinterpret_cast<unsigned long long *>(ws + WS_HIST + hist_bytes(max_a));
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e;

    // globals + partials + both histograms are one contiguous range of uint64
    const int64_t n_zero = (int64_t)(need / sizeof(unsigned long long));
    hipLaunchKernelGGL(zero_u64_kernel, dim3(stream_blocks(n_zero, 256, 1024)), dim3(256), 0, s,
                       reinterpret_cast<unsigned long long *>(ws), n_zero);
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "zeroing the compare workspace");

    PassArgs pa{};
    pa.map_a = map_a;
    pa.map_b = map_b;
    pa.npix = npix;
    pa.nr_a = n_rays_a;
    pa.nr_b = n_rays_b;
    pa.max_a = max_a;
    pa.max_b = max_b;
    pa.hist_a = hist_a;
    pa.hist_b = hist_b;
    pa.partials = partials;
    pa.g = g;
    pa.vec4 = (aligned(map_a, 16) && aligned(map_b, 16)) ? 1 : 0;
    const int blocks = pass_blocks(npix);
    hipLaunchKernelGGL(pass_kernel<true>, dim3(blocks), dim3(PASS_THREADS), 0, s, pa);
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "compare pass kernel");

    // tiled scan of both histograms: tile sums, their scan, the tiles
    auto *sums = reinterpret_cast<unsigned long long *>(ws + WS_HIST + hist_bytes(max_a) + hist_bytes(max_b));
    const int64_t ta = scan_tiles(max_a), tb = scan_tiles(max_b);
    const int64_t na = (int64_t)max_a + 1, nb = (int64_t)max_b + 1;
    hipLaunchKernelGGL(tile_sum_kernel, dim3((unsigned)(ta + tb)), dim3(SCAN_THREADS), 0, s,
                       (const unsigned long long *)hist_a, na, ta, (const unsigned long long *)hist_b, nb, sums);
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "histogram tile sums");
    hipLaunchKernelGGL(scan_kernel, dim3(2), dim3(SCAN_THREADS), 0, s, sums, ta, sums + ta, tb);
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "scan of tile sums");
    hipLaunchKernelGGL(tile_scan_kernel, dim3((unsigned)(ta + tb)), dim3(SCAN_THREADS), 0, s, hist_a, na, ta, hist_b,
                       nb, (const unsigned long long *)sums);
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "histogram tile scans");

    KsArgs ka{};
    ka.cum_a = hist_a;
    ka.cum_b = hist_b;
    ka.max_a = max_a;
    ka.max_b = max_b;
    ka.nr_a = n_rays_a;
    ka.nr_b = n_rays_b;
    ka.npix = (double)npix;
    ka.g = g;
    const int64_t cand = (int64_t)max_a + (int64_t)max_b + 2;
    hipLaunchKernelGGL(ks_kernel, dim3((unsigned)((cand + KS_THREADS - 1) / KS_THREADS)), dim3(KS_THREADS), 0, s, ka);
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "K-S kernel");

    FinalArgs fa{};
    fa.partials = partials;
    fa.n_blocks = blocks;
    fa.npix = npix;
    fa.nr_a = n_rays_a;
    fa.nr_b = n_rays_b;
    fa.hist_a = hist_a;
    fa.hist_b = hist_b;
    fa.max_a = max_a;
    fa.max_b = max_b;
    fa.g = g;
    hipLaunchKernelGGL(final_kernel, dim3(1), dim3(FINAL_THREADS), 0, s, fa);
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "compare final kernel");

    Globals host{};
    e = hipMemcpyAsync(&host, g, sizeof(Globals), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "reading the comparison");
    *result_host = host.result;
    if (host.overflow)
        return fail(RS_EINVAL, "a ray count exceeds its bound (max_a=%u max_b=%u, found %u and %u)", max_a, max_b,
                    host.result.max_a, host.result.max_b);
    return RS_OK;
}

}  // extern "C"
