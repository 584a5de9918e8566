// Far-field expansion (RS_FARFIELD): two levels of FP64 local expansions of the
// distant lenses, near lenses summed directly, a rigorous per-ray bound.
#include "far_ray.h"

namespace rs {
namespace {

// ---------------------------------------------------------------------------
// Far-field expansion (RS_FARFIELD). The paper's tree codes group distant
// lenses into pseudo-lenses with higher multipoles (Section 2, Eq.
// (hierarchical)); here distant lenses enter local expansions of the
// deflection, to order FAR_P, on two levels:
//   * super-patch (FF_SP_X x FF_SP_Y patches, centre zS, half-diagonal H):
//     lenses farther than FAR_RATIO H give C_n = sum_k m_k tS_k^(n+1),
//     tS_k = 1 / (zS - z_k); nearer lenses go to the super-patch's list;
//   * patch (64 x 32 rays, centre z0, half-diagonal h): the super expansion
//     is re-centred exactly on z0 (a polynomial translation), and the listed
//     lenses farther than FAR_RATIO h from z0 add c_n = sum_k m_k t_k^(n+1),
//     t_k = 1 / (z0 - z_k); the rest are summed directly.
// With z = x1 + i x2 and w = z - z0, sum_k m_k / (z - z_k) = sum_n (-w)^n T_n,
// and the deflection (a1, a2) is (Re, -Im) of that sum. All of it is FP64; each
// ray carries a rigorous bound (series truncation on both levels, rounding of
// the coefficients, the translation and the evaluation, the near sum) plus the
// definition's own rounding, and rays within it of a pixel edge go to the FP64
// re-check, so the map equals the definition's.
// ---------------------------------------------------------------------------
constexpr int FAR_THREADS = 256;
constexpr int FAR_ROWS = PATCH_X * PATCH_Y / FAR_THREADS;     // rays per thread (8)
static_assert(FAR_ROWS * (FAR_THREADS / 64) == (PATCH_X / 8) * (PATCH_Y / 8), "8 x 8 blocks cover the patch");
constexpr int NEAR_EXP = 512;

// binom(n, m) for n, m < FAR_P (Pascal's triangle; integers below 2^13, exact in FP64).
struct BinomTable {
    double v[FAR_P][FAR_P];
    constexpr BinomTable() : v() {
        for (int n = 0; n < FAR_P; ++n) {
            v[n][0] = 1.0;
            for (int m = 1; m <= n; ++m) v[n][m] = v[n - 1][m - 1] + (m < n ? v[n - 1][m] : 0.0);
        }
    }
};
__constant__ constexpr BinomTable BINOM_TABLE{};
#define BINOM BINOM_TABLE.v
// One lens's contribution to an expansion about (ox, oy) with half-diagonal h
// (the lens is at least FAR_RATIO h away): the powers m t^(n+1) and the bound
// terms m/|d|, m/|d| rho^P / (1 - rho) and sqrt(2) m / (|d| - h).
struct FarAcc {
    double c1[FAR_P], c2[FAR_P];
    double sfar, trunc, sdef, nfar;
    __device__ void zero() {
#pragma unroll
        for (int n = 0; n < FAR_P; ++n) {
            c1[n] = 0.0;
            c2[n] = 0.0;
        }
        sfar = trunc = sdef = nfar = 0.0;
    }
    __device__ __forceinline__ void add(double d1, double d2, double r2, double m, double h) {
        const double inv = rcp64(r2);
        const double t1 = d1 * inv, t2 = -d2 * inv;   // t = 1 / d, d = centre - lens
        double p1 = m * t1, p2 = m * t2;
        c1[0] += p1;
        c2[0] += p2;
#pragma unroll
        for (int n = 1; n < FAR_P; ++n) {
            const double q1 = __builtin_fma(p1, t1, -p2 * t2);
            const double q2 = __builtin_fma(p1, t2, p2 * t1);
            p1 = q1;
            p2 = q2;
            c1[n] += p1;
            c2[n] += p2;
        }
        // Bound terms from 1/|d| and 1/(1 - rho) (Newton-refined, within a few units of
        // 2^-53 relative; the decision's final factor 1.001 covers that): |m|/(|d| - h)
        // is |m|/|d| / (1 - rho).
        const double inv_ad = rsq64(r2);
        const double s = fabs(m) * inv_ad;
        const double rho = h * inv_ad;
        const double rho2 = rho * rho, rho4 = rho2 * rho2, rho8 = rho4 * rho4, rho16 = rho8 * rho8;
        const double g = rcp64(1.0 - rho);
        sfar += s;
        trunc += s * rho16 * g;
        sdef += 1.4142135623730951 * s * g;
        nfar += 1.0;
    }
    // Sum over the wave's lanes (butterfly): every lane ends with the totals.
    __device__ void butterfly() {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
            for (int n = 0; n < FAR_P; ++n) {
                c1[n] += __shfl_xor(c1[n], off);
                c2[n] += __shfl_xor(c2[n], off);
            }
            sfar += __shfl_xor(sfar, off);
            trunc += __shfl_xor(trunc, off);
            sdef += __shfl_xor(sdef, off);
            nfar += __shfl_xor(nfar, off);
        }
    }
    // Block sum into out[FAR_REC] (shared); lanes by butterfly, then waves in index order.
    template <int THREADS = FAR_THREADS>
    __device__ void reduce(double (*part)[FAR_REC], double *out) {
        const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
        butterfly();
        if (lane == 0) {
#pragma unroll
            for (int n = 0; n < FAR_P; ++n) {
                part[wave][n] = c1[n];
                part[wave][FAR_P + n] = c2[n];
            }
            part[wave][2 * FAR_P] = sfar;
            part[wave][2 * FAR_P + 1] = trunc;
            part[wave][2 * FAR_P + 2] = sdef;
            part[wave][2 * FAR_P + 3] = nfar;
        }
        __syncthreads();
        if (threadIdx.x < FAR_REC) {
            double v = 0.0;
            for (int w = 0; w < THREADS / 64; ++w) v += part[w][threadIdx.x];
            out[threadIdx.x] = v;
        }
        __syncthreads();
    }
};

// Shared memory of a level builder with THREADS threads.
template <int THREADS = FAR_THREADS>
struct FarLevelSmem {
    double part[THREADS / 64][FAR_REC];
    double out[FAR_REC];
    int count;
};
using FarSuperSmem = FarLevelSmem<FAR_THREADS>;
// Groups hold 2^19 rays and there are few of them: two blocks' worth of threads each.
constexpr int FAR_GROUP_THREADS = 2 * FAR_THREADS;

// Record of one level about (cx, cy) with half-diagonal H: of the candidates
// (cand(q, k, X, Y) gives candidate q's lens, or false when q is none), those
// farther than FAR_RATIO H add to the expansion C_n = sum m t^(n+1) and to the
// bound sums; the others go to list (count in list[0]; a count above cap means
// the list is incomplete and the level below scans every lens instead). With a
// parent record about (pcx, pcy) (a level above, whose own candidates these
// are; held as n_parts records to be added in order), the parent's expansion is
// re-centred exactly on (cx, cy),
//   E_m = sum_{n>=m} binom(n, m) e^(n-m) C_n, e = z_parent - z,
// and added, and its bound sums are added to this level's. The sums stay valid
// bounds below: their rounding constants allow for several translations.
template <bool UNIT, int THREADS = FAR_THREADS, class Cand>
__device__ __forceinline__ void build_level(const ShootArgs &a, double cx, double cy, double H, int64_t n_cand, Cand cand,
                                   int32_t *list, int cap, double *rec, const double *parent, int n_parts,
                                   double pcx, double pcy, FarLevelSmem<THREADS> &sm) {
    const double near_r2 = (FAR_RATIO * H) * (FAR_RATIO * H);
    if (threadIdx.x == 0) sm.count = 0;
    __syncthreads();
    FarAcc acc;
    acc.zero();
    // The next candidate's lens is loaded before this one is expanded, so its
    // memory latency overlaps the expansion.
    int64_t kn = 0;
    double Xn = 0.0, Yn = 0.0;
    bool vn = (int64_t)threadIdx.x < n_cand && cand(threadIdx.x, kn, Xn, Yn);
#pragma unroll 1
    for (int64_t q = threadIdx.x; q < n_cand; q += THREADS) {
        const int64_t k = kn;
        const double X = Xn, Y = Yn;
        const bool v = vn;
        vn = q + THREADS < n_cand && cand(q + THREADS, kn, Xn, Yn);
        if (!v) continue;
        const double d1 = cx - X, d2 = cy - Y;
        const double r2 = d1 * d1 + d2 * d2;
        if (!(r2 >= near_r2)) {
            const int j = atomicAdd(&sm.count, 1);
            if (j < cap) list[1 + j] = (int32_t)k;
            continue;
        }
        const double m = (UNIT || a.lens_m == nullptr) ? 1.0 : ((global_double *)a.lens_m)[k];
        acc.add(d1, d2, r2, m, H);
    }
    acc.template reduce<THREADS>(sm.part, sm.out);
    const int t = threadIdx.x;
    if (parent == nullptr) {
        if (t < FAR_REC) rec[t] = sm.out[t];
    } else {
        const global_double *Pp = (const global_double *)parent;
        auto P = [&](int n) {
            double v = Pp[n];
            for (int part = 1; part < n_parts; ++part) v += Pp[part * FAR_REC + n];
            return v;
        };
        if (t < FAR_P) {
            const double e1 = pcx - cx, e2 = pcy - cy;
            double s1 = 0.0, s2 = 0.0;
            double g1 = 1.0, g2 = 0.0;   // e^(n-m)
            for (int n = t; n < FAR_P; ++n) {
                const double binom = BINOM[n][t];   // exact in FP64 for n < 16
                const double C1 = P(n), C2 = P(FAR_P + n);
                s1 = __builtin_fma(binom, g1 * C1 - g2 * C2, s1);
                s2 = __builtin_fma(binom, g1 * C2 + g2 * C1, s2);
                const double q1 = g1 * e1 - g2 * e2, q2 = g1 * e2 + g2 * e1;
                g1 = q1;
                g2 = q2;
            }
            rec[t] = s1 + sm.out[t];
            rec[FAR_P + t] = s2 + sm.out[FAR_P + t];
        } else if (t < FAR_P + FAR_EXTRA) {
            rec[2 * FAR_P + (t - FAR_P)] = P(2 * FAR_P + (t - FAR_P)) + sm.out[2 * FAR_P + (t - FAR_P)];
        }
    }
    if (t == 0) list[0] = sm.count;
}

// Every lens from index first on is a candidate.
struct AllLenses {
    const double *xy;
    int64_t first;
    __device__ bool operator()(int64_t q, int64_t &k, double &X, double &Y) const {
        k = first + q;
        X = ((global_double *)xy)[2 * k];
        Y = ((global_double *)xy)[2 * k + 1];
        return true;
    }
};

// Records of super-patch sp from every lens (the mixed mode's re-check stage,
// random rays and batches): far lenses -> coefficients about zS; the others ->
// the super-patch's lens list.
template <bool UNIT>
__device__ __forceinline__ void build_super(const ShootArgs &a, int64_t sp, FarSuperSmem &sm) {
    double cx, cy, H;
    super_geometry(a, sp, cx, cy, H);
    build_level<UNIT>(a, cx, cy, H, a.n_lens, AllLenses{a.lens_xy, 0}, a.ff_near + sp * (int64_t)(1 + a.ff_cap), a.ff_cap,
                      a.ff_super + sp * (int64_t)FAR_REC, nullptr, 0, 0.0, 0.0, sm);
}

// Level 1 of one launch (or, for random rays, of the whole rectangle): one block
// per super-patch. RECHECK: the grid re-check stage needs the records only when
// the deflection launch queued rays.
template <bool UNIT, bool RECHECK>
__global__ __launch_bounds__(FAR_THREADS) void farfield_super_kernel(const ShootArgs a) {
    __shared__ FarSuperSmem sm;
    if (RECHECK && *a.qcount == 0) return;
    build_super<UNIT>(a, blockIdx.x, sm);
}

// Blocks that scan one group's lenses: one per 8192 lenses, at most FF_GROUP_PARTS.
__host__ __device__ inline int group_parts(int64_t n_lens) {
    return n_lens / 8192 + 1 < FF_GROUP_PARTS ? (int)(n_lens / 8192 + 1) : FF_GROUP_PARTS;
}

// Far-field mode, level 0: groups of FF_GROUP x FF_GROUP super-patches (centre
// zG, half-diagonal HG, one ray spacing of slack on each side, of the full box).
__device__ __forceinline__ void group_geometry(const ShootArgs &a, int64_t g, double &cx, double &cy, double &H) {
    constexpr int GX = FF_GROUP * FF_SP_X * PATCH_X, GY = FF_GROUP * FF_SP_Y * PATCH_Y;
    const int64_t gx = g % a.ff_gbx, gy = g / a.ff_gbx;
    const int64_t i_g = a.ff_i0 + gx * GX;
    const int64_t j_g = a.ff_j0 + gy * GY;
    cx = a.sx0 + ((double)i_g + 0.5 * GX) * a.spx;
    cy = a.sy0 + ((double)j_g + 0.5 * GY) * a.spy;
    const double hx = (0.5 * GX + 1.0) * a.spx;
    const double hy = (0.5 * GY + 1.0) * a.spy;
    H = sqrt(hx * hx + hy * hy) * (1.0 + 1e-12);
}

__device__ __forceinline__ int64_t group_of(const ShootArgs &a, int64_t sp) {
    return ((sp / a.ff_sbx) / FF_GROUP) * a.ff_gbx + (sp % a.ff_sbx) / FF_GROUP;
}

// Far-field mode with tops: top t of FF_TOP x FF_TOP groups, the same construction one
// level up (its box holds its groups' boxes).
__device__ __forceinline__ void top_geometry(const ShootArgs &a, int64_t t, double &cx, double &cy, double &H) {
    constexpr int TX = FF_TOP * FF_GROUP * FF_SP_X * PATCH_X, TY = FF_TOP * FF_GROUP * FF_SP_Y * PATCH_Y;
    const int64_t tx = t % a.ff_tbx, ty = t / a.ff_tbx;
    const int64_t i_t = a.ff_i0 + tx * TX;
    const int64_t j_t = a.ff_j0 + ty * TY;
    cx = a.sx0 + ((double)i_t + 0.5 * TX) * a.spx;
    cy = a.sy0 + ((double)j_t + 0.5 * TY) * a.spy;
    const double hx = (0.5 * TX + 1.0) * a.spx;
    const double hy = (0.5 * TY + 1.0) * a.spy;
    H = sqrt(hx * hx + hy * hy) * (1.0 + 1e-12);
}

__device__ __forceinline__ int64_t top_of(const ShootArgs &a, int64_t g) {
    return ((g / a.ff_gbx) / FF_TOP) * a.ff_tbx + (g % a.ff_gbx) / FF_TOP;
}

// A level's candidates: the lists of the level above (one per part, in part order), or,
// when one of them overflowed, every lens that level did not expand (the same test it
// made).
template <int P>
struct ListCandidates {
    const double *xy;
    const global_i32 *lists;   // the parts' lists, stride apart
    int64_t stride;
    int64_t e[P - 1];          // candidates before the end of parts 0 .. P - 2 (non-decreasing)
    bool scan_all;
    double cx, cy, r2;
    __device__ bool operator()(int64_t q, int64_t &k, double &X, double &Y) const {
        if (scan_all) {
            k = q;
        } else {
            // q's part is the number of part ends at or below q; its offset counts from the
            // last of them (unrolled, so e stays in registers)
            int64_t part = 0, before = 0;
#pragma unroll
            for (int i = 0; i < P - 1; ++i) {
                const bool past = q >= e[i];
                part += past;
                before = past ? e[i] : before;
            }
            k = (int64_t)lists[part * stride + 1 + (q - before)];
        }
        X = ((global_double *)xy)[2 * k];
        Y = ((global_double *)xy)[2 * k + 1];
        if (scan_all) {
            const double f1 = cx - X, f2 = cy - Y;
            if (f1 * f1 + f2 * f2 >= r2) return false;
        }
        return true;
    }
};

// Candidates from `used` lists of capacity cap, stride apart, of the level about (cx, cy)
// with half-diagonal H.
template <int P>
__device__ __forceinline__ ListCandidates<P> list_candidates(const ShootArgs &a, const int32_t *lists, int64_t stride,
                                                             int32_t cap, int used, double cx, double cy, double H,
                                                             int64_t &n) {
    ListCandidates<P> c;
    c.xy = a.lens_xy;
    c.cx = cx;
    c.cy = cy;
    c.r2 = (FAR_RATIO * H) * (FAR_RATIO * H);
    c.lists = (const global_i32 *)lists;
    c.stride = stride;
    c.scan_all = false;
    int64_t total = 0;
#pragma unroll
    for (int p = 0; p < P; ++p) {
        const int32_t np = p < used ? c.lists[p * stride] : 0;   // the lists past `used` were not written
        c.scan_all = c.scan_all || np > cap;
        total += np;
        if (p < P - 1) c.e[p] = total;
    }
    n = c.scan_all ? a.n_lens : total;
    return c;
}

// A super-patch's candidates: its group's lists (one per part), or with tops the
// group's one list.
__device__ __forceinline__ ListCandidates<FF_GROUP_PARTS> group_candidates(const ShootArgs &a, int64_t g, int64_t &n) {
    double cx, cy, H;
    group_geometry(a, g, cx, cy, H);
    const int32_t *lists = a.ff_glist + g * FF_GROUP_PARTS * (int64_t)(1 + FF_PART_CAP);
    if (a.ff_top) return list_candidates<FF_GROUP_PARTS>(a, lists, 0, FF_GROUP_ONE_CAP, 1, cx, cy, H, n);
    return list_candidates<FF_GROUP_PARTS>(a, lists, 1 + FF_PART_CAP, FF_PART_CAP, group_parts(a.n_lens), cx, cy,
                                           H, n);
}

// Far-field mode, level 0: group_parts(N) blocks per group, each over its range of
// lens indices.
template <bool UNIT>
__global__ __launch_bounds__(FAR_GROUP_THREADS) __attribute__((amdgpu_waves_per_eu(4))) void farfield_group_kernel(const ShootArgs a) {
    __shared__ FarLevelSmem<FAR_GROUP_THREADS> sm;
    const int used = group_parts(a.n_lens);
    const int64_t g = blockIdx.x / used;
    const int part = (int)(blockIdx.x % used);
    const int64_t first = a.n_lens * part / used;
    const int64_t last = a.n_lens * (part + 1) / used;
    double cx, cy, H;
    group_geometry(a, g, cx, cy, H);
    const int64_t slot = g * FF_GROUP_PARTS + part;
    build_level<UNIT, FAR_GROUP_THREADS>(a, cx, cy, H, last - first, AllLenses{a.lens_xy, first},
                                         a.ff_glist + slot * (int64_t)(1 + FF_PART_CAP), FF_PART_CAP,
                                         a.ff_group + slot * (int64_t)FAR_REC, nullptr, 0, 0.0, 0.0, sm);
}

// Far-field mode with tops, level 0: FF_TOP_PARTS blocks per top, each over its range of
// lens indices (the group kernel's scan one level up). A launch has few tops (a band of
// 2^27 rays holds about 30), so the blocks are as large as they can be.
constexpr int FAR_TOP_THREADS = 1024;
template <bool UNIT>
__global__ __launch_bounds__(FAR_TOP_THREADS) __attribute__((amdgpu_waves_per_eu(4))) void farfield_top_kernel(const ShootArgs a) {
    __shared__ FarLevelSmem<FAR_TOP_THREADS> sm;
    const int64_t t = blockIdx.x / FF_TOP_PARTS;
    const int part = (int)(blockIdx.x % FF_TOP_PARTS);
    const int64_t first = a.n_lens * part / FF_TOP_PARTS;
    const int64_t last = a.n_lens * (part + 1) / FF_TOP_PARTS;
    double cx, cy, H;
    top_geometry(a, t, cx, cy, H);
    const int64_t slot = t * FF_TOP_PARTS + part;
    build_level<UNIT, FAR_TOP_THREADS>(a, cx, cy, H, last - first, AllLenses{a.lens_xy, first},
                                         a.ff_tlist + slot * (int64_t)(1 + FF_TOP_PART_CAP), FF_TOP_PART_CAP,
                                         a.ff_top + slot * (int64_t)FAR_REC, nullptr, 0, 0.0, 0.0, sm);
}

// Far-field mode with tops, level 1: one block per group, candidates from its top's
// lists, the top's expansion re-centred and added; one record (part 0) and one list.
template <bool UNIT>
__global__ __launch_bounds__(FAR_GROUP_THREADS) __attribute__((amdgpu_waves_per_eu(4))) void farfield_group_top_kernel(const ShootArgs a) {
    __shared__ FarLevelSmem<FAR_GROUP_THREADS> sm;
    const int64_t g = blockIdx.x;
    const int64_t t = top_of(a, g);
    double tcx, tcy, tH;
    top_geometry(a, t, tcx, tcy, tH);
    int64_t n;
    const ListCandidates<FF_TOP_PARTS> c =
        list_candidates<FF_TOP_PARTS>(a, a.ff_tlist + t * FF_TOP_PARTS * (int64_t)(1 + FF_TOP_PART_CAP),
                                      1 + FF_TOP_PART_CAP, FF_TOP_PART_CAP, FF_TOP_PARTS, tcx, tcy, tH, n);
    double cx, cy, H;
    group_geometry(a, g, cx, cy, H);
    build_level<UNIT, FAR_GROUP_THREADS>(a, cx, cy, H, n, c, a.ff_glist + g * FF_GROUP_PARTS * (int64_t)(1 + FF_PART_CAP),
                                         FF_GROUP_ONE_CAP, a.ff_group + g * FF_GROUP_PARTS * (int64_t)FAR_REC,
                                         a.ff_top + t * FF_TOP_PARTS * (int64_t)FAR_REC, FF_TOP_PARTS, tcx, tcy, sm);
}

// Far-field mode, level 1: one block per super-patch, candidates from its group,
// the group's expansion re-centred and added.
template <bool UNIT>
__global__ __launch_bounds__(FAR_THREADS) void farfield_super_group_kernel(const ShootArgs a) {
    __shared__ FarSuperSmem sm;
    const int64_t sp = blockIdx.x;
    const int64_t g = group_of(a, sp);
    int64_t n;
    const ListCandidates<FF_GROUP_PARTS> c = group_candidates(a, g, n);
    double cx, cy, H;
    super_geometry(a, sp, cx, cy, H);
    build_level<UNIT>(a, cx, cy, H, n, c, a.ff_near + sp * (int64_t)(1 + a.ff_cap), a.ff_cap,
                      a.ff_super + sp * (int64_t)FAR_REC, a.ff_group + g * FF_GROUP_PARTS * (int64_t)FAR_REC,
                      a.ff_top ? 1 : group_parts(a.n_lens), c.cx, c.cy, sm);
}

// Level 1 of every map of a mixed batch that flagged rays: one block per
// (map, super-patch), maps found by binary search on their first record.
template <bool UNIT>
__global__ __launch_bounds__(FAR_THREADS) void batch_super_kernel(const BatchArgs b) {
    __shared__ FarSuperSmem sm;
    const int64_t t = blockIdx.x;
    int lo = 0, hi = b.n_maps - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (b.maps[mid].super_begin <= t) lo = mid;
        else hi = mid - 1;
    }
    const BatchMap &m = b.maps[lo];
    if (t - m.super_begin >= m.n_super || m.counters[C_RECHECK] == 0ull) return;
    const ShootArgs a = make_uniform(batch_far_args(m));
    build_super<UNIT>(a, t - m.super_begin, sm);
}

// One patch of a far-field launch: first ray (ib, jb), centre (ox, oy), half-
// diagonal h (one ray spacing of slack on each side), the radius inside which
// lenses are summed directly, and the super-patch that holds it. Window widths
// stay below 2^22 rays and launches below 2^31 patches, so 32-bit indices hold.
struct PatchFrame {
    int64_t ib, jb, sp;
    double ox, oy, h, near_r2;
};

__device__ __forceinline__ PatchFrame patch_frame(const ShootArgs &a, int64_t patch) {
    PatchFrame f;
    const int32_t nbx = (int32_t)a.nbx, p = (int32_t)patch;
    const int32_t pbx = p % nbx, pby = p / nbx;
    f.ib = a.i0 + (int64_t)pbx * PATCH_X;
    f.jb = a.jc0 + (int64_t)pby * PATCH_Y;
    f.sp = (int64_t)(pby / FF_SP_Y) * a.ff_sbx + pbx / FF_SP_X;
    f.ox = a.sx0 + ((double)f.ib + 0.5 * PATCH_X) * a.spx;
    f.oy = a.sy0 + ((double)f.jb + 0.5 * PATCH_Y) * a.spy;
    const double hx = (0.5 * PATCH_X + 1.0) * a.spx;
    const double hy = (0.5 * PATCH_Y + 1.0) * a.spy;
    f.h = sqrt(hx * hx + hy * hy) * (1.0 + 1e-12);
    f.near_r2 = (FAR_RATIO * f.h) * (FAR_RATIO * f.h);
    return f;
}

// The candidates of a patch: the super-patch's list, or, when that list
// overflowed, every lens that neither its group nor the super-patch expanded
// (the same tests those levels made).
struct Candidates {
    const global_i32 *list;
    int64_t n;
    bool scan_all;
    double cx, cy, super_r2;
    double gx, gy, group_r2;
};

__device__ __forceinline__ Candidates candidates(const ShootArgs &a, int64_t sp) {
    Candidates c;
    double H;
    super_geometry(a, sp, c.cx, c.cy, H);
    c.super_r2 = (FAR_RATIO * H) * (FAR_RATIO * H);
    c.list = (const global_i32 *)(a.ff_near + sp * (int64_t)(1 + a.ff_cap));
    const int32_t listed = c.list[0];
    c.scan_all = listed > a.ff_cap;
    c.n = c.scan_all ? a.n_lens : listed;
    group_geometry(a, group_of(a, sp), c.gx, c.gy, H);
    c.group_r2 = (FAR_RATIO * H) * (FAR_RATIO * H);
    return c;
}

// Candidate q: its lens index and position; false when an overflowed list's
// scan meets a lens a level above expanded.
__device__ __forceinline__ bool candidate(const ShootArgs &a, const Candidates &c, int64_t q, int64_t &k, double &X,
                                          double &Y) {
    k = c.scan_all ? q : (int64_t)c.list[1 + q];
    X = ((global_double *)a.lens_xy)[2 * k];
    Y = ((global_double *)a.lens_xy)[2 * k + 1];
    if (c.scan_all) {
        const double f1 = c.gx - X, f2 = c.gy - Y;
        if (f1 * f1 + f2 * f2 >= c.group_r2) return false;
        const double e1 = c.cx - X, e2 = c.cy - Y;
        if (e1 * e1 + e2 * e2 >= c.super_r2) return false;
    }
    return true;
}

// Level 2, part 1: the record of each patch, one wave per patch. The candidates
// farther than FAR_RATIO h from the patch centre add their own expansion about
// it; the super-patch expansion is re-centred exactly on it,
//   sum_n C_n (e + v)^n = sum_m v^m sum_{n>=m} binom(n, m) e^(n-m) C_n,
// v = -w = z0 - z, e = zS - z0; the record holds the sum of both, the bound terms
// of both levels (truncation, and rounding of the coefficients, the translation
// and the evaluation, with per-level factors and generous constants), and the
// nearer candidates, in candidate order, for the ray kernel's direct sum. Block 0
// also resets the ray kernel's patch counter.
template <bool UNIT>
__global__ __launch_bounds__(FAR_THREADS) void farfield_patch_kernel(const ShootArgs a, int64_t patches) {
    constexpr double U64 = 1.1102230246251565e-16;  // 2^-53
    if (blockIdx.x == 0 && threadIdx.x == 0) *a.ff_work = 0u;
    const int lane = threadIdx.x & 63;
    const int64_t patch = (int64_t)blockIdx.x * (FAR_THREADS / 64) + (threadIdx.x >> 6);
    if (patch >= patches) return;   // the whole wave
    const PatchFrame f = patch_frame(a, patch);
    const Candidates c = candidates(a, f.sp);
    double *rec = a.ff_patch + patch * (int64_t)FF_PATCH_DOUBLES;
    FarAcc acc;
    acc.zero();
    int n_near = 0;
    for (int64_t q0 = 0; q0 < c.n; q0 += 64) {
        const int64_t q = q0 + lane;
        int64_t k = 0;
        double X = 0.0, Y = 0.0, m = 1.0, d1 = 0.0, d2 = 0.0, r2 = 0.0;
        bool is_far = false, is_near = false;
        if (q < c.n && candidate(a, c, q, k, X, Y)) {
            d1 = f.ox - X;
            d2 = f.oy - Y;
            r2 = d1 * d1 + d2 * d2;
            m = (UNIT || a.lens_m == nullptr) ? 1.0 : ((global_double *)a.lens_m)[k];
            is_far = r2 >= f.near_r2;
            is_near = !is_far;
        }
        if (is_far) acc.add(d1, d2, r2, m, f.h);
        const uint64_t nb = __ballot(is_near);
        if (is_near) {
            const int pos = n_near + __builtin_popcountll(nb & ((1ull << lane) - 1ull));
            if (pos < FF_PATCH_NEAR) {
                rec[FF_PATCH_HEAD + pos] = X;
                rec[FF_PATCH_HEAD + FF_PATCH_NEAR + pos] = Y;
                rec[FF_PATCH_HEAD + 2 * FF_PATCH_NEAR + pos] = m;
            }
        }
        n_near += __builtin_popcountll(nb);
    }
    acc.butterfly();   // every lane now holds the wave's sums
    const global_double *sc = (const global_double *)(a.ff_super + f.sp * (int64_t)FAR_REC);
    if (lane < FAR_P) {
        const int mm = lane;
        double p1 = 0.0, p2 = 0.0;
#pragma unroll
        for (int n = 0; n < FAR_P; ++n) {
            if (n == mm) {
                p1 = acc.c1[n];
                p2 = acc.c2[n];
            }
        }
        const double e1 = c.cx - f.ox, e2 = c.cy - f.oy;
        double s1 = 0.0, s2 = 0.0;
        double g1 = 1.0, g2 = 0.0;   // e^(n-m)
        for (int n = mm; n < FAR_P; ++n) {
            const double binom = BINOM[n][mm];   // exact in FP64 for n < 16
            const double C1 = sc[n], C2 = sc[FAR_P + n];
            s1 = __builtin_fma(binom, g1 * C1 - g2 * C2, s1);
            s2 = __builtin_fma(binom, g1 * C2 + g2 * C1, s2);
            const double q1 = g1 * e1 - g2 * e2, q2 = g1 * e2 + g2 * e1;
            g1 = q1;
            g2 = q2;
        }
        rec[mm] = s1 + p1;
        rec[FAR_P + mm] = s2 + p2;
    } else if (lane == FAR_P) {
        const double SFAR_S = sc[2 * FAR_P], TRUNC_S = sc[2 * FAR_P + 1], SDEF_S = sc[2 * FAR_P + 2];
        const double NFAR_S = sc[2 * FAR_P + 3];
        rec[2 * FAR_P] = SFAR_S + acc.sfar;
        rec[2 * FAR_P + 1] = TRUNC_S + acc.trunc + (NFAR_S + 24.0 * FAR_P + 64.0) * U64 * 1.34 * SFAR_S +
                             (acc.nfar + 16.0 * FAR_P + 64.0) * U64 * 1.34 * acc.sfar;
        rec[2 * FAR_P + 2] = SDEF_S + acc.sdef;
        rec[2 * FAR_P + 3] = (double)n_near;
    } else if (lane <= FAR_P + FF_PATCH_HEAD - (2 * FAR_P + 4)) {
        rec[2 * FAR_P + 4 + (lane - FAR_P - 1)] = 0.0;   // the spare doubles
    }
}

struct FarSmem {
    PixelTable table;            // the patch's counts per pixel (map mode)
    double near_x[NEAR_EXP], near_y[NEAR_EXP], near_m[NEAR_EXP];
    double rec[FF_PATCH_HEAD];
    int near_count[2];           // by patch parity: one is filled while the other is cleared
    int next;                    // the patch after this one
};

// Level 2, part 2: the rays. Persistent blocks take patches from a counter. A
// patch's near lenses come from its record, or, when the record could not hold
// them all, from the candidates with the record kernel's test (beyond NEAR_EXP
// of them the patch is re-checked whole). Each thread then takes 8 rays: the
// series (Horner in v), the near lenses directly, the pixel decision against the
// bound, and the count in the block's pixel table, which is added to the map
// (one global atomic per distinct pixel) and cleared after every patch.
template <bool UNIT, bool PIX>
__global__ __launch_bounds__(FAR_THREADS, 3) void farfield_kernel(const ShootArgs a, int64_t patches) {
    __shared__ FarSmem sm;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    if (!PIX) table_clear<FAR_THREADS>(sm.table, tid);
    if (tid == 0) {
        sm.near_count[0] = 0;
        sm.near_count[1] = 0;
        sm.next = (int)atomicAdd(a.ff_work, 1u);
    }
    __syncthreads();
    int64_t patch = sm.next;
    unsigned long long n_in = 0, n_out = 0;
    const int64_t W = a.i1 - a.i0;
    for (int par = 0; patch < patches; par ^= 1) {
        uint32_t next = 0;
        if (tid == 0) next = atomicAdd(a.ff_work, 1u);   // used after the rays: its latency is hidden
        const PatchFrame f = patch_frame(a, patch);
        const int64_t ib = f.ib, jb = f.jb;
        const double ox = f.ox, oy = f.oy;
        const global_double *R = (const global_double *)(a.ff_patch + patch * (int64_t)FF_PATCH_DOUBLES);
        if (tid < FF_PATCH_HEAD) sm.rec[tid] = R[tid];
        const int stored = (int)R[2 * FAR_P + 3];
        if (stored <= FF_PATCH_NEAR) {
            if (tid < stored) {
                sm.near_x[tid] = R[FF_PATCH_HEAD + tid];
                sm.near_y[tid] = R[FF_PATCH_HEAD + FF_PATCH_NEAR + tid];
                sm.near_m[tid] = R[FF_PATCH_HEAD + 2 * FF_PATCH_NEAR + tid];
            }
            if (tid == 0) sm.near_count[par] = stored;
        } else {
            const Candidates c = candidates(a, f.sp);
            for (int64_t q = tid; q < c.n; q += FAR_THREADS) {
                int64_t k;
                double X, Y;
                if (!candidate(a, c, q, k, X, Y)) continue;
                const double d1 = ox - X, d2 = oy - Y;
                const double r2 = d1 * d1 + d2 * d2;
                if (r2 >= f.near_r2) continue;   // in the patch's expansion
                const double m = (UNIT || a.lens_m == nullptr) ? 1.0 : ((global_double *)a.lens_m)[k];
                const int j = atomicAdd(&sm.near_count[par], 1);
                if (j < NEAR_EXP) {
                    sm.near_x[j] = X;
                    sm.near_y[j] = Y;
                    sm.near_m[j] = m;
                }
            }
        }
        __syncthreads();
        const double SFAR = sm.rec[2 * FAR_P], far_err = sm.rec[2 * FAR_P + 1], SDEF = sm.rec[2 * FAR_P + 2];
        const int n_near_all = sm.near_count[par];
        if (tid == 0) sm.near_count[par ^ 1] = 0;   // every thread read it one patch ago
        const bool all_flagged = n_near_all > NEAR_EXP;
        const int n_near = all_flagged ? 0 : n_near_all;

        // A wave takes 8 x 8-ray blocks of the patch (block wave + 4 r, r < 8), so the
        // rays of one wave land on few pixels. Ray r of this thread has column
        // ib + 8 ((wave + 4 r) % 8) + lane % 8 (two values, r even or odd) and row
        // jb + 8 (r / 2) + lane / 8 (four values).
        const int wave = tid >> 6;
        auto col = [&](int c) { return ib + 8 * ((wave + 4 * c) % (PATCH_X / 8)) + (lane & 7); };
        auto row = [&](int rr) { return jb + 8 * rr + (lane >> 3); };
        double X1[2], X2[FAR_ROWS / 2];
#pragma unroll
        for (int c = 0; c < 2; ++c) X1[c] = ray_coord(a.sx0, col(c), a.spx);
#pragma unroll
        for (int rr = 0; rr < FAR_ROWS / 2; ++rr) X2[rr] = ray_coord(a.sy0, row(rr), a.spy);
        // The thread's rays in two passes of RPASS: per pass, (1) the expansion of each
        // ray (independent Horner chains), (2) the near lenses, each read from LDS once
        // per pass and added onto each ray's far part in list order, (3) the pixel
        // decision and binning into the block's pixel table.
        constexpr int RPASS = FAR_ROWS / 2;
#pragma unroll
        for (int pass = 0; pass < FAR_ROWS / RPASS; ++pass) {
            double A1[RPASS], A2[RPASS];
            {
                double T1[FAR_P], T2[FAR_P];
#pragma unroll
                for (int n = 0; n < FAR_P; ++n) {
                    T1[n] = sm.rec[n];
                    T2[n] = sm.rec[FAR_P + n];
                }
#pragma unroll
                for (int k = 0; k < RPASS; ++k) {
                    const int r = pass * RPASS + k;
                    const double nw1 = ox - X1[r & 1], nw2 = oy - X2[r >> 1];   // -w
                    double S1 = T1[FAR_P - 1], S2 = T2[FAR_P - 1];
#pragma unroll
                    for (int n = FAR_P - 2; n >= 0; --n) {
                        const double q1 = __builtin_fma(S1, nw1, __builtin_fma(-S2, nw2, T1[n]));
                        const double q2 = __builtin_fma(S1, nw2, __builtin_fma(S2, nw1, T2[n]));
                        S1 = q1;
                        S2 = q2;
                    }
                    A1[k] = S1;
                    A2[k] = -S2;
                }
            }
            double SN[RPASS];
#pragma unroll
            for (int k = 0; k < RPASS; ++k) SN[k] = 0.0;
            uint32_t tiny = 0u;
            for (int q = 0; q < n_near; ++q) {
                const double X = sm.near_x[q], Y = sm.near_y[q], M = sm.near_m[q];
#pragma unroll
                for (int k = 0; k < RPASS; ++k) {
                    const int r = pass * RPASS + k;
                    const double e1 = X1[r & 1] - X, e2 = X2[r >> 1] - Y;
                    const double r2 = __builtin_fma(e1, e1, e2 * e2);
                    if (!(r2 > 1e-200)) tiny |= 1u << k;
                    const double f = M * rcp64(r2);
                    A1[k] = __builtin_fma(f, e1, A1[k]);
                    A2[k] = __builtin_fma(f, e2, A2[k]);
                    SN[k] = __builtin_fma(fabs(e1) + fabs(e2), fabs(f), SN[k]);
                }
            }
#pragma unroll
            for (int k = 0; k < RPASS; ++k) {
                const int r = pass * RPASS + k;
                const int64_t i = col(r & 1), j = row(r >> 1);
                const bool valid = (i < a.i1) && (j < a.jc1);
                int code = far_decide(a, X1[r & 1], X2[r >> 1], A1[k], A2[k], far_err, SFAR, SDEF, SN[k], n_near,
                                      !((tiny >> k) & 1u) && !all_flagged);
                if (!valid) code = INT32_MIN;

                n_in += __builtin_popcountll(__ballot(code >= 0));
                n_out += __builtin_popcountll(__ballot(code == OUT));
                if (PIX) {
                    if (valid && code != FLAGGED) a.pix_out[(j - a.j0) * W + (i - a.i0)] = code;
                } else {
                    table_add(sm.table, a.map, code);
                }
                const uint64_t fl = __ballot(code == FLAGGED);
                if (fl) SingleSink{}.append(a, fl, lane, code == FLAGGED, i, j);
            }
        }
        if (tid == 0) sm.next = (int)next;
        __syncthreads();   // every ray of the patch is in the table
        if (!PIX) table_flush_clear<FAR_THREADS>(sm.table, a.map, tid);
        patch = sm.next;
    }
    if (lane == 0) {
        if (n_in) global_add(a.counters + C_IN, n_in);
        if (n_out) global_add(a.counters + C_OUT, n_out);
    }
}

// Re-check stage of the mixed mode on the regular grid, one thread per queued
// ray (far_recheck_ray). A ray it places is binned and its entry marked
// RESOLVED; the others are counted in *qlive and left for the FP64 stage over
// every lens. Queue entries of one deflection wave are adjacent and share a
// super-patch, so a wave walks one list.
template <bool UNIT>
__global__ __launch_bounds__(256) void recheck_far_kernel(const ShootArgs a, uint32_t *qlive) {
    const uint32_t n = *a.qcount;
    const int64_t W = a.i1 - a.i0;
    unsigned long long n_in = 0, n_out = 0;
    uint32_t left = 0;
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t idx = blockIdx.x * blockDim.x + threadIdx.x; idx < n; idx += stride) {
        const uint32_t q = a.queue[idx];
        const int64_t i = a.i0 + (int64_t)(q % (uint64_t)W);
        const int64_t j = a.jc0 + (int64_t)(q / (uint64_t)W);
        const int code = far_recheck_ray<UNIT>(a, i, j);
        if (code == FLAGGED) {
            ++left;
        } else {
            a.queue[idx] = q | RESOLVED;
            if (code >= 0) ++n_in;
            else ++n_out;
            if (a.pix_out) a.pix_out[(j - a.j0) * W + (i - a.i0)] = code;
            else if (code >= 0) atomicAdd(a.map + code, 1u);
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        n_in += __shfl_xor(n_in, off);
        n_out += __shfl_xor(n_out, off);
        left += __shfl_xor(left, off);
    }
    if (__lane_id() == 0) {
        if (n_in) atomicAdd(a.counters + C_IN, n_in);
        if (n_out) atomicAdd(a.counters + C_OUT, n_out);
        if (left) atomicAdd(qlive, left);
    }
}

}  // namespace

hipError_t launch_recheck_far(const ShootArgs &a, uint32_t *qlive, int64_t max_rays, hipStream_t stream) {
    if (max_rays <= 0) return hipSuccess;
    const bool unit = a.lens_m == nullptr;
    if (!a.random) {   // grid: this launch's records (random rays: the map's, built once)
        const int64_t rows = a.jc1 - a.jc0;
        const int64_t nby = (rows + PATCH_Y - 1) / PATCH_Y;
        const int64_t n_super = a.ff_sbx * ((nby + FF_SP_Y - 1) / FF_SP_Y);
        if (n_super <= 0) return hipSuccess;
        if (unit) hipLaunchKernelGGL((farfield_super_kernel<true, true>), dim3((unsigned)n_super), dim3(FAR_THREADS), 0, stream, a);
        else hipLaunchKernelGGL((farfield_super_kernel<false, true>), dim3((unsigned)n_super), dim3(FAR_THREADS), 0, stream, a);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    int64_t blocks = (max_rays + 255) / 256;
    if (blocks > 2048) blocks = 2048;
    if (unit) hipLaunchKernelGGL((recheck_far_kernel<true>), dim3((unsigned)blocks), dim3(256), 0, stream, a, qlive);
    else hipLaunchKernelGGL((recheck_far_kernel<false>), dim3((unsigned)blocks), dim3(256), 0, stream, a, qlive);
    return hipGetLastError();
}

hipError_t launch_super_records(const ShootArgs &a, int64_t n_super, hipStream_t stream) {
    if (n_super <= 0) return hipSuccess;
    if (a.lens_m == nullptr) hipLaunchKernelGGL((farfield_super_kernel<true, false>), dim3((unsigned)n_super), dim3(FAR_THREADS), 0, stream, a);
    else hipLaunchKernelGGL((farfield_super_kernel<false, false>), dim3((unsigned)n_super), dim3(FAR_THREADS), 0, stream, a);
    return hipGetLastError();
}

hipError_t launch_batch_super(const BatchArgs &b, hipStream_t stream) {
    if (b.total_super <= 0) return hipSuccess;
    if (b.unit_masses) hipLaunchKernelGGL((batch_super_kernel<true>), dim3((unsigned)b.total_super), dim3(FAR_THREADS), 0, stream, b);
    else hipLaunchKernelGGL((batch_super_kernel<false>), dim3((unsigned)b.total_super), dim3(FAR_THREADS), 0, stream, b);
    return hipGetLastError();
}

hipError_t launch_farfield(const ShootArgs &a, hipStream_t stream) {
    const int64_t rows = a.jc1 - a.jc0;
    const int64_t nby = (rows + PATCH_Y - 1) / PATCH_Y;
    const int64_t patches = a.nbx * nby;
    if (patches <= 0) return hipSuccess;
    const int64_t n_super = a.ff_sbx * ((nby + FF_SP_Y - 1) / FF_SP_Y);
    const bool unit = a.lens_m == nullptr;
    const bool pix = a.pix_out != nullptr;
    const dim3 block(FAR_THREADS);
    const int64_t n_group = a.ff_gbx * ((((nby + FF_SP_Y - 1) / FF_SP_Y) + FF_GROUP - 1) / FF_GROUP);
    const dim3 group_block(FAR_GROUP_THREADS);
    if (a.ff_top) {
        const int64_t n_gy = (((nby + FF_SP_Y - 1) / FF_SP_Y) + FF_GROUP - 1) / FF_GROUP;
        const int64_t n_top = a.ff_tbx * ((n_gy + FF_TOP - 1) / FF_TOP);
        const dim3 top_grid((unsigned)(n_top * FF_TOP_PARTS));
        if (unit) hipLaunchKernelGGL((farfield_top_kernel<true>), top_grid, dim3(FAR_TOP_THREADS), 0, stream, a);
        else hipLaunchKernelGGL((farfield_top_kernel<false>), top_grid, dim3(FAR_TOP_THREADS), 0, stream, a);
        if (unit) hipLaunchKernelGGL((farfield_group_top_kernel<true>), dim3((unsigned)n_group), group_block, 0, stream, a);
        else hipLaunchKernelGGL((farfield_group_top_kernel<false>), dim3((unsigned)n_group), group_block, 0, stream, a);
    } else {
        const dim3 group_grid((unsigned)(n_group * group_parts(a.n_lens)));
        if (unit) hipLaunchKernelGGL((farfield_group_kernel<true>), group_grid, group_block, 0, stream, a);
        else hipLaunchKernelGGL((farfield_group_kernel<false>), group_grid, group_block, 0, stream, a);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (unit) hipLaunchKernelGGL((farfield_super_group_kernel<true>), dim3((unsigned)n_super), block, 0, stream, a);
    else hipLaunchKernelGGL((farfield_super_group_kernel<false>), dim3((unsigned)n_super), block, 0, stream, a);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const dim3 rec_grid((unsigned)((patches + FAR_THREADS / 64 - 1) / (FAR_THREADS / 64)));
    if (unit) hipLaunchKernelGGL((farfield_patch_kernel<true>), rec_grid, block, 0, stream, a, patches);
    else hipLaunchKernelGGL((farfield_patch_kernel<false>), rec_grid, block, 0, stream, a, patches);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    auto launch_rays = [&](auto kernel) {
        int64_t blocks = persistent_blocks(kernel, FAR_THREADS, 0);
        if (blocks > patches) blocks = patches;
        hipLaunchKernelGGL(kernel, dim3((unsigned)blocks), block, 0, stream, a, patches);
    };
    if (unit) {
        if (pix) launch_rays(farfield_kernel<true, true>);
        else launch_rays(farfield_kernel<true, false>);
    } else {
        if (pix) launch_rays(farfield_kernel<false, true>);
        else launch_rays(farfield_kernel<false, false>);
    }
    return hipGetLastError();
}

}  // namespace rs
