/*
 * FP64 CPU oracle for inverse ray-shooting magnification maps.
 *
 * TEST INFRASTRUCTURE ONLY. Only the tests, the smoke check and the bench's
 * CPU-baseline leg may load this library. The HIP product path never calls it
 * and shares no code, header, table or helper with it.
 *
 * What it computes (Bate et al., "Computational advances in gravitational
 * microlensing"):
 *   - Section 2, Eq. (sigma): the lens equation with N* point masses, a smooth
 *     convergence sigma_c and an external shear gamma,
 *         y1 = (1 - gamma - sigma_c) x1 - sum_k m_k (x1 - X_k) / |x - x_k|^2
 *         y2 = (1 + gamma - sigma_c) x2 - sum_k m_k (x2 - Y_k) / |x - x_k|^2
 *   - Section 2, Eq. (mu_ij): inverse ray-shooting; rays are deflected from the
 *     image plane and counted per source-plane pixel, N_ij.
 *   - Section 3.1: rays are shot on a regular grid (CPU-T/CPU-P), so that with
 *     no lensing every pixel receives exactly N_rays rays. Rays are placed at
 *     cell centres, x1 = sx0 + (i + 1/2) sw/nx.
 *   - Section 3.1 (the GPU code's sampling): alternatively every ray sits at an
 *     independent uniformly random position in the shooting rectangle, so a
 *     pixel receives N_rays rays only on average, with Poisson noise. Ray (i, j)
 *     takes its two uniforms from the counter-based generator Philox4x64-10
 *     (Salmon, Moraes, Dror & Shaw 2011) at counter (j nx + i, 0, 0, 0) and key
 *     (seed, 0): U = (top 52 bits of a 64-bit output + 1/2) 2^-52, strictly
 *     inside (0, 1); x1 = sx0 + U1 sw, x2 = sy0 + U2 sh.
 *
 * Readings where the paper is silent (each is also listed in the design notes):
 *   - the sum runs over lenses in index order k = 0..N*-1, sequentially, with
 *     no fused multiply-add (this file is compiled with -ffp-contract=off);
 *   - pixels are half-open [p, p+1) in pixel units; a ray is binned if its
 *     source position is finite and lies in [0,npx) x [0,npy), else it is "out";
 *   - a ray that lands exactly on a lens (r^2 == 0) is dropped and counted
 *     as "singular";
 *   - masses default to 1 (Einstein-radius units) when no mass array is given;
 *   - the coefficient (1 - gamma - sigma_c) is evaluated as (1 - gamma) - sigma_c.
 *
 * Everything is plain FP64. Threads split the ray rows of the window; every
 * ray's arithmetic is independent of the thread count.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    double sigma_c, gamma;
    double sx0, sy0, sw, sh;
    int64_t nx, ny;
    int64_t i0, i1, j0, j1;
    double tx0, ty0, tw, th;
    int64_t npx, npy;
    int64_t random_rays;   /* 0: regular grid; 1: Philox-random positions */
    uint64_t seed;
} oracle_params;

enum { RAY_OUT = -1, RAY_SINGULAR = -2 };

/* One ray, start to finish: Section 3.1 grid position, Eq. (sigma), pixel. */
typedef struct {
    double u, v;     /* source position in pixel units (NaN when singular) */
    int64_t pix;     /* v*npx + u, RAY_OUT or RAY_SINGULAR */
} ray_result;

/* Philox4x64-10: ten rounds of two 64x64->128-bit products, the key bumped by
 * the Weyl constants between rounds. */
void oracle_philox4x64(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4])
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
    uint64_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += W0;
            k1 += W1;
        }
        const unsigned __int128 p0 = (unsigned __int128)M0 * c0;
        const unsigned __int128 p1 = (unsigned __int128)M1 * c2;
        const uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
        const uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
        c0 = hi1 ^ c1 ^ k0;
        c1 = lo1;
        c2 = hi0 ^ c3 ^ k1;
        c3 = lo0;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

/* Image-plane position of ray (i, j). */
static void ray_position(const oracle_params *p, int64_t i, int64_t j, double *x1, double *x2)
{
    if (p->random_rays) {
        const uint64_t ctr[4] = {(uint64_t)j * (uint64_t)p->nx + (uint64_t)i, 0, 0, 0};
        const uint64_t key[2] = {p->seed, 0};
        uint64_t out[4];
        oracle_philox4x64(ctr, key, out);
        const double u1 = ((double)(out[0] >> 12) + 0.5) * 0x1p-52;
        const double u2 = ((double)(out[1] >> 12) + 0.5) * 0x1p-52;
        *x1 = p->sx0 + u1 * p->sw;
        *x2 = p->sy0 + u2 * p->sh;
    } else {
        /* Section 3.1: regular grid, cell-centred. */
        *x1 = p->sx0 + ((double)i + 0.5) * (p->sw / (double)p->nx);
        *x2 = p->sy0 + ((double)j + 0.5) * (p->sh / (double)p->ny);
    }
}

static ray_result shoot_one(const oracle_params *p, const double *lens_xy, const double *lens_m,
                            int64_t n_lens, int64_t i, int64_t j)
{
    ray_result r;
    double x1, x2;
    ray_position(p, i, j, &x1, &x2);

    /* Eq. (sigma), the point-mass sum, in lens order. */
    double a1 = 0.0, a2 = 0.0;
    for (int64_t k = 0; k < n_lens; ++k) {
        const double d1 = x1 - lens_xy[2 * k];
        const double d2 = x2 - lens_xy[2 * k + 1];
        const double r2 = d1 * d1 + d2 * d2;
        if (r2 == 0.0) {
            r.u = NAN;
            r.v = NAN;
            r.pix = RAY_SINGULAR;
            return r;
        }
        const double m = lens_m ? lens_m[k] : 1.0;
        const double f = m / r2;
        a1 += f * d1;
        a2 += f * d2;
    }
    /* Eq. (sigma), macro terms: diag(1-gamma, 1+gamma) x - sigma_c x. */
    const double c1 = (1.0 - p->gamma) - p->sigma_c;
    const double c2 = (1.0 + p->gamma) - p->sigma_c;
    const double y1 = c1 * x1 - a1;
    const double y2 = c2 * x2 - a2;

    /* Source-plane pixel units; pixel (p,q) covers [p,p+1) x [q,q+1). */
    r.u = (y1 - p->tx0) / (p->tw / (double)p->npx);
    r.v = (y2 - p->ty0) / (p->th / (double)p->npy);
    if (isfinite(r.u) && isfinite(r.v) && r.u >= 0.0 && r.u < (double)p->npx &&
        r.v >= 0.0 && r.v < (double)p->npy) {
        r.pix = (int64_t)floor(r.v) * p->npx + (int64_t)floor(r.u);
    } else {
        r.pix = RAY_OUT;
    }
    return r;
}

/* Distance from c to the nearest integer edge in [0, n], for c within [-tol, n+tol]. */
static int near_edge_1d(double c, int64_t n, double tol)
{
    if (!(c >= -tol && c <= (double)n + tol))
        return 0;
    const double f = floor(c);
    const double d = fmin(c - f, f + 1.0 - c);
    return d < tol;
}

static int is_near_edge(const oracle_params *p, const ray_result *r, double tol)
{
    if (r->pix == RAY_SINGULAR)
        return 0;
    if (!isfinite(r->u) || !isfinite(r->v))
        return 0;
    const int in_u = r->u >= -tol && r->u <= (double)p->npx + tol;
    const int in_v = r->v >= -tol && r->v <= (double)p->npy + tol;
    if (!in_u || !in_v)
        return 0;
    return near_edge_1d(r->u, p->npx, tol) || near_edge_1d(r->v, p->npy, tol);
}

/* ------------------------------------------------------------------------- */
/* Threading: rows of the window are handed out one at a time.               */
/* ------------------------------------------------------------------------- */

typedef struct {
    const oracle_params *p;
    const double *lens_xy, *lens_m;
    int64_t n_lens;
    int64_t next_row;              /* shared, atomically incremented */
    /* make_map outputs */
    uint32_t *map;                 /* shared final map (reduced under lock) */
    pthread_mutex_t lock;
    uint64_t counts[4];            /* in, out, singular, near-edge */
    double near_tol;
    int64_t *near_ij;              /* optional list of (i, j) pairs */
    int64_t near_cap;
    /* ray_pixels outputs */
    int64_t *pix;
    double *uo, *vo;
} job;

static int64_t take_row(job *jb)
{
    return __atomic_fetch_add(&jb->next_row, 1, __ATOMIC_RELAXED);
}

static void *map_worker(void *arg)
{
    job *jb = (job *)arg;
    const oracle_params *p = jb->p;
    const size_t npix = (size_t)p->npx * (size_t)p->npy;
    uint32_t *local = (uint32_t *)calloc(npix, sizeof(uint32_t));
    if (!local)
        return (void *)1;
    uint64_t c_in = 0, c_out = 0, c_sing = 0;
    for (;;) {
        const int64_t j = p->j0 + take_row(jb);
        if (j >= p->j1)
            break;
        for (int64_t i = p->i0; i < p->i1; ++i) {
            const ray_result r = shoot_one(p, jb->lens_xy, jb->lens_m, jb->n_lens, i, j);
            if (r.pix >= (int64_t)npix) {
                /* cannot happen for 0 <= u < npx, 0 <= v < npy; refuse rather than write out of bounds */
                free(local);
                return (void *)1;
            }
            if (r.pix >= 0) {
                local[r.pix] += 1;
                ++c_in;
            } else if (r.pix == RAY_OUT) {
                ++c_out;
            } else {
                ++c_sing;
            }
            if (jb->near_tol > 0.0 && is_near_edge(p, &r, jb->near_tol)) {
                pthread_mutex_lock(&jb->lock);
                const uint64_t slot = jb->counts[3]++;
                if (jb->near_ij && (int64_t)slot < jb->near_cap) {
                    jb->near_ij[2 * slot] = i;
                    jb->near_ij[2 * slot + 1] = j;
                }
                pthread_mutex_unlock(&jb->lock);
            }
        }
    }
    pthread_mutex_lock(&jb->lock);
    for (size_t q = 0; q < npix; ++q)
        jb->map[q] += local[q];
    jb->counts[0] += c_in;
    jb->counts[1] += c_out;
    jb->counts[2] += c_sing;
    pthread_mutex_unlock(&jb->lock);
    free(local);
    return NULL;
}

static void *pix_worker(void *arg)
{
    job *jb = (job *)arg;
    const oracle_params *p = jb->p;
    const int64_t w = p->i1 - p->i0;
    for (;;) {
        const int64_t jj = take_row(jb);
        const int64_t j = p->j0 + jj;
        if (j >= p->j1)
            break;
        for (int64_t i = p->i0; i < p->i1; ++i) {
            const ray_result r = shoot_one(p, jb->lens_xy, jb->lens_m, jb->n_lens, i, j);
            const int64_t idx = jj * w + (i - p->i0);
            jb->pix[idx] = r.pix;
            if (jb->uo)
                jb->uo[idx] = r.u;
            if (jb->vo)
                jb->vo[idx] = r.v;
        }
    }
    return NULL;
}

static int check_params(const oracle_params *p, int64_t n_lens)
{
    if (!p || n_lens < 0)
        return -1;
    if (p->nx <= 0 || p->ny <= 0 || p->npx <= 0 || p->npy <= 0)
        return -1;
    if (!(p->sw > 0.0) || !(p->sh > 0.0) || !(p->tw > 0.0) || !(p->th > 0.0))
        return -1;
    if (p->i0 < 0 || p->i1 > p->nx || p->i0 > p->i1 || p->j0 < 0 || p->j1 > p->ny || p->j0 > p->j1)
        return -1;
    return 0;
}

static int run_threads(job *jb, void *(*fn)(void *), int nthreads)
{
    if (nthreads < 1)
        nthreads = 1;
    if (nthreads > 256)
        nthreads = 256;
    pthread_t th[256];
    int started = 0, rc = 0;
    for (int t = 0; t < nthreads; ++t) {
        if (pthread_create(&th[t], NULL, fn, jb) != 0)
            break;
        ++started;
    }
    if (started == 0)
        return -3;
    for (int t = 0; t < started; ++t) {
        void *ret = NULL;
        pthread_join(th[t], &ret);
        if (ret)
            rc = -2;
    }
    return rc;
}

/*
 * Build the count map of the ray window [i0,i1) x [j0,j1).
 *   lens_xy: [n_lens][2] positions; lens_m: [n_lens] masses or NULL (unit).
 *   map: [npy][npx] uint32, zeroed here, then filled.
 *   counts: [4] = rays in map, rays out, singular rays, near-edge rays.
 *   near_tol: rays whose (u,v) lies within near_tol pixels of a pixel edge
 *             are counted (and listed into near_ij as (i,j) pairs, up to
 *             near_cap pairs); 0 disables the check.
 * Returns 0, or -1 on invalid arguments, -2 on allocation failure.
 */
int oracle_make_map(const oracle_params *p, const double *lens_xy, const double *lens_m,
                    int64_t n_lens, uint32_t *map, uint64_t *counts, double near_tol,
                    int64_t *near_ij, int64_t near_cap, int nthreads)
{
    if (check_params(p, n_lens) != 0 || !map || !counts || (n_lens > 0 && !lens_xy))
        return -1;
    job jb;
    memset(&jb, 0, sizeof(jb));
    jb.p = p;
    jb.lens_xy = lens_xy;
    jb.lens_m = lens_m;
    jb.n_lens = n_lens;
    jb.map = map;
    jb.near_tol = near_tol;
    jb.near_ij = near_ij;
    jb.near_cap = near_cap;
    pthread_mutex_init(&jb.lock, NULL);
    memset(map, 0, sizeof(uint32_t) * (size_t)p->npx * (size_t)p->npy);
    const int rc = run_threads(&jb, map_worker, nthreads);
    pthread_mutex_destroy(&jb.lock);
    memcpy(counts, jb.counts, sizeof(jb.counts));
    return rc;
}

/*
 * Per-ray results for the window, row-major within the window
 * (index (j-j0)*(i1-i0) + (i-i0)): pixel index v*npx+u, -1 (out) or
 * -2 (singular), and optionally the FP64 source position in pixel units.
 */
int oracle_ray_pixels(const oracle_params *p, const double *lens_xy, const double *lens_m,
                      int64_t n_lens, int64_t *pix, double *u_out, double *v_out, int nthreads)
{
    if (check_params(p, n_lens) != 0 || !pix || (n_lens > 0 && !lens_xy))
        return -1;
    job jb;
    memset(&jb, 0, sizeof(jb));
    jb.p = p;
    jb.lens_xy = lens_xy;
    jb.lens_m = lens_m;
    jb.n_lens = n_lens;
    jb.pix = pix;
    jb.uo = u_out;
    jb.vo = v_out;
    return run_threads(&jb, pix_worker, nthreads);
}
