/*
 * rayshoot.h — C ABI of the MI355X inverse ray-shooting library.
 *
 * The operation (Bate et al., "Computational advances in gravitational
 * microlensing"):
 *   - Section 2, Eq. (sigma): a ray at image position x = (x1, x2) reaches
 *       y1 = (1 - gamma - sigma_c) x1 - sum_k m_k (x1 - X_k) / |x - x_k|^2
 *       y2 = (1 + gamma - sigma_c) x2 - sum_k m_k (x2 - Y_k) / |x - x_k|^2
 *     for N* point lenses (x_k, m_k), smooth convergence sigma_c and external
 *     shear gamma (sigma = sigma_c + sigma_* is the total convergence).
 *   - Section 2, Eq. (mu_ij): inverse ray-shooting counts the rays N_ij that
 *     reach each source pixel; mu_ij = N_ij / N_rays.
 *   - Section 3.1: rays sit on a regular image-plane grid. Here ray (i, j) is
 *     at the cell centre x1 = sx0 + (i + 1/2) sw/nx, x2 = sy0 + (j + 1/2) sh/ny.
 *   - Pixel (p, q) of the source map covers u in [p, p+1), v in [q, q+1), with
 *     u = (y1 - tx0) / (tw/npx) and v = (y2 - ty0) / (th/npy). Rays outside
 *     [0,npx) x [0,npy), or with a non-finite position, are counted as "out".
 *     A ray exactly on a lens (|x - x_k|^2 == 0) is "singular": dropped, counted.
 *
 * Precision modes:
 *   RS_MIXED  the deflection sum runs in FP32 with block-relative coordinates
 *             and FP64 folding of short FP32 partial sums; every ray carries a
 *             rigorous bound on its source-position error, and rays whose
 *             bound reaches a pixel edge are re-evaluated in FP64 with the
 *             plain definition (lens order, no fused multiply-add, IEEE
 *             division). A first FP64 stage with fused multiply-adds and a
 *             rigorous bound decides almost every queued ray; only rays it
 *             cannot place run the exact sequence. The count map equals the
 *             FP64 definition's map.
 *   RS_FP32   the same FP32 sum, binned directly (no bound, no re-check).
 *
 * Conventions for every call:
 *   - Array arguments are DEVICE pointers (hipMalloc'd or torch CUDA tensors)
 *     unless the comment says "host".
 *   - Calls that take a stream enqueue work on that HIP stream (NULL = the
 *     default stream) and return before it runs; results are valid after the
 *     stream is synchronised. Argument validation happens before anything is
 *     enqueued.
 *   - The caller owns every buffer. rs_make_map and rs_ray_pixels allocate
 *     nothing; they use the caller's workspace.
 *   - Return codes: RS_OK (0) or a negative RS_E* code; rs_last_error() gives a
 *     thread-local message for the last failure. No C++ exception crosses the ABI.
 */
#ifndef RAYSHOOT_H
#define RAYSHOOT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RS_OK 0
#define RS_EINVAL (-1)     /* bad argument (sizes, extents, window, null pointer, mode) */
#define RS_ENOMEM (-2)     /* workspace too small, or server budget cannot hold a request */
#define RS_EHIP (-3)       /* a HIP runtime call failed */
#define RS_EBUSY (-4)      /* server full (non-blocking submit) */
#define RS_ECANCELED (-5)  /* request cancelled */

#define RS_FP32 0
#define RS_MIXED 1

#define RS_ACCUMULATE 1      /* flag: add to the map instead of zeroing it first */
#define RS_EXACT_RECHECK 2   /* flag (RS_MIXED): re-check every queued ray with the definition's exact
                                FP64 sequence only, skipping the faster bounded FP64 first stage */

/* One map: macro model, shooting grid, ray window and source grid. */
typedef struct {
    double sigma_star;      /* compact-object convergence; informational (N* and lens masses carry it) */
    double sigma_c;         /* smooth convergence, Eq. (sigma) */
    double gamma;           /* external shear, Eq. (sigma); x1 carries 1 - gamma */
    double sx0, sy0;        /* lower-left corner of the shooting rectangle (image plane) */
    double sw, sh;          /* its width (along x1) and height (along x2), > 0 */
    int64_t nx, ny;         /* ray grid, > 0; ray (i,j) sits at the cell centre */
    int64_t i0, i1, j0, j1; /* ray window [i0,i1) x [j0,j1); {0,nx,0,ny} = the whole grid */
    double tx0, ty0;        /* lower-left corner of the source map */
    double tw, th;          /* source map width and height, > 0 */
    int64_t npx, npy;       /* source pixels, > 0; the map is uint32 [npy][npx] row-major */
    int32_t mode;           /* RS_FP32 or RS_MIXED */
    int32_t flags;          /* 0 or an OR of RS_ACCUMULATE, RS_EXACT_RECHECK */
} rs_map_params;

/* Counters of one map (or window), accumulated on the device. */
typedef struct {
    uint64_t rays_shot;       /* rays in the window */
    uint64_t rays_in_map;     /* rays binned */
    uint64_t rays_out;        /* rays outside the map or with a non-finite position */
    uint64_t rays_singular;   /* rays exactly on a lens */
    uint64_t rays_rechecked;  /* RS_MIXED: rays re-evaluated in FP64 */
} rs_map_stats;

/* Library version string. */
const char *rs_version(void);

/* Thread-local message describing the last non-zero return on this thread. */
const char *rs_last_error(void);

/*
 * Workspace bytes rs_make_map / rs_ray_pixels need for these parameters and
 * lens count (stats counters plus, for RS_MIXED, the FP64 re-check queue).
 * Returns 0 if the parameters are invalid.
 */
size_t rs_workspace_bytes(const rs_map_params *params, int64_t n_lens);

/*
 * Build the count map of the ray window (Section 2, Eq. (sigma) and Eq. (mu_ij)).
 *   lens_xy  device, float64 [n_lens][2] (x, y) positions, 16-byte aligned
 *   lens_m   device, float64 [n_lens] masses, or NULL for unit masses
 *   n_lens   >= 0
 *   map      device, uint32 [npy][npx]; zeroed first unless RS_ACCUMULATE
 *   workspace / workspace_bytes  device scratch of at least rs_workspace_bytes()
 *   stream   hipStream_t (NULL = default stream)
 * The stats of the call stay in the workspace: read them with rs_read_stats.
 * Errors: RS_EINVAL (bad params or pointers), RS_ENOMEM (workspace too small),
 * RS_EHIP (launch failure).
 */
int rs_make_map(const rs_map_params *params, const double *lens_xy, const double *lens_m,
                int64_t n_lens, uint32_t *map, void *workspace, size_t workspace_bytes,
                void *stream);

/*
 * Per-ray result of the window, for tests: pix[(j-j0)*(i1-i0) + (i-i0)] =
 * v*npx + u of the ray's pixel, -1 if out, -2 if singular. Same arithmetic and
 * the same re-check rule as rs_make_map in the given mode. No map is written.
 *   pix  device, int32 [(i1-i0)*(j1-j0)]; npx*npy must be < 2^31
 */
int rs_ray_pixels(const rs_map_params *params, const double *lens_xy, const double *lens_m,
                  int64_t n_lens, int32_t *pix, void *workspace, size_t workspace_bytes,
                  void *stream);

/*
 * Copy the counters of the last rs_make_map / rs_ray_pixels that used this
 * workspace into host memory. Synchronises the stream.
 */
int rs_read_stats(const void *workspace, rs_map_stats *stats_host, void *stream);

/*
 * Kernel timing. When enabled, rs_make_map records HIP events on its stream
 * around every deflection-kernel launch; rs_profile_read synchronises those
 * events and returns the summed kernel milliseconds, the number of launches
 * and the ray-lens interactions those launches covered, then resets the sums.
 * Used by the benchmark's roofline figure.
 */
int rs_profile_enable(int on);
int rs_profile_read(double *kernel_ms, int64_t *launches, double *interactions);

/* ------------------------------------------------------------------------- */
/* Autotuner of the deflection kernel's thread shape.                        */
/* The paper notes that the direct GPU code's batch and thread-group sizes    */
/* are hardware dependent (Section 2, GPU-D); here the choice is measured.    */
/* Every shape covers the same 64 x 32 ray patch per block, so the choice     */
/* changes speed only: maps are bit-identical across shapes in both modes.    */
/* ------------------------------------------------------------------------- */

#define RS_MAX_SHAPES 8

typedef struct {
    int32_t shape;               /* fastest shape id on the sample */
    int32_t n_shapes;            /* shapes available */
    int32_t rays_per_lane[RS_MAX_SHAPES][2];  /* (x, y) rays per lane of each shape */
    int32_t threads[RS_MAX_SHAPES];           /* threads per block of each shape */
    double ms[RS_MAX_SHAPES];    /* deflection-kernel time of each shape on the sample, ms */
    double sample_interactions;  /* ray-lens interactions in the sample */
} rs_tune_result;

/*
 * Time every shape on a sample of this map (a band of rows from the middle of
 * the window holding about sample_rays rays; <= 0 picks 2^22) and remember the
 * fastest for maps with the same signature (mode, unit or general masses,
 * N* rounded to a power of two). Later rs_make_map calls with that signature
 * use it. scratch_map (device, uint32 [npy][npx]) is overwritten. Synchronises
 * the stream. Errors as rs_make_map.
 */
int rs_tune(const rs_map_params *params, const double *lens_xy, const double *lens_m, int64_t n_lens,
            uint32_t *scratch_map, void *workspace, size_t workspace_bytes, int64_t sample_rays,
            void *stream, rs_tune_result *result_host);

/*
 * Force a shape for every later launch (0 .. n_shapes-1), or -1 to use the
 * tuner's cache and the built-in default. The previous setting is stored in
 * *previous when it is not NULL. Errors: RS_EINVAL (shape out of range).
 */
int rs_set_shape(int shape, int *previous);

/* Write / read the tuner's cache as text (one "mode unit n_bucket shape" line each). */
int rs_tune_save(const char *path);
int rs_tune_load(const char *path);

#ifdef __cplusplus
}
#endif

#endif /* RAYSHOOT_H */
