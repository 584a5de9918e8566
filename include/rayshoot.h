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
 *   - Section 3.1, the GPU code's sampling (flag RS_RANDOM_RAYS): ray (i, j)
 *     instead sits at an independent uniformly random point of the shooting
 *     rectangle, x1 = sx0 + U1 sw, x2 = sy0 + U2 sh, so a pixel receives N_rays
 *     only on average (Poisson noise). U1, U2 come from the counter-based
 *     generator Philox4x64-10 (Salmon et al. 2011) at counter (j nx + i, 0, 0, 0)
 *     and key (seed, 0): U = (output word >> 12, plus 1/2) * 2^-52, words 0
 *     and 1 of the block. A ray's position depends only on (i, j) and the seed,
 *     so windows of one map still sum to the whole map.
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
 *             division). On the regular grid a first stage evaluates each
 *             queued ray from its super-patch's FP64 far-field expansion (the
 *             RS_FARFIELD one, below) plus the lenses listed next to the
 *             super-patch, under that mode's rigorous bound; the rays it
 *             cannot place (and every queued random ray) go to an FP64 stage
 *             over every lens with fused multiply-adds and a rigorous bound,
 *             and only the rays that stage cannot place run the exact sequence.
 *             The count map equals the FP64 definition's map.
 *   RS_FP32   the same FP32 sum, binned directly (no bound, no re-check).
 *   RS_FARFIELD  the tree codes' idea (Section 2, Eq. (hierarchical): distant
 *             lenses grouped, with higher multipoles) taken to all orders: per
 *             64 x 32-ray patch, lenses farther than 4 half-diagonals enter an
 *             order-16 FP64 local expansion of the deflection about the patch
 *             centre, nearer ones are summed directly, and each ray carries a
 *             rigorous bound (truncation + rounding + the definition's own
 *             rounding); rays within it of a pixel edge get the same FP64
 *             re-check. The count map equals the FP64 definition's map, at
 *             about 100 FP64 operations per lens and patch instead of 2048
 *             interactions. Single maps only (not random rays, batches, the
 *             server or the tuner).
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
#define RS_EBUSY (-4)      /* the server's waiting queue is full (rs_server_submit never blocks) */
#define RS_ECANCELED (-5)  /* request cancelled */

#define RS_FP32 0
#define RS_MIXED 1
#define RS_FARFIELD 2

#define RS_ACCUMULATE 1      /* flag: add to the map instead of zeroing it first */
#define RS_EXACT_RECHECK 2   /* flag (RS_MIXED): re-check every queued ray with the definition's exact
                                FP64 sequence only, skipping the faster bounded FP64 first stage */
#define RS_RANDOM_RAYS 4     /* flag: Philox-random ray positions instead of the regular grid
                                (rs_make_map and rs_ray_pixels; not in batches or the server) */

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
    int32_t mode;           /* RS_FP32, RS_MIXED or RS_FARFIELD */
    int32_t flags;          /* 0 or an OR of RS_ACCUMULATE, RS_EXACT_RECHECK, RS_RANDOM_RAYS */
    uint64_t seed;          /* RS_RANDOM_RAYS: the generator key's first word */
} rs_map_params;

/* Counters of one map (or window), accumulated on the device. */
typedef struct {
    uint64_t rays_shot;       /* rays in the window */
    uint64_t rays_in_map;     /* rays binned */
    uint64_t rays_out;        /* rays outside the map or with a non-finite position */
    uint64_t rays_singular;   /* rays exactly on a lens */
    uint64_t rays_rechecked;  /* RS_MIXED: rays re-evaluated in FP64 */
    uint64_t rays_rechecked_direct; /* of those, rays re-evaluated against every lens (the far-field
                                       first stage could not place them, or did not apply) */
} rs_map_stats;

/* Library version string. */
const char *rs_version(void);

/* Thread-local message describing the last non-zero return on this thread. */
const char *rs_last_error(void);

/*
 * Workspace bytes rs_make_map / rs_ray_pixels need for these parameters and
 * lens count: the stats counters; for RS_MIXED and RS_FARFIELD the FP64
 * re-check queue (4 bytes per ray of the largest launch, up to 2^27 rays) and
 * the super-patch records of the far-field expansion or re-check stage (about
 * 16.7 KB per 32768 rays); for random rays the bin arrays and the sorted ray
 * list (20 bytes per ray of the largest launch, up to 2^26 rays or one 32-row
 * band of a wider window). Windows wider than 2^22 rays are refused (RS_EINVAL).
 * Returns 0 if the parameters are invalid.
 */
size_t rs_workspace_bytes(const rs_map_params *params, int64_t n_lens);

/*
 * Build the count map of the ray window (Section 2, Eq. (sigma) and Eq. (mu_ij)).
 *   lens_xy  device, float64 [n_lens][2] (x, y) positions, 8-byte aligned
 *   lens_m   device, float64 [n_lens] masses (8-byte aligned), or NULL for unit masses
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
 * rs_make_map without allocation, for callers that cannot allocate device memory
 * (code under HIP graph capture, serving loops or harnesses that forbid hipMalloc).
 * The same count map and counters as rs_make_map (same arguments, same errors),
 * computed with a static device scratch of RS_NOALLOC_SCRATCH_BYTES that the
 * library holds on each device it runs on until the process ends, instead of a
 * caller workspace; the map is built in launches of as many 32-row bands as the
 * scratch holds (on the regular grid every mode gives rs_make_map's map bit for
 * bit; with RS_RANDOM_RAYS the mixed mode does, while RS_FP32 may bin a few rays
 * differently, as launches of other sizes sort rays into other bins). The call
 * allocates nothing and never creates HIP events (rs_profile_enable does not
 * apply to it).
 *   stats_host  HOST; NULL, or filled with the call's counters after a device-to-host
 *               copy and a synchronisation of the stream (pass NULL under graph
 *               capture)
 * The scratch is on the current device; the stream must belong to it. Every call
 * on one device shares that device's scratch, which keeps the last call's contents
 * (each call clears what must start at zero): calls that overlap on one device,
 * on different streams or threads, race and corrupt each other's maps. Serialise them.
 * Errors: as rs_make_map; RS_ENOMEM when one 32-row band of the window needs more
 * than RS_NOALLOC_SCRATCH_BYTES (a window wider than about 500000 rays in RS_MIXED).
 */
#define RS_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int rs_make_map_noalloc(const rs_map_params *params, const double *lens_xy, const double *lens_m,
                        int64_t n_lens, uint32_t *map, rs_map_stats *stats_host, void *stream);

/*
 * Kernel timing. When enabled, rs_make_map records HIP events on its stream
 * around every deflection-kernel launch; rs_profile_read synchronises those
 * events and returns the summed kernel milliseconds, the number of launches
 * and the ray-lens interactions those launches covered, then resets the sums.
 * Used by the benchmark's roofline figure.
 * Two further aids need no call: the environment variable RAYSHOOT_DEBUG=1 makes
 * the library print each map's launch plan and each batch's choice to stderr (=2
 * also the request loop's steps), and named roctx ranges mark its phases for
 * rocprofv3 --marker-trace.
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
 * N* rounded down to a power of two, the window's 64 x 32-ray patches rounded
 * down to a power of two). Later rs_make_map calls with that signature use it.
 * scratch_map (device, uint32 [npy][npx]) is overwritten. Synchronises the
 * stream. When the environment variable RAYSHOOT_TUNE_CACHE names a file, the
 * cache is loaded from it on first use and written to it after every tuning run.
 * Errors as rs_make_map.
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

/* Write / read the tuner's cache as text, one line per entry:
   "kind mode unit n_bucket patch_bucket choice" (kind 0: single maps, choice = shape;
   kind 1: batches, choice = shape + 16 * blocks per CU, 0 blocks = as many as fit). */
int rs_tune_save(const char *path);
int rs_tune_load(const char *path);

/* ------------------------------------------------------------------------- */
/* Batched maps: many maps, each with its own lenses, grids and parameters,   */
/* in one persistent launch of the deflection kernel followed by one batched  */
/* FP64 re-check. Every map is bit-identical to what rs_make_map gives for it. */
/* ------------------------------------------------------------------------- */

typedef struct {
    rs_map_params params;    /* one map; every request of a batch has the same mode */
    const double *lens_xy;   /* device, float64 [n_lens][2] */
    const double *lens_m;    /* device, float64 [n_lens] or NULL (unit masses) */
    int64_t n_lens;
    uint32_t *map;           /* device, uint32 [npy][npx]; zeroed unless params.flags has RS_ACCUMULATE */
} rs_map_request;

/*
 * Workspace bytes for this batch: descriptors, counters, two bits per ray
 * (rays to re-check, rays left to the exact stage) and, in RS_MIXED, each
 * map's super-patch records for the far-field re-check stage (about 4.4 KB per
 * 32768 rays). Returns 0 if a request is invalid.
 */
size_t rs_batch_workspace_bytes(const rs_map_request *requests, int32_t n);

/*
 * Build n maps (1 <= n <= 65536) in one launch sequence on the stream: one
 * persistent deflection launch over the 64 x 32-ray patches of every map (most
 * expensive maps first), then one batched FP64 re-check. Each map's window must
 * hold fewer than 2^32 rays. The per-map counters stay in the workspace (read
 * them with rs_batch_read_stats). The library copies its work descriptors from
 * host memory into the workspace (hipMemcpyAsync) before returning.
 * Errors: RS_EINVAL (a bad request, mixed modes), RS_ENOMEM (workspace too
 * small), RS_EHIP.
 */
int rs_make_maps(const rs_map_request *requests, int32_t n, void *workspace, size_t workspace_bytes,
                 void *stream);

#define RS_MAX_BATCH_CHOICES 16

typedef struct {
    int32_t best;                                 /* index of the fastest candidate */
    int32_t n;                                    /* candidates timed */
    int32_t shape[RS_MAX_BATCH_CHOICES];          /* thread shape of each candidate */
    int32_t blocks_per_cu[RS_MAX_BATCH_CHOICES];  /* persistent blocks per CU (0 = as many as fit) */
    double ms[RS_MAX_BATCH_CHOICES];              /* persistent deflection launch on the sample, ms */
    double sample_interactions;                   /* ray-lens interactions in the sample */
} rs_tune_batch_result;

/*
 * Autotune a batch: time the persistent deflection launch for every thread shape
 * and persistent grid (all blocks that fit per CU, 3, 2) on a sample made of a
 * band of whole patch rows (about sample_rays rays; <= 0 picks 2^20) from the
 * middle of every map's window, and remember the fastest for batches with the
 * same signature (mode, unit or general masses, the heaviest map's N* and the
 * batch's patch count, each rounded down to a power of two; RAYSHOOT_TUNE_CACHE
 * as for rs_tune). The requests' maps are overwritten (scratch); the workspace
 * needs rs_batch_workspace_bytes of the requests. Synchronises the stream.
 * Errors as rs_make_maps.
 */
int rs_tune_batch(const rs_map_request *requests, int32_t n, void *workspace, size_t workspace_bytes,
                  int64_t sample_rays, void *stream, rs_tune_batch_result *result_host);

/* Counters of each map of the last rs_make_maps on this workspace, in request order. Synchronises. */
int rs_batch_read_stats(const void *workspace, int32_t n, rs_map_stats *stats_host, void *stream);

/* ------------------------------------------------------------------------- */
/* Request loop with continuous batching.                                      */
/* A scheduler thread admits requests in arrival order when a slot is free and */
/* their device footprint (lenses, masses, map) fits the server's pool, and    */
/* keeps two launch steps in flight. Each step hands out about slice_ms of GPU  */
/* work as bands of ray rows: requests waiting longer than starve_s since     */
/* submission first (oldest first), then least remaining work first, in whole  */
/* 32-row bands while the budget lasts (the first request always gets one),    */
/* and runs them as one rs_make_maps batch. A                                  */
/* request that arrives while the GPU is busy joins the next step; a small one */
/* then finishes without waiting for large ones. Each finished map equals      */
/* rs_make_map of the same request bit for bit (a map is the integer sum of its */
/* bands).                                                                      */
/* ------------------------------------------------------------------------- */

typedef struct {
    size_t hbm_budget_bytes;  /* device pool for admitted requests (allocated once, by the server) */
    int32_t max_inflight;     /* requests admitted at once (slots), >= 1 */
    int32_t mode;             /* RS_FP32 or RS_MIXED, for every request */
    double slice_ms;          /* target GPU time of one launch step; <= 0 selects 10 ms; four
                                 times that while requests wait for admission */
    double starve_s;          /* a request older than this is served first; <= 0 selects 0.5 s */
    int32_t max_waiting;      /* requests waiting for admission before rs_server_submit returns
                                 RS_EBUSY; <= 0 selects 4096 */
} rs_server_cfg;

typedef struct {
    uint64_t completed, canceled, failed;  /* finished requests by outcome */
    uint64_t steps;                        /* launch steps run */
    uint64_t waiting, active, max_waiting; /* queue depths (now, and the largest seen) */
    uint64_t hbm_in_use_bytes, hbm_peak_bytes;  /* pool bytes held by admitted requests */
    double interactions;                   /* ray-lens pairs computed */
    double gpu_busy_s;                     /* summed step time on the device */
    double maps_per_s;                     /* completed / (last completion - first submission) */
    double latency_p50_s, latency_p99_s;   /* submission -> map in host memory, completed requests */
    double latency_mean_s, latency_max_s;
    uint64_t rejected_busy;                /* submissions refused with RS_EBUSY */
} rs_server_stats;

typedef struct rs_server rs_server;

/* Start a server on the current device: allocates its pool, four streams (two for launch
   steps, one for admission, one for copies back) and pinned host buffers for the step
   counters, starts its thread. */
int rs_server_create(const rs_server_cfg *cfg, rs_server **server);

/*
 * Queue one map. The parameters and the HOST lens arrays are copied before the
 * call returns; map_host (HOST, uint32 [npy][npx], or NULL to discard) must stay
 * valid until rs_server_wait returns for the ticket. The window must hold fewer
 * than 2^32 rays. Errors: RS_EINVAL, RS_EBUSY (cfg.max_waiting requests are already
 * waiting for admission; nothing is queued, try again later), RS_ECANCELED (server
 * stopping), RS_EHIP (the server has stopped after a device error or found no device).
 */
int rs_server_submit(rs_server *server, const rs_map_params *params, const double *lens_xy_host,
                     const double *lens_m_host, int64_t n_lens, uint32_t *map_host, uint64_t *ticket);

/* *done = 1 once the request has finished (completed, cancelled or failed). */
int rs_server_poll(rs_server *server, uint64_t ticket, int *done);

/*
 * Block until the request has finished, then release the ticket. Returns
 * RS_OK (map written, stats and latency filled), RS_ECANCELED, RS_ENOMEM (its
 * footprint exceeds the whole pool) or RS_EHIP (a device error: the server then
 * fails every unfinished request and refuses new ones).
 */
int rs_server_wait(rs_server *server, uint64_t ticket, rs_map_stats *stats, double *latency_s);

/* Cancel a waiting or running request; work already on the device is discarded. */
int rs_server_cancel(rs_server *server, uint64_t ticket);

/* Counters, throughput and latency percentiles of the server so far. */
int rs_server_get_stats(rs_server *server, rs_server_stats *stats);

/* Stop admitting, drop waiting requests, finish running ones, release everything. */
void rs_server_destroy(rs_server *server);

/* ---------------------------------------------------------------------------
 * Map statistics (Section 3.1, Accuracy: the RMS and K-S assessment; Eq. deltam; Section 2, Eq. mu).
 *
 * A count map N (uint32, npix pixels, any layout: every statistic here is over
 * the set of pixels) gives the magnification mu = N / N_rays and the change in
 * magnitude dm = -2.5 log10(mu) of each pixel; a pixel without rays has mu = 0,
 * dm = +inf. Two maps of the same source grid are compared by
 *   - the root-mean-square of dm_a - dm_b over the pixels with rays in both
 *     maps (a pixel empty in either map has no finite difference and is left
 *     out; their number is reported), and
 *   - the two-sample Kolmogorov-Smirnov statistic D of the two dm samples (all
 *     pixels, +inf being the largest value), with its probability
 *     P(KS) = Q((sqrt(n_e) + 0.12 + 0.11 / sqrt(n_e)) D), n_e = npix / 2, where
 *     Q(l) = 2 sum_{j>=1} (-1)^(j-1) exp(-2 j^2 l^2) is the Kolmogorov survival
 *     function (Stephens' effective-size correction).
 * The histogram of counts, divided by npix, is the map's magnification
 * probability distribution P(mu = c / N_rays).
 * All arithmetic is FP64; the pass over the maps is bound by HBM bandwidth.
 * ------------------------------------------------------------------------- */

typedef struct {
    double rms_dm;        /* RMS of dm_a - dm_b over pixels with rays in both maps; NaN if none */
    double ks_d;          /* two-sample K-S statistic D of the dm distributions */
    double ks_p;          /* P(KS) as above */
    double mean_mu_a;     /* sum of map_a / (npix * n_rays_a) */
    double mean_mu_b;
    int64_t n_pix;
    int64_t n_both;       /* pixels in the RMS */
    int64_t n_zero_a;     /* pixels without rays */
    int64_t n_zero_b;
    uint32_t max_a;       /* largest count in each map */
    uint32_t max_b;
} rs_compare_result;

/* N_rays of a map: rays per unit area of the regular shooting grid,
 * (nx / sw)(ny / sh), times the area of one source pixel, (tw / npx)(th / npy)
 * (Section 3.1). Host only. Returns NaN (and sets rs_last_error) on bad params. */
double rs_rays_per_pixel(const rs_map_params *params);

/* max_dev[0] = the largest count of map[0..npix). Enqueued on stream. */
int rs_map_max(const uint32_t *map, int64_t npix, uint32_t *max_dev, void *stream);

/* hist[c] = number of pixels with count c, for c = 0..max_count, and
 * hist[max_count + 1] = number of pixels with a larger count. hist is a device
 * array of max_count + 2 uint64 (overwritten). Enqueued on stream. */
int rs_map_histogram(const uint32_t *map, int64_t npix, uint32_t max_count, uint64_t *hist, void *stream);

/* dm[p] = -2.5 log10(map[p] / n_rays) in FP64 (+inf where map[p] == 0).
 * dm is a device array of npix doubles. Enqueued on stream. */
int rs_delta_m(const uint32_t *map, int64_t npix, double n_rays, double *dm, void *stream);

/* Workspace bytes of rs_compare_maps for count bounds max_a, max_b. */
size_t rs_compare_workspace_bytes(uint32_t max_a, uint32_t max_b);

/* Compare two count maps of npix pixels each (device arrays). max_a and max_b
 * bound the counts of each map (rs_map_max gives them); the workspace is a
 * device buffer of at least rs_compare_workspace_bytes(max_a, max_b) bytes,
 * 256-byte aligned. Synchronous: waits for the stream, then fills
 * *result_host. Returns RS_EINVAL when a count exceeds its bound (result_host
 * still gets the true maxima), RS_ENOMEM when the workspace is too small. */
int rs_compare_maps(const uint32_t *map_a, const uint32_t *map_b, int64_t npix, double n_rays_a,
                    double n_rays_b, uint32_t max_a, uint32_t max_b, void *workspace, size_t workspace_bytes,
                    rs_compare_result *result_host, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* RAYSHOOT_H */
