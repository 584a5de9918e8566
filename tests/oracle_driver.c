/*
 * The FP64 oracle (oracle/oracle.c, included whole) run from a file of inputs,
 * for builds with AddressSanitizer + UndefinedBehaviorSanitizer or
 * ThreadSanitizer (tests/test_oracle_sanitized.py). Reads the parameters, the
 * lenses and the masses, runs oracle_make_map and oracle_ray_pixels, and writes
 * every output for comparison with the ordinary build.
 *
 * input:  oracle_params, int64 n_lens, int64 has_masses, double xy[2n], double m[n]
 * output: int32 rc_map, int32 rc_pix, uint64 counts[4], uint32 map[npy*npx],
 *         int64 near[2 * min(counts[3], 4096)], int64 pix[rays], double u[rays], v[rays]
 */
#include "../oracle/oracle.c"

#include <stdio.h>

static int read_all(FILE *f, void *dst, size_t bytes)
{
    return bytes == 0 || fread(dst, 1, bytes, f) == bytes;
}

int main(int argc, char **argv)
{
    if (argc < 4) return 2;
    FILE *f = fopen(argv[1], "rb");
    if (!f) return 3;
    oracle_params p;
    int64_t n = 0, has_m = 0;
    if (!read_all(f, &p, sizeof(p)) || !read_all(f, &n, 8) || !read_all(f, &has_m, 8) || n < 0) return 4;
    double *xy = malloc(16 * (size_t)n + 16);
    double *m = has_m ? malloc(8 * (size_t)n + 8) : NULL;
    if (!xy || (has_m && !m)) return 5;
    if (!read_all(f, xy, 16 * (size_t)n) || (has_m && !read_all(f, m, 8 * (size_t)n))) return 6;
    fclose(f);
    const int threads = atoi(argv[3]);
    const size_t npix = (size_t)p.npx * (size_t)p.npy;
    const size_t rays = (size_t)((p.i1 - p.i0) * (p.j1 - p.j0));
    uint32_t *map = malloc(4 * npix + 4);
    uint64_t counts[4] = {0, 0, 0, 0};
    const int64_t near_cap = 4096;
    int64_t *near = malloc(16 * (size_t)near_cap);
    int64_t *pix = malloc(8 * rays + 8);
    double *u = malloc(8 * rays + 8), *v = malloc(8 * rays + 8);
    if (!map || !near || !pix || !u || !v) return 7;
    const int32_t rc_map = oracle_make_map(&p, n ? xy : NULL, m, n, map, counts, 1e-9, near, near_cap, threads);
    const int32_t rc_pix = oracle_ray_pixels(&p, n ? xy : NULL, m, n, pix, u, v, threads);
    FILE *o = fopen(argv[2], "wb");
    if (!o) return 8;
    const size_t n_near = counts[3] < (uint64_t)near_cap ? (size_t)counts[3] : (size_t)near_cap;
    fwrite(&rc_map, 4, 1, o);
    fwrite(&rc_pix, 4, 1, o);
    fwrite(counts, 8, 4, o);
    fwrite(map, 4, npix, o);
    fwrite(near, 16, n_near, o);
    fwrite(pix, 8, rays, o);
    fwrite(u, 8, rays, o);
    fwrite(v, 8, rays, o);
    fclose(o);
    free(xy);
    free(m);
    free(map);
    free(near);
    free(pix);
    free(u);
    free(v);
    return 0;
}
