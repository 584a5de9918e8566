// Entry point without device allocation: rs_make_map_noalloc builds the count
// map with the library's own static device scratch in place of a caller
// workspace, for callers that cannot allocate (HIP graph capture, serving loops
// that forbid hipMalloc). Each device holds its own copy of the array for the
// life of the process; its address is looked up once per device.
#include "rs_internal.h"
#include "rayshoot.h"

#include <mutex>

namespace rs {
int fail(int code, const char *fmt, ...);
int hip_fail(hipError_t e, const char *what);
int enqueue_map_fixed(const rs_map_params *p, const double *lens_xy, const double *lens_m, int64_t n_lens,
                      uint32_t *map, int (*scratch_of_device)(void **), size_t scratch_bytes,
                      hipStream_t stream, void **scratch_used);
}  // namespace rs

using namespace rs;

// The scratch: counters, queue lengths, the re-check queue of one launch, the
// far-field records and, for random rays, the bin arrays and sorted rays. In host
// code this name is only a handle for hipGetSymbolAddress, never an address.
static __device__ __align__(256) unsigned char scratch[RS_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
void *g_scratch[MAX_DEVICES];   // device address of scratch per device; nullptr until looked up

// Device address of this device's scratch (current device), looked up on first use.
int scratch_address(void **out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= MAX_DEVICES) return fail(RS_EINVAL, "device %d out of range", dev);
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!p) return fail(RS_EHIP, "hipGetSymbolAddress(scratch) returned NULL");
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return RS_OK;
}
}  // namespace

extern "C" int rs_make_map_noalloc(const rs_map_params *params, const double *lens_xy, const double *lens_m,
                                   int64_t n_lens, uint32_t *map, rs_map_stats *stats_host, void *stream) {
    void *ws = nullptr;
    hipStream_t s = static_cast<hipStream_t>(stream);
    int rc = enqueue_map_fixed(params, lens_xy, lens_m, n_lens, map, scratch_address, RS_NOALLOC_SCRATCH_BYTES, s,
                               &ws);
    if (rc || !stats_host) return rc;
    unsigned long long c[N_COUNTERS];
    hipError_t e = hipMemcpyAsync(c, static_cast<const char *>(ws) + WS_COUNTERS, sizeof(c),
                                  hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "reading stats");
    stats_host->rays_in_map = c[C_IN];
    stats_host->rays_out = c[C_OUT];
    stats_host->rays_singular = c[C_SING];
    stats_host->rays_rechecked = c[C_RECHECK];
    stats_host->rays_rechecked_direct = c[C_DIRECT];
    stats_host->rays_shot = c[C_IN] + c[C_OUT] + c[C_SING];
    return RS_OK;
}
