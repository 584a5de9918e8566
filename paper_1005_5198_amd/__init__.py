"""MI355X-native inverse ray-shooting for gravitational-microlensing magnification maps.

Public entry points (loaded lazily so that importing the package, e.g. for
``paper_1005_5198_amd.workloads``, does not need the HIP library):

    make_map(params, lens_xy, lens_m=None, mode="mixed") -> torch.uint32 [npy, npx]
    shoot_map(lens_xy, masses, sigma_star, sigma_c, gamma, shoot, src, mode="mixed")
                                          the same with the model and grids given directly
    make_map_noalloc(params, lens_xy, ...)  make_map with no device allocation in the library
    ray_pixels(params, lens_xy, lens_m=None, mode="mixed") -> torch.int32 [rays in window]
    read_stats(workspace) -> dict
    make_maps(maps) / Batch / Server      many maps: one persistent launch; a request loop
    compare_maps(map_a, map_b, n_rays_a)  RMS of dm and the K-S test between two maps
    delta_m / histogram / map_max         per-pixel dm, count histogram, largest count

``params`` is a dict with the fields of ``rs_map_params`` (see include/rayshoot.h);
``map_params(sigma_star, sigma_c, gamma, shoot, src)`` builds one.
"""
_API = ("make_map", "make_map_noalloc", "shoot_map", "map_params", "ray_pixels", "read_stats", "workspace_bytes", "new_workspace", "to_params",
        "lens_tensors", "profile_enable", "profile_read", "version", "tune", "set_shape", "tune_save",
        "tune_load", "make_maps", "Batch", "Server", "rays_per_pixel", "map_max", "histogram", "delta_m",
        "compare_maps", "compare_workspace_bytes")


def __getattr__(name):
    if name in _API:
        from . import api
        return getattr(api, name)
    raise AttributeError(name)
