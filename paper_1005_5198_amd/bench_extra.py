"""Batched and served measurements for bench.py.

batched(): the 64-map batch (config 3 distribution) in one persistent launch
sequence vs the same maps one at a time through rs_make_map; every batched map
is compared with its one-at-a-time result (bit-identical).
The other legs: the request loop (served), map statistics, the far-field mode,
random rays, the plain-FP32 mode's accuracy, and two more single-map workloads.
"""
from __future__ import annotations

import time

import numpy as np
import torch

from . import workloads as w


def batched(rs, n_maps: int = 64, mode: str = "mixed", repeats: int = 1, check: bool = True,
            tune: bool = True) -> dict:
    """The config-3 batch in one persistent launch (tuned first: thread shape and persistent
    grid timed on a band of every map) against the same maps one at a time (the single-map
    tuner's choice per map signature)."""
    specs = w.config3(n_maps)
    items = [(s.params, s.lens_xy, s.lens_m) for s in specs]
    b = rs.Batch(items, mode=mode)
    inter = b.interactions
    tuned = b.tune() if tune else None
    b.run()
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(repeats):
        outs = b.run()
    torch.cuda.synchronize()
    dt_batch = (time.perf_counter() - t) / repeats
    batch_maps = [o.cpu().numpy() for o in outs]
    # one at a time, same inputs already on the device
    plain_out = [torch.empty_like(o) for o in outs]
    # one workspace, sized for the largest map, reused by the sequential launches on one stream
    ws = torch.empty(max(rs.workspace_bytes(p, xy.shape[0], mode) for p, (xy, _) in zip(b.params, b.lenses)),
                     dtype=torch.uint8, device="cuda")
    for p, (xy, m), o in zip(b.params, b.lenses, plain_out):
        rs.make_map(p, xy, m, mode=mode, out=o, workspace=ws)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(repeats):
        for p, (xy, m), o in zip(b.params, b.lenses, plain_out):
            rs.make_map(p, xy, m, mode=mode, out=o, workspace=ws)
    torch.cuda.synchronize()
    dt_plain = (time.perf_counter() - t) / repeats
    identical = None
    if check:
        identical = all(np.array_equal(a, o.cpu().numpy()) for a, o in zip(batch_maps, plain_out))
    return {"workload": f"config3: {n_maps} maps (sigma*~U[0.2,0.8], s~U[0,0.5], gamma~U[0,0.4], "
                        f"256^2-1024^2 px, 200 rays/px), {mode} mode",
            "maps": n_maps, "interactions": inter,
            "batched_maps_per_s": n_maps / dt_batch, "batched_value": inter / dt_batch,
            "plain_maps_per_s": n_maps / dt_plain, "plain_value": inter / dt_plain,
            "speedup": dt_plain / dt_batch, "batched_s": dt_batch, "plain_s": dt_plain,
            "identical_to_plain": identical,
            "tuned": None if tuned is None else {
                "rays_per_lane": tuned["best"]["rays_per_lane"], "blocks_per_cu": tuned["best"]["blocks_per_cu"],
                "sample_ms": tuned["best"]["ms"], "candidates": len(tuned["candidates"]),
                "sample_interactions": tuned["sample_interactions"]}}


def _percentiles(lat):
    a = np.sort(np.asarray(lat))
    def rank(p):
        k = int(np.ceil(p / 100.0 * len(a)))
        return float(a[min(max(k, 1), len(a)) - 1])
    return rank(50), rank(99)


def served(rs, n_requests: int = 48, rho: float = 0.8, mode: str = "mixed", seed: int = 4,
           budget_bytes: int = 2 << 30, max_inflight: int = 16, slice_ms: float = 10.0,
           starve_s: float = 0.5) -> dict:
    """Poisson arrivals of config-3-distributed requests (each with its own lens set):
    the request loop vs the same arrivals served one at a time by plain rs_make_map calls."""
    import threading

    _, specs = w.config4_arrivals(n_requests, 1.0, seed=seed)
    # plain service rate of this request mix (one at a time, inputs from the host, map back to the host)
    def plain_one(s):
        out = rs.make_map(s.params, s.lens_xy, s.lens_m, mode=mode)
        return out.cpu().numpy()
    plain_one(specs[0])
    head = specs[: min(8, n_requests)]
    t = time.perf_counter()
    for s in head:
        plain_one(s)
    plain_ips = sum(s.interactions for s in head) / (time.perf_counter() - t)
    mean_inter = sum(s.interactions for s in specs) / n_requests
    rate = rho * plain_ips / mean_inter          # requests per second at load rho
    gaps = np.random.default_rng(seed).exponential(1.0 / rate, size=n_requests)
    arrivals = np.cumsum(gaps) - gaps[0]

    # one at a time (FIFO): latency = completion - arrival
    lat_plain = []
    t0 = time.perf_counter()
    for s, a in zip(specs, arrivals):
        now = time.perf_counter() - t0
        if now < a:
            time.sleep(a - now)
        plain_one(s)
        lat_plain.append(time.perf_counter() - t0 - a)
    span_plain = time.perf_counter() - t0

    # the request loop
    tickets = [None] * n_requests
    with rs.Server(hbm_budget_bytes=budget_bytes, max_inflight=max_inflight, mode=mode, slice_ms=slice_ms,
                   starve_s=starve_s) as srv:
        t0 = time.perf_counter()

        def feed():
            for k, (s, a) in enumerate(zip(specs, arrivals)):
                now = time.perf_counter() - t0
                if now < a:
                    time.sleep(a - now)
                tickets[k] = srv.submit(s.params, s.lens_xy, s.lens_m)

        th = threading.Thread(target=feed)
        th.start()
        th.join()
        served_maps = [srv.wait(tk)[0] for tk in tickets]
        span_served = time.perf_counter() - t0
        st = srv.stats()
    identical = all(np.array_equal(m, plain_one(s)) for m, s in zip(served_maps[:8], specs[:8]))
    p50p, p99p = _percentiles(lat_plain)
    inter = sum(s.interactions for s in specs)
    return {"workload": f"config4: {n_requests} Poisson requests at rho={rho} of the one-at-a-time rate "
                        f"({rate:.2f}/s), config-3 distribution, {mode} mode, device pool {budget_bytes >> 20} MiB",
            "requests": n_requests, "rho": rho, "arrival_rate_per_s": rate, "interactions": inter,
            "hbm_budget_bytes": budget_bytes,
            "served_maps_per_s": st["maps_per_s"], "served_p50_s": st["latency_p50_s"],
            "served_p99_s": st["latency_p99_s"], "served_span_s": span_served, "served_steps": st["steps"],
            "served_max_waiting": st["max_waiting"], "served_hbm_peak_bytes": st["hbm_peak_bytes"],
            "plain_maps_per_s": n_requests / span_plain, "plain_p50_s": p50p, "plain_p99_s": p99p,
            "plain_span_s": span_plain, "identical_first8": identical}


def served_legs(rs, n_requests: int = 96, mode: str = "mixed") -> dict:
    """The request loop at load 0.8 and 1.2 of the one-at-a-time rate, and at 0.8 with a
    device pool of 8 MiB, small enough that admission by footprint makes requests wait."""
    return {"rho_0.8": served(rs, n_requests=n_requests, rho=0.8, mode=mode),
            "rho_1.2": served(rs, n_requests=n_requests, rho=1.2, mode=mode),
            "rho_0.8_budget_8MiB": served(rs, n_requests=n_requests, rho=0.8, mode=mode, budget_bytes=8 << 20)}


def map_stats(rs, side: int = 4096, n_rays_a: float = 500.0, n_rays_b: float = 1000.0, reps: int = 20) -> dict:
    """Comparison of two side^2 count maps (the accuracy assessment's largest map size).

    Reports the whole rs_compare_maps call (five launches, the result read back),
    the histogram and dm calls, each averaged over reps after one warm-up, and
    the HBM rate of the comparison counted as the 8 bytes per pixel pair its
    pass reads."""
    a, b = w.count_map_pair(side, side, n_rays_a, n_rays_b, seed=16, spike_frac=2e-4)
    da, db = torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()
    ma, mb = rs.map_max(da), rs.map_max(db)
    ws = torch.empty(int(rs.compare_workspace_bytes(ma, mb)), dtype=torch.uint8, device="cuda")
    res = rs.compare_maps(da, db, n_rays_a, n_rays_b, ma, mb, workspace=ws)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(reps):
        res = rs.compare_maps(da, db, n_rays_a, n_rays_b, ma, mb, workspace=ws)
    dt_cmp = (time.perf_counter() - t) / reps

    def timed(fn):
        fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    ms_hist = timed(lambda: rs.histogram(da, ma))
    ms_dm = timed(lambda: rs.delta_m(da, n_rays_a))
    ms_max = timed(lambda: rs.map_max(da, out=torch.empty(1, dtype=torch.int32, device="cuda")))
    npix = side * side
    return {"pixels": npix, "max_counts": [ma, mb], "compare_ms": dt_cmp * 1e3,
            "compare_pass_bytes": 8 * npix, "compare_GBps_wall": 8 * npix / dt_cmp / 1e9,
            "histogram_ms": ms_hist, "delta_m_ms": ms_dm, "map_max_ms": ms_max,
            "delta_m_GBps": 12 * npix / (ms_dm * 1e-3) / 1e9,
            "rms_dm": res["rms_dm"], "ks_d": res["ks_d"], "ks_p": res["ks_p"]}


def phi_fiducial_both(rs, band_rows: int = 2400) -> dict:
    """The whole Phi_fiducial map twice: in far-field mode (one call, timed on the
    process's first call and on a second one), then with the direct kernel band by band
    (about 8 minutes, one progress line per band on stderr); the two count maps are compared
    pixel for pixel."""
    import sys
    spec = w.phi_fiducial()
    p = spec.params
    xy, _ = rs.lens_tensors(spec.lens_xy)
    ff = torch.zeros((p["npy"], p["npx"]), dtype=torch.uint32, device="cuda")
    ws = rs.new_workspace(p, spec.n_lens, "farfield")
    times = []
    for _ in range(2):
        torch.cuda.synchronize()
        t = time.perf_counter()
        rs.make_map(p, xy, None, mode="farfield", out=ff, workspace=ws)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t)
    t_first, t_ff = times
    st_ff = rs.read_stats(ws)
    print(f"phi_fiducial far field: {t_first:.3f} s first call, {t_ff:.3f} s second", file=sys.stderr, flush=True)
    r = phi_fiducial(rs, full=True, band_rows=band_rows, mode="mixed", out_map=True)
    direct = r.pop("map")
    diff = int((direct != ff).sum().item())
    r.update({"farfield_seconds": t_ff, "farfield_first_call_seconds": t_first,
              "farfield_rate_direct_equivalent": spec.interactions / t_ff,
              "farfield_recheck_fraction": st_ff["rays_rechecked"] / spec.n_rays,
              "pixels_differing": diff, "maps_equal": diff == 0})
    return r


def phi_fiducial(rs, rows: int = 64, full: bool = False, band_rows: int = 2400, mode: str = "mixed",
                 out_map: bool = False) -> dict:
    """The 1e6-lens, 2500^2-pixel, 3.1e15-interaction map of Section 2's Phi_fiducial (the cost model Phi).

    By default a band of `rows` ray rows through the middle of the map is timed
    (3.6e12 interactions at 64 rows) and the full map's time is projected from
    its rate; with full=True the whole map is made band by band (about 8 minutes
    on one GPU), printing one progress line per band."""
    import sys
    spec = w.phi_fiducial()
    p = spec.params
    nx, ny = p["nx"], p["ny"]
    xy, _ = rs.lens_tensors(spec.lens_xy)
    if not full:
        j0 = ny // 2 - rows // 2
        sub = spec.window(0, nx, j0, j0 + rows)
        ws = rs.new_workspace(sub.params, spec.n_lens, mode)
        torch.cuda.synchronize()
        t = time.perf_counter()
        rs.make_map(sub.params, xy, None, mode=mode, workspace=ws)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        st = rs.read_stats(ws)
        rate = sub.interactions / dt
        return {"workload": spec.name, "rows": rows, "rays": sub.n_rays, "lenses": spec.n_lens,
                "interactions": sub.interactions, "seconds": dt, "rate": rate,
                "pct_fp32_peak": 10.0 * rate / 157.3e12, "recheck_fraction": st["rays_rechecked"] / sub.n_rays,
                "projected_full_map_s": spec.interactions / rate}
    out = torch.zeros((p["npy"], p["npx"]), dtype=torch.uint32, device="cuda")
    ws = None
    total = {"rays_in_map": 0, "rays_out": 0, "rays_singular": 0, "rays_rechecked": 0}
    t = time.perf_counter()
    for j0 in range(0, ny, band_rows):
        j1 = min(ny, j0 + band_rows)
        sub = spec.window(0, nx, j0, j1)
        if ws is None:
            ws = rs.new_workspace(sub.params, spec.n_lens, mode)
        rs.make_map(sub.params, xy, None, mode=mode, out=out, accumulate=True, workspace=ws)
        st = rs.read_stats(ws)
        for k in total:
            total[k] += st[k]
        print(f"phi_fiducial band rows {j0}..{j1} of {ny}: {time.perf_counter() - t:.1f} s", file=sys.stderr,
              flush=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t
    rate = spec.interactions / dt
    res = {"workload": spec.name, "rows": ny, "rays": spec.n_rays, "lenses": spec.n_lens,
           "interactions": spec.interactions, "seconds": dt, "rate": rate,
           "pct_fp32_peak": 10.0 * rate / 157.3e12, "recheck_fraction": total["rays_rechecked"] / spec.n_rays,
           "rays_in_map": total["rays_in_map"], "rays_out": total["rays_out"],
           "map_sum": int(out.to(torch.int64).sum().item())}
    if out_map:
        res["map"] = out
    return res


def far_field(rs, reps: int = 5) -> dict:
    """The config-2 map in RS_FARFIELD mode (per-patch FP64 local expansion of the distant
    lenses, bound, FP64 re-check): time per map, the direct-sum interactions it stands for per
    second, and whether the map equals the mixed (direct) mode's, bit for bit."""
    spec = w.config2()
    xy, _ = rs.lens_tensors(spec.lens_xy)
    ws = rs.new_workspace(spec.params, spec.n_lens, "farfield")   # holds the mixed mode's needs too
    out = torch.empty((spec.params["npy"], spec.params["npx"]), dtype=torch.uint32, device="cuda")
    ref = rs.make_map(spec.params, xy, None, mode="mixed", workspace=ws).clone()
    rs.make_map(spec.params, xy, None, mode="farfield", out=out, workspace=ws)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(reps):
        rs.make_map(spec.params, xy, None, mode="farfield", out=out, workspace=ws)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t) / reps
    st = rs.read_stats(ws)
    return {"workload": "config2", "ms_per_map": dt * 1e3, "maps_per_s": 1.0 / dt,
            "direct_equivalent_interactions_per_s": spec.interactions / dt,
            "recheck_fraction": st["rays_rechecked"] / spec.n_rays,
            "equals_mixed_map": bool(torch.equal(out, ref))}


def random_rays(rs, reps: int = 3, mode: str = "mixed") -> dict:
    """The config-2 map with Philox-random ray positions (the paper's GPU code's sampling):
    time per map and interactions/s against the regular grid's, plus the re-check fraction."""
    spec = w.config2()
    p = dict(spec.params)
    p.update(random_rays=1, seed=2)
    xy, _ = rs.lens_tensors(spec.lens_xy)
    ws = rs.new_workspace(p, spec.n_lens, mode)
    out = torch.empty((p["npy"], p["npx"]), dtype=torch.uint32, device="cuda")
    rs.make_map(p, xy, None, mode=mode, out=out, workspace=ws)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(reps):
        rs.make_map(p, xy, None, mode=mode, out=out, workspace=ws)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t) / reps
    st = rs.read_stats(ws)
    return {"workload": "config2, random rays", "mode": mode, "ms_per_map": dt * 1e3,
            "interactions_per_s": spec.interactions / dt, "recheck_fraction": st["rays_rechecked"] / spec.n_rays}


def fp32_accuracy(rs) -> dict:
    """Plain-FP32 mode against the definition on the config-2 map (19200 x 3840 rays, 17240
    lenses): the fraction of rays whose pixel changes, from the per-ray pixel indices of both
    modes (the mixed mode's equal the definition's ray for ray), and the relative L1 error
    sum|fp32 - exact| / sum(exact) of the count map."""
    spec = w.config2()
    xy, _ = rs.lens_tensors(spec.lens_xy)
    pix_m = rs.ray_pixels(spec.params, xy, None, mode="mixed")
    pix_f = rs.ray_pixels(spec.params, xy, None, mode="fp32")
    changed = int((pix_m != pix_f).sum().item())
    del pix_m, pix_f
    map_m = rs.make_map(spec.params, xy, None, mode="mixed").to(torch.int64)
    map_f = rs.make_map(spec.params, xy, None, mode="fp32").to(torch.int64)
    l1 = int((map_f - map_m).abs().sum().item())
    total = int(map_m.sum().item())
    return {"workload": "config2", "rays": spec.n_rays, "rays_changed_pixel": changed,
            "changed_fraction": changed / spec.n_rays, "budget": 1e-4,
            "map_relative_l1": l1 / max(total, 1)}


def _time_map(rs, spec, mode: str, reps: int) -> tuple:
    xy, m = rs.lens_tensors(spec.lens_xy, spec.lens_m)
    ws = rs.new_workspace(spec.params, spec.n_lens, mode)
    out = torch.empty((spec.params["npy"], spec.params["npx"]), dtype=torch.uint32, device="cuda")
    rs.make_map(spec.params, xy, m, mode=mode, out=out, workspace=ws)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(reps):
        rs.make_map(spec.params, xy, m, mode=mode, out=out, workspace=ws)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t) / reps
    return dt, rs.read_stats(ws), out


def single_map(rs, spec, label: str, reps: int = 3, modes=("mixed", "fp32", "farfield")) -> dict:
    """One workload in each mode: time per map, interactions/s and %FP32 peak (direct modes),
    the re-check fraction, and whether the far-field map equals the mixed one."""
    res = {"workload": label, "rays": spec.n_rays, "lenses": spec.n_lens, "interactions": spec.interactions}
    maps = {}
    for mode in modes:
        dt, st, out = _time_map(rs, spec, mode, reps)
        r = {"ms_per_map": dt * 1e3, "interactions_per_s": spec.interactions / dt,
             "recheck_fraction": st["rays_rechecked"] / max(spec.n_rays, 1)}
        if mode != "farfield":
            r["pct_fp32_peak"] = 10.0 * spec.interactions / dt / 157.3e12
        res[mode] = r
        maps[mode] = out
    if "mixed" in maps and "farfield" in maps:
        res["farfield_equals_mixed"] = bool(torch.equal(maps["mixed"], maps["farfield"]))
    return res


def config1(rs, reps: int = 3) -> dict:
    """The 32768^2-ray paper-scale map (462 lenses, 1024^2 px): plain FP32 vs mixed (and far field)."""
    return single_map(rs, w.config1(), "config1: sigma*=0.4, 462 unit lenses (R=34), 32768^2 rays over 40^2, "
                                       "1024^2 px source of side 20", reps)


def paper_fig1_point(rs, reps: int = 2) -> dict:
    """The paper's Section 3.1 parameter point sigma=0.4, gamma=0 at 1024^2 px and 2000 rays per
    pixel (N* = 558 with the paper-rule disc; 5.8e9 rays, 3.25e12 interactions)."""
    spec = w.paper_point(0.4, 0.0)
    return single_map(rs, spec, "paper point sigma=0.4 gamma=0: 1024^2 px, 2000 rays/px, paper-rule lens disc",
                      reps, modes=("mixed", "farfield"))
