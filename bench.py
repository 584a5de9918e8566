"""Benchmark: inverse ray-shooting magnification maps on one MI355X.

One step = one whole magnification map of the high-optical-depth workload
(sigma* = 0.8, gamma = 0.3, 17240 unit lenses in a disc of radius 146.8,
19200 x 3840 rays at spacing 0.0125 over a 240 x 48 shooting rectangle,
1024^2-pixel source map of side 20; 1.271e12 ray-lens interactions) in the
oracle-matching mixed mode (FP32 deflection + FP64 edge re-check).
Inputs (lenses) are resident in HBM before the timed region.

Prints ONE JSON line:
  value       ray-lens interactions per second over the timed steps
  roofline    FP32 VALU roofline of the deflection kernel: algorithmic
              10 FLOP per interaction / mean kernel duration (HIP events on
              the kernel's stream), against the 157.3 TFLOP/s FP32 peak
  cpu_baseline  the FP64 oracle timed on the host cores on a bounded sample
              of the same map (a band of ray rows)
Also reported: the plain-FP32 mode rate, the re-check fraction, the 64-map
batch (one persistent launch) against the same maps one at a time, and the
request loop (continuous batching, Poisson arrivals) against the same arrivals
served one at a time, with maps/s and p50/p99 latency, the map comparison
(RMS of dm, K-S test) of two 4096^2 maps, and the same map in the far-field
expansion mode (same count map, far fewer operations).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import hashlib
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP32_PEAK_TFLOPS = 157.3       # 256 CU x 2.4 GHz x 128 FP32 lanes x 2 FLOP (FMA)
FLOP_PER_INTERACTION = 10      # the paper's N_FLOP (Section 2, Phi); one deflection term
METRIC = "ray·lens interactions/s (%FP32 peak); maps/s + p50/p99 latency, batched vs plain"

# HBM bytes per launch of the mixed-mode deflection kernel on this workload: rocprofv3 --pmc
# FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0 KiB (factors from a 1 GiB copy), from the counters in
# profiles/shoot_kernel_config2.md, taken with the kernel sources whose digest follows. When any
# of those sources differs, the figure no longer describes the kernel and is reported as null.
TRAFFIC_BYTES_PER_LAUNCH = 1.480e9
TRAFFIC_SOURCES = tuple(os.path.join("paper_1005_5198_amd", "csrc", f) for f in (
    "shoot.hip", "shoot_common.h", "recheck_ray.h", "philox.h", "rs_internal.h", "rs_layout.h")) + (
    os.path.join("include", "rayshoot.h"),)
TRAFFIC_SOURCES_DIGEST = "dabdd5d46d8c4c59"


def kernel_sources_digest() -> str:
    h = hashlib.sha256()
    for name in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic():
    """The counters' bytes per launch when they were taken on the sources built here, else None."""
    return TRAFFIC_BYTES_PER_LAUNCH if kernel_sources_digest() == TRAFFIC_SOURCES_DIGEST else None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--mode", default="mixed", choices=("mixed", "fp32"))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=20.0, help="target CPU time of the oracle sample")
    ap.add_argument("--no-batched", action="store_true", help="skip the 64-map batch vs one-at-a-time")
    ap.add_argument("--no-serve", action="store_true", help="skip the request loop vs one-at-a-time")
    ap.add_argument("--no-stats", action="store_true", help="skip the map-comparison statistics timing")
    ap.add_argument("--no-farfield", action="store_true", help="skip the far-field expansion mode timing")
    ap.add_argument("--no-tune", action="store_true", help="keep the default thread shape (skip the autotuner)")
    ap.add_argument("--no-random", action="store_true", help="skip the random-ray map timing")
    ap.add_argument("--no-accuracy", action="store_true",
                    help="skip the plain-FP32 mode's changed-ray fraction and map error on the config-2 map")
    ap.add_argument("--no-other-maps", action="store_true",
                    help="skip the 32768^2-ray map and the paper's sigma=0.4 point (each mode)")
    ap.add_argument("--serve-requests", type=int, default=96,
                    help="requests per request-loop leg (load 0.8, 1.2, and 0.8 with an 8 MiB pool)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy three times (scales HBM byte counters)")
    return ap.parse_args()


def copy_calibration():
    """A plain copy of known size: 1 GiB read + 1 GiB written per launch, three launches."""
    import torch
    n = 1 << 28
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_per_launch": n * 4, "launches": 3}), flush=True)


def cpu_baseline(spec, target_s: float):
    """Time the FP64 oracle on a band of ray rows of the same map, all host cores (<= 16)."""
    import oracle
    oracle.build(force=False)
    threads = max(1, min(len(os.sched_getaffinity(0)), 16))
    nx = spec.params["nx"]
    # calibrate on a thin band, then size the sample to about target_s seconds
    rows = 24
    j0 = spec.params["ny"] // 2
    sub = spec.window(0, nx, j0, j0 + rows)
    t = time.perf_counter()
    oracle.make_map(sub.params, sub.lens_xy, sub.lens_m, nthreads=threads)
    dt = time.perf_counter() - t
    rate = sub.interactions / max(dt, 1e-6)
    rows = int(max(4, min(spec.params["ny"] - j0, target_s * rate / (nx * spec.n_lens))))
    sub = spec.window(0, nx, j0, j0 + rows)
    t = time.perf_counter()
    oracle.make_map(sub.params, sub.lens_xy, sub.lens_m, nthreads=threads)
    dt = time.perf_counter() - t
    # the whole 1024^2-ray, 462-lens map on one core
    from paper_1005_5198_amd import workloads as w
    c0 = w.config0()
    t = time.perf_counter()
    oracle.make_map(c0.params, c0.lens_xy, c0.lens_m, nthreads=1)
    dt0 = time.perf_counter() - t
    return {"value": sub.interactions / dt, "unit": "ray·lens/s", "cores": threads, "kind": "oracle",
            "sample": f"rows {j0}..{j0 + rows} of the {nx}x{spec.params['ny']}-ray map "
                      f"({sub.n_rays} rays x {spec.n_lens} lenses, {dt:.1f} s)",
            "cpu": _cpu_model(), "host_cpus": os.cpu_count(),
            "one_core_small_map": {"value": c0.interactions / dt0, "unit": "ray·lens/s", "seconds": dt0,
                                   "sample": "the whole 1024^2-ray, 462-lens map"}}


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              f"(the multi-GPU design shards ray rows and sum-reduces the uint32 maps).", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration()
        return
    import torch
    import paper_1005_5198_amd as rs
    from paper_1005_5198_amd import workloads as w

    torch.cuda.set_device(0)
    spec = w.config2()
    xy, m = rs.lens_tensors(spec.lens_xy, spec.lens_m)
    ws = rs.new_workspace(spec.params, spec.n_lens, args.mode)
    out = torch.empty((spec.params["npy"], spec.params["npx"]), dtype=torch.uint32, device="cuda")
    tuned = None
    if not args.no_tune:   # untimed: the autotuner times each thread shape on a band of the map
        tuned = rs.tune(spec.params, xy, m, mode=args.mode)

    for _ in range(args.warmup):
        rs.make_map(spec.params, xy, m, mode=args.mode, out=out, workspace=ws)
    torch.cuda.synchronize()

    rs.profile_enable(True)
    rs.profile_read()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        rs.make_map(spec.params, xy, m, mode=args.mode, out=out, workspace=ws)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    kernel_ms, launches, inter_launched = rs.profile_read()
    rs.profile_enable(False)
    stats = rs.read_stats(ws)

    inter = spec.interactions
    value = inter * args.steps / elapsed
    ms_per_step = elapsed * 1e3 / args.steps
    achieved_tflops = FLOP_PER_INTERACTION * inter_launched / (kernel_ms * 1e-3) / 1e12
    result = {
        "metric": METRIC,
        "value": value,
        "unit": "ray·lens/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded lens disc; no dataset)",
        "config": {"workload": "config2: sigma*=0.8 gamma=0.3, 17240 unit lenses (R=146.8), "
                               "19200x3840 rays over 240x48, 1024^2 px source of side 20, "
                               f"{args.mode} mode",
                   "rays": spec.n_rays, "lenses": spec.n_lens, "interactions_per_map": inter,
                   "mode": args.mode},
        "pct_fp32_peak": FLOP_PER_INTERACTION * value / (FP32_PEAK_TFLOPS * 1e12),
        "maps_per_s": args.steps / elapsed,
        "recheck_fraction": stats["rays_rechecked"] / spec.n_rays,
        # wall time per map outside the deflection launches: map fill, super-patch records,
        # the FP64 re-check stages and launch gaps, and its share of the step
        "non_deflection_ms_per_map": ms_per_step - kernel_ms / args.steps,
        "non_deflection_share": (ms_per_step - kernel_ms / args.steps) / ms_per_step,
        "roofline": {"bound": "alu", "achieved": achieved_tflops, "peak": FP32_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved_tflops / FP32_PEAK_TFLOPS,
                     "traffic": measured_traffic(), "traffic_sources_digest": kernel_sources_digest(),
                     "kernel": "shoot_kernel (deflection + binning)",
                     "launches": launches, "mean_launch_ms": kernel_ms / max(launches, 1)},
        "thread_shape": None if tuned is None else tuned["shapes"][tuned["best"]]["rays_per_lane"],
    }
    if args.mode == "mixed":
        # the plain-FP32 mode on the same map, for comparison
        ws32 = rs.new_workspace(spec.params, spec.n_lens, "fp32")
        rs.make_map(spec.params, xy, m, mode="fp32", out=out, workspace=ws32)
        torch.cuda.synchronize()
        n32 = max(2, args.steps // 2)
        t = time.perf_counter()
        for _ in range(n32):
            rs.make_map(spec.params, xy, m, mode="fp32", out=out, workspace=ws32)
        torch.cuda.synchronize()
        result["fp32_mode_value"] = inter * n32 / (time.perf_counter() - t)
    if not (args.no_batched and args.no_serve and args.no_stats and args.no_farfield and args.no_random
            and args.no_other_maps and args.no_accuracy):
        from paper_1005_5198_amd import bench_extra
        if not args.no_batched:
            result["batched"] = bench_extra.batched(rs, mode=args.mode)
        if not args.no_serve:
            result["served"] = bench_extra.served_legs(rs, n_requests=args.serve_requests, mode=args.mode)
        if not args.no_stats:
            result["map_stats"] = bench_extra.map_stats(rs)
        if not args.no_farfield:
            result["far_field"] = bench_extra.far_field(rs)
        if not args.no_random:
            result["random_rays"] = bench_extra.random_rays(rs, mode=args.mode)
        if not args.no_accuracy:
            result["fp32_accuracy"] = bench_extra.fp32_accuracy(rs)
        if not args.no_other_maps:
            result["config1"] = bench_extra.config1(rs)
            result["paper_point"] = bench_extra.paper_fig1_point(rs)
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(spec, args.cpu_seconds)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
