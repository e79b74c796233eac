"""Benchmark: single-slice parallel-beam FBP at 512^2, 720 angles, 725 bins on one MI355X.

A step is one whole reconstruction (Ram-Lak filter GEMM + backprojection) of
the seeded 20-ellipse Poisson-noise phantom through the C ABI, inputs resident
in HBM.  Prints one JSON line with throughput, per-step p50/p99, the error
against the FP64 oracle, a roofline entry for the dominant kernel
(backprojection) and the oracle's own throughput on the host cores.

python bench.py [--gpus 1] [--steps 1000] [--warmup 20] [--precision fp32] [--no-cpu-baseline]
               [--no-autotune] [--copy-mb MiB] [--latency-samples 1000] [--kernel-launches 1000]
               [--workload c2|c1]

--workload c1 runs the same measurement on the small 128^2 / 180-angle / 183-bin
slice (a reported side result; the default and the headline line is c2).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "pixel-angle updates/s & slices/s (512², 720 ang) at stated err vs FP64; p99 ms"
UNIT = "pixel-angle updates/s"
FP32_VECTOR_PEAK_TFLOPS = 157.3      # MI355X published FP32 vector peak
FP32_MATRIX_PEAK_TFLOPS = 157.3      # MI355X published FP32 matrix peak
HBM_PEAK_GBS = 8000.0
BP_FLOPS_PER_UPDATE = 7              # coordinate FMA (2) + fraction (1) + lerp (3) + accumulate (1)
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "bp_c2_hbm_traffic.txt")
BP_SOURCES = {"bp_qt_grid_kernel": os.path.join(ROOT, "paper_2109_02174_amd", "csrc", "bp_qt_kernels.hip"),
              "bp_grid_kernel": os.path.join(ROOT, "paper_2109_02174_amd", "csrc", "bp_kernels.hip")}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "bf16", "fp16"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="skip tile autotuning (default shapes, or FBP_FORCE_CONFIG): for profiler runs")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--kernel-launches", type=int, default=1000,
                    help="back-to-back launches each kernel's own duration is averaged over")
    ap.add_argument("--latency-samples", type=int, default=1000,
                    help="requests timed one at a time after the timed region (p50/p99)")
    ap.add_argument("--workload", default="c2", choices=["c2", "c1"],
                    help="c2: 512^2 / 720 angles / 725 bins (default); c1: 128^2 / 180 / 183")
    ap.add_argument("--copy-mb", type=int, default=0,
                    help="after the timed region, one device copy of this many MiB (counter calibration)")
    return ap.parse_args()


def source_hash(path: str) -> str:
    return hashlib.sha256(open(path, "rb").read()).hexdigest()[:16]


def recorded_traffic(kernel: str):
    """HBM bytes per backprojection launch from the committed rocprofv3 counter summary,
    or None when the summary is absent, covers another kernel, or was taken on a
    different source of that kernel."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    fields = {}
    for line in open(TRAFFIC_FILE):
        if "=" in line and not line.lstrip().startswith("#"):
            k, v = line.split("=", 1)
            fields[k.strip()] = v.strip()
    if fields.get("kernel") != kernel or kernel not in BP_SOURCES:
        return None
    if fields.get("bp_source_sha256_16") != source_hash(BP_SOURCES[kernel]):
        return None
    try:
        return int(float(fields["hbm_bytes_per_launch"]))
    except (KeyError, ValueError):
        return None


def time_launches(fn, stream, n: int) -> float:
    """Average device duration (ms) of n back-to-back launches of fn on `stream`.

    Blocker GEMMs are queued first, enough to outlast the host's enqueueing of all n
    launches (about 20 us of host time each, and a 4096^3 GEMM takes about 0.9 ms),
    so that every launch is queued before the first one starts: the events then see
    device time, not host launch gaps, also for kernels shorter than a launch's
    host time.
    """
    import torch
    blocker = torch.empty((4096, 4096), device="cuda")
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    n_block = max(2, math.ceil(n * 20e-6 / 0.8e-3))
    with torch.cuda.stream(stream):
        for _ in range(n_block):
            blocker = blocker @ blocker.T   # device work ahead of the timed launches
        e0.record(stream)
        for _ in range(n):
            fn()
        e1.record(stream)
    e1.synchronize()
    return e0.elapsed_time(e1) / n


def bp_kernel_name(shape_name: str) -> str:
    """The backprojection kernel(s) one launch of a tile shape runs."""
    if "angle chunks" in shape_name:
        return "bp_qt_grid_kernel"
    if "1 angle group" in shape_name:
        return "bp_grid_kernel + combine_parts_kernel (angle-split single slice)"
    return "bp_grid_kernel"


def cpu_baseline(sl, seconds: float):
    """The FP64 oracle timed on the host cores over repeated whole reconstructions,
    with all threads (the reported value) and with one thread (3 runs)."""
    import oracle
    threads = oracle.num_threads()
    oracle.set_num_threads(1)
    one = []
    for _ in range(3):
        t0 = time.perf_counter()
        oracle.fbp(sl.sino, sl.N, sl.dt, sl.angles)
        one.append(time.perf_counter() - t0)
    oracle.set_num_threads(threads)
    times = []
    out = None
    t_end = time.perf_counter() + seconds
    while len(times) < 3 or time.perf_counter() < t_end:
        t0 = time.perf_counter()
        out = oracle.fbp(sl.sino, sl.N, sl.dt, sl.angles)
        times.append(time.perf_counter() - t0)
        if len(times) >= 200:
            break
    times.sort()
    med = times[len(times) // 2]
    upd = sl.N * sl.N * sl.K
    return {
        "value": upd / med, "unit": UNIT, "cores": threads, "kind": "oracle",
        "sample": (f"{len(times)} whole FP64 reconstructions (filter + backprojection) of the "
                   f"{sl.N}x{sl.N}/{sl.K}-angle/{sl.D}-bin slice, median {med * 1e3:.1f} ms each, "
                   f"{threads} OpenMP threads"),
        "slices_per_s": 1.0 / med,
        "value_1_thread": sl.N * sl.N * sl.K / sorted(one)[1],
    }, out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); slices are "
              "independent, so a multi-GPU run would shard them with no exchange.", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_2109_02174_amd as fbp
    from paper_2109_02174_amd import configs, metrics

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    sl = configs.c2_slice() if args.workload == "c2" else configs.c1_slice()
    geom = fbp.Geometry(sl.K, sl.D, sl.N, sl.dt, sl.angles)
    stream = torch.cuda.current_stream()
    tuned = None if args.no_autotune else fbp.fbp_autotune(geom)
    cfg = fbp.fbp_plan_config(geom)
    sino = torch.tensor(sl.sino[None].astype(np.float32), device="cuda")
    img = torch.empty((1, sl.N, sl.N), dtype=torch.float32, device="cuda")
    ws = fbp.alloc_workspace(fbp.fbp_workspace_bytes(geom, 1, args.precision))
    filt = torch.empty_like(sino)

    def step():
        fbp.fbp_reconstruct(geom, sino, out=img, workspace=ws, precision=args.precision)

    # The dominant kernel alone (backprojection) and the filter GEMM alone, same stream,
    # each averaged over back-to-back launches, measured before the throughput run.
    # Besides their own figures they keep the GPU busy for some 35 ms, so that the
    # timed steps find it at the clock it holds under load: an idle GPU takes tens of
    # milliseconds of continuous work to ramp up, which a run of a few steps (under a
    # millisecond) would otherwise measure.
    fbp.fbp_filter(geom, sino, out=filt, precision=args.precision)
    n_k = max(args.kernel_launches, 1)
    bp_ms = time_launches(lambda: fbp.fbp_backproject(geom, filt, out=img), stream, n_k)
    flt_ms = time_launches(lambda: fbp.fbp_filter(geom, sino, out=filt, precision=args.precision),
                           stream, n_k)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    # timed region: exactly `steps` steps back to back, synchronised on both sides
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = wall * 1e3 / args.steps

    # latency, after the timed region: each request submitted alone on an idle GPU and
    # timed from submission to completion on the host (at least 1000 samples)
    n_lat = max(args.latency_samples, 1)
    lat = []
    for _ in range(n_lat):
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        step()
        torch.cuda.synchronize()
        lat.append((time.perf_counter() - t1) * 1e3)
    lat.sort()
    updates = sl.N * sl.N * sl.K
    p50 = lat[len(lat) // 2]
    p99 = lat[min(len(lat) - 1, int(math.ceil(0.99 * len(lat))) - 1)]

    bp_tflops = BP_FLOPS_PER_UPDATE * updates / (bp_ms * 1e-3) / 1e12
    bp_kernel = bp_kernel_name(fbp.fbp_tile_config_name(cfg))
    traffic = recorded_traffic(bp_kernel) if args.workload == "c2" else None   # summary is for c2
    gemm_flops = 2.0 * sl.K * sl.D * sl.D

    if args.copy_mb > 0:
        src = torch.empty(args.copy_mb << 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
    fbp.fbp_reconstruct(geom, sino, out=img, workspace=ws, precision=args.precision)
    torch.cuda.synchronize()
    result_img = img[0].cpu().numpy().astype(np.float64)

    line = {
        "metric": METRIC, "value": updates / (ms_per_step * 1e-3), "unit": UNIT, "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if args.precision == "fp32" else f"{args.precision} filter operands, f32",
        "data": "synthetic (seeded 20-ellipse phantom, analytic sinogram, Poisson I0=1e5)",
        "config": {"workload": f"single slice {sl.N}x{sl.N}, {sl.K} angles in [0,pi), {sl.D} bins",
                   "image": sl.N, "angles": sl.K, "detectors": sl.D, "det_spacing": sl.dt,
                   "filter_precision": args.precision, "tile_config": cfg,
                   "tile_config_name": fbp.fbp_tile_config_name(cfg), "autotuned": tuned},
        "slices_per_s": 1e3 / ms_per_step,
        "latency_ms": {"p50": p50, "p99": p99, "min": lat[0], "max": lat[-1], "samples": len(lat),
                       "timing": "host submit to completion, one request at a time on an idle GPU"},
        "roofline": {"bound": "alu", "achieved": bp_tflops, "peak": FP32_VECTOR_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": bp_tflops / FP32_VECTOR_PEAK_TFLOPS,
                     "traffic": traffic,
                     "kernel": bp_kernel,
                     "kernel_ms": bp_ms, "kernel_launches": n_k, "flops_per_update": BP_FLOPS_PER_UPDATE,
                     "updates_per_launch": updates},
        "filter_gemm": {"kernel_ms": flt_ms, "dense_tflops": gemm_flops / (flt_ms * 1e-3) / 1e12,
                        "peak_tflops": FP32_MATRIX_PEAK_TFLOPS if args.precision == "fp32" else 2500.0,
                        "hbm_gbs": 2 * sl.K * sl.D * 4 / (flt_ms * 1e-3) / 1e9},
    }
    if not args.no_cpu_baseline:
        cb, ref = cpu_baseline(sl, args.cpu_seconds)
        line["cpu_baseline"] = cb
        line["error_vs_fp64"] = metrics.compare(result_img, ref, sl.value_range)
    else:
        line["cpu_baseline"] = None
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
