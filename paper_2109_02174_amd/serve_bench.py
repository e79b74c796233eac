"""Serving benchmark: Poisson arrivals of mixed-geometry reconstruction requests.

Each request is a stack of U{1..64} slices of one geometry drawn as in the
mixed batch (side {256,384,512,1024}, angles {360,720,1440}, detectors
ceil(sqrt(2) side)+2), FP32.  Sinograms are placed in HBM before the run (a pool
of 64 seeded phantom slices per geometry that requests read from; host-to-device
transfer is outside the measurement).  The server admits requests under a 200 GB
HBM budget and batches continuously over four streams, each batch bounded in
cost (pixel-angle updates).

First the saturation throughput is measured (all requests offered at once),
then a sweep of offered loads from 25% to 120% of it.  At every point the same
arrival sequence is also served by the plain baseline: FIFO, one slice per
fbp_reconstruct call, one stream, synchronous.  Latency is arrival to completion.

python -m paper_2109_02174_amd.serve_bench [--requests 2000] [--points 0.25,0.5,0.75,1.0,1.2]
                                           [--streams 4] [--batch-cost 1e10]
"""
from __future__ import annotations

import argparse
import json
import math
import threading
import time

import numpy as np

BUDGET_BYTES = 200 * 10 ** 9


def make_requests(n: int):
    from . import configs
    from .phantom import SEED_TAG_ARRIVALS, SEED_TAG_GEOM, rng_for
    rg = rng_for(5, SEED_TAG_GEOM)
    sides = rg.integers(0, len(configs.C4_SIDES), size=n)
    angs = rg.integers(0, len(configs.C4_ANGLES), size=n)
    nsl = rg.integers(1, 65, size=n)
    gaps = rng_for(5, SEED_TAG_ARRIVALS).exponential(1.0, size=n)   # scaled by 1/QPS later
    reqs = [(configs.C4_SIDES[s], configs.C4_ANGLES[a], int(b)) for s, a, b in zip(sides, angs, nsl)]
    return reqs, gaps


def build_pools(device="cuda", per_geom: int = 64):
    import torch

    from . import _binding as fbp
    from . import configs
    from . import phantom as ph
    pools, geoms = {}, {}
    gi = 0
    for side in configs.C4_SIDES:
        for K in configs.C4_ANGLES:
            D = configs.c4_detectors(side)
            g = fbp.Geometry(K, D, side, 1.0, ph.uniform_angles(K))
            sl = []
            for b in range(per_geom):
                ells = ph.draw_ellipses(ph.rng_for(5, 1000 + gi * per_geom + b), 20)
                sl.append(ph.ellipse_sinogram_device(ells, side, D, 1.0, g.angles, device).to(torch.float32))
            pools[(side, K)] = torch.stack(sl).contiguous()
            geoms[(side, K)] = g
            gi += 1
    return pools, geoms


def run_server(reqs, arrivals, pools, geoms, n_streams=4, batch_cost=None, collect=None):
    """Serve the requests at the given arrival offsets (seconds); return stats."""
    from .serve import DEFAULT_BATCH_COST, GpuExecutor, Server
    srv = Server(GpuExecutor(n_streams=n_streams), BUDGET_BYTES,
                 max_batch_cost=DEFAULT_BATCH_COST if batch_cost is None else int(batch_cost))
    kept = {}
    t0 = time.perf_counter()
    for i, ((side, K, n), at) in enumerate(zip(reqs, arrivals)):
        now = time.perf_counter() - t0
        if at > now:
            time.sleep(at - now)
        f = srv.submit(geoms[(side, K)], pools[(side, K)][:n])
        if collect is not None and i in collect:
            kept[i] = f          # other results are dropped as they complete
    srv.drain()
    t_end = time.perf_counter()
    st = srv.stats()
    srv.shutdown()
    slices = sum(r[2] for r in reqs)
    st["slices_per_s"] = slices / (t_end - t0)
    st["requests_per_s"] = len(reqs) / (t_end - t0)
    if collect is not None:
        for i, f in kept.items():
            collect[i] = f.result()
    return st


def run_baseline(reqs, arrivals, pools, geoms):
    """FIFO, one slice per fbp_reconstruct call, one stream, synchronous."""
    import torch

    from . import _binding as fbp
    stream = torch.cuda.current_stream()
    ws = fbp.alloc_workspace(max(fbp.fbp_workspace_bytes(g, 1) for g in geoms.values()))
    outs = {k: torch.empty((1, g.image_size, g.image_size), device="cuda") for k, g in geoms.items()}
    lat = []
    t0 = time.perf_counter()
    for (side, K, n), at in zip(reqs, arrivals):
        now = time.perf_counter() - t0
        if at > now:
            time.sleep(at - now)
        g = geoms[(side, K)]
        for b in range(n):
            fbp.fbp_reconstruct(g, pools[(side, K)][b:b + 1], out=outs[(side, K)], workspace=ws)
        stream.synchronize()
        lat.append(time.perf_counter() - t0 - at)
    t_end = time.perf_counter()
    lat.sort()

    def pct(p):
        return lat[min(len(lat) - 1, int(math.ceil(p / 100.0 * len(lat))) - 1)] * 1e3
    slices = sum(r[2] for r in reqs)
    return {"p50_ms": pct(50), "p99_ms": pct(99), "slices_per_s": slices / (t_end - t0),
            "requests_per_s": len(reqs) / (t_end - t0)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--requests", type=int, default=2000)
    ap.add_argument("--points", default="0.25,0.5,0.75,1.0,1.2")
    ap.add_argument("--no-baseline", action="store_true")
    ap.add_argument("--streams", type=int, default=4)
    ap.add_argument("--batch-cost", type=float, default=None,
                    help="bound on a batch's pixel-angle updates (default: serve.DEFAULT_BATCH_COST)")
    args = ap.parse_args()
    if not 1 <= args.streams <= 4:
        ap.error("--streams must be 1 to 4")
    import torch

    from . import _binding as fbp
    pools, geoms = build_pools()
    tuned = {f"{k[0]}x{k[1]}": fbp.fbp_autotune(g) for k, g in sorted(geoms.items())}
    reqs, gaps = make_requests(args.requests)
    torch.cuda.synchronize()
    kw = {"n_streams": args.streams, "batch_cost": args.batch_cost}
    run_server(reqs[:50], np.zeros(50), pools, geoms, **kw)               # warm-up: plans, graphs
    sat = run_server(reqs, np.zeros(len(reqs)), pools, geoms, **kw)       # offered load: everything at t=0
    out = {"workload": "Poisson arrivals, requests of U{1..64} slices of one mixed geometry, FP32, "
                       f"sinograms resident in HBM, budget 200 GB, {args.streams} streams, batch cost bound "
                       f"{args.batch_cost or 'default'}",
           "requests_per_point": len(reqs), "saturation": sat, "tile_config_per_geometry": tuned,
           "points": []}
    sat_qps = sat["requests_per_s"]
    for f in [float(x) for x in args.points.split(",")]:
        qps = f * sat_qps
        arrivals = np.cumsum(gaps) / qps
        pt = {"load": f, "qps": qps, "served": run_server(reqs, arrivals, pools, geoms, **kw)}
        if not args.no_baseline:
            pt["one_slice_per_launch"] = run_baseline(reqs, arrivals, pools, geoms)
        out["points"].append(pt)
        print(json.dumps(pt), flush=True)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
