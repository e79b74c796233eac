"""Mixed-size batch benchmark: 1000 slices of random geometry in one batch call.

Image side from {256, 384, 512, 1024}, angles from {360, 720, 1440} (uniform on
[0, pi)), detectors ceil(sqrt(2) side) + 2, each slice a seeded 20-ellipse
phantom with an exact FP64 sinogram generated in HBM (rounded to FP32 for the
library).  Every geometry here is a quarter-turn geometry (even side, uniform
angles with even count), so all slices take the chunked quarter-turn
backprojector: the batch runs as grouped filter GEMMs plus one persistent
backprojection launch over every tile of every slice, replayed from a captured
HIP graph (the autotuner only picks the window pitch, which does not change the
bits).  Reported beside it: the same slices reconstructed one per launch
(fbp_reconstruct with one slice, no graph), and for a sample of slices whether
the two are bitwise equal.  (Agreement with the FP64 reference for one slice of
every geometry of this workload is checked by the GPU test-suite.)

python -m paper_2109_02174_amd.batch_bench [--slices 1000] [--reps 5]
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np


def build_jobs(n_slices: int, device="cuda", keep_host=()):
    """Jobs (Geometry, sino, image) of the mixed workload; FP64 host copies of the
    sinograms and phantom rasters of the slices in keep_host."""
    import torch

    from . import _binding as fbp
    from . import configs
    from . import phantom as ph

    geoms = configs.c4_geometries(n_slices)
    gobj = {}
    jobs, host = [], {}
    for i, g in enumerate(geoms):
        key = (g.N, g.K, g.D)
        if key not in gobj:
            gobj[key] = fbp.Geometry(g.K, g.D, g.N, g.dt, ph.uniform_angles(g.K))
        geo = gobj[key]
        ells = ph.draw_ellipses(ph.rng_for(4, i), 20)
        s64 = ph.ellipse_sinogram_device(ells, g.N, g.D, g.dt, geo.angles, device)
        if i in keep_host:
            host[i] = (s64.cpu().numpy(), ph.rasterise(ells, g.N))
        sino = s64.to(torch.float32).contiguous()
        img = torch.empty((g.N, g.N), dtype=torch.float32, device=device)
        jobs.append((geo, sino, img))
    return jobs, gobj, host


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--slices", type=int, default=1000)
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--no-baseline", action="store_true")
    args = ap.parse_args()

    import torch

    from . import _binding as fbp
    from . import configs

    geoms = configs.c4_geometries(args.slices)
    upd = np.array([g.N * g.N * g.K for g in geoms], dtype=np.float64)
    order = np.argsort(upd)
    sample = sorted({int(order[0]), int(order[-1]), int(order[len(order) // 2])})
    t0 = time.perf_counter()
    jobs, gobj, _ = build_jobs(args.slices)
    torch.cuda.synchronize()
    t_gen = time.perf_counter() - t0
    tuned = {}
    for k, g in sorted(gobj.items()):
        fbp.fbp_autotune(g)
        tuned[f"{k[0]}x{k[1]}x{k[2]}"] = {"single": fbp.fbp_plan_config(g), "stack": fbp.fbp_plan_stack_config(g)}
    ws = fbp.alloc_workspace(fbp.fbp_batch_workspace_bytes(jobs))
    stream = torch.cuda.current_stream()

    fbp.fbp_reconstruct_batch(jobs, workspace=ws)          # plans, capture, warm-up
    torch.cuda.synchronize()
    times = []
    for _ in range(args.reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        fbp.fbp_reconstruct_batch(jobs, workspace=ws)
        e1.record(stream)
        e1.synchronize()
        times.append(e0.elapsed_time(e1))
    batch_ms = sorted(times)[len(times) // 2]
    total_upd = float(upd.sum())
    out = {
        "workload": f"{args.slices} mixed slices (side {{256,384,512,1024}}, angles {{360,720,1440}}, "
                    "detectors ceil(sqrt2 side)+2), FP32, one batch call, persistent launches, HIP graph",
        "slices": args.slices, "updates": total_upd, "batch_ms": batch_ms,
        "slices_per_s": args.slices / (batch_ms * 1e-3), "updates_per_s": total_upd / (batch_ms * 1e-3),
        "input_generation_s": t_gen, "tile_config_per_geometry": tuned,
    }

    batched = {i: jobs[i][2].cpu().numpy().copy() for i in sample}
    if not args.no_baseline:
        imgs = [torch.empty_like(j[2]) for j in jobs]
        wss = fbp.alloc_workspace(max(fbp.fbp_workspace_bytes(g, 1) for g in gobj.values()))
        for (g, s, _), im in zip(jobs[:10], imgs[:10]):           # warm plans
            fbp.fbp_reconstruct(g, s[None], out=im[None], workspace=wss)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for (g, s, _), im in zip(jobs, imgs):
            fbp.fbp_reconstruct(g, s[None], out=im[None], workspace=wss)
        e1.record(stream)
        e1.synchronize()
        base_ms = e0.elapsed_time(e1)
        out["one_slice_per_launch"] = {"ms": base_ms, "slices_per_s": args.slices / (base_ms * 1e-3),
                                       "updates_per_s": total_upd / (base_ms * 1e-3)}
        out["speedup_vs_one_slice_per_launch"] = base_ms / batch_ms
        out["batch_vs_alone_bitwise"] = all(np.array_equal(batched[i], imgs[i].cpu().numpy()) for i in sample)
        out["batch_vs_alone_max_rel"] = max(
            float(np.max(np.abs(batched[i] - imgs[i].cpu().numpy())) / np.max(np.abs(batched[i])))
            for i in sample)

    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
