"""Filter-variant benchmark: 512^2, 720 angles, 725 bins with each filter kernel
(Ram-Lak, Shepp-Logan, Hann) and each angular weighting (pi/K; angle gaps on an
uneven angle list), FP32, inputs in HBM.

Per variant: the filter GEMM alone, one whole single-slice reconstruction, and a
64-slice stack (per slice).  Ram-Lak's kernel vanishes at even offsets, so its
GEMM does half the MACs of the other two.  (Agreement of every variant with the
FP64 reference is checked by the GPU test-suite.)

python -m paper_2109_02174_amd.variant_bench [--reps 20]
"""
from __future__ import annotations

import argparse
import json
import math


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--reps", type=int, default=20)
    ap.add_argument("--stack", type=int, default=64)
    args = ap.parse_args()
    import numpy as np
    import torch

    from . import _binding as fbp
    from . import phantom as ph

    N, K, D = 512, 720, 725
    uneven = np.sort(np.concatenate([np.linspace(0.0, 1.0, K // 2, endpoint=False),
                                     np.linspace(1.0, math.pi, K - K // 2, endpoint=False)]))
    stream = torch.cuda.current_stream()

    def timed(fn, reps):
        blocker = torch.empty((4096, 4096), device="cuda")
        for _ in range(2):
            blocker = blocker @ blocker.T   # queue ahead so host launch gaps are not timed
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        e1.synchronize()
        return e0.elapsed_time(e1) / reps

    out = {"workload": f"{N}x{N}, {K} angles, {D} bins, FP32; stack of {args.stack}", "variants": []}
    for weighting, ang in (("uniform", ph.uniform_angles(K)), ("angle-gaps", uneven)):
        sino1 = ph.ellipse_sinogram_device(ph.draw_ellipses(ph.rng_for(6, 0), 20), N, D, 1.0, ang)
        sino1 = sino1.to(torch.float32)[None].contiguous()
        stack = sino1.expand(args.stack, K, D).contiguous()
        for kind in ("ramlak", "shepp-logan", "hann"):
            g = fbp.Geometry(K, D, N, 1.0, ang, filter=kind, weighting=weighting)
            tuned = fbp.fbp_autotune(g)
            img1 = torch.empty((1, N, N), device="cuda")
            imgs = torch.empty((args.stack, N, N), device="cuda")
            filt = torch.empty_like(sino1)
            ws1 = fbp.alloc_workspace(fbp.fbp_workspace_bytes(g, 1))
            wss = fbp.alloc_workspace(fbp.fbp_workspace_bytes(g, args.stack))
            fbp.fbp_reconstruct(g, sino1, out=img1, workspace=ws1)
            fbp.fbp_reconstruct(g, stack, out=imgs, workspace=wss)
            torch.cuda.synchronize()
            f_ms = timed(lambda: fbp.fbp_filter(g, sino1, out=filt), args.reps)
            one_ms = timed(lambda: fbp.fbp_reconstruct(g, sino1, out=img1, workspace=ws1), args.reps)
            st_ms = timed(lambda: fbp.fbp_reconstruct(g, stack, out=imgs, workspace=wss), max(2, args.reps // 10))
            upd = float(N * N * K)
            out["variants"].append({
                "filter": kind, "weighting": weighting, "tile_single": tuned,
                "tile_stack": fbp.fbp_plan_stack_config(g),
                "filter_us": f_ms * 1e3, "single_slice_us": one_ms * 1e3,
                "single_slice_updates_per_s": upd / (one_ms * 1e-3),
                "stack_us_per_slice": st_ms * 1e3 / args.stack,
                "stack_updates_per_s": upd * args.stack / (st_ms * 1e-3)})
            print(json.dumps(out["variants"][-1]), flush=True)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
