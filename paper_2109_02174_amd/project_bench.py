"""Forward-projector benchmark: 512^2 image, 720 angles, 725 bins, FP32, inputs in HBM
(and the fan beam: 720 views over a full turn, 801 bins, source at R = 1024).

Times fbp_project (one slice and a stack) beside fbp_backproject of the same
shape, and reports pixel-angle pairs per second for both (N^2 K per slice; each
pair is one hat-weighted multiply-add per bin the pixel reaches).  Agreement
with the FP64 reference is checked by the GPU test-suite.

python -m paper_2109_02174_amd.project_bench [--reps 50] [--stack 16]
"""
from __future__ import annotations

import argparse
import json


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--reps", type=int, default=50)
    ap.add_argument("--stack", type=int, default=16)
    args = ap.parse_args()
    import torch

    from . import _binding as fbp
    from . import phantom as ph

    N, K, D = 512, 720, 725
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

    img = torch.tensor(ph.rasterise(ph.draw_ellipses(ph.rng_for(7, 0), 20), N), dtype=torch.float32,
                       device="cuda")[None].contiguous()
    imgs = img.expand(args.stack, N, N).contiguous()
    back1 = torch.empty((1, N, N), device="cuda")
    backs = torch.empty((args.stack, N, N), device="cuda")
    res = {"workload": f"{N}x{N}, {K} angles, {D} bins, FP32; stack of {args.stack}; "
                       f"fan beam: {K} views over 2 pi, 801 bins, R = 1024"}
    for prefix, g in (("", fbp.Geometry(K, D, N, 1.0)), ("fan_", fbp.Geometry(K, 801, N, 1.0, source_distance=1024.0))):
        Dg = g.n_det
        sino1 = torch.empty((1, K, Dg), device="cuda")
        sinos = torch.empty((args.stack, K, Dg), device="cuda")
        fbp.fbp_project(g, img, out=sino1)
        fbp.fbp_project(g, imgs, out=sinos)
        fbp.fbp_backproject(g, sino1, out=back1)
        fbp.fbp_backproject(g, sinos, out=backs)
        torch.cuda.synchronize()
        upd = float(N * N * K)
        for name, fn, n in (("project_single", lambda: fbp.fbp_project(g, img, out=sino1), 1),
                            ("project_stack", lambda: fbp.fbp_project(g, imgs, out=sinos), args.stack),
                            ("backproject_single", lambda: fbp.fbp_backproject(g, sino1, out=back1), 1),
                            ("backproject_stack", lambda: fbp.fbp_backproject(g, sinos, out=backs), args.stack)):
            ms = timed(fn, args.reps if n == 1 else max(4, args.reps // 5))
            res[prefix + name + "_us_per_slice"] = ms * 1e3 / n
            res[prefix + name + "_pixel_angles_per_s"] = upd * n / (ms * 1e-3)
            print(json.dumps({prefix + name: ms * 1e3 / n}), flush=True)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
