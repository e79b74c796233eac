"""Fan-beam benchmark: 512 x 512 image, 720 views over a full turn, 801 bins of unit
width on a flat detector, source at 1024 pixels from the centre, FP32, inputs in HBM.

Times the filter (pre-weight + GEMM), the backprojection and the whole
reconstruction, for one slice and per slice of a stack, and reports pixel-view
updates per second (N^2 K per slice).  Agreement with the FP64 reference is
checked by the GPU test-suite.

python -m paper_2109_02174_amd.fan_bench [--reps 50] [--stack 16]
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

    N, K, D, R = 512, 720, 801, 1024.0
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

    sl = ph.fan_slice(8, 0, N, K, D, 1.0, R, n_ellipses=20)
    g = fbp.Geometry(K, D, N, 1.0, sl.angles, source_distance=R)
    sino1 = torch.tensor(sl.sino, dtype=torch.float32, device="cuda")[None].contiguous()
    sinos = sino1.expand(args.stack, K, D).contiguous()
    filt1, filts = torch.empty_like(sino1), torch.empty_like(sinos)
    img1 = torch.empty((1, N, N), device="cuda")
    imgs = torch.empty((args.stack, N, N), device="cuda")
    ws1 = fbp.alloc_workspace(fbp.fbp_workspace_bytes(g, 1))
    wss = fbp.alloc_workspace(fbp.fbp_workspace_bytes(g, args.stack))
    fbp.fbp_reconstruct(g, sino1, out=img1, workspace=ws1)
    fbp.fbp_reconstruct(g, sinos, out=imgs, workspace=wss)
    fbp.fbp_filter(g, sino1, out=filt1)
    fbp.fbp_filter(g, sinos, out=filts)
    torch.cuda.synchronize()
    upd = float(N * N * K)
    res = {"workload": f"fan beam {N}x{N}, {K} views over 2 pi, {D} bins, R = {R:g}, FP32; stack of {args.stack}"}
    for name, fn, n in (("filter_single", lambda: fbp.fbp_filter(g, sino1, out=filt1), 1),
                        ("backproject_single", lambda: fbp.fbp_backproject(g, filt1, out=img1), 1),
                        ("reconstruct_single", lambda: fbp.fbp_reconstruct(g, sino1, out=img1, workspace=ws1), 1),
                        ("filter_stack", lambda: fbp.fbp_filter(g, sinos, out=filts), args.stack),
                        ("backproject_stack", lambda: fbp.fbp_backproject(g, filts, out=imgs), args.stack),
                        ("reconstruct_stack", lambda: fbp.fbp_reconstruct(g, sinos, out=imgs, workspace=wss),
                         args.stack)):
        ms = timed(fn, args.reps if n == 1 else max(4, args.reps // 5))
        res[name + "_us_per_slice"] = ms * 1e3 / n
        if "filter" not in name:
            res[name + "_updates_per_s"] = upd * n / (ms * 1e-3)
        print(json.dumps({name: ms * 1e3 / n}), flush=True)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
