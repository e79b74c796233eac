"""Filter-path benchmark: the ramp filter of one sinogram (K rows of D bins, FP32,
inputs in HBM) through the MFMA GEMM and through the FFT path, for detector
lengths from the workloads (183 ... 1451 bins) up to 4096, and the whole 512^2 /
720-angle / 725-bin reconstruction with each.  Agreement with the FP64
reference is checked by the GPU test-suite.

python -m paper_2109_02174_amd.filter_bench [--reps 50]
"""
from __future__ import annotations

import argparse
import json


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--reps", type=int, default=50)
    args = ap.parse_args()
    import torch

    from . import _binding as fbp
    from . import phantom as ph

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

    res = {"filter": []}
    for K, D in ((180, 183), (360, 365), (720, 725), (1440, 1451), (1440, 2897), (720, 4096)):
        g = fbp.Geometry(K, D, 64, 1.0)
        P = torch.tensor(ph.rng_for(9, D).normal(size=(1, K, D)).astype("float32"), device="cuda")
        out = torch.empty_like(P)
        row = {"K": K, "D": D}
        for prec in ("fp32", "fft"):
            fbp.fbp_filter(g, P, out=out, precision=prec)
            torch.cuda.synchronize()
            row[prec + "_us"] = timed(lambda: fbp.fbp_filter(g, P, out=out, precision=prec), args.reps) * 1e3
        res["filter"].append(row)
        print(json.dumps(row), flush=True)
    N, K, D = 512, 720, 725
    g = fbp.Geometry(K, D, N, 1.0)
    sino = torch.tensor(ph.ellipse_sinogram(ph.draw_ellipses(ph.rng_for(10, 0), 20), N, D, 1.0,
                                            ph.uniform_angles(K))[None].astype("float32"), device="cuda")
    img = torch.empty((1, N, N), device="cuda")
    ws = fbp.alloc_workspace(fbp.fbp_workspace_bytes(g, 1))
    for prec in ("fp32", "fft"):
        fbp.fbp_reconstruct(g, sino, out=img, workspace=ws, precision=prec)
        torch.cuda.synchronize()
        res["reconstruct_512_720_725_" + prec + "_us"] = timed(
            lambda: fbp.fbp_reconstruct(g, sino, out=img, workspace=ws, precision=prec), args.reps) * 1e3
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
