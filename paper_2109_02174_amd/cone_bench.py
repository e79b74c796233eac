"""Cone-beam (FDK) benchmark: 256^3 volume, 360 views over a full turn, flat
detector of 256 rows x 384 columns (unit spacing), source at 512 voxels from
the axis, FP32, inputs in HBM.  Times the filter (pre-weight + row GEMM), the
backprojection and the whole reconstruction, and reports voxel-view updates
per second (N^2 Nz K).  Agreement with the FP64 reference is checked by the
GPU test-suite.

python -m paper_2109_02174_amd.cone_bench [--reps 10]
"""
from __future__ import annotations

import argparse
import json


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--reps", type=int, default=10)
    args = ap.parse_args()
    import torch

    from . import _binding as fbp
    from . import phantom as ph

    N, Nz, K, Dv, Du, R = 256, 256, 360, 256, 384, 512.0
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

    g = fbp.ConeGeometry(K, Du, Dv, N, Nz, R)
    proj = torch.tensor(ph.rng_for(11, 0).normal(size=(K, Dv, Du)).astype("float32"), device="cuda")
    filt = torch.empty_like(proj)
    vol = torch.empty((Nz, N, N), device="cuda")
    ws = fbp.alloc_workspace(fbp.fbp_cone_workspace_bytes(g))
    fbp.fbp_cone_reconstruct(g, proj, out=vol, workspace=ws)
    fbp.fbp_cone_filter(g, proj, out=filt)
    torch.cuda.synchronize()
    upd = float(N * N * Nz * K)
    res = {"workload": f"cone beam {N}x{N}x{Nz}, {K} views over 2 pi, detector {Dv}x{Du}, R = {R:g}, FP32"}
    for name, fn in (("filter", lambda: fbp.fbp_cone_filter(g, proj, out=filt)),
                     ("backproject", lambda: fbp.fbp_cone_backproject(g, filt, out=vol)),
                     ("reconstruct", lambda: fbp.fbp_cone_reconstruct(g, proj, out=vol, workspace=ws))):
        ms = timed(fn, args.reps)
        res[name + "_ms"] = ms
        if name != "filter":
            res[name + "_updates_per_s"] = upd / (ms * 1e-3)
        print(json.dumps({name: ms}), flush=True)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
