"""GPU: the mixed-size batch path (grouped GEMM + persistent backprojection from a
captured HIP graph) against reconstructing each slice alone and against the oracle.
A batch gives a geometry with fewer than 4 slices its single-slice tile shape,
unsplit: bitwise the shape's one-slice kernel, and bitwise fbp_reconstruct alone
unless that splits the slice's angles over workgroups (then within the FP32
tolerance)."""
import math

import numpy as np
import pytest
import torch

import oracle
import paper_2109_02174_amd as fbp
from paper_2109_02174_amd import metrics
from paper_2109_02174_amd import phantom as ph

pytestmark = pytest.mark.gpu

# (N, K, D, dt, angle kind)
MIX = [
    (64, 90, 93, 1.0, "uniform"),
    (100, 120, 145, 1.0, "uniform"),
    (33, 37, 49, 0.8, "random"),
    (128, 180, 183, 1.0, "uniform"),
    (128, 180, 183, 1.0, "uniform"),
    (17, 5, 26, 1.3, "random"),
    (256, 360, 365, 1.0, "uniform"),
    (1, 3, 2, 1.0, "uniform"),
]


def _angles(K, kind, seed):
    if kind == "uniform":
        return ph.uniform_angles(K)
    return np.sort(ph.rng_for(1100, seed).uniform(0.0, math.pi, K))


def _jobs(seed, mix=MIX):
    jobs, refs = [], []
    for i, (N, K, D, dt, kind) in enumerate(mix):
        ang = _angles(K, kind, i)
        sl = ph.ellipse_slice(1100 + seed, i, N, K, D, dt, n_ellipses=6, angles=ang)
        g = fbp.Geometry(K, D, N, dt, ang)
        sino = torch.tensor(sl.sino.astype(np.float32), device="cuda")
        img = torch.full((N, N), float("nan"), device="cuda")
        jobs.append((g, sino, img))
        refs.append(sl)
    return jobs, refs


def _alone(g, sino, prec="fp32"):
    out = fbp.fbp_reconstruct(g, sino[None].contiguous(), precision=prec)
    torch.cuda.synchronize()
    return out[0].cpu().numpy()


def _unsplit(g, sino, prec="fp32"):
    """The slice through the plan's single-slice shape without angle split, as the
    batch runs it: the shape's stack path on 4 copies (its stack kernel gives each
    slice the one-slice kernel's bits)."""
    filt = fbp.fbp_filter(g, sino[None].contiguous(), precision=prec)
    q4 = filt.expand(4, g.n_angles, g.n_det).contiguous()
    out = fbp.fbp_backproject_with_config(g, q4, fbp.fbp_plan_config(g))
    torch.cuda.synchronize()
    return out[0].cpu().numpy()


def _check_vs_alone(got, g, sino, prec="fp32"):
    """Bitwise equal to the unsplit single-slice shape, and to fbp_reconstruct alone
    unless that angle-splits the slice (then within the FP32 tolerance)."""
    assert np.array_equal(got, _unsplit(g, sino, prec)), f"batch differs from the shape's kernel, N={g.image_size}"
    alone = _alone(g, sino, prec)
    if "1 angle group" in fbp.fbp_tile_config_name(fbp.fbp_plan_config(g)):
        assert np.max(np.abs(got - alone)) <= 2e-4 * np.max(np.abs(alone)) + 1e-30
    else:
        assert np.array_equal(got, alone), f"batch differs from alone, N={g.image_size}"


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_batch_equals_alone_and_matches_oracle(prec):
    jobs, refs = _jobs(0)
    fbp.fbp_reconstruct_batch(jobs, precision=prec)
    torch.cuda.synchronize()
    for (g, sino, img), sl in zip(jobs, refs):
        got = img.cpu().numpy()
        assert np.all(np.isfinite(got))
        _check_vs_alone(got, g, sino, prec)
        if prec == "fp32":
            ref = oracle.fbp(sl.sino, sl.N, sl.dt, sl.angles)
            m = metrics.compare(got, ref, sl.value_range)
            assert m["max_abs_rel"] <= 2e-4 and m["rmse_rel"] <= 2e-5, m


def test_graph_replays_with_new_inputs_and_sizes():
    """One workspace, several batches: each replay of the captured graph is checked
    against the eager single-slice path, with host work and syncs in between."""
    ws = fbp.alloc_workspace(64 << 20)
    for rep, mix in enumerate([MIX, MIX[:3], MIX[2:], MIX]):
        jobs, _ = _jobs(10 + rep, mix)
        fbp.fbp_reconstruct_batch(jobs, workspace=ws)
        torch.cuda.synchronize()
        for g, sino, img in jobs:
            _check_vs_alone(img.cpu().numpy(), g, sino)


def test_graphs_disabled_gives_same_bits(monkeypatch):
    jobs, _ = _jobs(20)
    fbp.fbp_reconstruct_batch(jobs)
    torch.cuda.synchronize()
    first = [img.cpu().numpy().copy() for _, _, img in jobs]
    monkeypatch.setenv("FBP_DISABLE_GRAPHS", "1")
    for _, _, img in jobs:
        img.fill_(float("nan"))
    fbp.fbp_reconstruct_batch(jobs)
    torch.cuda.synchronize()
    for x, (_, _, img) in zip(first, jobs):
        assert np.array_equal(x, img.cpu().numpy())


def test_batch_rejects_small_workspace():
    jobs, _ = _jobs(30, MIX[:2])
    need = fbp.fbp_batch_workspace_bytes(jobs)
    ws = fbp.alloc_workspace(need - 256)
    with pytest.raises(fbp.FbpError) as e:
        fbp.fbp_reconstruct_batch(jobs, workspace=ws)
    assert e.value.status == fbp.FBP_EWORKSPACE


def test_batches_on_two_streams_overlapping():
    """Two batches in flight on two streams with their own workspaces."""
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    j1, _ = _jobs(40)
    j2, _ = _jobs(41)
    w1 = fbp.alloc_workspace(fbp.fbp_batch_workspace_bytes(j1))
    w2 = fbp.alloc_workspace(fbp.fbp_batch_workspace_bytes(j2))
    torch.cuda.synchronize()
    with torch.cuda.stream(s1):
        fbp.fbp_reconstruct_batch(j1, workspace=w1, stream=s1)
    with torch.cuda.stream(s2):
        fbp.fbp_reconstruct_batch(j2, workspace=w2, stream=s2)
    torch.cuda.synchronize()
    for g, sino, img in j1 + j2:
        _check_vs_alone(img.cpu().numpy(), g, sino)
