"""GPU: stacks of slices that share a geometry, and angle-split single slices.

Stacks of 4 or more slices run with the plan's stack tile shape; tile shapes
with a stack kernel backproject 2 or 4 slices per workgroup (one coordinate,
truncation and LDS address for 2M pixels), the rest of the stack one slice per
workgroup.  Each slice's arithmetic and summation order are those of the
one-slice kernel of the shape, so a slice comes out bitwise the same in any
position of a stack and in a batch group.  Single slices with a one-group shape
split their angles over workgroups and add the parts in a fixed order.  Both
paths agree with the FP64 oracle (here and, for every shape, in the parity
tests) and with each other within the FP32 tolerance.
"""
import math

import numpy as np
import pytest
import torch

import oracle
import paper_2109_02174_amd as fbp
from paper_2109_02174_amd import phantom as ph

pytestmark = pytest.mark.gpu


def _geom(K, D, N, dt, seed, kind="random"):
    if kind == "uniform":
        ang = ph.uniform_angles(K)
    else:
        ang = np.sort(ph.rng_for(1300, seed).uniform(0.0, math.pi, K))
    return fbp.Geometry(K, D, N, dt, ang)


def _q(B, K, D, seed):
    return torch.tensor(ph.rng_for(1301, seed).normal(size=(B, K, D)).astype(np.float32), device="cuda")


def _plain_shapes():
    return [c for c in range(fbp.fbp_num_tile_configs()) if "rotations" not in fbp.fbp_tile_config_name(c)]


def bp_tolerance(Q):
    Q = np.asarray(Q, np.float64)
    dq = np.max(np.abs(np.diff(Q, axis=-1)))
    return math.pi * (1e-4 * max(dq, np.max(np.abs(Q))) + 1e-5 * np.max(np.abs(Q))) + 1e-6


def test_some_shapes_have_stack_kernels():
    names = [fbp.fbp_tile_config_name(c) for c in range(fbp.fbp_num_tile_configs())]
    assert sum("slice stacks" in n for n in names) >= 2


@pytest.mark.parametrize("K,D,N,dt,B", [(50, 101, 70, 1.0, 9), (24, 230, 48, 0.35, 7), (33, 49, 33, 1.0, 4)])
def test_stack_position_does_not_change_a_slice(K, D, N, dt, B):
    # B copies of one slice: the grouped kernel (every position in a group) and the
    # one-slice kernel of the ragged tail must give the same bits
    g = _geom(K, D, N, dt, K + D)
    one = _q(1, K, D, K)
    q = one.expand(B, K, D).contiguous()
    for cfg in _plain_shapes():
        out = torch.full((B, N, N), float("nan"), device="cuda")
        fbp.fbp_backproject_with_config(g, q, cfg, out=out)
        got = out.cpu().numpy()
        assert np.all(np.isfinite(got)), f"tile {cfg}: pixel left unwritten"
        for s in range(1, B):
            assert np.array_equal(got[0], got[s]), f"tile {cfg}, slice {s}"


@pytest.mark.parametrize("K,D,N,dt", [(90, 101, 70, 1.0), (40, 230, 48, 0.35), (180, 183, 128, 1.0)])
def test_single_slice_and_stack_paths_match_oracle(K, D, N, dt):
    g = _geom(K, D, N, dt, 3 * K + D)
    Q = ph.rng_for(1305, K).normal(size=(5, K, D)).astype(np.float32)
    ref = oracle.backproject(Q.astype(np.float64), N, dt, np.asarray(g.angles))
    tol = bp_tolerance(Q)
    q = torch.tensor(Q, device="cuda")
    for cfg in _plain_shapes():
        stack = fbp.fbp_backproject_with_config(g, q, cfg).cpu().numpy()           # stack path
        assert np.max(np.abs(stack - ref)) <= tol, f"tile {cfg}: stack"
        for s in (0, 4):
            one = fbp.fbp_backproject_with_config(g, q[s:s + 1].contiguous(), cfg).cpu().numpy()[0]
            assert np.max(np.abs(one - ref[s])) <= tol, f"tile {cfg}: single slice {s}"
            again = fbp.fbp_backproject_with_config(g, q[s:s + 1].contiguous(), cfg).cpu().numpy()[0]
            assert np.array_equal(one, again)


def test_split_single_slices_on_two_streams():
    # the plan's partial-sum buffer is shared: calls on two streams must not mix
    K, D, N = 120, 145, 100
    g = _geom(K, D, N, 1.0, 11)
    cfg = next(c for c in _plain_shapes() if "1 angle group" in fbp.fbp_tile_config_name(c))
    q = _q(6, K, D, 12)
    ref = [fbp.fbp_backproject_with_config(g, q[i:i + 1].contiguous(), cfg).cpu().numpy()[0] for i in range(6)]
    torch.cuda.synchronize()
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    outs = [torch.full((1, N, N), float("nan"), device="cuda") for _ in range(6)]
    for rep in range(3):
        for i in range(6):
            st = streams[i % 2]
            with torch.cuda.stream(st):
                fbp.fbp_backproject_with_config(g, q[i:i + 1].contiguous(), cfg, out=outs[i], stream=st)
        torch.cuda.synchronize()
        for i in range(6):
            assert np.array_equal(outs[i].cpu().numpy()[0], ref[i]), f"rep {rep}, slice {i}"


def test_stack_reconstruction_matches_oracle():
    K, D, N, dt, B = 60, 97, 64, 1.0, 7
    g = _geom(K, D, N, dt, 7, kind="uniform")
    rng = ph.rng_for(1302, 0)
    sino = rng.normal(size=(B, K, D)).astype(np.float32)
    out = fbp.fbp_reconstruct(g, torch.tensor(sino, device="cuda")).cpu().numpy()
    ref = oracle.fbp(sino.astype(np.float64), N, dt, np.asarray(g.angles))
    scale = np.max(np.abs(ref))
    assert np.max(np.abs(out - ref)) <= 2e-4 * scale
    for s in (0, 3, 6):
        one = fbp.fbp_reconstruct(g, torch.tensor(sino[s:s + 1], device="cuda")).cpu().numpy()[0]
        assert np.max(np.abs(one - ref[s])) <= 2e-4 * scale


def test_batch_groups_equal_the_stack_call_bitwise():
    # 9 slices of one geometry (stack shape: groups and a single), 5 of another
    # (stack shape), 2 of a third (single-slice shape, unsplit)
    geoms = [(_geom(90, 93, 64, 1.0, 0, "uniform"), 9), (_geom(120, 145, 100, 1.0, 1), 5),
             (_geom(37, 49, 33, 0.8, 2), 2)]
    jobs, per_geom = [], []
    i = 0
    for g, n in geoms:
        sinos = torch.tensor(ph.rng_for(1303, i).normal(size=(n, g.n_angles, g.n_det)).astype(np.float32),
                             device="cuda")
        per_geom.append((g, sinos))
        for s in range(n):
            img = torch.full((g.image_size, g.image_size), float("nan"), device="cuda")
            jobs.append((g, sinos[s], img, len(per_geom) - 1, s))
        i += 1
    order = list(ph.rng_for(1304, 0).permutation(len(jobs)))   # interleave the geometries
    jobs = [jobs[j] for j in order]
    fbp.fbp_reconstruct_batch([(g, sino, img) for g, sino, img, _, _ in jobs])
    torch.cuda.synchronize()
    whole = []
    for g, sinos in per_geom:
        if sinos.shape[0] >= 4:
            whole.append(fbp.fbp_reconstruct(g, sinos).cpu().numpy())
        else:
            whole.append(np.stack([fbp.fbp_reconstruct(g, sinos[s:s + 1].contiguous()).cpu().numpy()[0]
                                   for s in range(sinos.shape[0])]))
    for g, sino, img, gi, s in jobs:
        got = img.cpu().numpy()
        if per_geom[gi][1].shape[0] >= 4 or "1 angle group" not in fbp.fbp_tile_config_name(fbp.fbp_plan_config(g)):
            assert np.array_equal(got, whole[gi][s]), f"geometry {gi}, slice {s}"
        else:
            assert np.max(np.abs(got - whole[gi][s])) <= 2e-4 * np.max(np.abs(whole[gi][s]))
