"""GPU: stacks of slices that share a geometry.

Tile shapes with a stack kernel backproject 4 slices per workgroup (one
coordinate, truncation and LDS address per 8 pixels); the rest of a stack, and
shapes without one, go one slice per workgroup.  Each slice's arithmetic and
summation order are those of the one-slice kernel, so a slice comes out bitwise
the same alone, in a stack (any position, ragged tail included) and in a batch.
Agreement with the FP64 oracle is checked for stacks in the parity tests.
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


def test_some_shapes_have_stack_kernels():
    names = [fbp.fbp_tile_config_name(c) for c in range(fbp.fbp_num_tile_configs())]
    assert sum("slice stacks" in n for n in names) >= 2


@pytest.mark.parametrize("K,D,N,dt,B", [(50, 101, 70, 1.0, 9), (24, 230, 48, 0.35, 6), (33, 49, 33, 1.0, 4),
                                        (20, 61, 40, 1.0, 3)])
def test_stack_equals_single_slices_bitwise(K, D, N, dt, B):
    g = _geom(K, D, N, dt, K + D)
    q = _q(B, K, D, K)
    for cfg in range(fbp.fbp_num_tile_configs()):
        if "rotations" in fbp.fbp_tile_config_name(cfg):
            continue
        out = torch.full((B, N, N), float("nan"), device="cuda")
        fbp.fbp_backproject_with_config(g, q, cfg, out=out)
        stack = out.cpu().numpy()
        assert np.all(np.isfinite(stack)), f"tile {cfg}: pixel left unwritten"
        for s in range(B):
            one = fbp.fbp_backproject_with_config(g, q[s:s + 1].contiguous(), cfg)
            assert np.array_equal(one.cpu().numpy()[0], stack[s]), f"tile {cfg}, slice {s}"


def test_stack_reconstruction_matches_oracle_and_single_calls():
    K, D, N, dt, B = 60, 97, 64, 1.0, 7
    g = _geom(K, D, N, dt, 7, kind="uniform")
    rng = ph.rng_for(1302, 0)
    sino = rng.normal(size=(B, K, D)).astype(np.float32)
    out = fbp.fbp_reconstruct(g, torch.tensor(sino, device="cuda")).cpu().numpy()
    ref = oracle.fbp(sino.astype(np.float64), N, dt, np.asarray(g.angles))
    scale = np.max(np.abs(ref))
    assert np.max(np.abs(out - ref)) <= 2e-4 * scale
    for s in (0, 3, 4, 6):
        one = fbp.fbp_reconstruct(g, torch.tensor(sino[s:s + 1], device="cuda")).cpu().numpy()[0]
        assert np.array_equal(one, out[s])


def test_batch_groups_of_one_geometry_equal_alone_bitwise():
    # 9 slices of one geometry (two groups of 4 and a single), 5 of another, 1 of a third
    geoms = [(_geom(90, 93, 64, 1.0, 0, "uniform"), 9), (_geom(120, 145, 100, 1.0, 1), 5),
             (_geom(37, 49, 33, 0.8, 2), 1)]
    jobs = []
    i = 0
    for g, n in geoms:
        for _ in range(n):
            sino = torch.tensor(ph.rng_for(1303, i).normal(size=(g.n_angles, g.n_det)).astype(np.float32),
                                device="cuda")
            img = torch.full((g.image_size, g.image_size), float("nan"), device="cuda")
            jobs.append((g, sino, img))
            i += 1
    order = list(ph.rng_for(1304, 0).permutation(len(jobs)))   # interleave the geometries
    jobs = [jobs[j] for j in order]
    fbp.fbp_reconstruct_batch(jobs)
    torch.cuda.synchronize()
    for g, sino, img in jobs:
        alone = fbp.fbp_reconstruct(g, sino[None].contiguous())[0]
        assert np.array_equal(img.cpu().numpy(), alone.cpu().numpy())
