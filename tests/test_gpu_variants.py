"""GPU: filter kernels other than Ram-Lak, and angle weights for uneven angle lists.

Shepp-Logan and Hann kernels do not vanish at even offsets, so the filter GEMM
adds the same-parity product (even taps) to the parity-split one; angle-gap
weighting scales each staged filtered row by w_k/(pi/K).  Both are checked
against the FP64 oracle's own definitions (oracle.filter_rows,
oracle.angle_weights, oracle.fbp_variant), element by element.
"""
import math

import numpy as np
import pytest
import torch

import oracle
import paper_2109_02174_amd as fbp
from paper_2109_02174_amd import metrics
from paper_2109_02174_amd import phantom as ph

pytestmark = pytest.mark.gpu

KINDS = ["ramlak", "shepp-logan", "hann"]


def _clustered(K, seed):
    """Uneven angles: a dense cluster and a sparse remainder, shuffled."""
    rng = ph.rng_for(1400, seed)
    a = np.concatenate([rng.uniform(0.0, 0.6, K // 2), rng.uniform(0.6, math.pi, K - K // 2)])
    return a[rng.permutation(K)]


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("K,D,dt,B", [(180, 183, 1.0, 1), (33, 64, 0.6, 2), (7, 725, 1.0, 1), (5, 1451, 1.0, 1)])
def test_filter_kinds_match_oracle(kind, K, D, dt, B):
    g = fbp.Geometry(K, D, 64, dt, filter=kind)
    P = ph.rng_for(1401, K + D).normal(size=(B, K, D)).astype(np.float32)
    got = fbp.fbp_filter(g, torch.tensor(P, device="cuda")).cpu().numpy()
    ref = oracle.filter_rows(P.astype(np.float64), dt, kind)
    # FP32 dot product over D terms, sum |dt h| <= 1/(2 dt) for all three kernels
    bound = D * 2.0 ** -24 * np.max(np.abs(P)) / (2 * dt) * 4
    assert np.max(np.abs(got - ref)) <= bound, kind


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("weighting", ["uniform", "angle-gaps"])
def test_reconstruction_variants_match_oracle(kind, weighting):
    K, D, N, dt = 120, 149, 100, 1.0
    ang = _clustered(K, 1) if weighting == "angle-gaps" else ph.uniform_angles(K)
    sl = ph.ellipse_slice(1402, 0, N, K, D, dt, n_ellipses=8, angles=ang)
    g = fbp.Geometry(K, D, N, dt, ang, filter=kind, weighting=weighting)
    got = fbp.fbp_reconstruct(g, torch.tensor(sl.sino[None].astype(np.float32), device="cuda")).cpu().numpy()[0]
    ref = oracle.fbp_variant(sl.sino, N, dt, ang, kind, weighted=(weighting == "angle-gaps"))
    m = metrics.compare(got, ref, sl.value_range)
    assert m["max_abs_rel"] <= 2e-4 and m["rmse_rel"] <= 2e-5, (kind, weighting, m)


@pytest.mark.parametrize("K,D,N", [(90, 101, 70), (61, 95, 45)])
def test_weighted_backprojection_every_tile_shape(K, D, N):
    """Angle weights through every tile shape (one-slice, stack and quarter-turn kernels)."""
    ang = _clustered(K, K)
    g = fbp.Geometry(K, D, N, 1.0, ang, weighting="angle-gaps")
    Q = ph.rng_for(1403, K).normal(size=(5, K, D)).astype(np.float32)
    ref = oracle.backproject(Q.astype(np.float64), N, 1.0, ang, oracle.angle_weights(ang))
    tol = 1e-4 * np.max(np.abs(ref)) + 1e-5 * math.pi * np.max(np.abs(Q))
    q = torch.tensor(Q, device="cuda")
    for cfg in range(fbp.fbp_num_tile_configs()):
        try:
            stack = fbp.fbp_backproject_with_config(g, q, cfg).cpu().numpy()
            one = fbp.fbp_backproject_with_config(g, q[:1].contiguous(), cfg).cpu().numpy()
        except fbp.FbpError as e:
            assert e.status == fbp.FBP_EUNSUPPORTED and "rotations" in fbp.fbp_tile_config_name(cfg)
            continue
        assert np.max(np.abs(stack - ref)) <= tol, f"tile {cfg}: stack"
        assert np.max(np.abs(one[0] - ref[0])) <= tol, f"tile {cfg}: single slice"


def test_quarter_turn_shapes_with_weights():
    """Uniform angles with angle-gap weighting (the weights are all pi/K, the
    quarter-turn shapes apply) give the uniform result bit for bit."""
    K, D, N = 120, 145, 100
    Q = torch.tensor(ph.rng_for(1404, 0).normal(size=(2, K, D)).astype(np.float32), device="cuda")
    gu = fbp.Geometry(K, D, N, 1.0)
    gw = fbp.Geometry(K, D, N, 1.0, weighting="angle-gaps")
    for cfg in range(fbp.fbp_num_tile_configs()):
        a = fbp.fbp_backproject_with_config(gu, Q, cfg).cpu().numpy()
        b = fbp.fbp_backproject_with_config(gw, Q, cfg).cpu().numpy()
        assert np.array_equal(a, b), cfg


@pytest.mark.parametrize("prec,min_psnr", [("bf16", 20.0), ("fp16", 55.0)])
@pytest.mark.parametrize("kind", ["shepp-logan", "hann"])
def test_reduced_precision_variants_are_stated(prec, min_psnr, kind):
    K, D, N, dt = 180, 183, 128, 1.0
    sl = ph.ellipse_slice(1405, 0, N, K, D, dt, n_ellipses=10)
    g = fbp.Geometry(K, D, N, dt, filter=kind)
    got = fbp.fbp_reconstruct(g, torch.tensor(sl.sino[None].astype(np.float32), device="cuda"),
                              precision=prec).cpu().numpy()[0]
    m = metrics.compare(got, oracle.fbp_variant(sl.sino, N, dt, sl.angles, kind), sl.value_range)
    print(kind, prec, m)
    assert np.all(np.isfinite(got)) and m["psnr_db"] >= min_psnr, m


def test_batch_mixes_filters_and_weights():
    """One batch with all three kernels and both weightings: every image matches the
    oracle of its own geometry, and equals reconstructing it alone."""
    jobs, refs = [], []
    specs = [(64, 90, 93, "ramlak", "uniform"), (64, 90, 93, "shepp-logan", "uniform"),
             (100, 120, 145, "hann", "angle-gaps"), (48, 40, 71, "shepp-logan", "angle-gaps"),
             (33, 37, 49, "ramlak", "angle-gaps")] * 2
    for i, (N, K, D, kind, w) in enumerate(specs):
        ang = _clustered(K, 10 + i) if w == "angle-gaps" else ph.uniform_angles(K)
        sl = ph.ellipse_slice(1406, i, N, K, D, 1.0, n_ellipses=6, angles=ang)
        g = fbp.Geometry(K, D, N, 1.0, ang, filter=kind, weighting=w)
        img = torch.full((N, N), float("nan"), device="cuda")
        jobs.append((g, torch.tensor(sl.sino.astype(np.float32), device="cuda"), img))
        refs.append((sl, oracle.fbp_variant(sl.sino, N, 1.0, ang, kind, weighted=(w == "angle-gaps"))))
    fbp.fbp_reconstruct_batch(jobs)
    torch.cuda.synchronize()
    for (g, sino, img), (sl, ref) in zip(jobs, refs):
        got = img.cpu().numpy()
        m = metrics.compare(got, ref, sl.value_range)
        assert m["max_abs_rel"] <= 2e-4 and m["rmse_rel"] <= 2e-5, (g.filter, g.weighting, m)
        alone = fbp.fbp_reconstruct(g, sino[None].contiguous()).cpu().numpy()[0]
        assert np.max(np.abs(got - alone)) <= 2e-5 * sl.value_range


@pytest.mark.parametrize("kind", ["ramlak", "hann"])
@pytest.mark.parametrize("K,D", [(720, 725), (180, 183), (90, 1451), (33, 64)])
def test_filter_one_slice_equals_its_place_in_a_stack(kind, K, D):
    """A single slice's filter grid is small, so each tile runs as two groups of
    four waves splitting the k-steps; in a 24-slice stack the tiles run as one
    group (and at other tile widths): the arithmetic order is the same, so the
    filtered rows are bitwise equal."""
    g = fbp.Geometry(K, D, 64, 1.0, filter=kind)
    P = torch.tensor(ph.rng_for(1402, K + D).normal(size=(24, K, D)).astype(np.float32), device="cuda")
    stack = fbp.fbp_filter(g, P).cpu().numpy()
    for s in (0, 11, 23):
        one = fbp.fbp_filter(g, P[s:s + 1].contiguous()).cpu().numpy()[0]
        assert np.array_equal(one, stack[s]), (kind, K, D, s)
