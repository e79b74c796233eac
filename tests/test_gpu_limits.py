"""GPU: the largest sizes the library accepts, against the FP64 oracle.

* Filter at the largest detector count (D = 8192): the convolution Q = P * H of
  section "Computed tomography" with the Ram-Lak and Hann kernels (Hann: even taps
  too, the largest tap tables in LDS), for a small grid (two four-wave groups per
  tile) and a grid of more tiles than CUs (one group), element by element.
* Backprojection (Eq. 2) at the largest image side (N = 16384, a 1 GiB image,
  detector capped at 8192 bins, so rays near the corners see zero-extended rows)
  and at the largest angle count (K = 65536: 2048 angle pairs per wave of the
  quarter-turn kernel, 32 rounds of window origins), and at K = 4096 (two rounds)
  for a quarter-turn list and for a list that takes the general tile shapes.

Tolerances as in test_gpu_parity (FP32 dot products of D terms; per-update FP32
coordinate and interpolation error).
"""
import math

import numpy as np
import pytest
import torch

import oracle
import paper_2109_02174_amd as fbp
from paper_2109_02174_amd import phantom as ph

pytestmark = pytest.mark.gpu


def _bp_tol(Q):
    dq = np.max(np.abs(np.diff(Q, axis=-1))) if Q.shape[-1] > 1 else 0.0
    return math.pi * (1e-4 * max(dq, np.max(np.abs(Q))) + 1e-5 * np.max(np.abs(Q))) + 1e-6


@pytest.mark.parametrize("kind", ["ramlak", "hann"])
@pytest.mark.parametrize("K,B", [(32, 1), (96, 1)])   # 1 row tile (small grid); 3 row tiles x 128 column tiles
def test_filter_at_max_detector_count(kind, K, B):
    D = 8192
    g = fbp.Geometry(K, D, 16, 1.0, filter=kind)
    P = ph.rng_for(1700, K).normal(size=(B, K, D)).astype(np.float32)
    got = fbp.fbp_filter(g, torch.tensor(P, device="cuda")).cpu().numpy()
    ref = oracle.filter_rows(P.astype(np.float64), 1.0, kind)
    bound = D * 2.0 ** -24 * np.max(np.abs(P)) / 2.0 * 4
    assert np.max(np.abs(got - ref)) <= bound


def test_detector_count_past_the_limit_is_refused():
    g = fbp.Geometry(2, 8193, 16, 1.0)
    with pytest.raises(fbp.FbpError) as e:
        fbp.fbp_filter(g, torch.zeros((1, 2, 8193), device="cuda"))
    assert e.value.status == fbp.FBP_EUNSUPPORTED


def test_backprojection_at_max_image_side():
    N, K, D = 16384, 4, 8192
    ang = ph.uniform_angles(K)
    g = fbp.Geometry(K, D, N, 1.0, ang)
    Q = ph.rng_for(1701, 0).normal(size=(1, K, D)).astype(np.float32)
    got = fbp.fbp_backproject(g, torch.tensor(Q, device="cuda")).cpu().numpy()[0].astype(np.float64)
    ref = oracle.backproject(Q.astype(np.float64), N, 1.0, ang)[0]
    assert np.max(np.abs(got - ref)) <= _bp_tol(Q)


@pytest.mark.parametrize("K,N,D,kind", [(65536, 16, 25, "uniform"), (4096, 64, 91, "uniform"),
                                        (4096, 64, 91, "random")])
def test_backprojection_at_many_angles(K, N, D, kind):
    if kind == "uniform":
        ang = ph.uniform_angles(K)
    else:
        ang = np.sort(ph.rng_for(1702, K).uniform(0.0, math.pi, K))
    g = fbp.Geometry(K, D, N, 1.0, ang)
    Q = ph.rng_for(1703, K).normal(size=(2, K, D)).astype(np.float32)
    q = torch.tensor(Q, device="cuda")
    ref = oracle.backproject(Q.astype(np.float64), N, 1.0, ang)
    tol = _bp_tol(Q)
    one = fbp.fbp_backproject(g, q[:1].contiguous()).cpu().numpy().astype(np.float64)
    two = fbp.fbp_backproject(g, q).cpu().numpy().astype(np.float64)
    assert np.max(np.abs(one[0] - ref[0])) <= tol
    assert np.max(np.abs(two - ref)) <= tol
    if kind == "uniform":   # quarter-turn kernel: the same bits alone and in a stack
        assert np.array_equal(one[0], two[0])
