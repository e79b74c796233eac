"""GPU: cone-beam FDK (circular orbit, flat detector) element by element against
the FP64 oracle's definition (oracle.cone_filter, oracle.cone_backproject,
oracle.cone_fdk, pinned in test_oracle_pins).

Tolerances.  Filter: an FP32 dot product over Du terms, kernel mass
sum |du h/2| <= 1/(4 du).  Backprojection: per view the column and row
coordinates carry a few FP32 ulps (the row coordinate v = z rho/dv of up to
|z| M / dv rows, rho = R/L relative error a few 2^-24), the weight (R/L)^2 a few
ulps; over K views of weight 2 pi/K the error stays within
2 pi M^2 (1e-5 (1 + |z|max M / dv / 16) max|dQ| + 1e-6 max|Q|), M = R/(R - r).
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


def _views(K, kind, seed):
    if kind == "turn":
        return np.arange(K, dtype=np.float64) * (2.0 * math.pi / K)
    return ph.rng_for(1800, seed).uniform(0.0, 2.0 * math.pi, K)


def _tol(Q, N, Nz, dv, R):
    Q = np.asarray(Q, np.float64)
    M = R / (R - (N - 1) / math.sqrt(2.0))
    dq = max(np.max(np.abs(np.diff(Q, axis=-1))) if Q.shape[-1] > 1 else 0.0,
             np.max(np.abs(np.diff(Q, axis=-2))) if Q.shape[-2] > 1 else 0.0)
    zmax = 0.5 * (Nz - 1)
    return 2.0 * math.pi * M * M * (1e-5 * (1.0 + zmax * M / dv / 16.0) * max(dq, np.max(np.abs(Q))) +
                                    1e-6 * np.max(np.abs(Q))) + 1e-6


@pytest.mark.parametrize("kind", ["ramlak", "hann"])
def test_cone_filter_matches_oracle(kind):
    K, Dv, Du, du, dv, R = 12, 9, 101, 0.8, 1.2, 60.0
    g = fbp.ConeGeometry(K, Du, Dv, 64, 8, R, du, dv, filter=kind)
    P = ph.rng_for(1801, 0).normal(size=(K, Dv, Du)).astype(np.float32)
    got = fbp.fbp_cone_filter(g, torch.tensor(P, device="cuda")).cpu().numpy()
    ref = oracle.cone_filter(P.astype(np.float64), du, dv, R, kind)
    assert np.max(np.abs(got - ref)) <= Du * 2.0 ** -24 * np.max(np.abs(P)) / (4 * du) * 4


@pytest.mark.parametrize("K,Dv,Du,N,Nz,du,dv,Rf,kind", [
    (24, 21, 61, 32, 20, 1.0, 1.0, 1.6, "turn"),
    (17, 45, 49, 27, 33, 1.0, 1.0, 2.0, "random"),     # odd sizes, a ragged second block of slices
    (20, 60, 90, 30, 24, 0.6, 0.7, 1.4, "random"),     # fine detector
    (16, 80, 120, 24, 40, 1.0, 1.0, 1.05, "random"),   # source close to the volume: strong magnification
    (1, 15, 41, 20, 9, 1.0, 1.0, 1.5, "random"),       # one view
    (12, 30, 40, 16, 70, 1.0, 1.5, 2.5, "turn"),       # tall volume: three blocks of slices
    (30, 36, 52, 40, 40, 1.0, 1.0, 2.0, "random"),     # four-column staging, windows past both detector edges
    (30, 36, 44, 40, 40, 1.0, 1.0, 3.0, "turn"),       # four-column staging, a ragged tile and z block
])
def test_cone_backprojection_matches_oracle(K, Dv, Du, N, Nz, du, dv, Rf, kind):
    R = Rf * N / math.sqrt(2.0)
    b = _views(K, kind, K * Du + N)
    g = fbp.ConeGeometry(K, Du, Dv, N, Nz, R, du, dv, b)
    Q = ph.rng_for(1802, K + N).normal(size=(K, Dv, Du)).astype(np.float32)
    got = fbp.fbp_cone_backproject(g, torch.tensor(Q, device="cuda")).cpu().numpy()
    ref = oracle.cone_backproject(Q.astype(np.float64), N, Nz, du, dv, R, b)
    assert np.all(np.isfinite(got))
    assert np.max(np.abs(got - ref)) <= _tol(Q, N, Nz, dv, R)


def test_cone_reconstruction_matches_oracle():
    N, Nz, K, Dv, Du, du, dv = 64, 48, 180, 71, 121, 1.0, 1.0
    R = 2.0 * N / math.sqrt(2.0)
    ells = ph.draw_ellipsoids(ph.rng_for(1803, 0), 8)
    b = _views(K, "turn", 0)
    P = ph.ellipsoid_cone_projections(ells, N, Nz, Dv, Du, du, dv, R, b)
    g = fbp.ConeGeometry(K, Du, Dv, N, Nz, R, du, dv, b)
    got = fbp.fbp_cone_reconstruct(g, torch.tensor(P.astype(np.float32), device="cuda")).cpu().numpy()
    ref = oracle.cone_fdk(P, N, Nz, du, dv, R, b)
    vol = ph.rasterise_volume(ells, N, Nz)
    rng = float(vol.max() - vol.min()) or 1.0
    m = metrics.compare(got, ref, rng)
    print(m)
    assert m["max_abs_rel"] <= 2e-4 and m["rmse_rel"] <= 2e-5, m


def test_cone_paths_agree_bitwise_and_repeat():
    N, Nz, K, Dv, Du = 32, 24, 60, 31, 51
    g = fbp.ConeGeometry(K, Du, Dv, N, Nz, 1.8 * N / math.sqrt(2.0))
    P = torch.tensor(ph.rng_for(1804, 0).normal(size=(K, Dv, Du)).astype(np.float32), device="cuda")
    whole = fbp.fbp_cone_reconstruct(g, P).cpu().numpy()
    two = fbp.fbp_cone_backproject(g, fbp.fbp_cone_filter(g, P)).cpu().numpy()
    assert np.array_equal(whole, two)
    assert np.array_equal(fbp.fbp_cone_reconstruct(g, P).cpu().numpy(), whole)


def test_cone_unaligned_views_match_oracle():
    """Projections at an address that is not a multiple of 16 bytes (a view of a
    larger buffer) are staged one column at a time; the result still agrees with
    the oracle, and with the aligned call within the FP32 tolerance."""
    N, Nz, K, Dv, Du = 40, 40, 30, 36, 52
    R = 2.0 * N / math.sqrt(2.0)
    b = _views(K, "random", 7)
    g = fbp.ConeGeometry(K, Du, Dv, N, Nz, R, 1.0, 1.0, b)
    Q = ph.rng_for(1805, 0).normal(size=(K, Dv, Du)).astype(np.float32)
    buf = torch.zeros(K * Dv * Du + 1, device="cuda")
    buf[1:] = torch.tensor(Q.ravel(), device="cuda")
    shifted = buf[1:].view(K, Dv, Du)
    assert shifted.data_ptr() % 16 != 0
    got = fbp.fbp_cone_backproject(g, shifted).cpu().numpy()
    ref = oracle.cone_backproject(Q.astype(np.float64), N, Nz, 1.0, 1.0, R, b)
    tol = _tol(Q, N, Nz, 1.0, R)
    assert np.max(np.abs(got - ref)) <= tol
    aligned = fbp.fbp_cone_backproject(g, torch.tensor(Q, device="cuda")).cpu().numpy()
    assert np.max(np.abs(aligned - ref)) <= tol


@pytest.mark.parametrize("K,Dv,Du,N,Nz", [(4, 1, 1, 1, 1), (3, 1, 5, 2, 1), (6, 4, 1, 3, 2), (2, 2, 8, 1, 33)])
def test_cone_degenerate_sizes(K, Dv, Du, N, Nz):
    """One voxel, one slice, one detector row or column: still the oracle's values."""
    R = 3.0 + N
    b = _views(K, "random", K + Dv + Du)
    g = fbp.ConeGeometry(K, Du, Dv, N, Nz, R, 1.0, 1.0, b)
    Q = ph.rng_for(1806, K + N).normal(size=(K, Dv, Du)).astype(np.float32)
    got = fbp.fbp_cone_backproject(g, torch.tensor(Q, device="cuda")).cpu().numpy()
    ref = oracle.cone_backproject(Q.astype(np.float64), N, Nz, 1.0, 1.0, R, b)
    assert np.max(np.abs(got - ref)) <= _tol(Q, N, Nz, 1.0, R)


def test_cone_full_size_backprojection_matches_oracle():
    """The benchmark's workload (256^3 volume, 360 views over a full turn, 256 x 384
    detector, R = 512): every voxel of the GPU backprojection against the FP64 oracle
    (about half a minute of host time)."""
    N, Nz, K, Dv, Du, R = 256, 256, 360, 256, 384, 512.0
    b = _views(K, "turn", 0)
    g = fbp.ConeGeometry(K, Du, Dv, N, Nz, R)
    Q = ph.rng_for(1807, 0).normal(size=(K, Dv, Du)).astype(np.float32)
    got = fbp.fbp_cone_backproject(g, torch.tensor(Q, device="cuda")).cpu().numpy()
    print("gpu done", flush=True)
    ref = oracle.cone_backproject(Q.astype(np.float64), N, Nz, 1.0, 1.0, R, b)
    err = np.max(np.abs(got - ref))
    print("max abs error", err, "bound", _tol(Q, N, Nz, 1.0, R), flush=True)
    assert err <= _tol(Q, N, Nz, 1.0, R)
