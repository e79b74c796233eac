"""CPU replay of the cone-beam backprojector's window set-up, packing and LDS indexing.

The cone-beam kernel stages, per block of views, each view's detector window in
LDS, packed back to back, and reads two rows of two columns per voxel from it.
This test restates, in NumPy, the host plan parameters (window bounds, row pitch,
LDS capacity) and the kernel's per-(tile, slice block, view block) steps: the
FP64 window bounds from the tile corners and the block's z extent, the column
alignment, the prefix-sum packing and the views a block takes, the staging
units and their LDS offsets, and the clamps on the sample coordinates.  It
asserts that every LDS write and read stays inside its view's window and the
workgroup's LDS, that every block makes progress, and that the float reciprocal
the staging uses for its row quotient is exact, for the GPU test geometries
and the benchmark workload (256^3 volume, 360 views, 256 x 384 detector, R = 512).
No GPU is involved; a change to the kernel's window arithmetic must be mirrored
here before it runs on a GPU.
"""
import math

import numpy as np
import pytest

TILE, ZB, KB = 16, 32, 16                 # columns per tile side, slices per block, views per block
LDS_BUDGET = 40 * 1024                    # bytes of dynamic LDS per workgroup
COEF = 12                                 # per-view floats before the integer block
PITCHES = [16, 24, 32, 40, 48, 64, 80, 96, 128, 160, 192, 248]


def fan_max_gradient(R, r):
    L = (R - r) + 2.0 * r * np.arange(4097) / 4096
    v2 = np.maximum(0.0, r * r - (R - L) ** 2)
    return 1.01 * float(np.max(R * np.sqrt(L * L + v2) / (L * L)))


def cone_pitch(wl):
    for p in PITCHES:
        if p >= wl + 1:
            return p
    return (wl + 4) // 4 * 4


def plan(N, Nz, Du, Dv, du, dv, R):
    r = 0.70710678118654752 * (N - 1)
    diag = (TILE - 1) * 1.4142135623730951
    half_span = 0.5 * diag * fan_max_gradient(R, r) / du
    rho_max = R / (R - r)
    drho = diag * R / ((R - r) * (R - r))
    span_v = ((ZB - 1) * rho_max + 0.5 * (Nz - 1) * drho) / dv
    WL = int(math.ceil(2.0 * half_span)) + 4
    WV = int(math.ceil(span_v)) + 5
    pitch = cone_pitch(WL + 6 if Du % 4 == 0 else WL)
    head = 4 * COEF * KB + 4 * 8 * KB + 4 * 4           # coefficients, integers, view count
    cap = (LDS_BUDGET - head) // 4
    staged = (WV + 1) * pitch <= cap
    vec4 = staged and Du % 4 == 0 and pitch % 4 == 0 and pitch >= WL + 7
    return dict(WL=WL, WV=WV, pitch=pitch, cap=cap, staged=staged, vec4=vec4)


def check_row_quotient(ng, units):
    """rr = int((e + 1/2) * (1/ng)) in FP32 equals e // ng for every unit e."""
    e = np.arange(units, dtype=np.int64)
    inv = np.float32(1.0) / np.float32(ng)
    rr = ((e.astype(np.float32) + np.float32(0.5)) * inv).astype(np.int64)
    assert np.array_equal(rr, e // ng), f"row quotient inexact for ng={ng}"


def replay(N, Nz, K, Du, Dv, du, dv, R, betas, plan_fn=plan):
    P = plan_fn(N, Nz, Du, Dv, du, dv, R)
    if not P["staged"]:
        return P, 0
    pitch, cap, RW = P["pitch"], P["cap"], P["WV"] + 1
    A = 4 if P["vec4"] else 1
    G = A
    cu, cv = 0.5 * (Du - 1), 0.5 * (Dv - 1)
    half_pix, half_z = 0.5 * (N - 1), 0.5 * (Nz - 1)
    tiles_x = (N + TILE - 1) // TILE
    c = np.cos(betas)
    sn = np.sin(betas)
    # every workgroup (tile, slice block) at once, each with its own view cursor
    t_idx, z_idx = np.meshgrid(np.arange(tiles_x * tiles_x), np.arange((Nz + ZB - 1) // ZB), indexing="ij")
    t_idx, z_idx = t_idx.ravel(), z_idx.ravel()
    c0 = (t_idx % tiles_x) * TILE
    r0 = (t_idx // tiles_x) * TILE
    z0 = z_idx * ZB
    zn = np.minimum(ZB, Nz - z0)
    cw = np.minimum(TILE, N - c0)
    rh = np.minimum(TILE, N - r0)
    zlo = z0 - half_z
    zhi = zlo + (zn - 1)
    xt = c0 - half_pix
    yt = r0 - half_pix
    k0 = np.zeros(t_idx.shape, dtype=np.int64)
    quotients = set()
    blocks = 0
    while np.any(k0 < K):
        live = k0 < K
        nmax = np.minimum(KB, K - k0)
        lanes = np.arange(KB)
        valid = (lanes[None, :] < nmax[:, None]) & live[:, None]
        k = np.minimum(k0[:, None] + lanes[None, :], K - 1)
        ck, sk = c[k], sn[k]
        Lt = R - (ck * xt[:, None] + sk * yt[:, None])
        Nt = R * (-sk * xt[:, None] + ck * yt[:, None])
        Lmin = np.full(k.shape, np.inf)
        Lmax = np.full(k.shape, -np.inf)
        umin = np.full(k.shape, np.inf)
        umax = np.full(k.shape, -np.inf)
        for q in range(4):
            ex = (cw - 1.0) if q & 1 else np.zeros_like(xt)
            ey = (rh - 1.0) if q & 2 else np.zeros_like(yt)
            L = Lt - ck * ex[:, None] - sk * ey[:, None]
            u = (Nt + R * (-sk * ex[:, None] + ck * ey[:, None])) / (L * du)
            Lmin, Lmax = np.minimum(Lmin, L), np.maximum(Lmax, L)
            umin, umax = np.minimum(umin, u), np.maximum(umax, u)
        assert np.all(Lmin[valid] > 0.0)
        rlo, rhi = R / Lmax, R / Lmin
        zl, zh = zlo[:, None], zhi[:, None]
        cand = np.stack([zl * rlo, zl * rhi, zh * rlo, zh * rhi])
        vmin = cand.min(axis=0) / dv
        vmax = cand.max(axis=0) / dv
        i0 = np.floor(umin + cu).astype(np.int64) - 1
        i0a = i0 - np.mod(i0, A)
        j0 = np.floor(vmin + cv).astype(np.int64) - 1
        ncw = np.floor(umax + cu).astype(np.int64) + 3 - i0a
        nc = np.minimum(pitch, (ncw + A - 1) // A * A)
        nr = np.minimum(RW, np.floor(vmax + cv).astype(np.int64) + 4 - j0)
        size = np.where(valid, nr * pitch, 0)
        incl = np.cumsum(size, axis=1)
        off = incl - size
        fit = valid & (incl <= cap)
        nk = fit.sum(axis=1)
        # the views taken are a prefix, and every live block takes at least one
        assert np.all(fit == (lanes[None, :] < nk[:, None]))
        assert np.all(nk[live] >= 1), "a block would take no view"
        take = fit
        # window shape: at least two columns and rows (the clamps of the samples are
        # nc - 2 and nr - 2), no wider than the pitch, no taller than the largest window
        assert np.all(nc[take] >= 2) and np.all(nr[take] >= 2)
        assert np.all(nc[take] <= pitch) and np.all(nr[take] <= RW)
        assert np.all(nc[take] % A == 0)
        # staging: unit e -> (row e // ng, columns G (e % ng) .. + G - 1) at
        # off + row * pitch + col; the last float of the last unit ends the window
        ng = nc // G
        units = ng * nr
        last = off + (nr - 1) * pitch + G * (ng - 1) + (G - 1)
        assert np.all(last[take] < off[take] + nr[take] * pitch)
        assert np.all((off + nr * pitch)[take] <= cap)
        assert np.all(units[take] < 1 << 16)
        for g, n in zip(ng[take].ravel(), units[take].ravel()):
            quotients.add((int(g), int(n)))
        # samples: column iu in [0, nc - 2] (clamp), row iv in [0, nr - 2] (clamp, or
        # the unclamped path when the first and last slices' rows lie in [0, nr - 2]);
        # the reads at iv * pitch + iu + {0, 1, pitch, pitch + 1} stay in the window
        max_read = off + (nr - 2) * pitch + (nc - 2) + pitch + 1
        assert np.all(max_read[take] < off[take] + nr[take] * pitch)
        k0 = np.where(live, k0 + nk, k0)
        blocks += int(live.sum())
    for g, n in sorted(quotients):
        check_row_quotient(g, n)
    return P, blocks


GEOMS = [
    # (K, Dv, Du, N, Nz, du, dv, R / (N / sqrt 2), views)  -- the GPU tests' geometries
    (24, 21, 61, 32, 20, 1.0, 1.0, 1.6, "turn"),
    (17, 45, 49, 27, 33, 1.0, 1.0, 2.0, "random"),
    (20, 60, 90, 30, 24, 0.6, 0.7, 1.4, "random"),
    (16, 80, 120, 24, 40, 1.0, 1.0, 1.05, "random"),
    (1, 15, 41, 20, 9, 1.0, 1.0, 1.5, "random"),
    (12, 30, 40, 16, 70, 1.0, 1.5, 2.5, "turn"),
    (30, 36, 52, 40, 40, 1.0, 1.0, 2.0, "random"),
    (30, 36, 44, 40, 40, 1.0, 1.0, 3.0, "turn"),
    (180, 71, 121, 64, 48, 1.0, 1.0, 2.0, "turn"),
    (60, 31, 51, 32, 24, 1.0, 1.0, 1.8, "turn"),
]


def _views(K, kind, seed):
    if kind == "turn":
        return np.arange(K) * (2.0 * math.pi / K)
    return np.sort(np.random.default_rng(seed).uniform(0.0, 2.0 * math.pi, K))


@pytest.mark.parametrize("geom", GEOMS, ids=[f"K{g[0]}N{g[3]}Nz{g[4]}" for g in GEOMS])
def test_cone_windows_stay_in_bounds(geom):
    K, Dv, Du, N, Nz, du, dv, Rf, kind = geom
    R = Rf * N / math.sqrt(2.0)
    P, blocks = replay(N, Nz, K, Du, Dv, du, dv, R, _views(K, kind, K * Du + N))
    assert P["pitch"] >= P["WL"] + 1


def test_cone_benchmark_geometry_stays_in_bounds():
    N, Nz, K, Dv, Du, R = 256, 256, 360, 256, 384, 512.0
    P, blocks = replay(N, Nz, K, Du, Dv, 1.0, 1.0, R, _views(K, "turn", 0))
    assert P["staged"] and P["vec4"]
    assert blocks > 0


def test_replay_catches_a_plan_whose_windows_overflow_the_lds():
    """The replay has teeth: a plan that keeps staging while its LDS capacity holds
    four rows (every window has at least five) is reported as a block that takes no
    view, which on the GPU would never end."""
    def short_plan(*args):
        P = plan(*args)
        P["cap"] = 4 * P["pitch"]
        return P

    N, Nz, K, Dv, Du, R = 64, 48, 24, 71, 121, 2.0 * 64 / math.sqrt(2.0)
    replay(N, Nz, K, Du, Dv, 1.0, 1.0, R, _views(K, "turn", 0))
    with pytest.raises(AssertionError):
        replay(N, Nz, K, Du, Dv, 1.0, 1.0, R, _views(K, "turn", 0), plan_fn=short_plan)
