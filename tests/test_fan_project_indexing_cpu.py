"""CPU replay of the fan-beam forward projector's windows.

The kernel gives each (view, bin) lane, on every image line it walks, a window of
T = floor(2r) + 1 pixels starting at floor(q* - r) + 1, where q* is where the
bin's ray crosses the line and r bounds 1 / |du/dq| over the image grown by a
margin m >= r (r per view and line); the window's start is clamped into the
padded line.  This file
restates in NumPy the host's layout (margin search, tap count, pad, pitch) and
the kernel's FP64 window arithmetic, and asserts for every line of every lane of
the test geometries (sampled for the large ones) that

  * the window stays inside the padded line: 0 <= start, start + T <= pitch, and
    T <= pad, so a clamped window that left the line reads only padding;
  * every image pixel on the line whose hat weight max(0, 1 - |u - j|) is nonzero
    lies inside the window (the weights themselves are recomputed per pixel).

No GPU is involved.
"""
import math

import numpy as np
import pytest


INFL = 1.000244140625


def line_half_width(cb, sb, R, ds, hp, margin, lc, rows):
    ext = hp + 0.5 + margin
    across = np.abs(lc - R * sb) if rows else np.abs(R * cb - lc)
    Lmax = (R + ext * abs(cb) - lc * sb) if rows else (R + ext * abs(sb) - lc * cb)
    return ds * Lmax * Lmax / (R * across) * INFL + 0.000244140625


def layout(N, D, ds, R, betas):
    """(T, margin, pad, pitch), or None where the library refuses the geometry."""
    if not (0.5 * (D - 1) * ds < R):
        return None
    hp = 0.5 * (N - 1)
    lc = np.arange(N, dtype=np.float64) - hp
    m, r_max = 2.0, -1.0
    for _ in range(12):
        r_all = 0.0
        ext = hp + 0.5 + m
        for b in betas:
            cb, sb = math.cos(b), math.sin(b)
            rows = abs(sb) >= abs(cb)
            Lmin = (R - ext * abs(cb) - lc * sb) if rows else (R - ext * abs(sb) - lc * cb)
            if np.any(Lmin <= 0.0):
                return None
            r_all = max(r_all, float(np.max(line_half_width(cb, sb, R, ds, hp, m, lc, rows))))
        if not (r_all < 1024.0):
            return None
        if r_all <= m:
            r_max = r_all
            break
        m = math.ceil(r_all) + 1.0
    if not (r_max > 0.0):
        return None
    T = int(math.floor(2.0 * r_max)) + 1
    return T, m, T + 2, N + 2 * (T + 2)


def check(N, D, ds, R, betas, views=None, bins=None):
    lay = layout(N, D, ds, R, betas)
    assert lay is not None
    T_host, margin, pad, pitch = lay
    hp, cd = 0.5 * (N - 1), 0.5 * (D - 1)
    views = range(len(betas)) if views is None else views
    j = np.arange(D, dtype=np.float64) if bins is None else np.asarray(bins, dtype=np.float64)
    lc = np.arange(N, dtype=np.float64) - hp                 # line coordinates
    q_pix = np.arange(N, dtype=np.float64) - hp              # pixel coordinates along a line
    for k in views:
        cb, sb = math.cos(betas[k]), math.sin(betas[k])
        rows = abs(sb) >= abs(cb)
        # the kernel's per-line half-width, evaluated in FP32 as there
        f = np.float32
        r = line_half_width(f(cb), f(sb), f(R), f(ds), f(hp), f(margin), lc.astype(np.float32), rows)
        r = np.asarray(r, dtype=np.float32).astype(np.float64)
        T = np.floor(2.0 * r).astype(np.int64) + 1           # per line
        assert np.all(T >= 1) and np.all(T <= pad) and np.all(T <= T_host + 1)
        g = cd - j
        Ea = g * R
        Ex = -R * sb / ds - g * cb
        Ey = R * cb / ds - g * sb
        Eq, El = (Ex, Ey) if rows else (Ey, Ex)
        Lq, Ll = (-cb, -sb) if rows else (-sb, -cb)
        q_off = pad + hp
        qs = -(Ea[:, None] + El[:, None] * lc[None, :]) / Eq[:, None]          # [bins, lines]
        st = np.clip(np.floor(qs + q_off - r[None, :]) + 1.0, 0.0, (pitch - T)[None, :])
        assert np.all(st >= 0) and np.all(st + T[None, :] <= pitch)
        # exact weights of every pixel of every line: u - j = E / L
        E = Ea[:, None, None] + Eq[:, None, None] * q_pix[None, None, :] + El[:, None, None] * lc[None, :, None]
        L = R + Lq * q_pix[None, None, :] + Ll * lc[None, :, None]
        assert np.all(L > 0)
        hit = np.abs(E / L) < 1.0                                # [bins, lines, pixels]
        p_idx = q_pix[None, None, :] + q_off                     # padded index of each pixel
        inside = (p_idx >= st[:, :, None]) & (p_idx < st[:, :, None] + T[None, :, None])
        missed = hit & ~inside
        assert not missed.any(), f"view {k}: {int(missed.sum())} weighted pixels outside their windows"


def fan_angles(K):
    return np.arange(K, dtype=np.float64) * (2.0 * math.pi / K)


@pytest.mark.parametrize("N,K,D,ds,R", [
    (40, 96, 61, 1.0, 80.0),
    (33, 40, 41, 1.3, 45.0),        # odd N, dt > 1, source close to the image
    (8, 8, 9, 0.7, 10.0),            # 45-degree views (rows/columns switch), tiny image
    (64, 720, 101, 1.0, 120.0),      # fine view spacing: every octant boundary met
    (1, 4, 1, 1.0, 4.0),             # one pixel, one bin
    (50, 60, 201, 0.5, 60.0),        # dt < 1, long detector (still shorter than R)
])
def test_windows_cover_every_weighted_pixel(N, K, D, ds, R):
    check(N, D, ds, R, fan_angles(K))


def test_benchmark_geometry_sampled():
    # 512^2, 720 views over 2 pi, 801 bins, R = 1024: views near every octant
    # boundary and a spread of bins, every line
    betas = fan_angles(720)
    views = sorted({0, 1, 89, 90, 91, 179, 180, 269, 270, 359, 450, 539, 630, 719})
    check(512, 801, 1.0, 1024.0, betas, views=views, bins=range(0, 801, 7))


def test_refused_geometries():
    # a detector reaching the source distance, and a source too close for the bound
    assert layout(64, 301, 1.0, 100.0, fan_angles(8)) is None
    assert layout(64, 61, 1.0, 46.0, fan_angles(8)) is None


def test_source_close_to_the_image():
    # R = 1.1 N / sqrt(2): wide fan, windows up to 31 pixels on the edge lines
    check(512, 725, 1.0, 400.0, fan_angles(720), views=[0, 45, 90, 135, 180], bins=range(0, 725, 11))


def _gpu_views(K, kind, seed):
    # the views of the GPU fan projector tests (tests/test_gpu_project.py)
    from paper_2109_02174_amd import phantom as ph
    if kind == "uniform":
        return fan_angles(K)
    return np.sort(ph.rng_for(1510, seed).uniform(0.0, 2.0 * math.pi, K))


@pytest.mark.parametrize("K,D,N,dt,R,kind", [
    (96, 61, 40, 1.0, 80.0, "uniform"), (40, 41, 33, 1.3, 45.0, "random"), (64, 49, 32, 1.0, 60.0, "uniform"),
    (25, 31, 17, 0.7, 30.0, "random"), (12, 13, 9, 1.0, 20.0, "random"), (5, 3, 1, 1.0, 4.0, "random"),
    (9, 1, 40, 1.0, 80.0, "random"), (3, 300, 40, 0.25, 80.0, "uniform"), (90, 101, 64, 1.0, 120.0, "uniform"),
])
def test_gpu_test_geometries(K, D, N, dt, R, kind):
    check(N, D, dt, R, _gpu_views(K, kind, K * D + N))


def test_gpu_adjoint_geometry_sampled():
    check(256, 401, 1.0, 400.0, fan_angles(360), views=[0, 45, 90, 135, 200, 359], bins=range(0, 401, 5))


def emulate(img, D, ds, R, betas):
    """The kernel's sums in FP64: per lane and line, the T taps of its window with
    the weight computed from E and L at each tap (padding reads zero)."""
    N = img.shape[0]
    T_host, margin, pad, pitch = layout(N, D, ds, R, betas)
    hp, cd = 0.5 * (N - 1), 0.5 * (D - 1)
    padded_rows = np.zeros((N, pitch))
    padded_rows[:, pad:pad + N] = img
    padded_cols = np.zeros((N, pitch))
    padded_cols[:, pad:pad + N] = img.T
    K = len(betas)
    out = np.zeros((K, D))
    for k, b in enumerate(betas):
        cb, sb = math.cos(b), math.sin(b)
        rows = abs(sb) >= abs(cb)
        plane = padded_rows if rows else padded_cols
        for j in range(D):
            g = cd - j
            Ea, Ex, Ey = g * R, -R * sb / ds - g * cb, R * cb / ds - g * sb
            Eq, El = (Ex, Ey) if rows else (Ey, Ex)
            Lq, Ll = (-cb, -sb) if rows else (-sb, -cb)
            acc = 0.0
            for l in range(N):
                lc = l - hp
                r = float(line_half_width(cb, sb, R, ds, hp, margin, lc, rows))
                T = int(math.floor(2.0 * r)) + 1
                qs = -(Ea + El * lc) / Eq
                st = int(min(max(math.floor(qs + pad + hp - r) + 1.0, 0.0), pitch - T))
                for m in range(T):
                    q = st + m - pad - hp
                    E = Ea + Eq * q + El * lc
                    L = R + Lq * q + Ll * lc
                    acc += max(0.0, 1.0 - abs(E / L)) * (R / L) ** 2 * plane[l, st + m]
            out[k, j] = acc * 2.0 * math.pi / K
    return out


@pytest.mark.parametrize("N,K,D,ds,R", [(12, 16, 17, 1.0, 24.0), (9, 12, 13, 0.8, 20.0), (10, 8, 21, 1.2, 30.0)])
def test_window_sums_equal_the_oracle_adjoint(N, K, D, ds, R):
    import oracle
    betas = fan_angles(K) + 0.1
    img = np.random.default_rng(N * K + D).normal(size=(N, N))
    ref = oracle.fan_splat(img, K, D, ds, R, betas)
    got = emulate(img, D, ds, R, betas)
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))
