"""Seeded synthetic inputs: analytic sinograms of ellipse phantoms and test objects.

This module is the one input generator shared by the tests, the benchmark and
the serving demo.  It holds none of the reconstruction arithmetic (no filter,
no backprojection): it only evaluates exact line integrals of simple objects
along the rays  x cos(theta) + y sin(theta) = t  (arXiv 2109.02174, section
"Computed tomography") and draws noise.

Conventions (shared with the library and the oracle by specification only):
  * detector bin j sits at t_j = (j - (D-1)/2) * dt, in pixel units;
  * pixel (r, c) of an N x N image sits at x = c - (N-1)/2, y = r - (N-1)/2;
  * ellipse parameters are drawn in normalised units (the image spans
    [-1, 1]^2) and scaled by N/2 to pixel units.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

# Integer tags standing for the string seeds 'geom' and 'arr' of the workload recipes.
SEED_TAG_GEOM = 0x67656F6D
SEED_TAG_ARRIVALS = 0x617272


def rng_for(*key: int) -> np.random.Generator:
    """PCG64 generator seeded by SeedSequence(key), e.g. rng_for(config_id, slice_id)."""
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([int(k) for k in key])))


def uniform_angles(K: int) -> np.ndarray:
    """theta_k = k*pi/K, k = 0..K-1, in FP64."""
    return np.arange(K, dtype=np.float64) * (math.pi / K)


@dataclass(frozen=True)
class Ellipse:
    """One ellipse in normalised units: centre, semi-axes, rotation, density."""
    cx: float
    cy: float
    a: float
    b: float
    phi: float
    rho: float


def draw_ellipses(rng: np.random.Generator, n: int) -> list:
    """Draw n ellipses; per ellipse the draw order is cx, cy, a, b, phi, rho."""
    out = []
    for _ in range(n):
        cx = rng.uniform(-0.7, 0.7)
        cy = rng.uniform(-0.7, 0.7)
        a = rng.uniform(0.05, 0.5)
        b = rng.uniform(0.05, 0.5)
        phi = rng.uniform(0.0, math.pi)
        rho = rng.uniform(-0.5, 1.0)
        out.append(Ellipse(cx, cy, a, b, phi, rho))
    return out


def detector_coords(D: int, dt: float) -> np.ndarray:
    return (np.arange(D, dtype=np.float64) - 0.5 * (D - 1)) * dt


def ellipse_line_integrals(ellipses, N: int, theta, t) -> np.ndarray:
    """Exact line integrals (pixel units) of a sum of ellipses along the lines
    x cos(theta) + y sin(theta) = t (theta, t: arrays of one shape).

    For an ellipse with semi-axes A, B (pixels), rotation phi, centre (x0, y0)
    and density rho, the line integral at (theta, t) is
        2 rho A B sqrt(s^2 - tau^2) / s^2   for |tau| <= s, else 0,
    with s^2 = A^2 cos^2(theta-phi) + B^2 sin^2(theta-phi) and
    tau = t - x0 cos(theta) - y0 sin(theta)  (Kak & Slaney 1988, ch. 3).
    """
    ang = np.asarray(theta, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    half = 0.5 * N
    out = np.zeros(np.broadcast(ang, t).shape, dtype=np.float64)
    ct, st = np.cos(ang), np.sin(ang)
    for e in ellipses:
        A, B = e.a * half, e.b * half
        x0, y0 = e.cx * half, e.cy * half
        s2 = (A * np.cos(ang - e.phi)) ** 2 + (B * np.sin(ang - e.phi)) ** 2
        tau = t - x0 * ct - y0 * st
        rad = s2 - tau * tau
        inside = rad > 0.0
        out += np.where(inside, 2.0 * e.rho * A * B * np.sqrt(np.where(inside, rad, 0.0)) / s2, 0.0)
    return out


def ellipse_sinogram(ellipses, N: int, D: int, dt: float, angles) -> np.ndarray:
    """Exact parallel-beam projections [K][D] (pixel units) of a sum of ellipses."""
    ang = np.asarray(angles, dtype=np.float64).reshape(-1, 1)
    t = detector_coords(D, dt).reshape(1, -1)
    return ellipse_line_integrals(ellipses, N, ang, t)


def fan_rays(R: float, D: int, ds: float, betas):
    """(theta, t) [K][D] of the fan-beam rays: source at R (cos b, sin b), flat
    detector through the centre along (-sin b, cos b), bin j at s_j.  The ray
    through the source and s e has normal angle b + pi/2 - atan(s/R) and
    distance R s / sqrt(R^2 + s^2) from the centre."""
    b = np.asarray(betas, dtype=np.float64).reshape(-1, 1)
    s = detector_coords(D, ds).reshape(1, -1)
    theta = b + 0.5 * math.pi - np.arctan(s / R)
    t = R * s / np.sqrt(R * R + s * s)
    return np.broadcast_to(theta, (b.shape[0], D)), np.broadcast_to(t, (b.shape[0], D))


def ellipse_fan_sinogram(ellipses, N: int, D: int, ds: float, R: float, betas) -> np.ndarray:
    """Exact fan-beam projections [K][D] (pixel units) of a sum of ellipses."""
    theta, t = fan_rays(R, D, ds, betas)
    return ellipse_line_integrals(ellipses, N, theta, t)


def ellipse_sinogram_device(ellipses, N: int, D: int, dt: float, angles, device="cuda"):
    """ellipse_sinogram evaluated with torch in FP64 on `device` (same formula, all
    ellipses at once); for generating large synthetic workloads directly in HBM."""
    import torch
    f64 = torch.float64
    ang = torch.as_tensor(np.asarray(angles, dtype=np.float64), dtype=f64, device=device).view(1, -1, 1)
    t = torch.as_tensor(detector_coords(D, dt), dtype=f64, device=device).view(1, 1, -1)
    half = 0.5 * N
    prm = torch.tensor([[e.a * half, e.b * half, e.cx * half, e.cy * half, e.phi, e.rho] for e in ellipses],
                       dtype=f64, device=device).view(-1, 6, 1, 1)
    A, B, x0, y0, phi, rho = (prm[:, i] for i in range(6))
    s2 = (A * torch.cos(ang - phi)) ** 2 + (B * torch.sin(ang - phi)) ** 2
    tau = t - x0 * torch.cos(ang) - y0 * torch.sin(ang)
    rad = torch.clamp(s2 - tau * tau, min=0.0)
    return (2.0 * rho * A * B * torch.sqrt(rad) / s2).sum(dim=0)


def rasterise(ellipses, N: int) -> np.ndarray:
    """Pixel-centre point samples [N][N] of the phantom (rows = y, columns = x)."""
    half = 0.5 * N
    coord = np.arange(N, dtype=np.float64) - 0.5 * (N - 1)
    x = coord.reshape(1, -1)
    y = coord.reshape(-1, 1)
    img = np.zeros((N, N), dtype=np.float64)
    for e in ellipses:
        A, B = e.a * half, e.b * half
        dx, dy = x - e.cx * half, y - e.cy * half
        u = dx * math.cos(e.phi) + dy * math.sin(e.phi)
        v = -dx * math.sin(e.phi) + dy * math.cos(e.phi)
        img += np.where((u / A) ** 2 + (v / B) ** 2 <= 1.0, e.rho, 0.0)
    return img


def gaussian_sinogram(sigma: float, D: int, dt: float, angles, x0: float = 0.0,
                      y0: float = 0.0) -> np.ndarray:
    """Projections of f = exp(-((x-x0)^2 + (y-y0)^2) / (2 sigma^2)) (peak 1, pixel units)."""
    ang = np.asarray(angles, dtype=np.float64).reshape(-1, 1)
    t = detector_coords(D, dt).reshape(1, -1)
    tau = t - x0 * np.cos(ang) - y0 * np.sin(ang)
    return math.sqrt(2.0 * math.pi) * sigma * np.exp(-tau * tau / (2.0 * sigma * sigma))


def disk_sinogram(radius: float, rho: float, D: int, dt: float, angles, x0: float = 0.0,
                  y0: float = 0.0) -> np.ndarray:
    """Projections of a uniform disk: 2 rho sqrt(R^2 - tau^2) for |tau| <= R."""
    ang = np.asarray(angles, dtype=np.float64).reshape(-1, 1)
    t = detector_coords(D, dt).reshape(1, -1)
    tau = t - x0 * np.cos(ang) - y0 * np.sin(ang)
    rad = radius * radius - tau * tau
    return np.where(rad > 0.0, 2.0 * rho * np.sqrt(np.maximum(rad, 0.0)), 0.0)


def add_gaussian_noise(sino: np.ndarray, rng: np.random.Generator, rel_sigma: float) -> np.ndarray:
    """i.i.d. N(0, (rel_sigma * max(sino))^2) on every bin."""
    sigma = rel_sigma * float(np.max(sino))
    return sino + rng.normal(0.0, sigma, size=sino.shape)


def add_poisson_noise(sino: np.ndarray, rng: np.random.Generator, I0: float, N: int) -> np.ndarray:
    """Photon-count noise on the Lambert-Beer model I = I0 exp(-mu d).

    Line integrals are taken in normalised length units (image half-width 1):
    counts n ~ Poisson(I0 exp(-p/(N/2))), n <- max(n, 1), and the noisy line
    integral is -ln(n/I0) * (N/2) in pixel units.
    """
    half = 0.5 * N
    lam = I0 * np.exp(-sino / half)
    counts = np.maximum(rng.poisson(lam), 1).astype(np.float64)
    return -np.log(counts / I0) * half


@dataclass(frozen=True)
class SliceInput:
    sino: np.ndarray        # FP64 [K][D]
    phantom: np.ndarray     # FP64 [N][N] pixel-centre raster
    ellipses: tuple
    N: int
    K: int
    D: int
    dt: float
    angles: np.ndarray

    @property
    def value_range(self) -> float:
        """Phantom range R = max - min of the raster (1.0 if the raster is flat)."""
        r = float(self.phantom.max() - self.phantom.min())
        return r if r > 0 else 1.0


def ellipse_slice(config_id: int, slice_id: int, N: int, K: int, D: int, dt: float = 1.0,
                  n_ellipses: int = 20, noise: str | None = None, angles=None,
                  gauss_rel_sigma: float = 0.01, I0: float = 1e5) -> SliceInput:
    """One seeded ellipse-phantom slice: ellipses first, then noise, from one generator."""
    rng = rng_for(config_id, slice_id)
    ells = draw_ellipses(rng, n_ellipses)
    ang = uniform_angles(K) if angles is None else np.asarray(angles, dtype=np.float64)
    sino = ellipse_sinogram(ells, N, D, dt, ang)
    if noise == "gauss":
        sino = add_gaussian_noise(sino, rng, gauss_rel_sigma)
    elif noise == "poisson":
        sino = add_poisson_noise(sino, rng, I0, N)
    elif noise is not None:
        raise ValueError(f"unknown noise model {noise!r}")
    return SliceInput(sino, rasterise(ells, N), tuple(ells), N, K, D, dt, ang)



def disk_fan_sinogram(radius: float, rho: float, D: int, ds: float, R: float, betas, x0: float = 0.0,
                      y0: float = 0.0) -> np.ndarray:
    """Fan-beam projections of a uniform disk: 2 rho sqrt(radius^2 - tau^2) along each ray."""
    theta, t = fan_rays(R, D, ds, betas)
    tau = t - x0 * np.cos(theta) - y0 * np.sin(theta)
    rad = radius * radius - tau * tau
    return np.where(rad > 0.0, 2.0 * rho * np.sqrt(np.maximum(rad, 0.0)), 0.0)


def fan_slice(config_id: int, slice_id: int, N: int, K: int, D: int, ds: float, R: float,
              n_ellipses: int = 20, betas=None) -> SliceInput:
    """One seeded ellipse-phantom fan-beam slice (views evenly spread over a full turn
    unless given); `angles` of the result holds the source angles."""
    rng = rng_for(config_id, slice_id)
    ells = draw_ellipses(rng, n_ellipses)
    b = np.arange(K, dtype=np.float64) * (2.0 * math.pi / K) if betas is None else np.asarray(betas, np.float64)
    sino = ellipse_fan_sinogram(ells, N, D, ds, R, b)
    return SliceInput(sino, rasterise(ells, N), tuple(ells), N, K, D, ds, b)


# ---------------------------------------------------------------- cone beam (3D)
# Circular orbit: source at (R cos b, R sin b, 0); flat detector through the axis,
# columns along (-sin b, cos b, 0) at s_i = (i - (Du-1)/2) du, rows along z at
# z_j = (j - (Dv-1)/2) dv; volume voxel (p, r, c) at (c - (N-1)/2, r - (N-1)/2,
# p - (Nz-1)/2) in voxel units.

@dataclass(frozen=True)
class Ellipsoid:
    cx: float
    cy: float
    cz: float
    a: float
    b: float
    c: float
    phi: float      # rotation about z
    rho: float


def draw_ellipsoids(rng: np.random.Generator, n: int) -> list:
    """n ellipsoids in normalised units (the volume spans [-1, 1]^3)."""
    out = []
    for _ in range(n):
        cx, cy, cz = rng.uniform(-0.5, 0.5, 3)
        a, b, c = rng.uniform(0.08, 0.4, 3)
        out.append(Ellipsoid(float(cx), float(cy), float(cz), float(a), float(b), float(c),
                             float(rng.uniform(0.0, math.pi)), float(rng.uniform(-0.5, 1.0))))
    return out


def cone_rays(R: float, Dv: int, Du: int, du: float, dv: float, betas):
    """Source points [K][3] and unit ray directions [K][Dv][Du][3]."""
    b = np.asarray(betas, dtype=np.float64).reshape(-1)
    S = np.stack([R * np.cos(b), R * np.sin(b), np.zeros_like(b)], axis=-1)
    e = np.stack([-np.sin(b), np.cos(b), np.zeros_like(b)], axis=-1)
    s = detector_coords(Du, du)
    z = detector_coords(Dv, dv)
    P = (e[:, None, None, :] * s[None, None, :, None] +
         np.array([0.0, 0.0, 1.0])[None, None, None, :] * z[None, :, None, None])
    d = P - S[:, None, None, :]
    d /= np.linalg.norm(d, axis=-1, keepdims=True)
    return S, d


def ellipsoid_cone_projections(ellipsoids, N: int, Nz: int, Dv: int, Du: int, du: float, dv: float, R: float,
                               betas) -> np.ndarray:
    """Exact cone-beam line integrals [K][Dv][Du] (voxel units) of a sum of ellipsoids:
    each ray is mapped into the ellipsoid's unit-sphere frame, where the chord length
    follows from a quadratic."""
    S, d = cone_rays(R, Dv, Du, du, dv, betas)
    half = 0.5 * N
    out = np.zeros(d.shape[:3], dtype=np.float64)
    for el in ellipsoids:
        C = np.array([el.cx * half, el.cy * half, el.cz * half])
        cph, sph = math.cos(el.phi), math.sin(el.phi)
        rot_t = np.array([[cph, sph, 0.0], [-sph, cph, 0.0], [0.0, 0.0, 1.0]])   # world -> body
        scale = np.array([1.0 / (el.a * half), 1.0 / (el.b * half), 1.0 / (el.c * half)])
        Y0 = (rot_t @ (S - C).T).T * scale                      # [K][3]
        Dy = np.einsum("ij,kvuj->kvui", rot_t, d) * scale       # [K][Dv][Du][3]
        aa = np.sum(Dy * Dy, axis=-1)
        bb = np.sum(Dy * Y0[:, None, None, :], axis=-1)
        cc = np.sum(Y0 * Y0, axis=-1)[:, None, None] - 1.0
        disc = bb * bb - aa * cc
        out += np.where(disc > 0.0, el.rho * 2.0 * np.sqrt(np.maximum(disc, 0.0)) / aa, 0.0)
    return out


def ball_cone_projections(radius: float, rho: float, Dv: int, Du: int, du: float, dv: float, R: float, betas,
                          centre=(0.0, 0.0, 0.0)) -> np.ndarray:
    """Cone-beam projections of a uniform ball: 2 rho sqrt(radius^2 - dist^2) along each ray."""
    S, d = cone_rays(R, Dv, Du, du, dv, betas)
    C = np.asarray(centre, dtype=np.float64)
    w = C[None, :] - S                                           # source -> centre
    t = np.sum(d * w[:, None, None, :], axis=-1)
    dist2 = np.sum(w * w, axis=-1)[:, None, None] - t * t
    rad = radius * radius - dist2
    return np.where(rad > 0.0, 2.0 * rho * np.sqrt(np.maximum(rad, 0.0)), 0.0)


def rasterise_volume(ellipsoids, N: int, Nz: int) -> np.ndarray:
    """Voxel-centre samples [Nz][N][N] of the ellipsoid phantom."""
    half = 0.5 * N
    x = (np.arange(N, dtype=np.float64) - 0.5 * (N - 1)).reshape(1, 1, -1)
    y = (np.arange(N, dtype=np.float64) - 0.5 * (N - 1)).reshape(1, -1, 1)
    z = (np.arange(Nz, dtype=np.float64) - 0.5 * (Nz - 1)).reshape(-1, 1, 1)
    vol = np.zeros((Nz, N, N), dtype=np.float64)
    for el in ellipsoids:
        dx, dy, dz = x - el.cx * half, y - el.cy * half, z - el.cz * half
        u = dx * math.cos(el.phi) + dy * math.sin(el.phi)
        v = -dx * math.sin(el.phi) + dy * math.cos(el.phi)
        vol += np.where((u / (el.a * half)) ** 2 + (v / (el.b * half)) ** 2 + (dz / (el.c * half)) ** 2 <= 1.0,
                        el.rho, 0.0)
    return vol
