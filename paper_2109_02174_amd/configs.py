"""The five workloads: geometry and phantom recipe of each.

These stand in for the paper's Visible Human slice set (arXiv 2109.02174,
section "Benchmark"), which is not available: seeded random-ellipse phantoms
with exact analytic sinograms, at the sizes below.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from .phantom import SEED_TAG_GEOM, rng_for


@dataclass(frozen=True)
class SliceGeom:
    N: int          # image side (pixels)
    K: int          # angles, theta_k = k pi / K
    D: int          # detector bins
    dt: float = 1.0 # bin width in pixel units

    @property
    def updates(self) -> int:
        """Pixel-angle updates of one backprojection: N^2 K."""
        return self.N * self.N * self.K


# Single slice 128^2, 180 angles, 183 bins, 10 ellipses, Gaussian noise 1% of max.
C1 = dict(config_id=1, geom=SliceGeom(128, 180, 183), n_ellipses=10, noise="gauss")
# Single slice 512^2, 720 angles, 725 bins, 20 ellipses, Poisson noise I0 = 1e5.
C2 = dict(config_id=2, geom=SliceGeom(512, 720, 725), n_ellipses=20, noise="poisson")
# 256-slice stack of the C2 geometry, noise-free, three filter precisions.
C3 = dict(config_id=3, geom=SliceGeom(512, 720, 725), n_ellipses=20, noise=None, n_slices=256)

C4_SIDES = (256, 384, 512, 1024)
C4_ANGLES = (360, 720, 1440)


def c4_detectors(side: int) -> int:
    """ceil(sqrt(2) side) + 2 bins: the image diagonal plus a margin."""
    return int(math.ceil(math.sqrt(2.0) * side)) + 2


def c4_geometries(n_slices: int = 1000) -> list:
    """Mixed-size batch: side and angle count drawn independently per slice."""
    rng = rng_for(4, SEED_TAG_GEOM)
    sides = rng.integers(0, len(C4_SIDES), size=n_slices)
    angs = rng.integers(0, len(C4_ANGLES), size=n_slices)
    return [SliceGeom(C4_SIDES[s], C4_ANGLES[a], c4_detectors(C4_SIDES[s]))
            for s, a in zip(sides, angs)]


def c1_slice():
    from .phantom import ellipse_slice
    g = C1["geom"]
    return ellipse_slice(1, 0, g.N, g.K, g.D, g.dt, n_ellipses=10, noise="gauss")


def c2_slice():
    from .phantom import ellipse_slice
    g = C2["geom"]
    return ellipse_slice(2, 0, g.N, g.K, g.D, g.dt, n_ellipses=20, noise="poisson")


def uniform_angles(K: int) -> np.ndarray:
    return np.arange(K, dtype=np.float64) * (math.pi / K)
