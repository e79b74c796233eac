"""FP64 CPU oracle for parallel-beam filtered backprojection.

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the CPU-baseline
leg of the benchmark are the only callers.  The HIP library never imports,
links or executes anything here, and nothing here imports the library.

The arithmetic lives in ``fbp_oracle.c`` (plain FP64 C, OpenMP over output
rows); this module compiles it with gcc when the shared object is missing or
older than the source, and wraps it for NumPy arrays.  See the header of
``fbp_oracle.c`` for the definitions and the readings of the paper
(arXiv 2109.02174, section "Computed tomography", Eq. 2 and the filtered
projection Q = P * H).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fbp_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None


def build(force: bool = False) -> str:
    """Compile ``fbp_oracle.c`` into ``liboracle.so`` with gcc (-O2, OpenMP)."""
    stale = (not os.path.exists(_LIB)) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC)
    if force or stale:
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp", "-fPIC",
               "-shared", "-std=c11", _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def load_library(path: str):
    """Open an oracle shared object and declare its C signatures."""
    lib = ctypes.CDLL(path)
    dp = ctypes.POINTER(ctypes.c_double)
    lib.oracle_filter.argtypes = [dp, ctypes.c_int64, ctypes.c_int32, ctypes.c_double, dp]
    lib.oracle_backproject.argtypes = [dp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                       ctypes.c_int32, ctypes.c_double, dp, dp]
    lib.oracle_fbp.argtypes = lib.oracle_backproject.argtypes
    lib.oracle_forward_splat.argtypes = lib.oracle_backproject.argtypes
    lib.oracle_filter_kind.argtypes = [dp, ctypes.c_int64, ctypes.c_int32, ctypes.c_double, ctypes.c_int32, dp]
    lib.oracle_angle_weights.argtypes = [dp, ctypes.c_int32, dp]
    lib.oracle_backproject_weighted.argtypes = [dp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                                ctypes.c_int32, ctypes.c_double, dp, dp, dp]
    lib.oracle_fan_filter.argtypes = [dp, ctypes.c_int64, ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                                      ctypes.c_int32, dp]
    lib.oracle_fan_backproject.argtypes = [dp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                           ctypes.c_double, ctypes.c_double, dp, dp]
    lib.oracle_fan_fbp.argtypes = [dp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                   ctypes.c_double, ctypes.c_double, dp, dp]
    lib.oracle_fan_splat.argtypes = lib.oracle_fan_fbp.argtypes
    i32, f64 = ctypes.c_int32, ctypes.c_double
    lib.oracle_cone_filter.argtypes = [dp, i32, i32, i32, f64, f64, f64, i32, dp]
    lib.oracle_cone_backproject.argtypes = [dp, i32, i32, i32, i32, i32, f64, f64, f64, dp, dp]
    lib.oracle_cone_fdk.argtypes = lib.oracle_cone_backproject.argtypes
    lib.oracle_cone_splat.argtypes = lib.oracle_cone_backproject.argtypes
    for fn in (lib.oracle_cone_filter, lib.oracle_cone_backproject, lib.oracle_cone_fdk, lib.oracle_cone_splat):
        fn.restype = ctypes.c_int
    for fn in (lib.oracle_filter, lib.oracle_backproject, lib.oracle_fbp,
               lib.oracle_forward_splat, lib.oracle_filter_kind, lib.oracle_angle_weights,
               lib.oracle_backproject_weighted, lib.oracle_fan_filter, lib.oracle_fan_backproject,
               lib.oracle_fan_fbp, lib.oracle_fan_splat):
        fn.restype = ctypes.c_int
    lib.oracle_num_threads.restype = ctypes.c_int
    lib.oracle_set_num_threads.argtypes = [ctypes.c_int]
    lib.oracle_set_num_threads.restype = None
    return lib


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build()
            _lib = load_library(_LIB)
        return _lib


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def num_threads() -> int:
    """OpenMP threads the oracle uses."""
    return int(_load().oracle_num_threads())


def set_num_threads(n: int) -> None:
    _load().oracle_set_num_threads(int(n))


def ramlak_filter(P, dt: float) -> np.ndarray:
    """Ram-Lak filtered rows ``Q[..., n] = dt * sum_m h(n-m) P[..., m]`` (last axis = bins)."""
    P = _f64(P)
    D = P.shape[-1]
    rows = int(np.prod(P.shape[:-1])) if P.ndim > 1 else 1
    Q = np.empty_like(P)
    rc = _load().oracle_filter(_ptr(P), rows, D, float(dt), _ptr(Q))
    if rc != 0:
        raise ValueError("oracle_filter rejected its arguments")
    return Q


FILTERS = {"ramlak": 0, "shepp-logan": 1, "hann": 2}


def filter_rows(P, dt: float, kind: str = "ramlak") -> np.ndarray:
    """Rows filtered with the Ram-Lak, Shepp-Logan or Hann kernel (last axis = bins)."""
    P = _f64(P)
    D = P.shape[-1]
    rows = int(np.prod(P.shape[:-1])) if P.ndim > 1 else 1
    Q = np.empty_like(P)
    rc = _load().oracle_filter_kind(_ptr(P), rows, D, float(dt), FILTERS[kind], _ptr(Q))
    if rc != 0:
        raise ValueError("oracle_filter_kind rejected its arguments")
    return Q


def angle_weights(angles) -> np.ndarray:
    """Quadrature weight of every angle (half the gaps to its neighbours on the half-turn)."""
    ang = _f64(angles).reshape(-1)
    w = np.empty_like(ang)
    rc = _load().oracle_angle_weights(_ptr(ang), ang.shape[0], _ptr(w))
    if rc != 0:
        raise ValueError("oracle_angle_weights rejected its arguments")
    return w


def _geom(arr: np.ndarray, angles):
    ang = _f64(angles).reshape(-1)
    K = ang.shape[0]
    return ang, K


def backproject(Q, N: int, dt: float, angles, weights=None) -> np.ndarray:
    """Backprojection of filtered rows Q[B][K][D] (or [K][D]) onto N x N images, with
    weight pi/K per angle, or the given per-angle weights."""
    Q = _f64(Q)
    squeeze = Q.ndim == 2
    if squeeze:
        Q = Q[None]
    B, K, D = Q.shape
    ang, Ka = _geom(Q, angles)
    if Ka != K:
        raise ValueError("angle count does not match the sinogram")
    img = np.empty((B, N, N), dtype=np.float64)
    if weights is not None:
        w = _f64(weights).reshape(-1)
        if w.shape[0] != K:
            raise ValueError("weight count does not match the angles")
        rc = _load().oracle_backproject_weighted(_ptr(Q), B, K, D, int(N), float(dt), _ptr(ang), _ptr(w),
                                                 _ptr(img))
    else:
        rc = _load().oracle_backproject(_ptr(Q), B, K, D, int(N), float(dt), _ptr(ang), _ptr(img))
    if rc != 0:
        raise ValueError("oracle_backproject rejected its arguments")
    return img[0] if squeeze else img


def fbp(P, N: int, dt: float, angles) -> np.ndarray:
    """Filter then backproject sinograms P[B][K][D] (or [K][D])."""
    P = _f64(P)
    squeeze = P.ndim == 2
    if squeeze:
        P = P[None]
    B, K, D = P.shape
    ang, Ka = _geom(P, angles)
    if Ka != K:
        raise ValueError("angle count does not match the sinogram")
    img = np.empty((B, N, N), dtype=np.float64)
    rc = _load().oracle_fbp(_ptr(P), B, K, D, int(N), float(dt), _ptr(ang), _ptr(img))
    if rc != 0:
        raise ValueError("oracle_fbp rejected its arguments")
    return img[0] if squeeze else img


def fbp_variant(P, N: int, dt: float, angles, kind: str = "ramlak", weighted: bool = False) -> np.ndarray:
    """Filter with the given kernel, then backproject with pi/K or the angle weights."""
    Q = filter_rows(P, dt, kind)
    return backproject(Q, N, dt, angles, angle_weights(angles) if weighted else None)


def forward_splat(img, K: int, D: int, dt: float, angles) -> np.ndarray:
    """Exact adjoint of :func:`backproject` (pixel-driven hat-function splat)."""
    img = _f64(img)
    squeeze = img.ndim == 2
    if squeeze:
        img = img[None]
    B, N, N2 = img.shape
    if N != N2:
        raise ValueError("image must be square")
    ang, Ka = _geom(img, angles)
    if Ka != K:
        raise ValueError("angle count mismatch")
    sino = np.empty((B, K, D), dtype=np.float64)
    rc = _load().oracle_forward_splat(_ptr(img), B, int(K), int(D), N, float(dt), _ptr(ang),
                                      _ptr(sino))
    if rc != 0:
        raise ValueError("oracle_forward_splat rejected its arguments")
    return sino[0] if squeeze else sino


# ---------------------------------------------------------------- fan beam
# Flat detector through the rotation centre, source at distance R (see the
# fan-beam block of fbp_oracle.c for the conventions).

def _views(arr, betas):
    ang = _f64(betas).reshape(-1)
    return ang, ang.shape[0]


def fan_filter(P, ds: float, R: float, kind: str = "ramlak") -> np.ndarray:
    """Pre-weighted, half-kernel filtered views of P[..., D]."""
    P = _f64(P)
    shape = P.shape
    D = shape[-1]
    rows = int(np.prod(shape[:-1])) if len(shape) > 1 else 1
    Q = np.empty_like(P)
    rc = _load().oracle_fan_filter(_ptr(P), rows, D, float(ds), float(R), FILTERS[kind], _ptr(Q))
    if rc != 0:
        raise ValueError("oracle_fan_filter rejected its arguments")
    return Q


def fan_backproject(Q, N: int, ds: float, R: float, betas) -> np.ndarray:
    """Distance-weighted backprojection of filtered views Q[B][K][D] (or [K][D]),
    weight 2 pi / K per view."""
    Q = _f64(Q)
    squeeze = Q.ndim == 2
    if squeeze:
        Q = Q[None]
    B, K, D = Q.shape
    ang, Ka = _views(Q, betas)
    if Ka != K:
        raise ValueError("view count does not match the sinogram")
    img = np.empty((B, N, N), dtype=np.float64)
    rc = _load().oracle_fan_backproject(_ptr(Q), B, K, D, int(N), float(ds), float(R), _ptr(ang), _ptr(img))
    if rc != 0:
        raise ValueError("oracle_fan_backproject rejected its arguments")
    return img[0] if squeeze else img


def fan_fbp(P, N: int, ds: float, R: float, betas) -> np.ndarray:
    """Fan-beam reconstruction (Ram-Lak, weights 2 pi / K) of P[B][K][D] (or [K][D])."""
    P = _f64(P)
    squeeze = P.ndim == 2
    if squeeze:
        P = P[None]
    B, K, D = P.shape
    ang, Ka = _views(P, betas)
    if Ka != K:
        raise ValueError("view count does not match the sinogram")
    img = np.empty((B, N, N), dtype=np.float64)
    rc = _load().oracle_fan_fbp(_ptr(P), B, K, D, int(N), float(ds), float(R), _ptr(ang), _ptr(img))
    if rc != 0:
        raise ValueError("oracle_fan_fbp rejected its arguments")
    return img[0] if squeeze else img


def fan_splat(img, K: int, D: int, ds: float, R: float, betas) -> np.ndarray:
    """Exact adjoint of :func:`fan_backproject` with weights 2 pi / K (tiny grids)."""
    img = _f64(img)
    squeeze = img.ndim == 2
    if squeeze:
        img = img[None]
    B, N, N2 = img.shape
    if N != N2:
        raise ValueError("image must be square")
    ang, Ka = _views(img, betas)
    if Ka != K:
        raise ValueError("view count mismatch")
    sino = np.empty((B, K, D), dtype=np.float64)
    rc = _load().oracle_fan_splat(_ptr(img), B, int(K), int(D), N, float(ds), float(R), _ptr(ang), _ptr(sino))
    if rc != 0:
        raise ValueError("oracle_fan_splat rejected its arguments")
    return sino[0] if squeeze else sino


# ---------------------------------------------------------------- cone beam (FDK)
# Circular source orbit at distance R, flat detector through the axis: columns
# (u, width du) along (-sin b, cos b, 0), rows (v, width dv) along z; projections
# [K][Dv][Du], volumes [Nz][N][N] (see the cone-beam block of fbp_oracle.c).

def cone_filter(P, du: float, dv: float, R: float, kind: str = "ramlak") -> np.ndarray:
    """Pre-weighted, half-kernel row-filtered views P[K][Dv][Du]."""
    P = _f64(P)
    K, Dv, Du = P.shape
    Q = np.empty_like(P)
    rc = _load().oracle_cone_filter(_ptr(P), K, Dv, Du, float(du), float(dv), float(R), FILTERS[kind], _ptr(Q))
    if rc != 0:
        raise ValueError("oracle_cone_filter rejected its arguments")
    return Q


def cone_backproject(Q, N: int, Nz: int, du: float, dv: float, R: float, betas) -> np.ndarray:
    """Distance-weighted bilinear backprojection of filtered views Q[K][Dv][Du]."""
    Q = _f64(Q)
    K, Dv, Du = Q.shape
    ang = _f64(betas).reshape(-1)
    if ang.shape[0] != K:
        raise ValueError("view count does not match the projections")
    vol = np.empty((Nz, N, N), dtype=np.float64)
    rc = _load().oracle_cone_backproject(_ptr(Q), K, Dv, Du, int(N), int(Nz), float(du), float(dv), float(R),
                                         _ptr(ang), _ptr(vol))
    if rc != 0:
        raise ValueError("oracle_cone_backproject rejected its arguments")
    return vol


def cone_fdk(P, N: int, Nz: int, du: float, dv: float, R: float, betas) -> np.ndarray:
    """FDK reconstruction (Ram-Lak) of P[K][Dv][Du]."""
    P = _f64(P)
    K, Dv, Du = P.shape
    ang = _f64(betas).reshape(-1)
    if ang.shape[0] != K:
        raise ValueError("view count does not match the projections")
    vol = np.empty((Nz, N, N), dtype=np.float64)
    rc = _load().oracle_cone_fdk(_ptr(P), K, Dv, Du, int(N), int(Nz), float(du), float(dv), float(R), _ptr(ang),
                                 _ptr(vol))
    if rc != 0:
        raise ValueError("oracle_cone_fdk rejected its arguments")
    return vol


def cone_splat(vol, K: int, Dv: int, Du: int, du: float, dv: float, R: float, betas) -> np.ndarray:
    """Exact adjoint of :func:`cone_backproject` (tiny grids)."""
    vol = _f64(vol)
    Nz, N, N2 = vol.shape
    if N != N2:
        raise ValueError("volume slices must be square")
    ang = _f64(betas).reshape(-1)
    proj = np.empty((K, Dv, Du), dtype=np.float64)
    rc = _load().oracle_cone_splat(_ptr(vol), int(K), int(Dv), int(Du), N, Nz, float(du), float(dv), float(R),
                                   _ptr(ang), _ptr(proj))
    if rc != 0:
        raise ValueError("oracle_cone_splat rejected its arguments")
    return proj
