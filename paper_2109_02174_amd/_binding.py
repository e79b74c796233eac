"""ctypes binding of libfbp (include/fbp.h): argument marshalling only.

Every function here has the name of the C entry point it wraps and does no
arithmetic of the method: it checks tensor dtype/device/shape, passes device
pointers and the current HIP stream, and raises FbpError on a nonzero status.
All reconstruction work runs in the library's HIP kernels; there is no
fallback of any kind when the library is missing.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfbp.so")

FBP_OK = 0
FBP_EINVAL = -1
FBP_ENOMEM = -2
FBP_EHIP = -3
FBP_EUNSUPPORTED = -4
FBP_EWORKSPACE = -5
FBP_ENOTREADY = -6
NOALLOC_WORKSPACE_BYTES = 64 << 20   # FBP_NOALLOC_WORKSPACE_BYTES

PRECISIONS = {"fp32": 0, "bf16": 1, "fp16": 2, "fft": 3}
FILTERS = {"ramlak": 0, "shepp-logan": 1, "hann": 2}
WEIGHTINGS = {"uniform": 0, "angle-gaps": 1}


class FbpError(RuntimeError):
    def __init__(self, status: int, where: str):
        msg = f"{where}: {fbp_status_string(status)} ({status})"
        if status in (FBP_EHIP, FBP_ENOMEM):
            detail = fbp_last_error()
            if detail:
                msg += f" [{detail}]"
        super().__init__(msg)
        self.status = status


class c_geom(ctypes.Structure):
    _fields_ = [("n_angles", ctypes.c_int32), ("n_det", ctypes.c_int32),
                ("image_size", ctypes.c_int32), ("det_spacing", ctypes.c_double),
                ("angles", ctypes.POINTER(ctypes.c_double)),
                ("filter", ctypes.c_int32), ("weighting", ctypes.c_int32),
                ("source_distance", ctypes.c_double)]


class c_cone_geom(ctypes.Structure):
    _fields_ = [("n_views", ctypes.c_int32), ("n_det_u", ctypes.c_int32), ("n_det_v", ctypes.c_int32),
                ("volume_size", ctypes.c_int32), ("volume_depth", ctypes.c_int32), ("filter", ctypes.c_int32),
                ("det_spacing_u", ctypes.c_double), ("det_spacing_v", ctypes.c_double),
                ("source_distance", ctypes.c_double), ("angles", ctypes.POINTER(ctypes.c_double))]


class c_job(ctypes.Structure):
    _fields_ = [("geom", c_geom), ("sino", ctypes.c_void_p), ("image", ctypes.c_void_p)]


_lib = None


def load():
    """Open libfbp.so (built in-tree by __graft_entry__.build or paper_2109_02174_amd.build)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libfbp.so is not built ({LIB_PATH}); run "
                          "`python -m paper_2109_02174_amd.build` first")
    lib = ctypes.CDLL(LIB_PATH)
    G = ctypes.POINTER(c_geom)
    vp, i32, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_size_t
    sig = {
        "fbp_filter": (ctypes.c_int, [G, i32, vp, vp, i32, vp]),
        "fbp_backproject": (ctypes.c_int, [G, i32, vp, vp, vp]),
        "fbp_project": (ctypes.c_int, [G, i32, vp, vp, vp]),
        "fbp_cone_filter": (ctypes.c_int, [ctypes.POINTER(c_cone_geom), vp, vp, vp]),
        "fbp_cone_backproject": (ctypes.c_int, [ctypes.POINTER(c_cone_geom), vp, vp, vp]),
        "fbp_cone_reconstruct": (ctypes.c_int, [ctypes.POINTER(c_cone_geom), vp, vp, vp, sz, vp]),
        "fbp_cone_workspace_bytes": (sz, [ctypes.POINTER(c_cone_geom)]),
        "fbp_reconstruct": (ctypes.c_int, [G, i32, vp, vp, vp, sz, i32, vp]),
        "fbp_reconstruct_noalloc": (ctypes.c_int, [G, i32, vp, vp, i32, vp]),
        "fbp_workspace_bytes": (sz, [G, i32, i32]),
        "fbp_reconstruct_batch": (ctypes.c_int, [ctypes.POINTER(c_job), i32, vp, sz, i32, vp]),
        "fbp_batch_workspace_bytes": (sz, [ctypes.POINTER(c_job), i32, i32]),
        "fbp_autotune": (ctypes.c_int, [G, vp, ctypes.POINTER(i32)]),
        "fbp_plan_config": (ctypes.c_int, [G]),
        "fbp_plan_stack_config": (ctypes.c_int, [G]),
        "fbp_backproject_with_config": (ctypes.c_int, [G, i32, vp, vp, i32, vp]),
        "fbp_num_tile_configs": (i32, []),
        "fbp_tile_config_name": (ctypes.c_char_p, [i32]),
        "fbp_status_string": (ctypes.c_char_p, [ctypes.c_int]),
        "fbp_version": (ctypes.c_char_p, []),
        "fbp_last_error": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


@dataclass
class Geometry:
    """Geometry: K angles (radians), D bins of width dt, N x N image, the filter kernel
    ("ramlak", "shepp-logan", "hann"), the angular weights ("uniform" pi/K, or
    "angle-gaps" for uneven angle lists) and the source distance (0: parallel beam;
    R > N/sqrt(2): fan beam with a flat detector, the angles being the source
    angles, by default spread over a full turn)."""
    n_angles: int
    n_det: int
    image_size: int
    det_spacing: float = 1.0
    angles: np.ndarray = field(default=None)
    filter: str = "ramlak"
    weighting: str = "uniform"
    source_distance: float = 0.0

    def __post_init__(self):
        if self.angles is None:
            turn = 2.0 * np.pi if self.source_distance > 0 else np.pi
            self.angles = np.arange(self.n_angles, dtype=np.float64) * (turn / self.n_angles)
        self.angles = np.ascontiguousarray(self.angles, dtype=np.float64)

    def as_c(self) -> c_geom:
        """The C struct (cached; the angle array is kept alive with it)."""
        # keyed by the angle array object: the cached struct keeps a reference to it,
        # so numpy refuses to reallocate its buffer in place while the cache holds it
        key = (self.n_angles, self.n_det, self.image_size, self.det_spacing, id(self.angles), self.filter,
               self.weighting, self.source_distance)
        cached = getattr(self, "_c_cache", None)
        if cached is not None and cached[0] == key:
            return cached[1]
        g = c_geom(int(key[0]), int(key[1]), int(key[2]), float(key[3]),
                   self.angles.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                   FILTERS.get(self.filter, -1) if isinstance(self.filter, str) else int(self.filter),
                   WEIGHTINGS.get(self.weighting, -1) if isinstance(self.weighting, str) else int(self.weighting),
                   float(key[7]))
        g._keep = self.angles
        self._c_cache = (key, g)
        return g


def _stream_ptr(stream=None) -> int:
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return int(s.cuda_stream)


def _check_tensor(t, shape, name):
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous float32 tensor on the GPU")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")


def _prec(p) -> int:
    return PRECISIONS[p] if isinstance(p, str) else int(p)


def _raise(rc, where):
    if rc != FBP_OK:
        raise FbpError(rc, where)


def fbp_status_string(status: int) -> str:
    return load().fbp_status_string(int(status)).decode()


def fbp_last_error() -> str:
    """The HIP call behind this thread's last FBP_EHIP / FBP_ENOMEM ("" if none)."""
    return load().fbp_last_error().decode()


def fbp_version() -> str:
    return load().fbp_version().decode()


def fbp_num_tile_configs() -> int:
    return int(load().fbp_num_tile_configs())


def fbp_tile_config_name(i: int) -> str:
    return load().fbp_tile_config_name(int(i)).decode()


def fbp_workspace_bytes(geom: Geometry, n_slices: int, precision="fp32") -> int:
    g = geom.as_c()
    return int(load().fbp_workspace_bytes(ctypes.byref(g), int(n_slices), _prec(precision)))


def _shapes(geom: Geometry, n: int):
    return (n, geom.n_angles, geom.n_det), (n, geom.image_size, geom.image_size)


def fbp_filter(geom: Geometry, sino, out=None, precision="fp32", stream=None):
    """Ramp-filter every row of sino[B][K][D] (device, float32) into out."""
    import torch
    n = sino.shape[0]
    sshape, _ = _shapes(geom, n)
    _check_tensor(sino, sshape, "sino")
    if out is None:
        out = torch.empty_like(sino)
    _check_tensor(out, sshape, "out")
    g = geom.as_c()
    rc = load().fbp_filter(ctypes.byref(g), n, sino.data_ptr(), out.data_ptr(), _prec(precision),
                           _stream_ptr(stream))
    _raise(rc, "fbp_filter")
    return out


def fbp_backproject(geom: Geometry, filtered, out=None, stream=None):
    """Backproject filtered[B][K][D] onto out[B][N][N] (weight pi/K)."""
    import torch
    n = filtered.shape[0]
    sshape, ishape = _shapes(geom, n)
    _check_tensor(filtered, sshape, "filtered")
    if out is None:
        out = torch.empty(ishape, dtype=torch.float32, device=filtered.device)
    _check_tensor(out, ishape, "out")
    g = geom.as_c()
    rc = load().fbp_backproject(ctypes.byref(g), n, filtered.data_ptr(), out.data_ptr(),
                                _stream_ptr(stream))
    _raise(rc, "fbp_backproject")
    return out


def fbp_project(geom: Geometry, image, out=None, stream=None):
    """Forward projection (adjoint of fbp_backproject): image [B][N][N] -> rows [B][K][D]."""
    import torch
    n = image.shape[0]
    sshape, ishape = _shapes(geom, n)
    _check_tensor(image, ishape, "image")
    if out is None:
        out = torch.empty(sshape, dtype=torch.float32, device=image.device)
    _check_tensor(out, sshape, "out")
    g = geom.as_c()
    rc = load().fbp_project(ctypes.byref(g), n, image.data_ptr(), out.data_ptr(), _stream_ptr(stream))
    _raise(rc, "fbp_project")
    return out


def fbp_backproject_with_config(geom: Geometry, filtered, config: int, out=None, stream=None):
    import torch
    n = filtered.shape[0]
    sshape, ishape = _shapes(geom, n)
    _check_tensor(filtered, sshape, "filtered")
    if out is None:
        out = torch.empty(ishape, dtype=torch.float32, device=filtered.device)
    _check_tensor(out, ishape, "out")
    g = geom.as_c()
    rc = load().fbp_backproject_with_config(ctypes.byref(g), n, filtered.data_ptr(), out.data_ptr(),
                                            int(config), _stream_ptr(stream))
    _raise(rc, "fbp_backproject_with_config")
    return out


def alloc_workspace(nbytes: int, device=None):
    """A 256-byte aligned device buffer of at least nbytes (torch allocations are aligned)."""
    import torch
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device or "cuda")


def fbp_reconstruct(geom: Geometry, sino, out=None, workspace=None, precision="fp32", stream=None):
    """Filter + backproject sino[B][K][D] into out[B][N][N]."""
    import torch
    n = sino.shape[0]
    sshape, ishape = _shapes(geom, n)
    _check_tensor(sino, sshape, "sino")
    if out is None:
        out = torch.empty(ishape, dtype=torch.float32, device=sino.device)
    _check_tensor(out, ishape, "out")
    if workspace is None:
        workspace = alloc_workspace(fbp_workspace_bytes(geom, n, precision), sino.device)
    g = geom.as_c()
    rc = load().fbp_reconstruct(ctypes.byref(g), n, sino.data_ptr(), out.data_ptr(),
                                workspace.data_ptr(), workspace.numel() * workspace.element_size(),
                                _prec(precision), _stream_ptr(stream))
    _raise(rc, "fbp_reconstruct")
    return out


def fbp_reconstruct_noalloc(geom: Geometry, sino, out, precision="fp32", stream=None):
    """fbp_reconstruct with the filtered rows in the library's static workspace:
    allocates nothing (`out` is required), and needs the geometry's plan and the
    precision's taps made by an earlier fbp_reconstruct or fbp_filter."""
    n = sino.shape[0]
    sshape, ishape = _shapes(geom, n)
    _check_tensor(sino, sshape, "sino")
    _check_tensor(out, ishape, "out")
    g = geom.as_c()
    rc = load().fbp_reconstruct_noalloc(ctypes.byref(g), n, sino.data_ptr(), out.data_ptr(),
                                        _prec(precision), _stream_ptr(stream))
    _raise(rc, "fbp_reconstruct_noalloc")
    return out


def _jobs_array(jobs):
    """jobs: sequence of (Geometry, sino[K][D] tensor, image[N][N] tensor).  Jobs that
    share a Geometry object share its C struct (and so its angle array)."""
    import torch
    arr = (c_job * max(len(jobs), 1))()
    keep = []
    per_geom = {}
    f32 = torch.float32
    for i, (geom, sino, img) in enumerate(jobs):
        ent = per_geom.get(id(geom))
        if ent is None:
            g = geom.as_c()
            ent = (g, (geom.n_angles, geom.n_det), (geom.image_size, geom.image_size))
            per_geom[id(geom)] = ent
            keep.append((geom, g))
        g, sshape, ishape = ent
        # the checks of _check_tensor, inlined; the named error comes from it
        if not (isinstance(sino, torch.Tensor) and sino.dtype == f32 and sino.is_cuda and sino.is_contiguous()
                and sino.shape == sshape):
            _check_tensor(sino, sshape, f"jobs[{i}].sino")
        if not (isinstance(img, torch.Tensor) and img.dtype == f32 and img.is_cuda and img.is_contiguous()
                and img.shape == ishape):
            _check_tensor(img, ishape, f"jobs[{i}].image")
        job = arr[i]
        job.geom = g
        job.sino = sino.data_ptr()
        job.image = img.data_ptr()
    return arr, keep


def fbp_batch_workspace_bytes(jobs, precision="fp32") -> int:
    arr, _keep = _jobs_array(jobs)
    return int(load().fbp_batch_workspace_bytes(arr, len(jobs), _prec(precision)))


def fbp_reconstruct_batch(jobs, workspace=None, precision="fp32", stream=None):
    """Reconstruct a mixed list of (Geometry, sino, image) slices in one batch."""
    arr, _keep = _jobs_array(jobs)
    nbytes = int(load().fbp_batch_workspace_bytes(arr, len(jobs), _prec(precision)))
    if workspace is None:
        workspace = alloc_workspace(nbytes, jobs[0][1].device if jobs else None)
    rc = load().fbp_reconstruct_batch(arr, len(jobs), workspace.data_ptr(),
                                      workspace.numel() * workspace.element_size(), _prec(precision),
                                      _stream_ptr(stream))
    _raise(rc, "fbp_reconstruct_batch")
    return workspace


def fbp_autotune(geom: Geometry, stream=None) -> int:
    g = geom.as_c()
    out = ctypes.c_int32(-1)
    rc = load().fbp_autotune(ctypes.byref(g), _stream_ptr(stream), ctypes.byref(out))
    _raise(rc, "fbp_autotune")
    return int(out.value)


def fbp_plan_config(geom: Geometry) -> int:
    g = geom.as_c()
    rc = int(load().fbp_plan_config(ctypes.byref(g)))
    if rc < 0:
        raise FbpError(rc, "fbp_plan_config")
    return rc


def fbp_plan_stack_config(geom: Geometry) -> int:
    g = geom.as_c()
    rc = int(load().fbp_plan_stack_config(ctypes.byref(g)))
    if rc < 0:
        raise FbpError(rc, "fbp_plan_stack_config")
    return rc


# ---------------------------------------------------------------- cone beam (FDK)

@dataclass
class ConeGeometry:
    """Circular cone-beam geometry: K source angles (default: a full turn), a flat
    detector of Dv rows x Du columns (spacings dv, du) through the rotation axis,
    source distance R > N/sqrt(2), an Nz x N x N volume, and the filter kernel."""
    n_views: int
    n_det_u: int
    n_det_v: int
    volume_size: int
    volume_depth: int
    source_distance: float
    det_spacing_u: float = 1.0
    det_spacing_v: float = 1.0
    angles: np.ndarray = field(default=None)
    filter: str = "ramlak"

    def __post_init__(self):
        if self.angles is None:
            self.angles = np.arange(self.n_views, dtype=np.float64) * (2.0 * np.pi / self.n_views)
        self.angles = np.ascontiguousarray(self.angles, dtype=np.float64)

    def as_c(self) -> c_cone_geom:
        g = c_cone_geom(int(self.n_views), int(self.n_det_u), int(self.n_det_v), int(self.volume_size),
                        int(self.volume_depth),
                        FILTERS.get(self.filter, -1) if isinstance(self.filter, str) else int(self.filter),
                        float(self.det_spacing_u), float(self.det_spacing_v), float(self.source_distance),
                        self.angles.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        g._keep = self.angles
        return g

    def proj_shape(self):
        return (self.n_views, self.n_det_v, self.n_det_u)

    def volume_shape(self):
        return (self.volume_depth, self.volume_size, self.volume_size)


def fbp_cone_filter(geom: ConeGeometry, proj, out=None, stream=None):
    """FDK pre-weighting and row filter: projections [K][Dv][Du] -> filtered views."""
    import torch
    _check_tensor(proj, geom.proj_shape(), "proj")
    if out is None:
        out = torch.empty(geom.proj_shape(), dtype=torch.float32, device=proj.device)
    _check_tensor(out, geom.proj_shape(), "out")
    g = geom.as_c()
    _raise(load().fbp_cone_filter(ctypes.byref(g), proj.data_ptr(), out.data_ptr(), _stream_ptr(stream)),
           "fbp_cone_filter")
    return out


def fbp_cone_backproject(geom: ConeGeometry, filtered, out=None, stream=None):
    """FDK distance-weighted bilinear backprojection: filtered views -> volume [Nz][N][N]."""
    import torch
    _check_tensor(filtered, geom.proj_shape(), "filtered")
    if out is None:
        out = torch.empty(geom.volume_shape(), dtype=torch.float32, device=filtered.device)
    _check_tensor(out, geom.volume_shape(), "out")
    g = geom.as_c()
    _raise(load().fbp_cone_backproject(ctypes.byref(g), filtered.data_ptr(), out.data_ptr(), _stream_ptr(stream)),
           "fbp_cone_backproject")
    return out


def fbp_cone_workspace_bytes(geom: ConeGeometry) -> int:
    g = geom.as_c()
    return int(load().fbp_cone_workspace_bytes(ctypes.byref(g)))


def fbp_cone_reconstruct(geom: ConeGeometry, proj, out=None, workspace=None, stream=None):
    """FDK reconstruction of projections [K][Dv][Du] into a volume [Nz][N][N]."""
    import torch
    _check_tensor(proj, geom.proj_shape(), "proj")
    if out is None:
        out = torch.empty(geom.volume_shape(), dtype=torch.float32, device=proj.device)
    _check_tensor(out, geom.volume_shape(), "out")
    if workspace is None:
        workspace = alloc_workspace(fbp_cone_workspace_bytes(geom), proj.device)
    g = geom.as_c()
    rc = load().fbp_cone_reconstruct(ctypes.byref(g), proj.data_ptr(), out.data_ptr(), workspace.data_ptr(),
                                     workspace.numel() * workspace.element_size(), _stream_ptr(stream))
    _raise(rc, "fbp_cone_reconstruct")
    return out
