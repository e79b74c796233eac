"""Host-side checks of libfbp that need no GPU.

The library loads and exports every function include/fbp.h declares, and its
argument validation returns the documented status codes before any HIP call
(so these run on a machine without a GPU).  Also static checks of the kernel
sources: no atomics, no CUDA headers.
"""
import ctypes
import math
import os
import re

import numpy as np
import pytest

import paper_2109_02174_amd as fbp
from paper_2109_02174_amd import _binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fbp.h")
CSRC = os.path.join(ROOT, "paper_2109_02174_amd", "csrc")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(B.LIB_PATH):
        from paper_2109_02174_amd import build
        build.build()
    return B.load()


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fbp_[a-z_0-9]+)\s*\(", text)))


def test_header_symbols_exported(lib):
    names = _declared_functions()
    assert "fbp_filter" in names and "fbp_backproject" in names and "fbp_reconstruct" in names
    for name in names:
        assert hasattr(lib, name), f"{name} declared in fbp.h but not exported"


def test_status_strings(lib):
    assert fbp.fbp_status_string(0) == "ok"
    for code in (-1, -2, -3, -4, -5, -6):
        s = fbp.fbp_status_string(code)
        assert s and s != "unknown status"
    assert fbp.fbp_status_string(12345) == "unknown status"
    assert "gfx950" in fbp.fbp_version()
    n = fbp.fbp_num_tile_configs()
    assert n >= 1
    for i in range(n):
        assert "tile" in fbp.fbp_tile_config_name(i)
    assert fbp.fbp_tile_config_name(n) == "invalid tile id"


def _geom(K=4, D=7, N=5, dt=1.0, angles=None):
    g = fbp.Geometry(K, D, N, dt, angles)
    return g, g.as_c()


FAKE = 0x100000       # never dereferenced: validation fails before any use
FAKE2 = 0x200000
FAKE3 = 0x300000


@pytest.mark.parametrize("K,D,N,dt", [(0, 7, 5, 1.0), (4, 0, 5, 1.0), (4, 7, 0, 1.0), (4, 7, 5, 0.0),
                                      (4, 7, 5, -1.0), (4, 7, 5, float("nan")), (4, 7, 5, float("inf"))])
def test_invalid_geometry_rejected(lib, K, D, N, dt):
    g = B.c_geom(K, D, N, dt, (ctypes.c_double * max(K, 1))())
    assert lib.fbp_filter(ctypes.byref(g), 1, FAKE, FAKE2, 0, None) == B.FBP_EINVAL
    assert lib.fbp_backproject(ctypes.byref(g), 1, FAKE, FAKE2, None) == B.FBP_EINVAL
    assert lib.fbp_project(ctypes.byref(g), 1, FAKE, FAKE2, None) == B.FBP_EINVAL
    assert lib.fbp_reconstruct(ctypes.byref(g), 1, FAKE, FAKE2, FAKE3, 1 << 20, 0, None) == B.FBP_EINVAL
    assert lib.fbp_workspace_bytes(ctypes.byref(g), 1, 0) == 0


@pytest.mark.parametrize("filt,weighting", [(-1, 0), (3, 0), (0, -1), (0, 2)])
def test_unknown_filter_or_weighting_rejected(lib, filt, weighting):
    ang = (ctypes.c_double * 4)(0.0, 0.5, 1.0, 1.5)
    g = B.c_geom(4, 7, 5, 1.0, ang, filt, weighting)
    assert lib.fbp_filter(ctypes.byref(g), 1, FAKE, FAKE2, 0, None) == B.FBP_EINVAL
    assert lib.fbp_backproject(ctypes.byref(g), 1, FAKE, FAKE2, None) == B.FBP_EINVAL
    assert lib.fbp_workspace_bytes(ctypes.byref(g), 1, 0) == 0


def test_geometry_struct_matches_the_header():
    # the binding's structs follow include/fbp.h field for field
    assert ctypes.sizeof(B.c_geom) == 48 and B.c_geom.filter.offset == 32 and B.c_geom.weighting.offset == 36
    assert B.c_geom.source_distance.offset == 40
    assert ctypes.sizeof(B.c_job) == 64


def test_null_and_nonfinite_angles_rejected(lib):
    g = B.c_geom(4, 7, 5, 1.0, None)
    assert lib.fbp_backproject(ctypes.byref(g), 1, FAKE, FAKE2, None) == B.FBP_EINVAL
    ang = (ctypes.c_double * 4)(0.0, 1.0, float("nan"), 2.0)
    g = B.c_geom(4, 7, 5, 1.0, ang)
    assert lib.fbp_backproject(ctypes.byref(g), 1, FAKE, FAKE2, None) == B.FBP_EINVAL
    assert lib.fbp_backproject(None, 1, FAKE, FAKE2, None) == B.FBP_EINVAL


def test_oversized_geometry_is_unsupported(lib):
    _, g = _geom(D=100000)
    assert lib.fbp_backproject(ctypes.byref(g), 1, FAKE, FAKE2, None) == B.FBP_EUNSUPPORTED
    assert lib.fbp_project(ctypes.byref(g), 1, FAKE, FAKE2, None) == B.FBP_EUNSUPPORTED


def test_pointer_checks(lib):
    _, g = _geom()
    gp = ctypes.byref(g)
    assert lib.fbp_filter(gp, 1, None, FAKE2, 0, None) == B.FBP_EINVAL
    assert lib.fbp_filter(gp, 1, FAKE, None, 0, None) == B.FBP_EINVAL
    assert lib.fbp_filter(gp, 1, FAKE + 2, FAKE2, 0, None) == B.FBP_EINVAL       # misaligned
    assert lib.fbp_filter(gp, 1, FAKE, FAKE + 8, 0, None) == B.FBP_EINVAL         # overlap
    assert lib.fbp_filter(gp, 1, FAKE, FAKE2, 7, None) == B.FBP_EINVAL            # precision
    assert lib.fbp_filter(gp, -1, FAKE, FAKE2, 0, None) == B.FBP_EINVAL
    assert lib.fbp_backproject(gp, 1, FAKE, FAKE + 4, None) == B.FBP_EINVAL      # overlap
    assert lib.fbp_backproject(gp, 1, FAKE, FAKE2 + 1, None) == B.FBP_EINVAL
    assert lib.fbp_project(gp, 1, FAKE, FAKE + 4, None) == B.FBP_EINVAL          # overlap
    assert lib.fbp_project(gp, 1, FAKE + 1, FAKE2, None) == B.FBP_EINVAL          # misaligned
    assert lib.fbp_project(gp, 1, None, FAKE2, None) == B.FBP_EINVAL
    assert lib.fbp_project(gp, -1, FAKE, FAKE2, None) == B.FBP_EINVAL
    # empty calls are valid no-ops that touch nothing
    assert lib.fbp_filter(gp, 0, None, None, 0, None) == B.FBP_OK
    assert lib.fbp_backproject(gp, 0, None, None, None) == B.FBP_OK
    assert lib.fbp_project(gp, 0, None, None, None) == B.FBP_OK
    assert lib.fbp_reconstruct(gp, 0, None, None, None, 0, 0, None) == B.FBP_OK


def test_workspace_checks(lib):
    _, g = _geom(K=4, D=7, N=5)
    gp = ctypes.byref(g)
    need = lib.fbp_workspace_bytes(gp, 3, 0)
    assert need >= 3 * 4 * 7 * 4 and need % 256 == 0
    assert lib.fbp_reconstruct(gp, 3, FAKE, FAKE2, None, need, 0, None) == B.FBP_EWORKSPACE
    assert lib.fbp_reconstruct(gp, 3, FAKE, FAKE2, FAKE3, need - 256, 0, None) == B.FBP_EWORKSPACE
    assert lib.fbp_reconstruct(gp, 3, FAKE, FAKE2, FAKE3 + 16, need, 0, None) == B.FBP_EINVAL
    assert lib.fbp_reconstruct(gp, 3, FAKE, FAKE2, FAKE, need, 0, None) == B.FBP_EINVAL  # aliases sino


def test_batch_validation(lib):
    ang = np.zeros(4)
    jobs = (B.c_job * 2)()
    for j in jobs:
        j.geom = B.c_geom(4, 7, 5, 1.0, ang.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        j.sino = FAKE
        j.image = FAKE2
    jobs[1].sino = FAKE3
    jobs[1].image = FAKE2 + 4096
    need = lib.fbp_batch_workspace_bytes(jobs, 2, 0)
    assert need > 2 * 4 * 7 * 4
    assert lib.fbp_reconstruct_batch(jobs, 2, None, need, 0, None) == B.FBP_EWORKSPACE
    assert lib.fbp_reconstruct_batch(jobs, 2, 0x400000, need - 1, 0, None) == B.FBP_EWORKSPACE
    assert lib.fbp_reconstruct_batch(jobs, 2, 0x400010, need, 0, None) == B.FBP_EINVAL
    assert lib.fbp_reconstruct_batch(jobs, -1, 0x400000, need, 0, None) == B.FBP_EINVAL
    assert lib.fbp_reconstruct_batch(jobs, 0, None, 0, 0, None) == B.FBP_OK
    jobs[1].image = FAKE2 + 16    # two images overlap
    assert lib.fbp_reconstruct_batch(jobs, 2, 0x400000, need, 0, None) == B.FBP_EINVAL
    jobs[1].image = None
    assert lib.fbp_reconstruct_batch(jobs, 2, 0x400000, need, 0, None) == B.FBP_EINVAL


def test_batch_validation_over_many_jobs(lib):
    # 64 jobs sharing two geometry structs: every refusal still comes before any HIP
    # call, whichever job carries the fault and wherever in the list it sits
    ang = np.zeros(4)
    angp = ang.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    n = 64
    jobs = (B.c_job * n)()
    img_bytes = 5 * 5 * 4
    for i, j in enumerate(jobs):
        j.geom = B.c_geom(4, 7, 5, 1.0 if i % 2 else 2.0, angp)
        j.sino = 0x1000000 + 256 * i
        j.image = 0x2000000 + 256 * i          # 100-byte images, 256 bytes apart
    need = lib.fbp_batch_workspace_bytes(jobs, n, 0)
    assert need > 0
    ws = 0x4000000
    # an overlap between two jobs far apart in the list (not neighbours in input order)
    jobs[50].image = jobs[10].image + img_bytes - 4
    assert lib.fbp_reconstruct_batch(jobs, n, ws, need, 0, None) == B.FBP_EINVAL
    jobs[50].image = jobs[10].image + img_bytes   # touching is not overlapping
    jobs[11].image = 0x3000000
    # one job of a repeated geometry made invalid (a struct of its own): still refused
    bad = B.c_geom(4, 7, 5, float("nan"), angp)
    jobs[33].geom = bad
    assert lib.fbp_batch_workspace_bytes(jobs, n, 0) == 0
    assert lib.fbp_reconstruct_batch(jobs, n, ws, need, 0, None) == B.FBP_EINVAL
    jobs[33].geom = B.c_geom(4, 7, 5, 1.0, angp)
    # non-finite angle in the array every job shares
    ang[2] = float("inf")
    assert lib.fbp_reconstruct_batch(jobs, n, ws, need, 0, None) == B.FBP_EINVAL
    ang[2] = 0.0


def test_autotune_and_plan_validation(lib):
    assert lib.fbp_autotune(None, None, None) == B.FBP_EINVAL
    assert lib.fbp_plan_config(None) == B.FBP_EINVAL
    _, g = _geom()
    assert lib.fbp_backproject_with_config(ctypes.byref(g), 1, FAKE, FAKE2, 99, None) == B.FBP_EINVAL


def _kernel_sources():
    return [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".hip", ".cpp", ".hpp"))]


def test_kernels_use_no_atomics_and_no_cuda():
    for path in _kernel_sources():
        text = open(path).read()
        code = re.sub(r"//.*", "", re.sub(r"/\*.*?\*/", "", text, flags=re.S))
        # memory-order constants of a fence are not atomic operations
        code = re.sub(r"__builtin_amdgcn_fence\(__ATOMIC_(RELEASE|ACQUIRE), \"wavefront\"\)", "", code)
        assert not re.search(r"atomic", code, re.I), f"atomic operation in {path}"
        assert "cuda" not in code.lower(), f"CUDA reference in {path}"
        assert "__HIP_PLATFORM" not in code


def test_product_never_touches_oracle():
    pkg = os.path.join(ROOT, "paper_2109_02174_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".cpp", ".hpp", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"^\s*(import|from)\s+oracle\b|liboracle|fbp_oracle", text, re.M), \
                    f"{f} loads the oracle"


@pytest.mark.parametrize("R", [-1.0, float("nan"), float("inf"), 3.0, 5 / math.sqrt(2.0)])
def test_bad_source_distance_rejected(lib, R):
    # the source must stay outside the 5 x 5 image: R > 5 / sqrt(2)
    ang = (ctypes.c_double * 4)(0.0, 0.5, 1.0, 1.5)
    g = B.c_geom(4, 7, 5, 1.0, ang, 0, 0, R)
    assert lib.fbp_filter(ctypes.byref(g), 1, FAKE, FAKE2, 0, None) == B.FBP_EINVAL
    assert lib.fbp_backproject(ctypes.byref(g), 1, FAKE, FAKE2, None) == B.FBP_EINVAL


def test_fan_beam_entry_points(lib):
    ang = (ctypes.c_double * 4)(0.0, 1.5, 3.0, 4.5)
    g = B.c_geom(4, 9, 5, 1.0, ang, 0, 0, 10.0)
    gp = ctypes.byref(g)
    # the projector takes fan geometries (its refusals need the plan, made on a GPU)
    assert lib.fbp_project(gp, 0, None, None, None) == B.FBP_OK
    assert lib.fbp_project(gp, 1, FAKE, FAKE + 4, None) == B.FBP_EINVAL
    assert lib.fbp_plan_config(gp) == B.FBP_EUNSUPPORTED
    assert lib.fbp_plan_stack_config(gp) == B.FBP_EUNSUPPORTED
    assert lib.fbp_backproject_with_config(gp, 1, FAKE, FAKE2, 0, None) == B.FBP_EUNSUPPORTED
    # one fan-beam kernel: nothing to tune, no tile id
    out = ctypes.c_int32(7)
    assert lib.fbp_autotune(gp, None, ctypes.byref(out)) == B.FBP_OK and out.value == -1
    # batches take fan-beam jobs: the workspace is sized for them and checked first
    job = B.c_job(g, FAKE, FAKE2)
    need = lib.fbp_batch_workspace_bytes(ctypes.byref(job), 1, 0)
    assert need >= 4 * 9 * 4
    assert lib.fbp_reconstruct_batch(ctypes.byref(job), 1, FAKE3, need - 1, 0, None) == B.FBP_EWORKSPACE
    # angle-gap weights are parallel-beam only
    g2 = B.c_geom(4, 9, 5, 1.0, ang, 0, 1, 10.0)
    assert lib.fbp_backproject(ctypes.byref(g2), 1, FAKE, FAKE2, None) == B.FBP_EUNSUPPORTED
    # validation still runs first: overlapping buffers are invalid
    assert lib.fbp_backproject(gp, 1, FAKE, FAKE + 4, None) == B.FBP_EINVAL


def test_cone_geometry_struct_matches_the_header():
    assert ctypes.sizeof(B.c_cone_geom) == 56
    assert B.c_cone_geom.det_spacing_u.offset == 24 and B.c_cone_geom.angles.offset == 48


@pytest.mark.parametrize("field,value", [("n_views", 0), ("n_det_u", 0), ("n_det_v", 0), ("volume_size", 0),
                                         ("volume_depth", 0), ("filter", 5), ("det_spacing_u", 0.0),
                                         ("det_spacing_v", float("nan")), ("source_distance", 3.0),
                                         ("source_distance", float("inf"))])
def test_cone_geometry_validation(lib, field, value):
    ang = (ctypes.c_double * 4)(0.0, 1.5, 3.0, 4.5)
    g = B.c_cone_geom(4, 9, 5, 6, 3, 0, 1.0, 1.0, 20.0, ang)
    setattr(g, field, value)
    gp = ctypes.byref(g)
    assert lib.fbp_cone_filter(gp, FAKE, FAKE2, None) == B.FBP_EINVAL
    assert lib.fbp_cone_backproject(gp, FAKE, FAKE2, None) == B.FBP_EINVAL
    assert lib.fbp_cone_reconstruct(gp, FAKE, FAKE2, FAKE3, 1 << 20, None) == B.FBP_EINVAL
    assert lib.fbp_cone_workspace_bytes(gp) == 0


def test_cone_pointer_checks(lib):
    ang = (ctypes.c_double * 4)(0.0, 1.5, 3.0, 4.5)
    g = B.c_cone_geom(4, 9, 5, 6, 3, 0, 1.0, 1.0, 20.0, ang)
    gp = ctypes.byref(g)
    assert lib.fbp_cone_workspace_bytes(gp) == 4 * 5 * 9 * 4 + (256 - (4 * 5 * 9 * 4) % 256)
    assert lib.fbp_cone_filter(gp, None, FAKE2, None) == B.FBP_EINVAL
    assert lib.fbp_cone_filter(gp, FAKE, FAKE + 16, None) == B.FBP_EINVAL             # overlap
    assert lib.fbp_cone_backproject(gp, FAKE, FAKE2 + 2, None) == B.FBP_EINVAL        # misaligned
    assert lib.fbp_cone_reconstruct(gp, FAKE, FAKE2, None, 0, None) == B.FBP_EWORKSPACE
    assert lib.fbp_cone_reconstruct(gp, FAKE, FAKE2, FAKE3, 16, None) == B.FBP_EWORKSPACE
    assert lib.fbp_cone_reconstruct(gp, FAKE, FAKE2, FAKE3 + 4, 1 << 20, None) == B.FBP_EINVAL
    g.angles = None
    assert lib.fbp_cone_filter(gp, FAKE, FAKE2, None) == B.FBP_EINVAL


def test_noalloc_workspace_size_matches_the_header():
    text = open(HEADER).read()
    m = re.search(r"#define FBP_NOALLOC_WORKSPACE_BYTES \(\(size_t\)(\d+) << (\d+)\)", text)
    assert m, "FBP_NOALLOC_WORKSPACE_BYTES not found in fbp.h"
    assert B.NOALLOC_WORKSPACE_BYTES == int(m.group(1)) << int(m.group(2))
    assert "FBP_ENOTREADY = -6" in text and B.FBP_ENOTREADY == -6


def test_noalloc_static_workspace_lives_in_device_memory_of_the_library():
    # the static workspace is a file-scope __device__ array: it occupies no space
    # in the shared object itself (no initialiser), only on each GPU that loads it
    assert os.path.getsize(B.LIB_PATH) < B.NOALLOC_WORKSPACE_BYTES // 8


def test_noalloc_validation_before_any_hip_call(lib):
    # every refusal below comes before the entry point touches HIP (no GPU here)
    _, g = _geom(K=4, D=7, N=5)
    gp = ctypes.byref(g)
    f = lib.fbp_reconstruct_noalloc
    assert f(gp, 0, None, None, 0, None) == B.FBP_OK
    assert f(gp, -1, FAKE, FAKE2, 0, None) == B.FBP_EINVAL
    assert f(gp, 1, None, FAKE2, 0, None) == B.FBP_EINVAL
    assert f(gp, 1, FAKE, None, 0, None) == B.FBP_EINVAL
    assert f(gp, 1, FAKE + 2, FAKE2, 0, None) == B.FBP_EINVAL       # misaligned
    assert f(gp, 1, FAKE, FAKE + 4, 0, None) == B.FBP_EINVAL        # overlap
    assert f(gp, 1, FAKE, FAKE2, 7, None) == B.FBP_EINVAL           # unknown precision
    assert f(None, 1, FAKE, FAKE2, 0, None) == B.FBP_EINVAL
    # filtered rows beyond the static workspace: n * K * D * 4 > 64 MiB
    _, big = _geom(K=720, D=725, N=512)
    n = B.NOALLOC_WORKSPACE_BYTES // (720 * 725 * 4)
    assert f(ctypes.byref(big), n + 1, FAKE, 1 << 40, 0, None) == B.FBP_EWORKSPACE
