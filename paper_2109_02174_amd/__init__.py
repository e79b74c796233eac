"""MI355X (gfx950) filtered backprojection: parallel beam, fan beam and cone beam (FDK).

The reconstruction runs in libfbp.so (hand-written HIP kernels behind the C ABI
of include/fbp.h); this package holds the thin ctypes binding with the same
function names, the seeded synthetic-input generator, image metrics and the
continuous-batching serving loop.
"""
from ._binding import (FBP_EHIP, FBP_EINVAL, FBP_ENOMEM, FBP_ENOTREADY, FBP_EUNSUPPORTED, FBP_EWORKSPACE, FBP_OK,
                       NOALLOC_WORKSPACE_BYTES,
                       ConeGeometry, FbpError, Geometry, alloc_workspace, fbp_cone_backproject, fbp_cone_filter,
                       fbp_cone_reconstruct, fbp_cone_workspace_bytes, fbp_autotune, fbp_backproject,
                       fbp_backproject_with_config, fbp_batch_workspace_bytes, fbp_filter,
                       fbp_num_tile_configs, fbp_plan_config, fbp_plan_stack_config, fbp_project, fbp_reconstruct, fbp_reconstruct_noalloc,
                       fbp_reconstruct_batch, fbp_status_string, fbp_tile_config_name, fbp_version, fbp_last_error,
                       fbp_workspace_bytes, load)

__all__ = [
    "FBP_OK", "FBP_EINVAL", "FBP_ENOMEM", "FBP_EHIP", "FBP_EUNSUPPORTED", "FBP_EWORKSPACE", "FBP_ENOTREADY", "NOALLOC_WORKSPACE_BYTES",
    "ConeGeometry", "FbpError", "Geometry", "alloc_workspace", "fbp_cone_backproject", "fbp_cone_filter",
    "fbp_cone_reconstruct", "fbp_cone_workspace_bytes", "fbp_autotune", "fbp_backproject",
    "fbp_backproject_with_config", "fbp_batch_workspace_bytes", "fbp_filter",
    "fbp_num_tile_configs", "fbp_plan_config", "fbp_plan_stack_config", "fbp_project", "fbp_reconstruct", "fbp_reconstruct_noalloc", "fbp_reconstruct_batch",
    "fbp_status_string", "fbp_tile_config_name", "fbp_version", "fbp_last_error", "fbp_workspace_bytes", "load",
]
