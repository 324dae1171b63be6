"""MI355X-native batched robot-to-obstacle clearance against link-local
signed distance grids (Fujii & Pham, Sec. III-A).

The computation runs in liblsdf.so (HIP, gfx950); this package is its thin
Python binding.
"""
from .lsdf import (GridSet, LsdfError, build_link_sdf, build_robot_grids, fk_batch, last_error,  # noqa: F401
                   load_library, query_min_distance, query_workspace, query_workspace_size, version)

__all__ = ["GridSet", "LsdfError", "build_link_sdf", "build_robot_grids", "fk_batch", "last_error",
           "load_library", "query_min_distance", "query_workspace", "query_workspace_size", "version"]
