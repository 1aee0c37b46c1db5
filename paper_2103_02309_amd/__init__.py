"""tetrt: closest-hit ray traversal through a constrained tetrahedral mesh on
MI355X (gfx950).

The compute path is the C-ABI library ``libtetrt.so`` (HIP kernels and host
packing, declared in ``include/tetrt.h``).  This package is its Python binding:
the functions below carry the library's names and only marshal arguments;
PyTorch supplies device memory and the current stream.
"""
from .binding import (TetRTError, Mesh, upload, tetmesh_upload, trace_closest, trace_closest_noalloc,
                      NOALLOC_MAX_BINNED_RAYS, tetmesh_locate,
                      tetmesh_tri_vertices, tetmesh_info, tetmesh_free, tm_last_error,
                      tetrt_sfc_keys, tetmesh_trace_workspace, tetmesh_bin_rays, library_path, RAY_MISS, RAY_STEP_CAP, RAY_INVALID,
                      Batch, outputs, tm_batch_create, tm_batch_set, tm_batch_launch,
                      tm_batch_graph_launch, tm_batch_tune, tm_batch_free, Server,
                      tm_server_create, tm_server_submit, tm_server_step, tm_server_poll,
                      tm_server_drain, tm_server_pending, tm_server_free, tm_request_rays,
                      REQ_PRIMARY, REQ_SHADOW, REQ_AO)

__all__ = ["TetRTError", "Mesh", "upload", "tetmesh_upload", "trace_closest", "trace_closest_noalloc",
           "NOALLOC_MAX_BINNED_RAYS", "tetmesh_locate",
           "tetmesh_tri_vertices", "tetmesh_info", "tetmesh_free", "tm_last_error",
           "tetrt_sfc_keys", "tetmesh_trace_workspace", "tetmesh_bin_rays", "library_path", "RAY_MISS", "RAY_STEP_CAP", "RAY_INVALID",
           "Batch", "outputs", "tm_batch_create", "tm_batch_set", "tm_batch_launch",
           "tm_batch_graph_launch", "tm_batch_tune", "tm_batch_free", "Server",
           "tm_server_create", "tm_server_submit", "tm_server_step", "tm_server_poll",
           "tm_server_drain", "tm_server_pending", "tm_server_free", "tm_request_rays",
           "REQ_PRIMARY", "REQ_SHADOW", "REQ_AO"]
