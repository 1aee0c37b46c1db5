"""ctypes binding of libtetrt.so.  Argument marshalling only: every step of the
traversal runs in the library's kernels; PyTorch provides device buffers and
the current HIP stream."""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch  # loads the HIP runtime that the library then shares

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libtetrt.so")

TM_OK, TM_ERR_ARG, TM_ERR_MESH, TM_ERR_OOM, TM_ERR_HIP = 0, -1, -2, -3, -4
RAY_MISS, RAY_STEP_CAP, RAY_INVALID = -1, -2, -3
_LAYOUTS = {"tet20": 0, "tet16": 1, "tet32n": 2}
_SFC = {"hilbert": 0, "morton": 1, "none": 2}


class TetRTError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("tetrt error %d: %s" % (code, msg))
        self.code = code


class _UploadOpts(C.Structure):
    _fields_ = [("layout", C.c_int32), ("sfc", C.c_int32), ("validate", C.c_int32),
                ("seed_grid", C.c_int32)]


class _TraceOpts(C.Structure):
    _fields_ = [("max_steps", C.c_int32), ("block", C.c_int32), ("kernel", C.c_int32),
                ("refill", C.c_int32), ("grid_cap", C.c_int32), ("xcds", C.c_int32),
                ("sort", C.c_int32), ("sort_chunk_log2", C.c_int32), ("sort_cells_log2", C.c_int32),
                ("sort_dirq", C.c_int32), ("eps", C.c_float), ("workspace", C.c_void_p), ("workspace_bytes", C.c_int64),
                ("fp64_steps", C.c_void_p)]

_TRACE_KEYS = ("max_steps", "block", "kernel", "refill", "grid_cap", "xcds", "sort",
               "sort_chunk_log2", "sort_cells_log2", "sort_dirq")


def _trace_opts(kw, workspace=None, fp64_steps=None, n=0):
    o = _TraceOpts()
    for k in _TRACE_KEYS:
        setattr(o, k, int(kw.pop(k, 0)))
    o.eps = float(kw.pop("eps", 0.0))
    if fp64_steps is not None:
        o.fp64_steps = _dev(fp64_steps, torch.int32, n, (), "fp64_steps")
    if kw:
        raise TypeError("unknown trace options: %s" % ", ".join(sorted(kw)))
    if workspace is not None:
        if not isinstance(workspace, torch.Tensor) or workspace.device.type != "cuda":
            raise TypeError("workspace must be a HIP device tensor")
        o.workspace = workspace.data_ptr()
        o.workspace_bytes = workspace.numel() * workspace.element_size()
    return o


class _Info(C.Structure):
    _fields_ = [("n_tets", C.c_int64), ("n_points", C.c_int64), ("n_tris", C.c_int64),
                ("hot_bytes", C.c_int64), ("cold_bytes", C.c_int64), ("layout", C.c_int32),
                ("sfc", C.c_int32), ("seed_grid", C.c_int32), ("reserved", C.c_int32)]


_lib = None


def library_path() -> str:
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise ImportError("libtetrt.so is not built (%s); run __graft_entry__.build() or "
                          "python -m paper_2103_02309_amd.build" % _LIB_PATH)
    L = C.CDLL(_LIB_PATH)
    vp, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
    L.tm_last_error.restype = C.c_char_p
    L.tm_last_error.argtypes = []
    L.tetmesh_upload.restype = C.c_int
    L.tetmesh_upload.argtypes = [vp, i64, vp, vp, vp, i64, C.POINTER(_UploadOpts), C.POINTER(vp)]
    L.trace_closest.restype = C.c_int
    L.trace_closest.argtypes = [vp, i64, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp,
                                C.POINTER(_TraceOpts), vp]
    L.tetmesh_trace_workspace.restype = C.c_int
    L.tetmesh_trace_workspace.argtypes = [vp, i64, vp, C.POINTER(_TraceOpts), C.POINTER(i64)]
    L.tetmesh_locate.restype = C.c_int
    L.tetmesh_locate.argtypes = [vp, i64, vp, vp, vp]
    L.tetmesh_tri_vertices.restype = C.c_int
    L.tetmesh_tri_vertices.argtypes = [vp, i64, vp, vp]
    L.tetmesh_info.restype = C.c_int
    L.tetmesh_info.argtypes = [vp, C.POINTER(_Info)]
    L.tetmesh_free.restype = C.c_int
    L.tetmesh_free.argtypes = [vp]
    L.tetrt_sfc_keys.restype = C.c_int
    L.tetrt_sfc_keys.argtypes = [i32, i32, i64, vp, vp]
    _lib = L
    return L


def tm_last_error() -> str:
    return _load().tm_last_error().decode()


def _check(rc):
    if rc != TM_OK:
        raise TetRTError(rc, tm_last_error())


def _host(a, dtype, shape_tail=None, name="array"):
    a = np.ascontiguousarray(np.asarray(a), dtype=dtype)
    if shape_tail is not None and (a.ndim != 1 + len(shape_tail) or a.shape[1:] != shape_tail):
        raise ValueError("%s must have shape [n, %s]" % (name, ", ".join(map(str, shape_tail))))
    return a


def _dev(t, dtype, n, tail=(), name="tensor", optional=False):
    """Validate a device tensor and return its address (0 for None)."""
    if t is None:
        if optional:
            return None
        raise ValueError("%s is required" % name)
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError("%s must be a HIP device tensor" % name)
    if t.dtype != dtype:
        raise TypeError("%s must be %s, got %s" % (name, dtype, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if tuple(t.shape) != (n,) + tuple(tail):
        raise ValueError("%s must have shape %s, got %s" % (name, (n,) + tuple(tail), tuple(t.shape)))
    return t.data_ptr()


def _stream(stream):
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


# ---- the C-ABI, one function per entry point ---------------------------------------

def tetmesh_upload(points, tets, nbrs, cflag, layout="tet20", sfc="hilbert", validate=True,
                   seed_grid=0):
    """Pack and upload a mesh (host arrays); returns the raw handle (int)."""
    L = _load()
    P = _host(points, np.float32, (3,), "points")
    T = _host(tets, np.int32, (4,), "tets")
    N = _host(nbrs, np.int32, (4,), "nbrs")
    F = _host(cflag, np.uint8, (4,), "cflag")
    if N.shape != T.shape or F.shape != T.shape:
        raise ValueError("tets, nbrs and cflag must have the same shape")
    opts = _UploadOpts(_LAYOUTS[layout], _SFC[sfc], int(bool(validate)), int(seed_grid))
    h = C.c_void_p()
    _check(L.tetmesh_upload(P.ctypes.data, P.shape[0], T.ctypes.data, N.ctypes.data, F.ctypes.data,
                            T.shape[0], C.byref(opts), C.byref(h)))
    return h.value


def trace_closest(handle, orig, dirs, tri, t, bary, tmax=None, start_tet=None, start_face=None,
                  hit_tets=None, steps=None, workspace=None, fp64_steps=None, stream=None, **opts):
    """Enqueue a trace of ``orig``/``dirs`` ([n, 3] float32, device) writing into the
    given device tensors; asynchronous on ``stream`` (default: the current one).
    ``opts``: the tm_trace_opts fields (max_steps, block, kernel, refill, grid_cap,
    xcds, sort, sort_chunk_log2, sort_cells_log2, sort_dirq, eps)."""
    n = int(orig.shape[0]) if orig.dim() >= 1 else 0
    args = [_dev(orig, torch.float32, n, (3,), "orig"), _dev(dirs, torch.float32, n, (3,), "dirs"),
            _dev(tmax, torch.float32, n, (), "tmax", True),
            _dev(start_tet, torch.int32, n, (), "start_tet", True),
            _dev(start_face, torch.int32, n, (), "start_face", True),
            _dev(tri, torch.int32, n, (), "tri"), _dev(t, torch.float32, n, (), "t"),
            _dev(bary, torch.float32, n, (2,), "bary"),
            _dev(hit_tets, torch.int32, n, (2,), "hit_tets", True),
            _dev(steps, torch.int32, n, (), "steps", True)]
    o = _trace_opts(dict(opts), workspace, fp64_steps, n)
    _check(_load().trace_closest(C.c_void_p(handle), n, *args, C.byref(o), _stream(stream)))


def tetmesh_trace_workspace(handle, n_rays, has_tmax, **opts):
    o = _trace_opts(dict(opts))
    b = C.c_int64()
    _check(_load().tetmesh_trace_workspace(C.c_void_p(handle), int(n_rays),
                                           C.c_void_p(1 if has_tmax else 0), C.byref(o),
                                           C.byref(b)))
    return b.value


def tetmesh_locate(handle, pts, out, stream=None):
    n = int(pts.shape[0])
    _check(_load().tetmesh_locate(C.c_void_p(handle), n, _dev(pts, torch.float32, n, (3,), "pts"),
                                  _dev(out, torch.int32, n, (), "out"), _stream(stream)))


def tetmesh_tri_vertices(handle, tri):
    tri = _host(tri, np.int32).reshape(-1)
    out = np.empty((tri.shape[0], 3), np.int32)
    _check(_load().tetmesh_tri_vertices(C.c_void_p(handle), tri.shape[0], tri.ctypes.data,
                                        out.ctypes.data))
    return out


def tetmesh_info(handle):
    info = _Info()
    _check(_load().tetmesh_info(C.c_void_p(handle), C.byref(info)))
    return {k: getattr(info, k) for k, _ in _Info._fields_ if k != "reserved"}


def tetmesh_free(handle):
    _check(_load().tetmesh_free(C.c_void_p(handle)))


def tetrt_sfc_keys(xyz, bits=21, curve="hilbert"):
    xyz = _host(xyz, np.uint32, (3,), "xyz")
    out = np.empty(xyz.shape[0], np.uint64)
    _check(_load().tetrt_sfc_keys(_SFC[curve], int(bits), xyz.shape[0], xyz.ctypes.data,
                                  out.ctypes.data))
    return out


# ---- convenience wrapper --------------------------------------------------------------

class Mesh:
    """An uploaded mesh.  ``trace`` allocates its outputs; ``trace_into`` writes into
    caller tensors (no allocation)."""

    def __init__(self, handle):
        self.handle = handle
        self.info = tetmesh_info(handle)

    def __del__(self):
        self.free()

    def free(self):
        h = getattr(self, "handle", None)
        if h:
            self.handle = None
            tetmesh_free(h)

    def trace(self, orig, dirs, tmax=None, start_tet=None, start_face=None, want_tets=False,
              want_steps=False, want_fp64=False, workspace=None, stream=None, **opts):
        n = int(orig.shape[0])
        dev = orig.device
        out = {"tri": torch.empty(n, dtype=torch.int32, device=dev),
               "t": torch.empty(n, dtype=torch.float32, device=dev),
               "bary": torch.empty((n, 2), dtype=torch.float32, device=dev)}
        if want_tets:
            out["hit_tets"] = torch.empty((n, 2), dtype=torch.int32, device=dev)
        if want_steps:
            out["steps"] = torch.empty(n, dtype=torch.int32, device=dev)
        if want_fp64:
            out["fp64_steps"] = torch.empty(n, dtype=torch.int32, device=dev)
        self.trace_into(out, orig, dirs, tmax, start_tet, start_face, workspace, stream, **opts)
        return out

    def trace_into(self, out, orig, dirs, tmax=None, start_tet=None, start_face=None,
                   workspace=None, stream=None, **opts):
        trace_closest(self.handle, orig, dirs, out["tri"], out["t"], out["bary"], tmax=tmax,
                      start_tet=start_tet, start_face=start_face, hit_tets=out.get("hit_tets"),
                      steps=out.get("steps"), workspace=workspace,
                      fp64_steps=out.get("fp64_steps"), stream=stream, **opts)
        return out

    def workspace_bytes(self, n_rays, has_tmax, **opts):
        return tetmesh_trace_workspace(self.handle, n_rays, has_tmax, **opts)

    def locate(self, pts, stream=None):
        out = torch.empty(int(pts.shape[0]), dtype=torch.int32, device=pts.device)
        tetmesh_locate(self.handle, pts, out, stream)
        return out

    def tri_vertices(self, tri):
        return tetmesh_tri_vertices(self.handle, tri)


def upload(points, tets, nbrs, cflag, **kw) -> Mesh:
    return Mesh(tetmesh_upload(points, tets, nbrs, cflag, **kw))
