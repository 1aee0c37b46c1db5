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
_LAYOUTS = {"tet20": 0, "tet16": 1, "tet32n": 2, "tet32": 3}
_SFC = {"hilbert": 0, "morton": 1, "none": 2, "hilbert_regions": 3}


class TetRTError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("tetrt error %d: %s" % (code, msg))
        self.code = code


class _UploadOpts(C.Structure):
    _fields_ = [("layout", C.c_int32), ("sfc", C.c_int32), ("validate", C.c_int32),
                ("seed_grid", C.c_int32), ("bin_rays", C.c_int64)]


class _TraceOpts(C.Structure):
    _fields_ = [("max_steps", C.c_int32), ("block", C.c_int32), ("kernel", C.c_int32),
                ("refill", C.c_int32), ("grid_cap", C.c_int32), ("xcds", C.c_int32),
                ("sort", C.c_int32), ("sort_chunk_log2", C.c_int32), ("sort_cells_log2", C.c_int32),
                ("sort_dirq", C.c_int32), ("xcd_blocks", C.c_int32), ("eps", C.c_float), ("workspace", C.c_void_p), ("workspace_bytes", C.c_int64),
                ("fp64_steps", C.c_void_p), ("order", C.c_void_p), ("queue_chunk", C.c_int32),
                ("passes", C.c_int32)]

_TRACE_KEYS = ("max_steps", "block", "kernel", "refill", "grid_cap", "xcds", "sort",
               "sort_chunk_log2", "sort_cells_log2", "sort_dirq", "xcd_blocks", "queue_chunk", "passes")


def _trace_opts(kw, workspace=None, fp64_steps=None, n=0):
    o = _TraceOpts()
    for k in _TRACE_KEYS:
        setattr(o, k, int(kw.pop(k, 0)))
    o.eps = float(kw.pop("eps", 0.0))
    if fp64_steps is not None:
        o.fp64_steps = _dev(fp64_steps, torch.int32, n, (), "fp64_steps")
    order = kw.pop("order", None)
    if order is not None:
        o.order = _dev(order, torch.int32, n, (), "order")
    if kw:
        raise TypeError("unknown trace options: %s" % ", ".join(sorted(kw)))
    if workspace is not None:
        if not isinstance(workspace, torch.Tensor) or workspace.device.type != "cuda":
            raise TypeError("workspace must be a HIP device tensor")
        o.workspace = workspace.data_ptr()
        o.workspace_bytes = workspace.numel() * workspace.element_size()
    return o


class _Job(C.Structure):
    _fields_ = [("mesh", C.c_void_p), ("n_rays", C.c_int64), ("d_orig", C.c_void_p),
                ("d_dir", C.c_void_p), ("d_tmax", C.c_void_p), ("d_start_tet", C.c_void_p),
                ("d_start_face", C.c_void_p), ("d_tri", C.c_void_p), ("d_t", C.c_void_p),
                ("d_bary", C.c_void_p), ("d_hit_tets", C.c_void_p), ("d_steps", C.c_void_p)]


class _Request(C.Structure):
    _fields_ = [("mesh", C.c_int32), ("kind", C.c_int32), ("width", C.c_int32), ("height", C.c_int32),
                ("eye", C.c_float * 3), ("forward", C.c_float * 3), ("up", C.c_float * 3),
                ("fov_h_deg", C.c_float), ("light", C.c_float * 3), ("ao_tmax", C.c_float),
                ("seed", C.c_uint32), ("d_tri", C.c_void_p), ("d_t", C.c_void_p), ("d_bary", C.c_void_p)]


class _ServerOpts(C.Structure):
    _fields_ = [("max_rays", C.c_int64), ("max_requests", C.c_int32), ("ring", C.c_int32),
                ("block", C.c_int32), ("sort", C.c_int32), ("max_steps", C.c_int32),
                ("eps", C.c_float)]


class _Done(C.Structure):
    _fields_ = [("id", C.c_int64), ("submit_ns", C.c_int64), ("admit_ns", C.c_int64),
                ("done_ns", C.c_int64), ("rays", C.c_int64)]


REQ_PRIMARY, REQ_SHADOW, REQ_AO = 0, 1, 2
_KINDS = {"primary": 0, "shadow": 1, "ao": 2}


class _Info(C.Structure):
    _fields_ = [("n_tets", C.c_int64), ("n_points", C.c_int64), ("n_tris", C.c_int64),
                ("hot_bytes", C.c_int64), ("cold_bytes", C.c_int64), ("layout", C.c_int32),
                ("sfc", C.c_int32), ("seed_grid", C.c_int32), ("n_regions", C.c_int32)]


_lib = None


def library_path() -> str:
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise ImportError("libtetrt.so is not built (%s); run python -m paper_2103_02309_amd.build"
                          % _LIB_PATH)
    L = C.CDLL(_LIB_PATH)
    vp, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
    L.tm_last_error.restype = C.c_char_p
    L.tm_last_error.argtypes = []
    L.tetmesh_upload.restype = C.c_int
    L.tetmesh_upload.argtypes = [vp, i64, vp, vp, vp, i64, C.POINTER(_UploadOpts), C.POINTER(vp)]
    L.trace_closest.restype = C.c_int
    L.trace_closest.argtypes = [vp, i64, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp,
                                C.POINTER(_TraceOpts), vp]
    L.trace_closest_noalloc.restype = C.c_int
    L.trace_closest_noalloc.argtypes = [vp, i64, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp,
                                        C.POINTER(_TraceOpts), vp]
    L.tetmesh_trace_workspace.restype = C.c_int
    L.tetmesh_trace_workspace.argtypes = [vp, i64, vp, C.POINTER(_TraceOpts), C.POINTER(i64)]
    L.tetmesh_bin_rays.restype = C.c_int
    L.tetmesh_bin_rays.argtypes = [vp, i64, vp, vp, C.POINTER(_TraceOpts), vp, vp]
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
    L.tm_batch_create.restype = C.c_int
    L.tm_batch_create.argtypes = [i32, i64, C.POINTER(vp)]
    L.tm_batch_set.restype = C.c_int
    L.tm_batch_set.argtypes = [vp, i32, C.POINTER(_Job), C.POINTER(_TraceOpts), vp]
    L.tm_batch_launch.restype = C.c_int
    L.tm_batch_launch.argtypes = [vp, vp]
    L.tm_batch_graph_launch.restype = C.c_int
    L.tm_batch_graph_launch.argtypes = [vp, vp]
    L.tm_batch_tune.restype = C.c_int
    L.tm_batch_tune.argtypes = [vp, i32, vp, C.POINTER(_TraceOpts), C.POINTER(C.c_float)]
    L.tm_batch_free.restype = C.c_int
    L.tm_batch_free.argtypes = [vp]
    L.tm_server_create.restype = C.c_int
    L.tm_server_create.argtypes = [C.POINTER(vp), i32, C.POINTER(_ServerOpts), C.POINTER(vp)]
    L.tm_server_submit.restype = C.c_int
    L.tm_server_submit.argtypes = [vp, C.POINTER(_Request), C.POINTER(i64)]
    L.tm_server_step.restype = C.c_int
    L.tm_server_step.argtypes = [vp, vp, C.POINTER(i64)]
    L.tm_server_poll.restype = C.c_int
    L.tm_server_poll.argtypes = [vp, C.POINTER(_Done), i32, C.POINTER(i32)]
    L.tm_server_drain.restype = C.c_int
    L.tm_server_drain.argtypes = [vp, vp]
    L.tm_server_pending.restype = C.c_int
    L.tm_server_pending.argtypes = [vp, C.POINTER(i64), C.POINTER(i64), C.POINTER(i64)]
    L.tm_server_free.restype = C.c_int
    L.tm_server_free.argtypes = [vp]
    L.tm_request_rays.restype = C.c_int
    L.tm_request_rays.argtypes = [vp, C.POINTER(_Request), i32, vp, vp, vp, vp, vp, vp, vp]
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
                   seed_grid=0, bin_rays=0):
    """Pack and upload a mesh (host arrays); returns the raw handle (int).  ``bin_rays``:
    rays the handle's own binning workspace holds (allocated here; 0 = none)."""
    L = _load()
    P = _host(points, np.float32, (3,), "points")
    T = _host(tets, np.int32, (4,), "tets")
    N = _host(nbrs, np.int32, (4,), "nbrs")
    F = _host(cflag, np.uint8, (4,), "cflag")
    if N.shape != T.shape or F.shape != T.shape:
        raise ValueError("tets, nbrs and cflag must have the same shape")
    opts = _UploadOpts(_LAYOUTS[layout], _SFC[sfc], int(bool(validate)), int(seed_grid), int(bin_rays))
    h = C.c_void_p()
    _check(L.tetmesh_upload(P.ctypes.data, P.shape[0], T.ctypes.data, N.ctypes.data, F.ctypes.data,
                            T.shape[0], C.byref(opts), C.byref(h)))
    return h.value


def trace_closest(handle, orig, dirs, tri, t, bary, tmax=None, start_tet=None, start_face=None,
                  hit_tets=None, steps=None, workspace=None, fp64_steps=None, stream=None, **opts):
    """Enqueue a trace of ``orig``/``dirs`` ([n, 3] float32, device) writing into the
    given device tensors; asynchronous on ``stream`` (default: the current one).
    ``opts``: the tm_trace_opts fields (max_steps, block, kernel, refill, grid_cap,
    xcds, xcd_blocks, sort, sort_chunk_log2, sort_cells_log2, sort_dirq, eps, order)."""
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


def trace_closest_noalloc(handle, orig, dirs, tri, t, bary, tmax=None, start_tet=None,
                          start_face=None, hit_tets=None, steps=None, stream=None, **opts):
    """trace_closest for callers that cannot allocate: binning uses the library's
    fixed per-device array (at most TM_NOALLOC_MAX_BINNED_RAYS rays)."""
    n = int(orig.shape[0]) if orig.dim() >= 1 else 0
    args = [_dev(orig, torch.float32, n, (3,), "orig"), _dev(dirs, torch.float32, n, (3,), "dirs"),
            _dev(tmax, torch.float32, n, (), "tmax", True),
            _dev(start_tet, torch.int32, n, (), "start_tet", True),
            _dev(start_face, torch.int32, n, (), "start_face", True),
            _dev(tri, torch.int32, n, (), "tri"), _dev(t, torch.float32, n, (), "t"),
            _dev(bary, torch.float32, n, (2,), "bary"),
            _dev(hit_tets, torch.int32, n, (2,), "hit_tets", True),
            _dev(steps, torch.int32, n, (), "steps", True)]
    o = _trace_opts(dict(opts), None, None, n)
    _check(_load().trace_closest_noalloc(C.c_void_p(handle), n, *args, C.byref(o), _stream(stream)))


NOALLOC_MAX_BINNED_RAYS = 1 << 24


def tetmesh_trace_workspace(handle, n_rays, has_tmax, **opts):
    o = _trace_opts(dict(opts), n=int(n_rays))
    b = C.c_int64()
    _check(_load().tetmesh_trace_workspace(C.c_void_p(handle), int(n_rays),
                                           C.c_void_p(1 if has_tmax else 0), C.byref(o),
                                           C.byref(b)))
    return b.value


def tetmesh_bin_rays(handle, orig, dirs, order, stream=None, **opts):
    """Write the binning order of ``orig``/``dirs`` into ``order`` (int32 [n], device)."""
    n = int(orig.shape[0])
    o = _trace_opts(dict(opts))
    _check(_load().tetmesh_bin_rays(C.c_void_p(handle), n, _dev(orig, torch.float32, n, (3,), "orig"),
                                    _dev(dirs, torch.float32, n, (3,), "dirs"), C.byref(o),
                                    _dev(order, torch.int32, n, (), "order"), _stream(stream)))


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
    return {k: getattr(info, k) for k, _ in _Info._fields_}


def tetmesh_free(handle):
    _check(_load().tetmesh_free(C.c_void_p(handle)))


def tetrt_sfc_keys(xyz, bits=21, curve="hilbert"):
    xyz = _host(xyz, np.uint32, (3,), "xyz")
    out = np.empty(xyz.shape[0], np.uint64)
    _check(_load().tetrt_sfc_keys(_SFC[curve], int(bits), xyz.shape[0], xyz.ctypes.data,
                                  out.ctypes.data))
    return out


def tm_batch_create(max_jobs, max_rays):
    h = C.c_void_p()
    _check(_load().tm_batch_create(int(max_jobs), int(max_rays), C.byref(h)))
    return h.value


def _job(handle, orig, dirs, tri, t, bary, tmax=None, start_tet=None, start_face=None,
         hit_tets=None, steps=None):
    n = int(orig.shape[0])
    j = _Job()
    j.mesh = handle
    j.n_rays = n
    j.d_orig = _dev(orig, torch.float32, n, (3,), "orig")
    j.d_dir = _dev(dirs, torch.float32, n, (3,), "dirs")
    j.d_tmax = _dev(tmax, torch.float32, n, (), "tmax", True)
    j.d_start_tet = _dev(start_tet, torch.int32, n, (), "start_tet", True)
    j.d_start_face = _dev(start_face, torch.int32, n, (), "start_face", True)
    j.d_tri = _dev(tri, torch.int32, n, (), "tri")
    j.d_t = _dev(t, torch.float32, n, (), "t")
    j.d_bary = _dev(bary, torch.float32, n, (2,), "bary")
    j.d_hit_tets = _dev(hit_tets, torch.int32, n, (2,), "hit_tets", True)
    j.d_steps = _dev(steps, torch.int32, n, (), "steps", True)
    return j


def tm_batch_set(batch, jobs, stream=None, **opts):
    """``jobs``: sequence of dicts with the keyword arguments of trace_closest
    (``handle``, ``orig``, ``dirs``, ``tri``, ``t``, ``bary`` and the optional ones)."""
    arr = (_Job * max(1, len(jobs)))(*[_job(**j) for j in jobs])
    o = _trace_opts(dict(opts))
    _check(_load().tm_batch_set(C.c_void_p(batch), len(jobs), arr, C.byref(o), _stream(stream)))


def tm_batch_launch(batch, stream=None):
    _check(_load().tm_batch_launch(C.c_void_p(batch), _stream(stream)))


def tm_batch_graph_launch(batch, stream=None):
    _check(_load().tm_batch_graph_launch(C.c_void_p(batch), _stream(stream)))


def tm_batch_tune(batch, reps=5, stream=None):
    o = _TraceOpts()
    ms = C.c_float()
    _check(_load().tm_batch_tune(C.c_void_p(batch), int(reps), _stream(stream), C.byref(o),
                                 C.byref(ms)))
    return {k: getattr(o, k) for k in ("block", "sort", "sort_chunk_log2", "xcds", "kernel", "queue_chunk",
                                       "refill")}, ms.value


def tm_batch_free(batch):
    _check(_load().tm_batch_free(C.c_void_p(batch)))


def _request(mesh=0, kind="primary", width=64, height=64, eye=(0.5, 0.5, 0.5),
             forward=(0.0, 0.0, 1.0), up=(0.0, 1.0, 0.0), fov_h_deg=60.0, light=(0.0, 0.0, 0.0),
             ao_tmax=0.1, seed=0, out=None):
    r = _Request()
    r.mesh = int(mesh)
    r.kind = _KINDS[kind] if isinstance(kind, str) else int(kind)
    r.width, r.height = int(width), int(height)
    r.eye[:] = [float(v) for v in eye]
    r.forward[:] = [float(v) for v in forward]
    r.up[:] = [float(v) for v in up]
    r.fov_h_deg = float(fov_h_deg)
    r.light[:] = [float(v) for v in light]
    r.ao_tmax = float(ao_tmax)
    r.seed = int(seed) & 0xFFFFFFFF
    if out is not None:
        n = r.width * r.height
        r.d_tri = _dev(out["tri"], torch.int32, n, (), "out['tri']")
        r.d_t = _dev(out["t"], torch.float32, n, (), "out['t']")
        r.d_bary = _dev(out["bary"], torch.float32, n, (2,), "out['bary']")
    return r


def tm_server_create(handles, max_rays, max_requests=0, ring=0, block=0, sort=0, max_steps=0, eps=0.0):
    arr = (C.c_void_p * len(handles))(*handles)
    o = _ServerOpts(int(max_rays), int(max_requests), int(ring), int(block), int(sort), int(max_steps),
                    float(eps))
    h = C.c_void_p()
    _check(_load().tm_server_create(arr, len(handles), C.byref(o), C.byref(h)))
    return h.value


def tm_server_submit(server, **req):
    """``req``: the tm_request fields (mesh, kind, width, height, eye, forward, up,
    fov_h_deg, light, ao_tmax, seed) and ``out``, a dict of device tensors as from
    ``outputs(width * height, ...)``.  Returns the request id."""
    r = _request(**req)
    i = C.c_int64()
    _check(_load().tm_server_submit(C.c_void_p(server), C.byref(r), C.byref(i)))
    return i.value


def tm_server_step(server, stream=None):
    n = C.c_int64()
    _check(_load().tm_server_step(C.c_void_p(server), _stream(stream), C.byref(n)))
    return n.value


def tm_server_poll(server, max_items=1024):
    buf = (_Done * max_items)()
    n = C.c_int32()
    _check(_load().tm_server_poll(C.c_void_p(server), buf, int(max_items), C.byref(n)))
    return [{k: getattr(buf[i], k) for k, _ in _Done._fields_} for i in range(n.value)]


def tm_server_drain(server, stream=None):
    _check(_load().tm_server_drain(C.c_void_p(server), _stream(stream)))


def tm_server_pending(server):
    q, a, f = C.c_int64(), C.c_int64(), C.c_int64()
    _check(_load().tm_server_pending(C.c_void_p(server), C.byref(q), C.byref(a), C.byref(f)))
    return {"queued": q.value, "admitted": a.value, "finished": f.value}


def tm_server_free(server):
    _check(_load().tm_server_free(C.c_void_p(server)))


def tm_request_rays(handle, phase, orig, dirs, tmax, start_face, tri=None, t=None, stream=None, **req):
    """The rays a server generates for a request (phase 0 camera, phase 1 secondary),
    written into the given device tensors."""
    r = _request(**req)
    n = r.width * r.height
    _check(_load().tm_request_rays(
        C.c_void_p(handle), C.byref(r), int(phase), _dev(orig, torch.float32, n, (3,), "orig"),
        _dev(dirs, torch.float32, n, (3,), "dirs"), _dev(tmax, torch.float32, n, (), "tmax"),
        _dev(start_face, torch.int32, n, (), "start_face"),
        _dev(tri, torch.int32, n, (), "tri", True), _dev(t, torch.float32, n, (), "t", True),
        _stream(stream)))


# ---- convenience wrappers -------------------------------------------------------------

def outputs(n, device, want_tets=False, want_steps=False):
    """Output tensors of a trace of n rays."""
    out = {"tri": torch.empty(n, dtype=torch.int32, device=device),
           "t": torch.empty(n, dtype=torch.float32, device=device),
           "bary": torch.empty((n, 2), dtype=torch.float32, device=device)}
    if want_tets:
        out["hit_tets"] = torch.empty((n, 2), dtype=torch.int32, device=device)
    if want_steps:
        out["steps"] = torch.empty(n, dtype=torch.int32, device=device)
    return out


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
        out = outputs(n, dev, want_tets, want_steps)
        if want_fp64:
            out["fp64_steps"] = torch.empty(n, dtype=torch.int32, device=dev)
        self.trace_into(out, orig, dirs, tmax, start_tet, start_face, workspace, stream, **opts)
        return out

    def trace_into(self, out, orig, dirs, tmax=None, start_tet=None, start_face=None,
                   workspace=None, stream=None, **opts):
        """Trace into caller tensors.  A trace that bins its rays (``sort``) without a
        ``workspace`` gets one from torch's allocator here, held on the stream it runs
        on, so the library itself never allocates."""
        if workspace is None:
            wo = {k: v for k, v in opts.items() if k in _TRACE_KEYS or k in ("eps", "order")}
            need = self.workspace_bytes(int(orig.shape[0]), tmax is not None, **wo)
            if need > 0:
                workspace = torch.empty(need, dtype=torch.uint8, device=orig.device)
                if stream is not None and stream != torch.cuda.current_stream(orig.device):
                    workspace.record_stream(stream)
        trace_closest(self.handle, orig, dirs, out["tri"], out["t"], out["bary"], tmax=tmax,
                      start_tet=start_tet, start_face=start_face, hit_tets=out.get("hit_tets"),
                      steps=out.get("steps"), workspace=workspace,
                      fp64_steps=out.get("fp64_steps"), stream=stream, **opts)
        return out

    def bin_rays(self, orig, dirs, order=None, stream=None, **opts):
        """The binning order of the rays (int32 [n] device tensor), for trace(order=...)."""
        if order is None:
            order = torch.empty(int(orig.shape[0]), dtype=torch.int32, device=orig.device)
        tetmesh_bin_rays(self.handle, orig, dirs, order, stream, **opts)
        return order

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


class Batch:
    """Batched traces over many meshes (tm_batch_*).  ``set`` takes a list of jobs,
    each a dict: ``mesh`` (a Mesh), ``orig``, ``dirs``, ``out`` (a dict as from
    ``outputs``) and optionally ``tmax``, ``start_tet``, ``start_face``.  The
    batch keeps references to the tensors of its current jobs."""

    def __init__(self, max_jobs, max_rays):
        self.handle = tm_batch_create(max_jobs, max_rays)
        self._jobs = []

    def __del__(self):
        self.free()

    def free(self):
        h = getattr(self, "handle", None)
        if h:
            self.handle = None
            tm_batch_free(h)

    def set(self, jobs, stream=None, **opts):
        spec = []
        for j in jobs:
            out = j["out"]
            spec.append(dict(handle=j["mesh"].handle, orig=j["orig"], dirs=j["dirs"],
                             tri=out["tri"], t=out["t"], bary=out["bary"], tmax=j.get("tmax"),
                             start_tet=j.get("start_tet"), start_face=j.get("start_face"),
                             hit_tets=out.get("hit_tets"), steps=out.get("steps")))
        tm_batch_set(self.handle, spec, stream, **opts)
        self._jobs = list(jobs)

    def launch(self, stream=None):
        tm_batch_launch(self.handle, stream)

    def graph_launch(self, stream=None):
        tm_batch_graph_launch(self.handle, stream)

    def tune(self, reps=5, stream=None):
        return tm_batch_tune(self.handle, reps, stream)


class Server:
    """Serving loop over resident meshes (tm_server_*).  ``submit`` keeps the
    request's output tensors alive until ``poll`` reports it."""

    def __init__(self, meshes, max_rays, **opts):
        self.meshes = list(meshes)
        self.handle = tm_server_create([m.handle for m in self.meshes], max_rays, **opts)
        self._outs = {}

    def __del__(self):
        self.free()

    def free(self):
        h = getattr(self, "handle", None)
        if h:
            self.handle = None
            tm_server_free(h)

    def submit(self, out, **req):
        i = tm_server_submit(self.handle, out=out, **req)
        self._outs[i] = out
        return i

    @staticmethod
    def prepare(**req):
        """A request's fields (as for ``submit``) packed once, for ``submit_prepared``."""
        return _request(**req)

    def submit_prepared(self, r, out):
        """Submit a request packed by ``prepare`` into ``out`` (tri int32, t float32,
        bary float32 [., 2] device tensors, contiguous, holding at least width x
        height entries from their start): per call only the three output
        addresses are set, for a submitting loop whose own cost matters."""
        n = r.width * r.height
        tri, t, bary = out["tri"], out["t"], out["bary"]
        for x, dt, name in ((tri, torch.int32, "tri"), (t, torch.float32, "t"), (bary, torch.float32, "bary")):
            if not isinstance(x, torch.Tensor) or x.device.type != "cuda" or x.dtype != dt or not x.is_contiguous():
                raise TypeError("out['%s'] must be a contiguous %s device tensor" % (name, dt))
        if tri.numel() < n or t.numel() < n or bary.numel() < 2 * n or (bary.dim() != 2 or bary.shape[1] != 2):
            raise ValueError("output tensors hold fewer than %d entries" % n)
        r.d_tri, r.d_t, r.d_bary = tri.data_ptr(), t.data_ptr(), bary.data_ptr()
        i = C.c_int64()
        _check(_load().tm_server_submit(C.c_void_p(self.handle), C.byref(r), C.byref(i)))
        self._outs[i.value] = out
        return i.value

    def step(self, stream=None):
        return tm_server_step(self.handle, stream)

    def poll(self, max_items=1024):
        done = tm_server_poll(self.handle, max_items)
        for d in done:
            self._outs.pop(d["id"], None)
        return done

    def drain(self, stream=None):
        tm_server_drain(self.handle, stream)

    def pending(self):
        return tm_server_pending(self.handle)
