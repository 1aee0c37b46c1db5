"""CPU reference ("oracle") for closest-hit traversal of a constrained tet mesh.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the library.  It shares no code with the
HIP path.

* ``walk.c`` (built into ``liboracle.so``): single-threaded FP64 tet walk, point
  location and canonical triangle ids; see its header for what it follows.
* ``brute.py``: FP64 brute-force closest hit over every constrained triangle,
  used to pin the walk on small meshes.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "walk.c")
_LIB = os.path.join(_HERE, "liboracle.so")
# a prebuilt variant of walk.c to load instead (the mutation tests use this)
_LIB_OVERRIDE = os.environ.get("TETRT_ORACLE_LIB")
_lib = None


def build(force: bool = False) -> str:
    """Compile ``walk.c`` with the system C compiler (no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fPIC", "-shared",
                               "-std=c99", "-Wall", "-Wextra", "-Wno-unused-parameter",
                               _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if _LIB_OVERRIDE:
            L = C.CDLL(_LIB_OVERRIDE)
        else:
            build()
            L = C.CDLL(_LIB)
        vp, i64, i32, f32p, f64p, i32p = (C.c_void_p, C.c_int64, C.c_int32,
                                          C.POINTER(C.c_float), C.POINTER(C.c_double),
                                          C.POINTER(C.c_int32))
        L.oracle_mesh_new.restype = vp
        L.oracle_mesh_new.argtypes = [f32p, i64, i32p, i32p, C.POINTER(C.c_uint8), i64,
                                      C.c_char_p, i64]
        L.oracle_mesh_free.argtypes = [vp]
        L.oracle_mesh_ntri.restype = i64
        L.oracle_mesh_ntri.argtypes = [vp]
        L.oracle_mesh_tables.argtypes = [vp, i32p, i32p, i32p]
        L.oracle_get_exit_face.restype = C.c_int
        L.oracle_get_exit_face.argtypes = [f64p]
        L.oracle_onb.argtypes = [f64p, f64p, f64p]
        L.oracle_locate.restype = C.c_int
        L.oracle_locate.argtypes = [vp, i64, f32p, i32, i32p]
        L.oracle_trace.restype = C.c_int
        L.oracle_trace.argtypes = [vp, i64, f32p, f32p, f32p, i32p, i32p, i32, C.c_int, i64,
                                   i32p, f64p, f64p, i32p, i32p, i32p]
        _lib = L
    return _lib


def _p(a, ct):
    return None if a is None else a.ctypes.data_as(C.POINTER(ct))


class OracleMesh:
    """The user's mesh arrays plus the oracle's canonical triangle tables.

    Triangle ids: faces (t, j) are visited t-major in user order and each
    constrained face gets the next id when first seen (both sides share it).
    """

    def __init__(self, points, tets, nbrs, cflag):
        L = _load()
        self.points = np.ascontiguousarray(points, dtype=np.float32)
        self.tets = np.ascontiguousarray(tets, dtype=np.int32)
        self.nbrs = np.ascontiguousarray(nbrs, dtype=np.int32)
        self.cflag = np.ascontiguousarray(cflag, dtype=np.uint8)
        err = C.create_string_buffer(256)
        h = L.oracle_mesh_new(_p(self.points, C.c_float), self.points.shape[0],
                              _p(self.tets, C.c_int32), _p(self.nbrs, C.c_int32),
                              _p(self.cflag, C.c_uint8), self.tets.shape[0], err, 256)
        if not h:
            raise ValueError("oracle: inconsistent mesh: " + err.value.decode())
        self._h = C.c_void_p(h)
        self.ntri = int(L.oracle_mesh_ntri(self._h))
        self.face_tri = np.empty((self.tets.shape[0], 4), np.int32)
        self.tri_tets = np.empty((self.ntri, 2), np.int32)
        self.tri_verts = np.empty((self.ntri, 3), np.int32)
        L.oracle_mesh_tables(self._h, _p(self.face_tri, C.c_int32), _p(self.tri_tets, C.c_int32),
                             _p(self.tri_verts, C.c_int32))

    @classmethod
    def from_kuhn(cls, m):
        return cls(m.points, m.tets, m.nbrs, m.cflag)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.oracle_mesh_free(h)
            self._h = None

    def locate(self, xyz, source_tet: int = 0):
        xyz = np.ascontiguousarray(xyz, dtype=np.float32).reshape(-1, 3)
        out = np.empty(xyz.shape[0], np.int32)
        rc = _load().oracle_locate(self._h, xyz.shape[0], _p(xyz, C.c_float), int(source_tet),
                                   _p(out, C.c_int32))
        if rc != 0:
            raise ValueError("oracle_locate: bad source tet")
        return out

    def trace(self, orig, dirs, tmax=None, start_face=None, start_tet=None, source_tet: int = 0,
              early_out: bool = True, max_steps: int = 0):
        """Closest hit of each ray; returns a dict of numpy arrays:
        tri (id or code), t (float64), bary [n, 2] (float64), tets [n, 2],
        steps, start."""
        o = np.ascontiguousarray(orig, dtype=np.float32).reshape(-1, 3)
        d = np.ascontiguousarray(dirs, dtype=np.float32).reshape(-1, 3)
        n = o.shape[0]
        if d.shape[0] != n:
            raise ValueError("orig and dirs differ in length")
        tm = None if tmax is None else np.ascontiguousarray(np.broadcast_to(
            np.asarray(tmax, dtype=np.float32), (n,)))
        sf = None if start_face is None else np.ascontiguousarray(start_face, dtype=np.int32)
        st = None if start_tet is None else np.ascontiguousarray(np.broadcast_to(
            np.asarray(start_tet, dtype=np.int32), (n,)))
        out = dict(tri=np.empty(n, np.int32), t=np.empty(n, np.float64),
                   bary=np.empty((n, 2), np.float64), tets=np.empty((n, 2), np.int32),
                   steps=np.empty(n, np.int32), start=np.empty(n, np.int32))
        rc = _load().oracle_trace(self._h, n, _p(o, C.c_float), _p(d, C.c_float),
                                  _p(tm, C.c_float), _p(sf, C.c_int32), _p(st, C.c_int32),
                                  int(source_tet), int(bool(early_out)), int(max_steps),
                                  _p(out["tri"], C.c_int32), _p(out["t"], C.c_double),
                                  _p(out["bary"], C.c_double), _p(out["tets"], C.c_int32),
                                  _p(out["steps"], C.c_int32), _p(out["start"], C.c_int32))
        if rc != 0:
            raise ValueError("oracle_trace: bad source tet")
        return out


def get_exit_face(q):
    """Algorithm 1 on four 2-D points q [4, 2] (float64)."""
    q = np.ascontiguousarray(q, dtype=np.float64).reshape(8)
    return int(_load().oracle_get_exit_face(_p(q, C.c_double)))


def onb(n):
    """The oracle's orthonormal ray frame (b1, b2) for a unit vector n."""
    n = np.ascontiguousarray(n, dtype=np.float64).reshape(3)
    b1 = np.empty(3)
    b2 = np.empty(3)
    _load().oracle_onb(_p(n, C.c_double), _p(b1, C.c_double), _p(b2, C.c_double))
    return b1, b2


from .brute import brute_closest_hit  # noqa: E402

__all__ = ["OracleMesh", "get_exit_face", "onb", "brute_closest_hit", "build"]
