"""Host-side checks of the C-ABI library that need no GPU: every symbol the
header declares is exported, argument and mesh validation errors, and the
space-filling-curve keys."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tetrt.h")


@pytest.fixture(scope="module")
def tetrt():
    from paper_2103_02309_amd.build import build_library
    build_library(force=False)
    import paper_2103_02309_amd as tetrt
    tetrt.binding._load()
    return tetrt


def _declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[\w\s\*]+?\b(\w+)\s*\(", src, flags=re.M)) -
                  {"if", "while", "defined"})


def test_every_declared_symbol_exported(tetrt):
    names = _declared_functions()
    assert {"tetmesh_upload", "trace_closest", "tetmesh_locate", "tetmesh_free",
            "tm_last_error"} <= set(names)
    lib = C.CDLL(tetrt.library_path())
    for name in names:
        assert hasattr(lib, name), name


def _tiny():
    from synth import kuhn_mesh
    return kuhn_mesh(3, jitter=0.1, seed=1, spheres=[[0.5, 0.5, 0.5, 0.3]])


def _upload_err(tetrt, *args, **kw):
    with pytest.raises(tetrt.TetRTError) as ei:
        tetrt.tetmesh_upload(*args, **kw)
    return ei.value.code, str(ei.value)


def test_validation_rejects_corrupt_meshes(tetrt):
    m = _tiny()
    # vertex id out of range
    # (tets are checked in order, so the first bad one is named)
    t = m.tets.copy(); t[0, 2] = m.n_points + 3
    code, msg = _upload_err(tetrt, m.points, t, m.nbrs, m.cflag)
    assert code == -2 and "tet 0" in msg and "out of range" in msg
    # neighbour link not mutual
    nb = m.nbrs.copy(); j = int(np.nonzero(nb[7] >= 0)[0][0]); nb[7, j] = (nb[7, j] + 1) % m.n_tets
    code, msg = _upload_err(tetrt, m.points, m.tets, nb, m.cflag)
    assert code == -2
    # constrained flag on one side only
    cf = m.cflag.copy(); t0, j0 = np.argwhere(cf)[0]; cf[t0, j0] = 0
    code, msg = _upload_err(tetrt, m.points, m.tets, m.nbrs, cf)
    assert code == -2 and "flag" in msg
    # zero volume
    p = m.points.copy(); tt = m.tets[11]; p[tt[3]] = p[tt[0]]
    code, msg = _upload_err(tetrt, p, m.tets, m.nbrs, m.cflag)
    assert code == -2
    # repeated vertex
    t = m.tets.copy(); t[0, 1] = t[0, 0]
    code, msg = _upload_err(tetrt, m.points, t, m.nbrs, m.cflag)
    assert code == -2 and "tet 0" in msg and "repeated" in msg


def test_argument_errors(tetrt):
    m = _tiny()
    code, _ = _upload_err(tetrt, m.points[:3], m.tets, m.nbrs, m.cflag)
    assert code == -1
    with pytest.raises(ValueError):
        tetrt.tetmesh_upload(m.points, m.tets, m.nbrs[:5], m.cflag)
    lib = tetrt.binding._load()
    assert lib.trace_closest(None, 1, None, None, None, None, None, None, None, None, None, None,
                             None, None) == -1
    assert "NULL mesh" in tetrt.tm_last_error()
    assert lib.tetmesh_free(None) == 0
    out = C.c_void_p()
    opts = tetrt.binding._UploadOpts(7, 0, 1, 0)
    P = np.ascontiguousarray(m.points)
    T, N, F = (np.ascontiguousarray(a) for a in (m.tets, m.nbrs, m.cflag))
    assert lib.tetmesh_upload(P.ctypes.data, P.shape[0], T.ctypes.data, N.ctypes.data, F.ctypes.data,
                              T.shape[0], C.byref(opts), C.byref(out)) == -1
    assert "layout" in tetrt.tm_last_error()


def test_hilbert_keys_walk_adjacent_cells(tetrt):
    for bits in (1, 2, 3, 4):
        g = np.arange(1 << bits, dtype=np.uint32)
        xyz = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
        k = tetrt.tetrt_sfc_keys(xyz, bits=bits, curve="hilbert")
        assert sorted(k.tolist()) == list(range(len(xyz)))       # a bijection onto 0..8^bits-1
        path = xyz[np.argsort(k)].astype(np.int64)
        step = np.abs(np.diff(path, axis=0)).sum(axis=1)
        assert np.all(step == 1)                                  # consecutive cells share a face
        assert k[0] == 0                                           # the curve starts at the origin


def test_morton_keys_interleave_bits(tetrt):
    xyz = np.array([[1, 0, 0], [0, 1, 0], [0, 0, 1], [3, 5, 6]], np.uint32)
    k = tetrt.tetrt_sfc_keys(xyz, bits=3, curve="morton")
    assert k[:3].tolist() == [4, 2, 1]
    # x=011 y=101 z=110 -> per level (x y z): 0 1 1 | 1 0 1 | 1 1 0
    assert int(k[3]) == 0b011101110


def test_sfc_key_argument_checks(tetrt):
    with pytest.raises(tetrt.TetRTError):
        tetrt.tetrt_sfc_keys(np.array([[8, 0, 0]], np.uint32), bits=3)
    with pytest.raises(tetrt.TetRTError):
        tetrt.tetrt_sfc_keys(np.zeros((1, 3), np.uint32), bits=22)


def test_batch_argument_errors(tetrt):
    """tm_batch_* reject bad arguments before touching a device."""
    lib = tetrt.binding._load()
    h = C.c_void_p()
    assert lib.tm_batch_create(0, 10, C.byref(h)) == -1 and "max_jobs" in tetrt.tm_last_error()
    assert lib.tm_batch_create(70000, 10, C.byref(h)) == -1
    assert lib.tm_batch_create(4, -1, C.byref(h)) == -1 and "max_rays" in tetrt.tm_last_error()
    assert lib.tm_batch_create(4, 1 << 33, C.byref(h)) == -1
    assert lib.tm_batch_create(4, 10, None) == -1
    assert lib.tm_batch_set(None, 0, None, None, None) == -1 and "NULL batch" in tetrt.tm_last_error()
    assert lib.tm_batch_launch(None, None) == -1
    assert lib.tm_batch_graph_launch(None, None) == -1
    assert lib.tm_batch_tune(None, 3, None, None, None) == -1
    assert lib.tm_batch_free(None) == 0


def test_server_argument_errors(tetrt):
    """tm_server_* and tm_request_rays reject bad arguments before touching a device."""
    lib = tetrt.binding._load()
    h = C.c_void_p()
    assert lib.tm_server_create(None, 1, None, C.byref(h)) == -1 and "meshes" in tetrt.tm_last_error()
    assert lib.tm_server_create(None, 1, None, None) == -1
    i = C.c_int64()
    assert lib.tm_server_submit(None, None, C.byref(i)) == -1
    assert lib.tm_server_step(None, None, None) == -1
    n = C.c_int32()
    assert lib.tm_server_poll(None, None, 0, C.byref(n)) == -1
    assert lib.tm_server_drain(None, None) == -1
    assert lib.tm_server_pending(None, None, None, None) == -1
    assert lib.tm_request_rays(None, None, 0, None, None, None, None, None, None, None) == -1
    assert lib.tm_server_free(None) == 0


def test_probe_l1_argument_errors():
    """The calibration kernel's library (the benchmark's, apart from the
    traversal library) rejects bad shapes before any launch (the pointers below
    are never dereferenced)."""
    from bench import probe_lib
    L = probe_lib()
    buf, out = C.c_void_p(4096), C.c_void_p(8192)
    bad = [
        (buf, 1 << 20, 7, 128, 128, 16, 16, out),        # unknown mode
        (buf, 1 << 20, 0, 24, 128, 16, 16, out),         # unit not a multiple of 16
        (buf, 1 << 20, 0, 128, 96, 16, 16, out),         # units not a power of two
        (buf, 1 << 10, 0, 128, 128, 16, 16, out),        # set larger than the buffer
        (buf, 1 << 20, 0, 128, 128, 0, 16, out),         # no blocks
        (buf, 1 << 20, 0, 128, 128, 16, 1 << 21, out),   # too many iterations
        (None, 1 << 20, 0, 128, 128, 16, 16, out),       # NULL buffer
    ]
    for a in bad:
        assert L.tetrt_probe_l1(*a, None) == -1, a
        assert b"tetrt_probe_l1" in L.tetrt_probe_last_error()


def test_probe_not_in_traversal_library(tetrt):
    """The calibration kernel ships only in the benchmark's library."""
    lib = C.CDLL(tetrt.library_path())
    assert not hasattr(lib, "tetrt_probe_l1")
