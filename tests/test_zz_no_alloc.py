"""trace_closest_noalloc (for callers that cannot allocate) against
trace_closest: the same kernels, with the binning permutation (and the
precision variant's tie list) in the library's fixed per-device array instead
of a caller workspace.  Two calls in a row, the
second smaller, must both give trace_closest's results bit for bit; sizes
beyond the array and a workspace argument are refused."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from synth import config_mesh, random_interior_rays

pytestmark = pytest.mark.gpu


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def _host(res):
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in res.items()}


@pytest.fixture(scope="module")
def mesh():
    import paper_2103_02309_amd as tetrt
    m = config_mesh("tiny")
    h = tetrt.upload(m.points, m.tets, m.nbrs, m.cflag, layout="tet16")
    yield tetrt, h
    h.free()


def _rays(n, seed):
    o, d = random_interior_rays(n, seed)
    tm = np.random.default_rng(seed).uniform(0.05, 0.6, n).astype(np.float32)
    return _dev(o), _dev(d), _dev(tm)


def _noalloc(tetrt, mesh, O, D, T, out, **opts):
    tetrt.binding.trace_closest_noalloc(mesh.handle, O, D, out["tri"], out["t"], out["bary"], tmax=T,
                                        hit_tets=out.get("hit_tets"), steps=out.get("steps"), **opts)


@pytest.mark.parametrize("kw", [dict(sort=2), dict(sort=0), dict(sort=2, eps=1e-6)])
def test_noalloc_matches_trace_closest(mesh, kw):
    """eps > 0: the precision variant, with its tie list in the fixed array too."""
    tetrt, h = mesh
    for n, seed in ((300_000, 81), (70_001, 82)):   # the second call smaller, ragged
        O, D, T = _rays(n, seed)
        ref = _host(h.trace(O, D, tmax=T, want_tets=True, want_steps=True, **kw))
        out = tetrt.outputs(n, "cuda:0", want_tets=True, want_steps=True)
        for v in out.values():
            v.fill_(-7)
        _noalloc(tetrt, h, O, D, T, out, **kw)
        got = _host(out)
        for k in ref:
            assert np.array_equal(got[k], ref[k], equal_nan=True), (n, k)


def test_noalloc_refuses_what_it_cannot_hold(mesh):
    tetrt, h = mesh
    n = tetrt.binding.NOALLOC_MAX_BINNED_RAYS + 1
    O = torch.zeros((n, 3), dtype=torch.float32, device="cuda:0")
    D = torch.ones((n, 3), dtype=torch.float32, device="cuda:0")
    T = torch.full((n,), 0.1, dtype=torch.float32, device="cuda:0")
    out = tetrt.outputs(n, "cuda:0")
    with pytest.raises(tetrt.TetRTError, match="at most"):
        _noalloc(tetrt, h, O, D, T, out, sort=2)
    # a caller workspace is not what this entry point takes (the C-ABI refuses it)
    import ctypes as C
    B = tetrt.binding
    O2, D2, T2 = _rays(1000, 83)
    ws = torch.empty(1 << 16, dtype=torch.uint8, device="cuda:0")
    out2 = tetrt.outputs(1000, "cuda:0")
    o = B._trace_opts({"sort": 2}, ws, None, 1000)
    rc = B._load().trace_closest_noalloc(
        C.c_void_p(h.handle), 1000, O2.data_ptr(), D2.data_ptr(), T2.data_ptr(), None, None,
        out2["tri"].data_ptr(), out2["t"].data_ptr(), out2["bary"].data_ptr(), None, None, C.byref(o),
        B._stream(None))
    assert rc == B.TM_ERR_ARG and "workspace" in B.tm_last_error()
