"""Parity of the HIP path (through the C-ABI) with the FP64 oracle on the same
seeded inputs."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from oracle.compare import compare
from synth import (config_mesh, kuhn_mesh, pinhole_rays, ao_rays, tri_geometry,
                   random_interior_rays)
from synth.kuhn import random_spheres

pytestmark = pytest.mark.gpu


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def _host(res):
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in res.items()}


@pytest.fixture(scope="module")
def tetrt():
    import paper_2103_02309_amd as tetrt
    return tetrt


LAYOUTS = ["tet20", "tet16", "tet32n", "tet32"]


@pytest.fixture(scope="module", params=LAYOUTS)
def tiny(request, tetrt, tiny_mesh, tiny_oracle):
    mesh = tetrt.upload(tiny_mesh.points, tiny_mesh.tets, tiny_mesh.nbrs, tiny_mesh.cflag,
                        layout=request.param)
    yield tiny_mesh, tiny_oracle, mesh
    mesh.free()


def _ao_from(m, om, o, d, ref, k=8, seed=3, tmax=0.1):
    hit = ref["tri"] >= 0
    hp = o[hit].astype(np.float64) + ref["t"][hit, None] * d[hit].astype(np.float64)
    nrm, _ = tri_geometry(m.points, om.tri_verts[ref["tri"][hit]])
    ao, ad, atm, parent = ao_rays(hp, nrm, d[hit], k=k, seed=seed, tmax=tmax)
    return ao, ad, atm, ref["tri"][hit][parent].astype(np.int32)


KERNELS = [dict(kernel=1), dict(kernel=2), dict(kernel=2, grid_cap=2, refill=8),
           dict(kernel=3), dict(kernel=3, queue_chunk=64, refill=1, xcds=1),
           dict(eps=1e-6), dict(eps=1e-4)]   # the last two: the precision variant


@pytest.mark.parametrize("kw", KERNELS)
def test_tiny_primary(tiny, kw):
    m, om, mesh = tiny
    o, d, _ = pinhole_rays((0.5, 0.5, 0.05), 64, 64, 60.0)
    got = _host(mesh.trace(_dev(o), _dev(d), want_tets=True, want_steps=True, **kw))
    ref = om.trace(o, d)
    rep = compare(m.points, om.tri_verts, o, d, ref, got)
    assert rep["ok"], rep
    same = got["tri"] == ref["tri"]
    assert np.array_equal(got["hit_tets"][same], ref["tets"][same])
    assert (got["steps"] == ref["steps"]).mean() > 0.999


def test_tiny_without_step_counts(tiny):
    """Without per-ray step counts (the kernel the benchmark times) every layout
    matches the oracle and gives bit for bit what the counting kernel gives,
    primary and AO rays."""
    m, om, mesh = tiny
    o, d, _ = pinhole_rays((0.5, 0.5, 0.05), 64, 64, 60.0)
    ref = om.trace(o, d)
    plain = _host(mesh.trace(_dev(o), _dev(d)))
    counted = _host(mesh.trace(_dev(o), _dev(d), want_steps=True))
    rep = compare(m.points, om.tri_verts, o, d, ref, plain)
    assert rep["ok"], rep
    for k in plain:
        assert np.array_equal(plain[k], counted[k], equal_nan=True), k
    ao, ad, atm, sf = _ao_from(m, om, o, d, ref)
    A = [_dev(x) for x in (ao, ad, atm, sf)]
    plain = _host(mesh.trace(A[0], A[1], tmax=A[2], start_face=A[3]))
    counted = _host(mesh.trace(A[0], A[1], tmax=A[2], start_face=A[3], want_steps=True))
    rep = compare(m.points, om.tri_verts, ao, ad, om.trace(ao, ad, atm, start_face=sf), plain, tmax=atm)
    assert rep["ok"], rep
    for k in plain:
        assert np.array_equal(plain[k], counted[k], equal_nan=True), k


@pytest.mark.parametrize("kw", KERNELS)
def test_tiny_ao(tiny, kw):
    m, om, mesh = tiny
    o, d, _ = pinhole_rays((0.5, 0.5, 0.05), 64, 64, 60.0)
    ref0 = om.trace(o, d)
    ao, ad, atm, sf = _ao_from(m, om, o, d, ref0)
    got = _host(mesh.trace(_dev(ao), _dev(ad), tmax=_dev(atm), start_face=_dev(sf), want_tets=True,
                           **kw))
    ref = om.trace(ao, ad, atm, start_face=sf)
    rep = compare(m.points, om.tri_verts, ao, ad, ref, got, tmax=atm)
    assert rep["ok"], rep
    same = (got["tri"] == ref["tri"]) & (ref["tri"] >= 0)
    assert np.array_equal(got["hit_tets"][same], ref["tets"][same])


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("n,seed", [(4, 1), (8, 2), (13, 3)])
def test_random_rays_small_meshes(tetrt, n, seed, layout):
    m = kuhn_mesh(n, jitter=0.1, seed=seed, spheres=random_spheres(4, seed=seed, r_lo=0.1, r_hi=0.3))
    om = oracle.OracleMesh.from_kuhn(m)
    mesh = tetrt.upload(m.points, m.tets, m.nbrs, m.cflag, layout=layout)
    o, d = random_interior_rays(20000, seed)
    tm = np.random.default_rng(seed).uniform(0.05, 1.5, 20000).astype(np.float32)
    tm[::4] = np.inf
    ref_tm = om.trace(o, d, tm)
    ref = om.trace(o, d)
    for kw in KERNELS:
        got = _host(mesh.trace(_dev(o), _dev(d), tmax=_dev(tm), **kw))
        rep = compare(m.points, om.tri_verts, o, d, ref_tm, got, tmax=tm)
        assert rep["ok"], (kw, rep)
        # the same rays without tmax
        got = _host(mesh.trace(_dev(o), _dev(d), **kw))
        rep = compare(m.points, om.tri_verts, o, d, ref, got)
        assert rep["ok"], (kw, rep)
    mesh.free()


def test_start_tet_matches_location(tiny):
    m, om, mesh = tiny
    o, d = random_interior_rays(5000, 17)
    st = om.locate(o)
    a = _host(mesh.trace(_dev(o), _dev(d)))
    b = _host(mesh.trace(_dev(o), _dev(d), start_tet=_dev(st)))
    assert (a["tri"] == b["tri"]).mean() > 0.999
    ref = om.trace(o, d, start_tet=st)
    assert compare(m.points, om.tri_verts, o, d, ref, b)["ok"]


def test_locate_contains_points(tiny):
    m, om, mesh = tiny
    rng = np.random.default_rng(5)
    x = rng.uniform(0.0, 1.0, size=(20000, 3)).astype(np.float32)
    t = mesh.locate(_dev(x)).cpu().numpy()
    assert np.all(t >= 0)
    P = m.points.astype(np.float64)
    V = P[m.tets[t]]
    X = x.astype(np.float64)
    worst = np.zeros(len(x))
    for j in range(4):
        f = [s for s in range(4) if s != j]
        A, B, Cc, W = V[:, f[0]], V[:, f[1]], V[:, f[2]], V[:, j]
        nrm = np.cross(B - A, Cc - A)
        nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
        sx = np.einsum("ij,ij->i", nrm, X - A) * np.sign(np.einsum("ij,ij->i", nrm, W - A))
        worst = np.minimum(worst, sx)
    # inside up to float32 rounding of the walk (distance below 1e-6 of the extent)
    assert worst.min() > -1e-6
    ref = om.locate(x)
    assert (ref == t).mean() > 0.999
    out = mesh.locate(_dev(np.array([[1.5, 0.5, 0.5], [0.5, -0.2, 0.5]], np.float32))).cpu().numpy()
    assert out.tolist() == [-1, -1]


def test_invalid_inputs(tiny, tetrt):
    m, om, mesh = tiny
    o = np.array([[0.5, 0.5, 0.05]] * 4 + [[2.0, 0.5, 0.5]], np.float32)
    d = np.array([[0, 0, 0], [np.nan, 0, 1], [0, 0, np.inf], [0, 0, 1], [0, 0, 1]], np.float32)
    got = _host(mesh.trace(_dev(o), _dev(d)))
    assert got["tri"].tolist()[:3] == [tetrt.RAY_INVALID] * 3
    assert got["tri"][3] >= 0
    assert got["tri"][4] == tetrt.RAY_INVALID
    assert np.isnan(got["t"][[0, 1, 2, 4]]).all()
    sf = np.array([-1, -1, -1, om.ntri, -1], np.int32)
    got = _host(mesh.trace(_dev(o), _dev(d), start_face=_dev(sf)))
    assert got["tri"][3] == tetrt.RAY_INVALID
    st = np.array([-1, -1, -1, m.n_tets, -1], np.int32)
    got = _host(mesh.trace(_dev(o), _dev(d), start_tet=_dev(st)))
    assert got["tri"][3] == tetrt.RAY_INVALID
    # empty batch is a no-op
    e = torch.empty((0, 3), dtype=torch.float32, device="cuda:0")
    mesh.trace(e, e)


def test_sfc_orders_agree(tetrt, tiny_mesh, tiny_oracle):
    """Memory order changes no result.  Region order (Sec. "Reordering tetrahedral
    mesh data"): the small scene has two regions, inside and outside its sphere."""
    m = tiny_mesh
    o, d = random_interior_rays(20000, 23)
    outs = {}
    for sfc in ("hilbert", "morton", "none", "hilbert_regions"):
        mesh = tetrt.upload(m.points, m.tets, m.nbrs, m.cflag, sfc=sfc)
        assert mesh.info["n_regions"] == (2 if sfc == "hilbert_regions" else 0)
        outs[sfc] = _host(mesh.trace(_dev(o), _dev(d)))
        mesh.free()
    assert all(np.array_equal(outs["hilbert_regions"][k], outs["hilbert"][k], equal_nan=True)
               for k in outs["hilbert"])
    for sfc in ("morton", "none"):
        same = outs[sfc]["tri"] == outs["hilbert"]["tri"]
        assert same.mean() > 0.9999
        hit = same & (outs[sfc]["tri"] >= 0)
        # t and bary come from the same triangle and ray in float64: bit-identical
        assert np.array_equal(outs[sfc]["t"][hit], outs["hilbert"]["t"][hit])


def test_step_cap_reports_code(tiny, tetrt):
    m, om, mesh = tiny
    o, d, _ = pinhole_rays((0.5, 0.5, 0.05), 8, 8, 60.0)
    got = _host(mesh.trace(_dev(o), _dev(d), max_steps=1))
    ref = om.trace(o, d)
    # rays that need more than one step stop with the step-cap code
    assert np.all(got["tri"][ref["steps"] > 1] == tetrt.RAY_STEP_CAP)
    ok = ref["steps"] <= 1
    assert np.array_equal(got["tri"][ok], ref["tri"][ok])


def test_repeat_calls_identical(tiny):
    m, om, mesh = tiny
    o, d = random_interior_rays(50000, 29)
    a = _host(mesh.trace(_dev(o), _dev(d)))
    b = _host(mesh.trace(_dev(o), _dev(d), block=64))
    assert np.array_equal(a["tri"], b["tri"])
    assert np.array_equal(a["t"], b["t"], equal_nan=True)


@pytest.mark.parametrize("kw", [dict(kernel=2, grid_cap=3, refill=1), dict(kernel=2, grid_cap=3, refill=16),
                                dict(kernel=2, grid_cap=3, refill=64), dict(kernel=3),
                                dict(kernel=3, queue_chunk=64, refill=1), dict(kernel=3, queue_chunk=4096, refill=64),
                                dict(kernel=3, queue_chunk=128, refill=5, xcds=3)])
def test_persistent_matches_one_lane_per_ray(tiny, kw):
    """Persistent lanes (few blocks, so every lane takes many rays) give
    bit-identical results to one lane per ray: same arithmetic per ray."""
    m, om, mesh = tiny
    o, d = random_interior_rays(30000, 37)
    tm = np.random.default_rng(2).uniform(0.0, 0.6, 30000).astype(np.float32)
    tm[::5] = np.inf
    st = om.locate(o)
    st[::3] = -1                      # a third of the rays locate on the device
    a = _host(mesh.trace(_dev(o), _dev(d), tmax=_dev(tm), start_tet=_dev(st), want_tets=True,
                         want_steps=True, kernel=1))
    b = _host(mesh.trace(_dev(o), _dev(d), tmax=_dev(tm), start_tet=_dev(st), want_tets=True,
                         want_steps=True, **kw))
    for k in a:
        assert np.array_equal(a[k], b[k], equal_nan=True), k


def test_layouts_agree(tetrt, tiny_mesh):
    """All layouts run the same arithmetic on the same geometry: identical
    outputs (only the neighbour decoding differs)."""
    m = tiny_mesh
    o, d = random_interior_rays(30000, 41)
    tm = np.random.default_rng(4).uniform(0.0, 0.8, 30000).astype(np.float32)
    outs = []
    for layout in LAYOUTS:
        mesh = tetrt.upload(m.points, m.tets, m.nbrs, m.cflag, layout=layout)
        outs.append(_host(mesh.trace(_dev(o), _dev(d), tmax=_dev(tm), want_tets=True, want_steps=True)))
        mesh.free()
    for other in outs[1:]:
        for k in outs[0]:
            assert np.array_equal(outs[0][k], other[k], equal_nan=True), k


@pytest.mark.parametrize("layout,rec_bytes", [("tet20", 20), ("tet16", 16), ("tet32n", 32), ("tet32", 32)])
def test_hot_bytes_per_layout(tetrt, tiny_mesh, layout, rec_bytes):
    """The arrays a step reads: one record per tet and one unpadded 12-byte point
    per vertex."""
    m = tiny_mesh
    mesh = tetrt.upload(m.points, m.tets, m.nbrs, m.cflag, layout=layout)
    try:
        info = mesh.info
        assert info["n_tets"] == m.n_tets and info["n_points"] == m.n_points
        assert info["hot_bytes"] == rec_bytes * m.n_tets + 12 * m.n_points
    finally:
        mesh.free()


@pytest.mark.parametrize("kw", [dict(sort=2), dict(sort=2, sort_cells_log2=2, sort_dirq=1),
                                dict(sort=2, sort_chunk_log2=10, sort_cells_log2=7, sort_dirq=3),
                                dict(sort=2, sort_chunk_log2=13),
                                dict(sort=2, kernel=2, grid_cap=3, refill=8), dict(sort=2, kernel=3),
                                dict(sort=2, kernel=3, queue_chunk=64, refill=2)])
def test_binned_rays_match_unbinned(tiny, kw):
    """Tracing in bin order through the permutation changes no result, and the
    results stay at the caller's positions."""
    m, om, mesh = tiny
    o, d = random_interior_rays(40001, 43)            # a ragged last chunk
    tm = np.random.default_rng(6).uniform(0.0, 0.6, 40001).astype(np.float32)
    a = _host(mesh.trace(_dev(o), _dev(d), tmax=_dev(tm), want_tets=True, want_steps=True, sort=1))
    b = _host(mesh.trace(_dev(o), _dev(d), tmax=_dev(tm), want_tets=True, want_steps=True, **kw))
    for k in a:
        assert np.array_equal(a[k], b[k], equal_nan=True), k


def test_binning_with_caller_workspace(tiny, tetrt):
    m, om, mesh = tiny
    o, d = random_interior_rays(30000, 47)
    need = mesh.workspace_bytes(30000, True, sort=2)
    assert need >= 4 * 30000
    assert mesh.workspace_bytes(30000, True, sort=1) == 0
    ws = torch.empty(need, dtype=torch.uint8, device="cuda:0")
    a = _host(mesh.trace(_dev(o), _dev(d), tmax=_dev(np.full(30000, 0.3, np.float32)), sort=1))
    b = _host(mesh.trace(_dev(o), _dev(d), tmax=_dev(np.full(30000, 0.3, np.float32)), sort=2,
                         workspace=ws))
    for k in a:
        assert np.array_equal(a[k], b[k], equal_nan=True), k
    with pytest.raises(tetrt.TetRTError):
        mesh.trace(_dev(o), _dev(d), sort=2, workspace=ws[: need // 2])


@pytest.mark.parametrize("kw", [dict(xcds=8), dict(xcds=8, xcd_blocks=1), dict(xcds=8, xcd_blocks=4),
                                dict(xcds=2, xcd_blocks=3, block=64), dict(xcds=8, xcd_blocks=8, sort=2)])
def test_xcd_renumbering_changes_no_result(tiny, kw):
    """Block renumbering for the XCDs only moves rays between lanes."""
    m, om, mesh = tiny
    o, d = random_interior_rays(40001, 53)
    tm = np.random.default_rng(8).uniform(0.0, 0.6, 40001).astype(np.float32)
    a = _host(mesh.trace(_dev(o), _dev(d), tmax=_dev(tm), want_tets=True, want_steps=True, sort=1))
    b = _host(mesh.trace(_dev(o), _dev(d), tmax=_dev(tm), want_tets=True, want_steps=True, **kw))
    for k in a:
        assert np.array_equal(a[k], b[k], equal_nan=True), k


def test_caller_order(tiny, tetrt):
    """tetmesh_bin_rays + order= gives the results of the call's own binning; an
    order with entries out of range leaves those lanes idle."""
    m, om, mesh = tiny
    o, d = random_interior_rays(30001, 59)
    tm = _dev(np.full(30001, 0.4, np.float32))
    O, D = _dev(o), _dev(d)
    a = _host(mesh.trace(O, D, tmax=tm, want_tets=True, want_steps=True, sort=1))
    order = mesh.bin_rays(O, D, sort_chunk_log2=10)
    got = np.sort(order.cpu().numpy())
    assert np.array_equal(got, np.arange(30001))
    b = _host(mesh.trace(O, D, tmax=tm, want_tets=True, want_steps=True, order=order))
    for k in a:
        assert np.array_equal(a[k], b[k], equal_nan=True), k
    rev = torch.arange(30000, -1, -1, dtype=torch.int32, device="cuda:0")
    c = _host(mesh.trace(O, D, tmax=tm, want_tets=True, want_steps=True, order=rev))
    for k in a:
        assert np.array_equal(a[k], c[k], equal_nan=True), k
    bad = rev.clone()
    bad[:100] = 1 << 30                                 # out of range: those rays are skipped
    out = mesh.trace(O, D, tmax=tm, order=bad)
    out["tri"][:] = -9
    mesh.trace_into(out, O, D, tmax=tm, order=bad)
    h = _host(out)
    skipped = np.arange(30000, 29900, -1)               # the rays the first 100 lanes would take
    assert np.all(h["tri"][skipped] == -9)
    rest = np.setdiff1d(np.arange(30001), skipped)
    assert np.array_equal(h["tri"][rest], a["tri"][rest])


def test_concurrent_streams_on_one_handle(tiny, tetrt):
    """A handle is read-only after upload: traces enqueued on two streams at once
    (unbinned primary rays on one, binned secondary rays with their own workspace
    on the other) give the results of the same traces run one after the other."""
    m, om, mesh = tiny
    o1, d1 = random_interior_rays(50000, 61)
    o2, d2 = random_interior_rays(60000, 62)
    tm2 = np.random.default_rng(9).uniform(0.05, 0.5, 60000).astype(np.float32)
    O1, D1, O2, D2, T2 = _dev(o1), _dev(d1), _dev(o2), _dev(d2), _dev(tm2)
    ref1 = _host(mesh.trace(O1, D1, want_steps=True))
    ref2 = _host(mesh.trace(O2, D2, tmax=T2, want_steps=True, sort=2))
    ws = torch.empty(mesh.workspace_bytes(60000, True, sort=2), dtype=torch.uint8, device="cuda:0")
    out1 = tetrt.outputs(50000, "cuda:0", want_steps=True)
    out2 = tetrt.outputs(60000, "cuda:0", want_steps=True)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    torch.cuda.synchronize()
    for _ in range(3):
        with torch.cuda.stream(s1):
            mesh.trace_into(out1, O1, D1, stream=s1)
        with torch.cuda.stream(s2):
            mesh.trace_into(out2, O2, D2, tmax=T2, sort=2, workspace=ws, stream=s2)
        torch.cuda.synchronize()
        got1, got2 = _host(out1), _host(out2)
        for k in ref1:
            assert np.array_equal(got1[k], ref1[k], equal_nan=True), k
        for k in ref2:
            assert np.array_equal(got2[k], ref2[k], equal_nan=True), k


def _raw_trace(tetrt, handle, O, D, T, out, stream=None, **opts):
    """trace_closest through the C-ABI without the Mesh wrapper's workspace."""
    tetrt.binding.trace_closest(handle, O, D, out["tri"], out["t"], out["bary"], tmax=T,
                                steps=out.get("steps"), stream=stream, **opts)


def test_handle_workspace_and_no_workspace(tiny_mesh, tetrt):
    """Binning without a caller workspace: through the handle's own (sized at
    upload) the results are those of an unbinned trace, also for traces on two
    streams one after the other without a synchronisation between them; a handle
    without one refuses an explicit sort = 2 and traces an automatic one unbinned."""
    m = tiny_mesh
    n = 300000                                    # above the automatic binning threshold
    o, d = random_interior_rays(n, 71)
    tm = np.random.default_rng(10).uniform(0.05, 0.5, n).astype(np.float32)
    O, D, T = _dev(o), _dev(d), _dev(tm)
    plain = tetrt.upload(m.points, m.tets, m.nbrs, m.cflag, layout="tet16")
    ws_mesh = tetrt.upload(m.points, m.tets, m.nbrs, m.cflag, layout="tet16", bin_rays=n)
    ref = _host(plain.trace(O, D, tmax=T, want_steps=True, sort=1))
    # automatic binning with no workspace anywhere: unbinned, same results
    out = tetrt.outputs(n, "cuda:0", want_steps=True)
    _raw_trace(tetrt, plain.handle, O, D, T, out)
    got = _host(out)
    for k in ref:
        assert np.array_equal(got[k], ref[k], equal_nan=True), k
    with pytest.raises(tetrt.TetRTError, match="workspace"):
        _raw_trace(tetrt, plain.handle, O, D, T, out, sort=2)
    # the handle's workspace, on two streams back to back
    outs = [tetrt.outputs(n, "cuda:0", want_steps=True) for _ in range(2)]
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    torch.cuda.synchronize()
    for _ in range(2):
        _raw_trace(tetrt, ws_mesh.handle, O, D, T, outs[0], stream=s1, sort=2)
        _raw_trace(tetrt, ws_mesh.handle, O, D, T, outs[1], stream=s2, sort=2, sort_chunk_log2=10)
        torch.cuda.synchronize()
        for o_ in outs:
            got = _host(o_)
            for k in ref:
                assert np.array_equal(got[k], ref[k], equal_nan=True), k
    # more rays than the handle's workspace holds: refused when asked for
    with pytest.raises(tetrt.TetRTError, match="workspace"):
        big = 2 * n + (1 << 18)                   # past all the handle's workspace holds (2n + ~100K)
        O2, D2 = _dev(np.resize(o, (big, 3))), _dev(np.resize(d, (big, 3)))
        _raw_trace(tetrt, ws_mesh.handle, O2, D2, _dev(np.resize(tm, big)),
                   tetrt.outputs(big, "cuda:0"), sort=2)
    plain.free()
    ws_mesh.free()


def test_queue_kernel_needs_a_workspace(tiny_mesh, tetrt):
    """The queue kernel keeps its counters in a workspace: through the raw C-ABI
    without one it is refused; with the caller's or the handle's own it runs, and
    an order from tetmesh_bin_rays feeds its queue."""
    m = tiny_mesh
    mesh = tetrt.upload(m.points, m.tets, m.nbrs, m.cflag, layout="tet16")
    ws_mesh = tetrt.upload(m.points, m.tets, m.nbrs, m.cflag, layout="tet16", bin_rays=10)
    o, d = random_interior_rays(5000, 91)
    O, D = _dev(o), _dev(d)
    ref = _host(mesh.trace(O, D, want_steps=True))
    out = tetrt.outputs(5000, "cuda:0", want_steps=True)
    with pytest.raises(tetrt.TetRTError, match="queue kernel needs a workspace"):
        _raw_trace(tetrt, mesh.handle, O, D, None, out, kernel=3)
    _raw_trace(tetrt, ws_mesh.handle, O, D, None, out, kernel=3)
    got = _host(out)
    for k in ref:
        assert np.array_equal(got[k], ref[k], equal_nan=True), k
    order = mesh.bin_rays(O, D, sort_chunk_log2=10)
    got = _host(mesh.trace(O, D, want_steps=True, kernel=3, order=order))
    for k in ref:
        assert np.array_equal(got[k], ref[k], equal_nan=True), k
    with pytest.raises(tetrt.TetRTError, match="queue_chunk"):
        mesh.trace(O, D, kernel=3, queue_chunk=100)
    mesh.free()
    ws_mesh.free()
