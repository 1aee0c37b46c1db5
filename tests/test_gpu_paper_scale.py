"""Parity at full size: the 12.6M-tet scene with the 1920x1080 camera, traced in
the launch configuration the benchmark times (Hilbert order, 8x8 pixel tiles,
the library's automatic block size: 128 threads for camera rays, 256 for binned
AO rays).  The oracle checks a seeded sample of rays one by one;
properties that hold for any ray are checked on all of them."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from oracle.compare import compare, ray_triangle_gap
from synth import config_mesh, pinhole_rays, ao_rays, tri_geometry

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def scene():
    m = config_mesh("paper")
    om = oracle.OracleMesh.from_kuhn(m)
    o, d, _ = pinhole_rays((0.5, 0.5, 0.02), 1920, 1080, 60.0, tile=8)
    return m, om, o, d


# Tet16 is the benchmark's layout; Tet20 is the paper's GPU layout; Tet32 the paper's
# 32-byte layout; Tet32N the one-round-trip variant
@pytest.fixture(scope="module", params=["tet16", "tet20", "tet32", "tet32n"])
def paper(request, scene):
    import paper_2103_02309_amd as tetrt
    m, om, o, d = scene
    mesh = tetrt.upload(m.points, m.tets, m.nbrs, m.cflag, layout=request.param)
    res = mesh.trace(torch.from_numpy(o).cuda(), torch.from_numpy(d).cuda(), want_tets=True,
                     want_steps=True)
    torch.cuda.synchronize()
    got = {k: v.cpu().numpy() for k, v in res.items()}
    yield m, mesh, om, o, d, got
    mesh.free()


def _check_properties(m, mesh, o, d, got, tmax=None):
    """Hold for every ray: normal termination, t within (0, tmax], the reported
    triangle lies on the ray (the line passes within 1e-6 of it: float32 exit
    decisions can only err that close to an edge), NaN outputs on a miss."""
    tri = got["tri"]
    assert not np.any(tri <= -2), np.unique(tri[tri <= -2], return_counts=True)
    h = tri >= 0
    t = got["t"][h]
    assert np.all(np.isfinite(t)) and np.all(t > -1e-6)
    if tmax is not None:
        assert np.all(t <= tmax[h])
    b = got["bary"][h].astype(np.float64)
    off = np.nonzero(h)[0][(b.min(axis=1) < 0) | (b.sum(axis=1) > 1)]
    if off.size:
        tv = mesh.tri_vertices(tri[off])
        gap = ray_triangle_gap(m.points, tv, np.arange(off.size), o[off], d[off])
        assert gap.max() <= 1e-6, (gap.max(), off[np.argmax(gap)])
    assert np.all(np.isnan(got["t"][~h]))


def test_primary_all_rays_properties(paper):
    m, mesh, om, o, d, got = paper
    assert got["tri"].shape[0] == 1920 * 1080
    _check_properties(m, mesh, o, d, got)
    assert 0.3 < (got["tri"] >= 0).mean() < 0.95


def test_primary_benchmark_kernel_identical(paper):
    """The benchmark times the walk without per-ray step counts and tet ids (a
    kernel of its own): on all 2,073,600 rays it gives bit for bit the results
    of the counting kernel that the oracle comparisons below check."""
    m, mesh, om, o, d, got = paper
    res = mesh.trace(torch.from_numpy(o).cuda(), torch.from_numpy(d).cuda())
    torch.cuda.synchronize()
    for k, v in res.items():
        assert np.array_equal(v.cpu().numpy(), got[k], equal_nan=True), k
    # ... and with the camera located once on the device and shared as every ray's
    # start tet, as the benchmark runs it
    import paper_2103_02309_amd as tetrt
    cam = torch.tensor([[0.5, 0.5, 0.02]], dtype=torch.float32, device="cuda:0")
    cam_tet = torch.empty(1, dtype=torch.int32, device="cuda:0")
    tetrt.tetmesh_locate(mesh.handle, cam, cam_tet)
    start = cam_tet.expand(o.shape[0]).contiguous()
    assert int(cam_tet.item()) == int(om.locate(o[:1])[0])
    res = mesh.trace(torch.from_numpy(o).cuda(), torch.from_numpy(d).cuda(), start_tet=start)
    torch.cuda.synchronize()
    for k, v in res.items():
        assert np.array_equal(v.cpu().numpy(), got[k], equal_nan=True), k
    # ... and by persistent waves draining the queue (per-XCD ranges, the default
    # rays per fetch and refill)
    res = mesh.trace(torch.from_numpy(o).cuda(), torch.from_numpy(d).cuda(), start_tet=start, kernel=3)
    torch.cuda.synchronize()
    for k, v in res.items():
        assert np.array_equal(v.cpu().numpy(), got[k], equal_nan=True), ("queue", k)


def test_primary_sampled_vs_oracle(paper):
    m, mesh, om, o, d, got = paper
    idx = np.sort(np.random.default_rng(12).choice(o.shape[0], 20000, replace=False))
    cam = om.locate(o[:1])
    ref = om.trace(o[idx], d[idx], start_tet=np.full(idx.shape[0], cam[0], np.int32))
    sub = {k: v[idx] for k, v in got.items()}
    rep = compare(m.points, om.tri_verts, o[idx], d[idx], ref, sub)
    assert rep["ok"], rep
    same = sub["tri"] == ref["tri"]
    assert np.array_equal(sub["hit_tets"][same & (ref["tri"] >= 0)], ref["tets"][same & (ref["tri"] >= 0)])
    assert (sub["steps"] == ref["steps"]).mean() > 0.99
    # the precision variant on the same rays meets the same bar
    res = mesh.trace(torch.from_numpy(o).cuda(), torch.from_numpy(d).cuda(), eps=1e-6)
    torch.cuda.synchronize()
    sub = {k: v.cpu().numpy()[idx] for k, v in res.items()}
    rep = compare(m.points, om.tri_verts, o[idx], d[idx], ref, sub)
    assert rep["ok"], ("eps 1e-6", rep)


def test_plane_rays_vs_oracle(paper):
    """The camera rays that lie exactly in the plane x = y (every one of them,
    1,080 rays through the grid's diagonal faces; the 607 that reach the cube's
    unjittered far boundary are this workload's exact float64 ties, answered by
    the grid tie scan), traced by the precision variant: identical to the
    oracle, ray for ray (the standard bar, 99.99% of 1,080)."""
    m, mesh, om, o, d, got = paper
    idx = np.nonzero(d[:, 0] == d[:, 1])[0]
    assert idx.size == 1080
    cam = om.locate(o[:1])
    ref = om.trace(o[idx], d[idx], start_tet=np.full(idx.size, cam[0], np.int32))
    O, D = torch.from_numpy(o[idx]).cuda(), torch.from_numpy(d[idx]).cuda()
    res = mesh.trace(O, D, eps=1e-6, want_fp64=True)
    torch.cuda.synchronize()
    sub = {k: v.cpu().numpy() for k, v in res.items()}
    rep = compare(m.points, om.tri_verts, o[idx], d[idx], ref, sub)
    assert rep["ok"], rep
    # the same rays among all 2M of the benchmark's launch give the same answers
    res = mesh.trace(torch.from_numpy(o).cuda(), torch.from_numpy(d).cuda(), eps=1e-6)
    torch.cuda.synchronize()
    for k in ("tri", "t", "bary"):
        assert np.array_equal(res[k].cpu().numpy()[idx], sub[k], equal_nan=True), k


def test_ao_sampled_vs_oracle(paper):
    """AO rays built from oracle hits of a primary sample."""
    m, mesh, om, o, d, got = paper
    idx = np.sort(np.random.default_rng(13).choice(o.shape[0], 6000, replace=False))
    cam = om.locate(o[:1])
    ref0 = om.trace(o[idx], d[idx], start_tet=np.full(idx.shape[0], cam[0], np.int32))
    hit = ref0["tri"] >= 0
    hp = o[idx][hit].astype(np.float64) + ref0["t"][hit, None] * d[idx][hit].astype(np.float64)
    nrm, _ = tri_geometry(m.points, om.tri_verts[ref0["tri"][hit]])
    ao, ad, atm, parent = ao_rays(hp, nrm, d[idx][hit], k=8, seed=3, tmax=0.1)
    sf = ref0["tri"][hit][parent].astype(np.int32)
    # binned, with the automatic die placement: the benchmark's AO launch
    res = mesh.trace(torch.from_numpy(ao).cuda(), torch.from_numpy(ad).cuda(),
                     tmax=torch.from_numpy(atm).cuda(), start_face=torch.from_numpy(sf).cuda(),
                     want_tets=True, want_steps=True, sort=2)
    torch.cuda.synchronize()
    g = {k: v.cpu().numpy() for k, v in res.items()}
    ref = om.trace(ao, ad, atm, start_face=sf)
    rep = compare(m.points, om.tri_verts, ao, ad, ref, g, tmax=atm)
    assert rep["ok"], rep
    _check_properties(m, mesh, ao, ad, g, atm)
    # the benchmark's kernel (no step counts or tet ids) gives the same results, and
    # so do persistent waves draining the queue of the binned rays
    for kw in (dict(), dict(kernel=3)):
        res = mesh.trace(torch.from_numpy(ao).cuda(), torch.from_numpy(ad).cuda(),
                         tmax=torch.from_numpy(atm).cuda(), start_face=torch.from_numpy(sf).cuda(), sort=2, **kw)
        torch.cuda.synchronize()
        for k, v in res.items():
            assert np.array_equal(v.cpu().numpy(), g[k], equal_nan=True), (kw, k)
    # the precision variant on the same rays meets the same bar
    res = mesh.trace(torch.from_numpy(ao).cuda(), torch.from_numpy(ad).cuda(),
                     tmax=torch.from_numpy(atm).cuda(), start_face=torch.from_numpy(sf).cuda(), sort=2,
                     eps=1e-6)
    torch.cuda.synchronize()
    rep = compare(m.points, om.tri_verts, ao, ad, ref, {k: v.cpu().numpy() for k, v in res.items()}, tmax=atm)
    assert rep["ok"], ("eps 1e-6", rep)


def test_ao_from_device_hits_properties(paper):
    """The benchmark's AO set (built from the device's own primary hits): every
    ray terminates normally and respects tmax.  (These inputs come from the
    device, so they are checked by properties only, never against the oracle.)"""
    m, mesh, om, o, d, got = paper
    hit = got["tri"] >= 0
    hp = o[hit].astype(np.float64) + got["t"][hit, None].astype(np.float64) * d[hit].astype(np.float64)
    nrm, _ = tri_geometry(m.points, mesh.tri_vertices(got["tri"][hit]))
    ao, ad, atm, parent = ao_rays(hp, nrm, d[hit], k=8, seed=3, tmax=0.1)
    sf = got["tri"][hit][parent].astype(np.int32)
    A = [torch.from_numpy(x).cuda() for x in (ao, ad, atm, sf)]
    order = mesh.bin_rays(A[0], A[1])         # as the benchmark: binning, then the walk
    res = mesh.trace(A[0], A[1], tmax=A[2], start_face=A[3], order=order)
    torch.cuda.synchronize()
    g = {k: v.cpu().numpy() for k, v in res.items()}
    _check_properties(m, mesh, ao, ad, g, atm)
    # the call's own binning gives the same results
    g2 = {k: v.cpu().numpy() for k, v in mesh.trace(A[0], A[1], tmax=A[2], start_face=A[3]).items()}
    for k in g:
        assert np.array_equal(g[k], g2[k], equal_nan=True), k


def test_finer_grid_sampled_vs_oracle():
    """The same scene on a 160^3 grid (24.6M tets: Tet16 records and points are
    442 MB, past the 256 MB last-level cache), in the benchmark's launch
    configuration: 10,000 sampled primary rays and the AO rays of 2,000 of them
    against the oracle, every ray by properties."""
    import paper_2103_02309_amd as tetrt
    from synth import config_mesh
    from _oracle_threads import oracle_trace
    m = config_mesh("paper160")
    om = oracle.OracleMesh.from_kuhn(m)
    o, d, _ = pinhole_rays((0.5, 0.5, 0.02), 1920, 1080, 60.0, tile=8)
    mesh = tetrt.upload(m.points, m.tets, m.nbrs, m.cflag, layout="tet16")
    assert mesh.info["hot_bytes"] > 256e6
    try:
        res = mesh.trace(torch.from_numpy(o).cuda(), torch.from_numpy(d).cuda(), want_steps=True)
        torch.cuda.synchronize()
        got = {k: v.cpu().numpy() for k, v in res.items()}
        _check_properties(m, mesh, o, d, got)
        rng = np.random.default_rng(16)
        idx = np.sort(rng.choice(o.shape[0], 10000, replace=False))
        cam = om.locate(o[:1])
        ref = oracle_trace(om, o[idx], d[idx], start_tet=np.full(idx.shape[0], cam[0], np.int32))
        rep = compare(m.points, om.tri_verts, o[idx], d[idx], ref, {k: v[idx] for k, v in got.items()})
        assert rep["ok"], rep
        sub = idx[:2000]
        hit = ref["tri"][:2000] >= 0
        hp = o[sub][hit].astype(np.float64) + ref["t"][:2000][hit, None] * d[sub][hit].astype(np.float64)
        nrm, _ = tri_geometry(m.points, om.tri_verts[ref["tri"][:2000][hit]])
        ao, ad, atm, parent = ao_rays(hp, nrm, d[sub][hit], k=8, seed=3, tmax=0.1)
        sf = ref["tri"][:2000][hit][parent].astype(np.int32)
        res = mesh.trace(torch.from_numpy(ao).cuda(), torch.from_numpy(ad).cuda(),
                         tmax=torch.from_numpy(atm).cuda(), start_face=torch.from_numpy(sf).cuda(), sort=2)
        torch.cuda.synchronize()
        g = {k: v.cpu().numpy() for k, v in res.items()}
        ref_a = oracle_trace(om, ao, ad, atm, start_face=sf)
        rep = compare(m.points, om.tri_verts, ao, ad, ref_a, g, tmax=atm)
        assert rep["ok"], rep
    finally:
        mesh.free()
