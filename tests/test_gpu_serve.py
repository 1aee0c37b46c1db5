"""Serving loop (tm_server_*): generated rays match their definitions, each
request's results equal trace_closest on its rays, and a request's results are
the same alone and in a mix of requests batched together."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from synth import pinhole_rays
from synth.batch import batch_specs, spec_mesh

pytestmark = pytest.mark.gpu

KEYS = ("tri", "t", "bary")


def _host(res):
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in res.items()}


def _same(a, b, what):
    for k in KEYS:
        x, y = a[k], b[k]
        ok = (x == y) | (np.isnan(x) & np.isnan(y)) if x.dtype.kind == "f" else x == y
        assert ok.all(), (what, k, int((~ok).sum()))


@pytest.fixture(scope="module")
def tetrt():
    import paper_2103_02309_amd as tetrt
    return tetrt


@pytest.fixture(scope="module")
def scene(tetrt):
    specs = batch_specs(count=4, seed=31, n_lo=6, n_hi=16)
    hosts = [spec_mesh(s) for s in specs]
    meshes = [tetrt.upload(m.points, m.tets, m.nbrs, m.cflag, layout="tet16") for m in hosts]
    yield specs, hosts, meshes
    for m in meshes:
        m.free()


def _req(spec, k, kind, W, H, seed=7):
    return dict(mesh=k, kind=kind, width=W, height=H, eye=spec["eye"], forward=spec["forward"],
                up=spec["up"], fov_h_deg=60.0, light=(0.5, 0.95, 0.5), ao_tmax=0.15, seed=seed)


def _rays(tetrt, mesh, req, phase, prev=None):
    n = req["width"] * req["height"]
    dev = "cuda:0"
    if prev is None:
        o = torch.empty((n, 3), dtype=torch.float32, device=dev)
        d = torch.empty((n, 3), dtype=torch.float32, device=dev)
    else:
        o, d = prev["orig"].clone(), prev["dirs"].clone()
    tm = torch.empty(n, dtype=torch.float32, device=dev)
    sf = torch.empty(n, dtype=torch.int32, device=dev)
    tetrt.tm_request_rays(mesh.handle, phase, o, d, tm, sf,
                          None if prev is None else prev["tri"], None if prev is None else prev["t"], **req)
    return {"orig": o, "dirs": d, "tmax": tm, "sf": sf}


def _reference(tetrt, mesh, req):
    """trace_closest on the request's own rays, phase by phase."""
    r0 = _rays(tetrt, mesh, req, 0)
    res0 = mesh.trace(r0["orig"], r0["dirs"], tmax=r0["tmax"], start_face=r0["sf"])
    if req["kind"] == "primary":
        return _host(res0)
    r1 = _rays(tetrt, mesh, req, 1, dict(r0, tri=res0["tri"], t=res0["t"]))
    return _host(mesh.trace(r1["orig"], r1["dirs"], tmax=r1["tmax"], start_face=r1["sf"]))


def test_camera_rays_match_pinhole_definition(tetrt, scene):
    specs, hosts, meshes = scene
    s = specs[0]
    req = _req(s, 0, "primary", 64, 40)
    r = _rays(tetrt, meshes[0], req, 0)
    o, d, _ = pinhole_rays(s["eye"], 64, 40, 60.0, forward=s["forward"], up=s["up"], tile=8)
    got = _host(r)
    assert np.array_equal(got["orig"], o)
    assert np.abs(got["dirs"] - d).max() < 2e-6
    assert np.all(np.isinf(got["tmax"])) and np.all(got["sf"] == -1)


@pytest.mark.parametrize("kind", ["shadow", "ao"])
def test_secondary_rays_properties(tetrt, scene, kind):
    specs, hosts, meshes = scene
    k = 1
    s, hm, mesh = specs[k], hosts[k], meshes[k]
    req = _req(s, k, kind, 128, 128)
    r0 = _rays(tetrt, mesh, req, 0)
    res0 = mesh.trace(r0["orig"], r0["dirs"], tmax=r0["tmax"], start_face=r0["sf"])
    r1 = _host(_rays(tetrt, mesh, req, 1, dict(r0, tri=res0["tri"], t=res0["t"])))
    h0, c0 = _host(res0), _host(r0)
    hit = h0["tri"] >= 0
    assert hit.sum() >= 500
    # origins: the hit points; start faces: the hit triangles; no hit -> zero direction
    hp = c0["orig"].astype(np.float64) + h0["t"][:, None].astype(np.float64) * c0["dirs"].astype(np.float64)
    assert np.abs(r1["orig"][hit] - hp[hit]).max() < 1e-6
    assert np.array_equal(r1["sf"][hit], h0["tri"][hit])
    assert np.all(r1["dirs"][~hit] == 0.0) and np.all(r1["sf"][~hit] == -1)
    d = r1["dirs"][hit].astype(np.float64)
    if kind == "shadow":
        assert np.abs(r1["orig"][hit] + d - np.array([0.5, 0.95, 0.5])).max() < 1e-6
        assert np.all(r1["tmax"][hit] == 1.0)
    else:
        assert np.abs(np.linalg.norm(d, axis=1) - 1.0).max() < 1e-5
        assert np.all(r1["tmax"][hit] == np.float32(0.15))
        tv = mesh.tri_vertices(h0["tri"][hit])
        P = hm.points.astype(np.float64)
        n = np.cross(P[tv[:, 1]] - P[tv[:, 0]], P[tv[:, 2]] - P[tv[:, 0]])
        n /= np.linalg.norm(n, axis=1, keepdims=True)
        n *= np.where(np.einsum("ij,ij->i", n, c0["dirs"][hit]) > 0, -1.0, 1.0)[:, None]
        cos = np.einsum("ij,ij->i", n, d)
        assert cos.min() > -1e-5
        # cosine-weighted: E[cos] = 2/3 (standard deviation of cos is sqrt(1/18))
        assert abs(cos.mean() - 2.0 / 3.0) < 5.0 * np.sqrt(1.0 / 18.0 / hit.sum())


@pytest.mark.parametrize("kind", ["primary", "shadow", "ao"])
def test_server_equals_trace(tetrt, scene, kind):
    specs, hosts, meshes = scene
    k = 2
    req = _req(specs[k], k, kind, 96, 64)
    out = tetrt.outputs(96 * 64, "cuda:0")
    srv = tetrt.Server(meshes, max_rays=1 << 16)
    i = srv.submit(out, **req)
    srv.drain()
    done = srv.poll()
    assert [d["id"] for d in done] == [i]
    assert done[0]["submit_ns"] <= done[0]["admit_ns"] <= done[0]["done_ns"]
    assert done[0]["rays"] == 96 * 64 * (1 if kind == "primary" else 2)
    _same(_host(out), _reference(tetrt, meshes[k], req), kind)
    srv.free()


def test_prepared_submit_equals_submit(tetrt, scene):
    """A request packed once (Server.prepare) and submitted into larger output
    buffers gives what the plain submit gives, in the first width x height
    entries; too small outputs are refused on the host."""
    specs, hosts, meshes = scene
    k = 1
    req = _req(specs[k], k, "ao", 80, 48)
    a = tetrt.outputs(80 * 48, "cuda:0")
    b = tetrt.outputs(80 * 48 + 1000, "cuda:0")
    srv = tetrt.Server(meshes, max_rays=1 << 16)
    srv.submit(a, **req)
    srv.submit_prepared(srv.prepare(**req), b)
    srv.drain()
    assert len(srv.poll()) == 2
    hb = {key: v[:80 * 48] for key, v in _host(b).items()}
    _same(_host(a), hb, "prepared")
    small = tetrt.outputs(80 * 48 - 1, "cuda:0")
    with pytest.raises(ValueError):
        srv.submit_prepared(srv.prepare(**req), small)
    srv.free()


def test_server_alone_vs_mix(tetrt, scene):
    specs, hosts, meshes = scene
    rng = np.random.default_rng(5)
    kinds = ["primary", "primary", "shadow", "ao"]
    reqs = []
    for q in range(30):
        k = int(rng.integers(0, len(meshes)))
        W, H = 8 * int(rng.integers(1, 17)), 8 * int(rng.integers(1, 17))
        reqs.append(_req(specs[k], k, kinds[int(rng.integers(0, 4))], W, H, seed=int(rng.integers(0, 1 << 31))))
    # alone: one server call per request
    alone = []
    srv = tetrt.Server(meshes, max_rays=1 << 15)
    for r in reqs:
        out = tetrt.outputs(r["width"] * r["height"], "cuda:0")
        srv.submit(out, **r)
        srv.drain()
        alone.append(_host(out))
    srv.poll()
    srv.free()
    # mixed: all at once through a small pool (admission waits) and a ring of 2
    largest = max(r["width"] * r["height"] for r in reqs)
    srv = tetrt.Server(meshes, max_rays=3 * largest, ring=2, max_requests=8)
    outs, ids = [], []
    for r in reqs:
        outs.append(tetrt.outputs(r["width"] * r["height"], "cuda:0"))
        ids.append(srv.submit(outs[-1], **r))
    steps = 0
    while srv.pending()["queued"] + srv.pending()["admitted"] > 0:
        srv.step()
        steps += 1
        if steps % 4 == 0:
            torch.cuda.synchronize()
        assert steps < 10_000
    done = srv.poll()
    assert sorted(d["id"] for d in done) == sorted(ids)
    for q, (o, a) in enumerate(zip(outs, alone)):
        _same(_host(o), a, "request %d (%s)" % (q, reqs[q]["kind"]))
    srv.free()


def test_server_errors(tetrt, scene):
    specs, hosts, meshes = scene
    srv = tetrt.Server(meshes, max_rays=4096)
    out = tetrt.outputs(64 * 64, "cuda:0")
    with pytest.raises(tetrt.TetRTError, match="multiples of 8"):
        srv.submit(tetrt.outputs(60 * 64, "cuda:0"), **_req(specs[0], 0, "primary", 60, 64))
    with pytest.raises(tetrt.TetRTError, match="mesh index"):
        srv.submit(out, **dict(_req(specs[0], 0, "primary", 64, 64), mesh=9))
    with pytest.raises(tetrt.TetRTError, match="parallel"):
        srv.submit(out, **dict(_req(specs[0], 0, "primary", 64, 64), forward=(0, 1, 0), up=(0, 2, 0)))
    big = tetrt.outputs(128 * 128, "cuda:0")
    with pytest.raises(tetrt.TetRTError, match="exceed"):
        srv.submit(big, **_req(specs[0], 0, "primary", 128, 128))
    assert srv.pending() == {"queued": 0, "admitted": 0, "finished": 0}
    srv.free()
