"""Batched traces over many meshes (tm_batch_*): every job's results equal those
of trace_closest on its own mesh, bit for bit, and agree with the FP64 oracle;
binning, block sizes, graph replays, job-table updates and the autotuner leave
them unchanged."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from oracle.compare import compare
from synth.batch import batch_specs, spec_mesh, camera_rays, ao_from_hits

pytestmark = pytest.mark.gpu

KEYS = ("tri", "t", "bary", "hit_tets", "steps")


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def _host(res):
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in res.items()}


@pytest.fixture(scope="module")
def tetrt():
    import paper_2103_02309_amd as tetrt
    return tetrt


@pytest.fixture(scope="module")
def scenes():
    """Ten uneven meshes (n 4..20) with mixed primary + AO rays (AO from oracle hits)."""
    out = []
    for spec in batch_specs(count=10, seed=21, n_lo=4, n_hi=20, rays_lo=200, rays_hi=30_000):
        m = spec_mesh(spec)
        om = oracle.OracleMesh.from_kuhn(m)
        po, pd = camera_rays(spec)
        pref = om.trace(po, pd)
        ao, ad, atm, sf = ao_from_hits(m.points, lambda ids: om.tri_verts[ids], po, pd, pref["tri"],
                                       pref["t"], spec["rays"] - len(po), spec["ao_seed"])
        o = np.concatenate([po, ao])
        d = np.concatenate([pd, ad])
        tmax = np.concatenate([np.full(len(po), np.inf, np.float32), atm])
        sfc = np.concatenate([np.full(len(po), -1, np.int32), sf])
        out.append(dict(spec=spec, mesh=m, oracle=om, o=o, d=d, tmax=tmax, sf=sfc))
    return out


@pytest.fixture(scope="module", params=["tet16", "tet20"])
def uploaded(request, tetrt, scenes):
    meshes = [tetrt.upload(s["mesh"].points, s["mesh"].tets, s["mesh"].nbrs, s["mesh"].cflag,
                           layout=request.param) for s in scenes]
    yield meshes
    for m in meshes:
        m.free()


def _jobs(tetrt, scenes, meshes, empty_at=(3,), reverse=False):
    jobs = []
    for k, (s, mesh) in enumerate(zip(scenes, meshes)):
        if k in empty_at:
            z = torch.zeros((0, 3), dtype=torch.float32, device="cuda:0")
            jobs.append(dict(mesh=mesh, orig=z, dirs=z.clone(),
                             out=tetrt.outputs(0, "cuda:0", True, True)))
        sel = slice(None, None, -1) if reverse else slice(None)
        n = len(s["o"])
        jobs.append(dict(mesh=mesh, orig=_dev(s["o"][sel]), dirs=_dev(s["d"][sel]),
                         tmax=_dev(s["tmax"][sel]), start_face=_dev(s["sf"][sel]),
                         out=tetrt.outputs(n, "cuda:0", True, True)))
    z = torch.zeros((0, 3), dtype=torch.float32, device="cuda:0")
    jobs.append(dict(mesh=meshes[0], orig=z, dirs=z.clone(), out=tetrt.outputs(0, "cuda:0", True, True)))
    return jobs


def _single(job):
    """The same rays through trace_closest on the job's mesh."""
    res = job["mesh"].trace(job["orig"], job["dirs"], tmax=job.get("tmax"),
                            start_face=job.get("start_face"), want_tets=True, want_steps=True)
    return _host(res)


def _same(a, b, what):
    for k in KEYS:
        x, y = a[k], b[k]
        assert x.shape == y.shape, (what, k)
        if x.dtype.kind == "f":
            ok = (x == y) | (np.isnan(x) & np.isnan(y))
        else:
            ok = x == y
        assert ok.all(), (what, k, int((~ok).sum()))


def _fill(jobs):
    for j in jobs:
        j["out"]["tri"].fill_(-7)
        j["out"]["t"].fill_(123.0)
        j["out"]["bary"].fill_(5.0)
        j["out"]["steps"].fill_(-9)


@pytest.mark.parametrize("kw", [dict(block=64), dict(block=128), dict(block=256), dict(kernel=3),
                                dict(kernel=3, queue_chunk=64, refill=1), dict(kernel=3, queue_chunk=1024, refill=64),
                                dict(kernel=3, xcds=1, sort=2, sort_chunk_log2=10)])
def test_batch_matches_single(tetrt, scenes, uploaded, kw):
    """Every job's results equal trace_closest on its own mesh, bit for bit: the
    one-lane-per-ray batch kernel at each block size, and the persistent waves
    draining one queue over all jobs (rays per fetch, refill threshold, one range
    or one per XCD)."""
    jobs = _jobs(tetrt, scenes, uploaded)
    b = tetrt.Batch(max_jobs=len(jobs), max_rays=sum(int(j["orig"].shape[0]) for j in jobs))
    b.set(jobs, **kw)
    _fill(jobs)
    b.launch()
    for k, j in enumerate(jobs):
        _same(_host(j["out"]), _single(j), "job %d" % k)
    b.free()


@pytest.mark.parametrize("eps", [1e-6, 1e-4])
def test_batch_precision_matches_single(tetrt, scenes, uploaded, eps):
    """The precision variant in a batch gives each job what trace_closest with the
    same eps gives it, bit for bit (and the oracle's ids, as test_batch_oracle)."""
    jobs = _jobs(tetrt, scenes, uploaded)
    b = tetrt.Batch(max_jobs=len(jobs), max_rays=sum(int(j["orig"].shape[0]) for j in jobs))
    b.set(jobs, eps=eps)
    _fill(jobs)
    b.launch()
    for k, j in enumerate(jobs):
        res = j["mesh"].trace(j["orig"], j["dirs"], tmax=j.get("tmax"), start_face=j.get("start_face"),
                              want_tets=True, want_steps=True, eps=eps)
        _same(_host(j["out"]), _host(res), "job %d" % k)
    b.free()


def test_batch_without_step_counts(tetrt, scenes, uploaded):
    """Jobs without step-count or tet-id outputs take the batch kernel that keeps
    no per-ray counts; results equal the counting path bit for bit."""
    jobs = _jobs(tetrt, scenes, uploaded)
    for j in jobs:
        n = int(j["orig"].shape[0])
        j["out"] = tetrt.outputs(n, "cuda:0", False, False)
    b = tetrt.Batch(max_jobs=len(jobs), max_rays=sum(int(j["orig"].shape[0]) for j in jobs))
    b.set(jobs)
    b.launch()
    for k, j in enumerate(jobs):
        got, ref = _host(j["out"]), _single(j)
        for key in ("tri", "t", "bary"):
            assert np.array_equal(got[key], ref[key], equal_nan=True), (k, key)
    b.free()


def test_batch_oracle(tetrt, scenes, uploaded):
    jobs = [j for j in _jobs(tetrt, scenes, uploaded, empty_at=()) if j["orig"].shape[0] > 0]
    b = tetrt.Batch(max_jobs=len(jobs), max_rays=sum(int(j["orig"].shape[0]) for j in jobs))
    b.set(jobs)
    b.launch()
    for s, j in zip(scenes, jobs):
        got = _host(j["out"])
        ref = s["oracle"].trace(s["o"], s["d"], tmax=s["tmax"], start_face=s["sf"])
        rep = compare(s["mesh"].points, s["oracle"].tri_verts, s["o"], s["d"], ref, got,
                      tmax=s["tmax"])
        assert rep["ok"], (s["spec"]["n"], rep)
    b.free()


@pytest.mark.parametrize("chunk", [10, 13])
def test_batch_binned(tetrt, scenes, uploaded, chunk):
    jobs = _jobs(tetrt, scenes, uploaded)
    b = tetrt.Batch(max_jobs=len(jobs), max_rays=sum(int(j["orig"].shape[0]) for j in jobs))
    b.set(jobs, sort=2, sort_chunk_log2=chunk, sort_dirq=3)
    _fill(jobs)
    b.launch()
    for k, j in enumerate(jobs):
        _same(_host(j["out"]), _single(j), "binned job %d" % k)
    b.free()


@pytest.mark.parametrize("kernel", [1, 3])
def test_batch_graph_replays(tetrt, scenes, uploaded, kernel):
    jobs = _jobs(tetrt, scenes, uploaded)
    cap = sum(int(j["orig"].shape[0]) for j in jobs)
    b = tetrt.Batch(max_jobs=len(jobs), max_rays=cap)
    b.set(jobs, sort=2, sort_chunk_log2=10, kernel=kernel)
    want = [_single(j) for j in jobs]
    for rep in range(3):
        _fill(jobs)
        torch.cuda.synchronize()
        x = torch.randn(1 << 20, device="cuda:0")
        (x * 2.0).sum().item()          # unrelated eager work between replays
        b.graph_launch()
        for k, j in enumerate(jobs):
            _same(_host(j["out"]), want[k], "replay %d job %d" % (rep, k))
    # same shape, other rays: the captured graph reads the new table
    jobs2 = _jobs(tetrt, scenes, uploaded, reverse=True)
    b.set(jobs2, sort=2, sort_chunk_log2=10, kernel=kernel)
    _fill(jobs2)
    b.graph_launch()
    for k, j in enumerate(jobs2):
        _same(_host(j["out"]), _single(j), "new table job %d" % k)
    # another shape: fewer jobs, binning off -> captured again
    jobs3 = jobs2[:4]
    b.set(jobs3, sort=1, kernel=kernel)
    _fill(jobs3)
    b.graph_launch()
    for k, j in enumerate(jobs3):
        _same(_host(j["out"]), _single(j), "new shape job %d" % k)
    b.free()


def test_batch_tune(tetrt, scenes, uploaded):
    jobs = _jobs(tetrt, scenes, uploaded)
    b = tetrt.Batch(max_jobs=len(jobs), max_rays=sum(int(j["orig"].shape[0]) for j in jobs))
    b.set(jobs)
    chosen, ms = b.tune(reps=2)
    assert chosen["kernel"] in (1, 3) and chosen["sort"] in (1, 2) and ms > 0
    if chosen["kernel"] == 1:
        assert chosen["block"] in (64, 128, 256)
    else:
        assert chosen["queue_chunk"] in (64, 256, 1024) and chosen["refill"] in (16, 64)
    _fill(jobs)
    b.launch()
    for k, j in enumerate(jobs):
        _same(_host(j["out"]), _single(j), "tuned job %d" % k)
    b.free()


def test_batch_errors(tetrt, scenes, uploaded):
    s = scenes[0]
    other = tetrt.upload(s["mesh"].points, s["mesh"].tets, s["mesh"].nbrs, s["mesh"].cflag,
                         layout="tet32n")
    jobs = _jobs(tetrt, scenes[:2], uploaded[:2], empty_at=())
    n = sum(int(j["orig"].shape[0]) for j in jobs)
    b = tetrt.Batch(max_jobs=len(jobs), max_rays=n)
    mixed = list(jobs)
    mixed[1] = dict(jobs[1], mesh=other)
    with pytest.raises(tetrt.TetRTError, match="layout"):
        b.set(mixed)
    with pytest.raises(tetrt.TetRTError, match="precision"):
        b.set(jobs, eps=1e-6, kernel=3)
    with pytest.raises(tetrt.TetRTError, match="one lane per ray"):
        b.set(jobs, kernel=2)
    with pytest.raises(tetrt.TetRTError, match="queue_chunk"):
        b.set(jobs, kernel=3, queue_chunk=96)
    with pytest.raises(tetrt.TetRTError, match="n_jobs"):
        b.set(jobs + jobs)
    small = tetrt.Batch(max_jobs=len(jobs), max_rays=n - 1)
    with pytest.raises(tetrt.TetRTError, match="max_rays"):
        small.set(jobs)
    # a failed set leaves the previous jobs in place
    b.set(jobs)
    with pytest.raises(tetrt.TetRTError, match="layout"):
        b.set(mixed)
    _fill(jobs)
    b.launch()
    for k, j in enumerate(jobs):
        _same(_host(j["out"]), _single(j), "after errors job %d" % k)
    small.free()
    b.free()
    other.free()


def test_batch_full_size_sampled_oracle(tetrt):
    """The many-mesh workload at its sizes: the largest mesh of the 64-mesh set
    (n = 88, 4.1M tets) with its whole ray budget, beside a small and a middle
    one, in one batched launch (Tet16, the benchmark's layout); AO rays from the
    oracle's camera hits.  20,000 sampled rays per job against the oracle."""
    from _oracle_threads import oracle_trace
    specs = batch_specs(count=64, seed=10)
    order = np.argsort([s["n"] for s in specs])
    pick = [int(order[-1]), int(order[0]), int(order[len(order) // 2])]
    assert specs[pick[0]]["n"] == 88
    rng = np.random.default_rng(90)
    scenes, jobs, meshes = [], [], []
    for k in pick:
        spec = specs[k]
        m = spec_mesh(spec)
        om = oracle.OracleMesh.from_kuhn(m)
        po, pd = camera_rays(spec)
        pref = oracle_trace(om, po, pd)
        ao, ad, atm, sf = ao_from_hits(m.points, lambda ids: om.tri_verts[ids], po, pd, pref["tri"],
                                       pref["t"], spec["rays"] - len(po), spec["ao_seed"])
        o, d = np.concatenate([po, ao]), np.concatenate([pd, ad])
        tmax = np.concatenate([np.full(len(po), np.inf, np.float32), atm])
        sfc = np.concatenate([np.full(len(po), -1, np.int32), sf])
        mesh = tetrt.upload(m.points, m.tets, m.nbrs, m.cflag, layout="tet16")
        meshes.append(mesh)
        jobs.append(dict(mesh=mesh, orig=_dev(o), dirs=_dev(d), tmax=_dev(tmax), start_face=_dev(sfc),
                         out=tetrt.outputs(len(o), "cuda:0")))
        scenes.append((m, om, o, d, tmax, sfc))
    b = tetrt.Batch(max_jobs=len(jobs), max_rays=sum(int(j["orig"].shape[0]) for j in jobs))
    b.set(jobs)
    b.launch()
    for (m, om, o, d, tmax, sfc), j, k in zip(scenes, jobs, pick):
        got = _host(j["out"])
        n = len(o)
        idx = np.sort(rng.choice(n, min(n, 20000), replace=False))
        ref = oracle_trace(om, o[idx], d[idx], tmax[idx], start_face=sfc[idx])
        rep = compare(m.points, om.tri_verts, o[idx], d[idx], ref, {x: v[idx] for x, v in got.items()},
                      tmax=tmax[idx])
        assert rep["ok"], (specs[k]["n"], n, rep)
        assert not np.any(got["tri"] <= -2)
    b.free()
    for mm in meshes:
        mm.free()
