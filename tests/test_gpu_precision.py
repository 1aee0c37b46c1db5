"""Precision stress on the 16^3 scene: rays aimed through mesh vertices (10%),
along non-surface tet edges (10%) and random (80%), against the FP64 oracle,
for the plain float32 walk and the float64 re-evaluation variant over a sweep
of eps.  Each case prints one JSON line (mismatch rate, t error, fraction of
rays and steps that took the float64 path)."""
import json

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from oracle.compare import compare
from synth import precision_rays

pytestmark = pytest.mark.gpu

N_RAYS = 200_000
EPS = [0.0, 1e-7, 1e-6, 1e-5, 1e-4]
KINDS = {0: "random", 1: "through vertices", 2: "along edges"}
MIN_IDENTICAL = {0: 1.0, 1: 0.99, 2: 0.998}


@pytest.fixture(scope="module")
def stress(tiny_mesh, tiny_oracle):
    import paper_2103_02309_amd as tetrt
    m = tiny_mesh
    o, d, kind = precision_rays(m.points, m.tets, m.cflag, n=N_RAYS, seed=4)
    ref = tiny_oracle.trace(o, d)
    mesh = tetrt.upload(m.points, m.tets, m.nbrs, m.cflag, layout="tet16")
    yield m, tiny_oracle, mesh, o, d, kind, ref
    mesh.free()


def _run(mesh, o, d, eps, start_tet=None):
    st = None if start_tet is None else torch.from_numpy(start_tet).cuda()
    res = mesh.trace(torch.from_numpy(o).cuda(), torch.from_numpy(d).cuda(), start_tet=st,
                     want_steps=True, want_fp64=True, eps=eps, max_steps=20000)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in res.items()}


@pytest.mark.parametrize("eps", EPS)
def test_precision_sweep(stress, eps):
    m, om, mesh, o, d, kind, ref = stress
    got = _run(mesh, o, d, eps)
    report = {"eps": eps, "rays": int(len(o))}
    bad = np.nonzero(got["tri"] == -2)[0][:12]
    if bad.size:
        # the rays that ended at the step cap, for diagnosis
        print("PRECISION_CAP " + json.dumps({"eps": eps, "rays": [
            {"i": int(k), "kind": int(kind[k]), "o": o[k].tolist(), "d": d[k].tolist(),
             "steps": int(got["steps"][k]), "fp64": int(got["fp64_steps"][k]),
             "ref_tri": int(ref["tri"][k]), "ref_steps": int(ref["steps"][k])} for k in bad]}))
    for k, name in KINDS.items():
        s = kind == k
        rep = compare(m.points, om.tri_verts, o[s], d[s], {x: v[s] for x, v in ref.items()},
                      {x: v[s] for x, v in got.items()})
        report[name] = {
            "mismatch_rate": round(1.0 - rep["frac_identical"], 7),
            "unexplained": rep["n_unexplained"],
            "aborted": int((got["tri"][s] == -2).sum()),
            "aborted_before_walk": int(((got["tri"][s] == -2) & (got["steps"][s] == 0)).sum()),
            "invalid": int((got["tri"][s] == -3).sum()),
            "max_t_rel": rep["max_t_rel"],
            "rays_fp64": round(float((got["fp64_steps"][s] > 0).mean()), 5),
            "steps_fp64": round(float(got["fp64_steps"][s].sum() / max(1, got["steps"][s].clip(0).sum())), 6),
        }
        if k == 0:
            # generic rays meet the acceptance rule with or without the variant
            assert rep["ok"], (eps, rep)
        if eps >= 1e-6:
            # with float32 rounding covered, every disagreement is an edge/vertex tie
            assert rep["n_unexplained"] == 0 and rep["gpu_abort_or_invalid"] == 0, (eps, name, rep)
            assert rep["max_t_rel"] <= 1e-5
            # identical ids: every random ray; rays aimed at vertices or along edges
            # meet the surface where several triangles are correct, and the two walks
            # may settle such a tie differently (measured: 99.3% and 99.9% identical)
            assert rep["frac_identical"] >= MIN_IDENTICAL[k], (eps, name, rep["frac_identical"])
    if eps > 0.0:
        # the same rays started in the oracle's located tets: separates location from walk
        st = om.locate(o)
        got2 = _run(mesh, o, d, eps, st)
        s = kind == 2
        rep2 = compare(m.points, om.tri_verts, o[s], d[s], {x: v[s] for x, v in ref.items()},
                       {x: v[s] for x, v in got2.items()})
        report["along edges, oracle start tets"] = {
            "mismatch_rate": round(1.0 - rep2["frac_identical"], 7), "unexplained": rep2["n_unexplained"],
            "aborted": int((got2["tri"][s] == -2).sum()), "invalid": int((got2["tri"][s] == -3).sum())}
    ident = float((got["tri"] == ref["tri"]).mean())
    report["identical_all"] = round(ident, 6)
    if eps >= 1e-6:
        assert ident >= 0.999, ident   # against 99.99% asked: the vertex/edge ties above
    print("PRECISION " + json.dumps(report))
    if eps == 0.0:
        assert (got["fp64_steps"] == 0).all()


@pytest.mark.parametrize("eps", [1e-6, 1e-4])
def test_two_pass_equals_one_pass(stress, eps):
    """The two-pass form (a float32 walk that defers its unsure rays to a list, then
    the float64-capable kernel on the list; passes = 2 with a workspace) gives
    the one-pass precision variant's results bit for bit, also in bin order; and
    the one-pass form with a workspace (its ties listed and resolved by the whole
    grid, the list overflowing into the waves on this set) gives those of the
    one-pass form without one (every tie resolved by its wave)."""
    import paper_2103_02309_amd as tetrt
    m, om, mesh, o, d, kind, ref = stress
    n = len(o)
    O, D = torch.from_numpy(o).cuda(), torch.from_numpy(d).cuda()
    tm = torch.from_numpy(np.random.default_rng(3).uniform(0.1, 2.0, n).astype(np.float32)).cuda()
    for tmax in (None, tm):
        two = mesh.trace(O, D, tmax=tmax, want_steps=True, want_tets=True, want_fp64=True, eps=eps,
                         max_steps=20000, passes=2)
        one = tetrt.outputs(n, "cuda:0", want_tets=True, want_steps=True)
        one["fp64_steps"] = torch.empty(n, dtype=torch.int32, device="cuda:0")
        tetrt.binding.trace_closest(mesh.handle, O, D, one["tri"], one["t"], one["bary"], tmax=tmax,
                                    hit_tets=one["hit_tets"], steps=one["steps"], fp64_steps=one["fp64_steps"],
                                    eps=eps, max_steps=20000)
        torch.cuda.synchronize()
        listed = mesh.trace(O, D, tmax=tmax, want_steps=True, want_tets=True, want_fp64=True, eps=eps,
                            max_steps=20000)
        torch.cuda.synchronize()
        for k in two:
            a, b = two[k].cpu().numpy(), one[k].cpu().numpy()
            assert np.array_equal(a, b, equal_nan=True), (eps, tmax is None, k, int((a != b).sum()))
            c = listed[k].cpu().numpy()
            assert np.array_equal(c, b, equal_nan=True), ("listed ties", eps, tmax is None, k, int((c != b).sum()))
        binned = mesh.trace(O, D, tmax=tmax, want_steps=True, want_tets=True, want_fp64=True, eps=eps,
                            max_steps=20000, sort=2, passes=2)
        torch.cuda.synchronize()
        for k in two:
            assert np.array_equal(binned[k].cpu().numpy(), two[k].cpu().numpy(), equal_nan=True), ("binned", k)
