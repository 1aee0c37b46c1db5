"""The parity checker (oracle/compare.py) on planted disagreements: results are
taken from the oracle and one field is changed on the CPU, and the checker must
accept exactly the disagreements its rule allows (a ray meeting an edge that
several triangles share) and reject the rest."""
import numpy as np

import oracle
from oracle.compare import compare
from synth import kuhn_mesh, pinhole_rays


def _copy(r):
    return {k: np.array(v, copy=True) for k, v in r.items()}


def test_identical_results_pass(tiny_mesh, tiny_oracle):
    o, d, _ = pinhole_rays((0.5, 0.5, 0.05), 32, 32, 60.0)
    ref = tiny_oracle.trace(o, d)
    rep = compare(tiny_mesh.points, tiny_oracle.tri_verts, o, d, ref, _copy(ref))
    assert rep["ok"] and rep["identical"] == rep["n"]


def test_wrong_triangle_is_unexplained(tiny_mesh, tiny_oracle):
    o, d, _ = pinhole_rays((0.5, 0.5, 0.05), 32, 32, 60.0)
    ref = tiny_oracle.trace(o, d)
    got = _copy(ref)
    # a hit replaced by a triangle on the far side of the sphere
    i = int(np.nonzero(ref["tri"] >= 0)[0][100])
    far = int(np.argmax(tiny_mesh.points[tiny_oracle.tri_verts[:, 0], 2]))
    got["tri"][i] = far
    rep = compare(tiny_mesh.points, tiny_oracle.tri_verts, o, d, ref, got, min_identical=0.0)
    assert rep["n_unexplained"] == 1 and rep["unexplained"] == [i] and not rep["ok"]
    # and a hit reported as a miss, its point deep inside the triangle
    got = _copy(ref)
    got["tri"][i] = -1
    rep = compare(tiny_mesh.points, tiny_oracle.tri_verts, o, d, ref, got, min_identical=0.0)
    assert rep["n_unexplained"] == 1


def test_shared_edge_tie_is_explained():
    """Rays that meet the surface exactly on the diagonal edge two triangles share:
    reporting the other triangle is a correct answer."""
    m = kuhn_mesh(16, jitter=0.0)
    om = oracle.OracleMesh.from_kuhn(m)
    rng = np.random.default_rng(12)
    k = 400
    a = np.round(rng.uniform(0.2, 0.8, k) * 2 ** 20) / 2 ** 20
    c = rng.integers(-3, 4, k) / 16.0
    o = np.stack([a, a - c, np.full(k, 0.03125)], 1).astype(np.float32)
    d = np.tile(np.array([[0, 0, 1]], np.float32), (k, 1))
    ref = om.trace(o, d, max_steps=1)
    hit = np.nonzero(ref["tri"] >= 0)[0]
    t2, tt2, bb2 = oracle.brute_closest_hit(m.points, om.tri_verts, o[hit], d[hit], exclude=ref["tri"][hit])
    tied = hit[(t2 >= 0) & (np.abs(tt2 - ref["t"][hit]) <= 1e-12)]
    assert tied.size > 50
    got = _copy(ref)
    alt = dict(zip(hit.tolist(), t2.tolist()))
    for i in tied:
        got["tri"][i] = alt[int(i)]
    rep = compare(m.points, om.tri_verts, o, d, ref, got, min_identical=0.0)
    assert rep["mismatches"] == tied.size and rep["n_unexplained"] == 0
    # a triangle that is not on that edge is not explained
    got["tri"][tied[0]] = (alt[int(tied[0])] + 7) % om.ntri
    rep = compare(m.points, om.tri_verts, o, d, ref, got, min_identical=0.0)
    assert rep["n_unexplained"] == 1


def test_hit_beyond_tmax_and_t_error(tiny_mesh, tiny_oracle):
    o, d, _ = pinhole_rays((0.5, 0.5, 0.05), 32, 32, 60.0)
    ref = tiny_oracle.trace(o, d)
    hit = np.nonzero(ref["tri"] >= 0)[0]
    # tmax just below each hit: the oracle misses; a compared hit would lie beyond tmax
    tm = np.full(len(o), np.inf, np.float32)
    tm[hit] = (ref["t"][hit] * 0.5).astype(np.float32)
    ref_tm = tiny_oracle.trace(o, d, tm)
    assert np.all(ref_tm["tri"][hit] == -1)
    rep = compare(tiny_mesh.points, tiny_oracle.tri_verts, o, d, ref_tm, _copy(ref), tmax=tm,
                  min_identical=0.0)
    assert rep["n_unexplained"] == hit.size
    # t off by 1e-4 relative on one matched hit
    got = _copy(ref)
    got["t"][hit[5]] *= 1.0001
    rep = compare(tiny_mesh.points, tiny_oracle.tri_verts, o, d, ref, got)
    assert rep["t_bad"] == 1 and not rep["ok"]
    # an abort code where the oracle traces normally
    got = _copy(ref)
    got["tri"][hit[7]] = -2
    rep = compare(tiny_mesh.points, tiny_oracle.tri_verts, o, d, ref, got, min_identical=0.0)
    assert rep["gpu_abort_or_invalid"] == 1 and rep["n_unexplained"] == 1


def test_t_tolerances(tiny_mesh, tiny_oracle):
    """A matched hit's t: within t_rtol * t passes, beyond it fails; an absolute
    allowance (per ray) widens the bound by exactly that much."""
    o, d, _ = pinhole_rays((0.5, 0.5, 0.05), 32, 32, 60.0)
    ref = tiny_oracle.trace(o, d)
    i = int(np.nonzero(ref["tri"] >= 0)[0][7])
    for shift, atol, ok in ((0.5e-5, 0.0, True), (2e-5, 0.0, False), (2e-5, 2e-5 * ref["t"][i], True),
                            (4e-5, 2e-5 * ref["t"][i], False)):
        got = _copy(ref)
        got["t"][i] = ref["t"][i] * (1.0 + shift)
        at = np.zeros(len(o))
        at[i] = atol
        rep = compare(tiny_mesh.points, tiny_oracle.tri_verts, o, d, ref, got, t_atol=at)
        assert rep["ok"] == ok, (shift, atol, rep["max_t_rel"])
