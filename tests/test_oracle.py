"""Pins for the FP64 oracle: each check compares it with something other than
itself (brute force, explicit 2-D containment, closed forms on jitter-free grids,
hand-derived values, invariances of the definition)."""
import itertools
import os

import numpy as np
import pytest

import oracle
from synth import kuhn_mesh, pinhole_rays, random_interior_rays, ao_rays, tri_geometry, precision_rays
from synth.kuhn import random_spheres

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---- Algorithm 1 against explicit containment ---------------------------------

def _orient(a, b, c):
    return (b[0] - a[0]) * (c[1] - a[1]) - (b[1] - a[1]) * (c[0] - a[0])


def _edge(a, b):
    """Orientation of (a, b, origin); exactly zero when the origin is on line ab
    through the origin-anchored form a x b."""
    return a[0] * b[1] - a[1] * b[0]


def _containing_slots(q, strict=True):
    """Slots e such that the face with q3 in place of q[e] holds the origin
    (counter-clockwise, closed unless ``strict``)."""
    out = []
    for e in range(3):
        f = [q[0], q[1], q[2]]
        f[e] = q[3]
        o = [_edge(f[0], f[1]), _edge(f[1], f[2]), _edge(f[2], f[0])]
        if (all(v > 0 for v in o) if strict else all(v >= 0 for v in o)):
            out.append(e)
    return out


def _random_face(rng, scale):
    while True:
        q = rng.normal(size=(3, 2)) * scale
        o = [_orient(q[0], q[1], (0, 0)), _orient(q[1], q[2], (0, 0)), _orient(q[2], q[0], (0, 0))]
        if all(v > 0 for v in o):
            return q
        if all(v < 0 for v in o):
            return q[[0, 2, 1]]


def test_exit_face_matches_containment_random():
    rng = np.random.default_rng(11)
    checked = 0
    for it in range(20000):
        scale = 10.0 ** rng.uniform(-4, 1)
        q = np.zeros((4, 2))
        q[:3] = _random_face(rng, scale)
        q[3] = rng.normal(size=2) * scale * 10.0 ** rng.uniform(-1, 1)
        strict = _containing_slots(q)
        assert len(strict) <= 1
        if strict:
            assert oracle.get_exit_face(q) == strict[0]
            checked += 1
    assert checked > 19000


def test_exit_face_sign_exhaustive():
    """q3 on both sides of (and exactly on) each line origin-q_i."""
    rng = np.random.default_rng(5)
    for it in range(3000):
        q = np.zeros((4, 2))
        q[:3] = _random_face(rng, 1.0)
        for i, s in itertools.product(range(3), (-2.0, -0.5, 0.5, 2.0)):
            for eps in (-1e-3, 0.0, 1e-3):
                perp = np.array([-q[i][1], q[i][0]])
                q[3] = s * q[i] + eps * perp
                e = oracle.get_exit_face(q)
                assert e in _containing_slots(q, strict=False), (q, e)


# ---- the oracle's frame ----------------------------------------------------------

def test_onb_orthonormal_right_handed():
    rng = np.random.default_rng(2)
    ns = list(rng.normal(size=(2000, 3))) + [np.array(v, float) for v in
                                               ([0, 0, 1], [0, 0, -1], [1, 0, 0], [0, -1, 0],
                                                [1e-12, 0, -1], [0, 1e-9, 1])]
    for n in ns:
        n = n / np.linalg.norm(n)
        b1, b2 = oracle.onb(n)
        M = np.stack([b1, b2, n])
        assert np.allclose(M @ M.T, np.eye(3), atol=1e-12)
        assert np.allclose(np.cross(b1, b2), n, atol=1e-12)


# ---- hand-derived golden values --------------------------------------------------

def _read_golden(name):
    rows = []
    for line in open(os.path.join(GOLDEN, name)):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        lhs, rhs = line.split("|")
        rows.append(([float(x) for x in lhs.split()], [float(x) for x in rhs.split()]))
    return rows


def _golden_box(split):
    """The closed Kuhn box of the golden files: every cube boundary face is scene
    geometry; with ``split`` also the interior face (0,4,7) between t0 and t1."""
    m = kuhn_mesh(1, jitter=0.0)
    assert m.tets[0].tolist() == [0, 4, 6, 7] and m.tets[1].tolist() == [0, 4, 7, 5]
    cf = (m.nbrs < 0).astype(np.uint8)
    if split:
        j0 = int(np.nonzero(m.tets[0] == 6)[0][0])     # t0's face opposite vertex 6
        j1 = int(np.nonzero(m.tets[1] == 5)[0][0])     # t1's face opposite vertex 5
        assert m.nbrs[0, j0] == 1 and m.nbrs[1, j1] == 0
        cf[0, j0] = cf[1, j1] = 1
    return m, oracle.OracleMesh(m.points, m.tets, m.nbrs, cf)


@pytest.mark.parametrize("name,split,ntri", [("kuhn_cube_box.txt", False, 12),
                                             ("kuhn_cube_split.txt", True, 13)])
@pytest.mark.parametrize("max_steps", [0, 1])
def test_golden_cube_box(name, split, ntri, max_steps):
    """Hand-derived hits, step counts, start tets and front/back tets.  With a cap
    of one step, the rays whose walk takes two steps are answered by the oracle's
    fallback (the closest hit by its definition, steps = -1) and must give the
    same triangle, t, weights and tets."""
    m, om = _golden_box(split)
    assert om.ntri == ntri
    rows = _read_golden(name)
    inp = np.array([r[0] for r in rows])
    exp = np.array([r[1] for r in rows])
    r = om.trace(inp[:, 0:3], inp[:, 3:6], inp[:, 6], max_steps=max_steps)
    assert r["tri"].tolist() == exp[:, 0].astype(int).tolist()
    hit = exp[:, 0] >= 0
    assert np.allclose(r["t"][hit], exp[hit, 1], rtol=1e-14, atol=0)
    assert np.allclose(r["bary"][hit], exp[hit, 2:4], atol=1e-14)
    steps = exp[:, 4].astype(int)
    if max_steps:
        assert (steps > max_steps).any()
        steps = np.where(steps > max_steps, -1, steps)
    assert r["steps"].tolist() == steps.tolist()
    assert r["start"].tolist() == exp[:, 5].astype(int).tolist()
    assert r["tets"].tolist() == exp[:, 6:8].astype(int).tolist()


# ---- against brute force ---------------------------------------------------------

def _check_vs_brute(om, points, orig, dirs, tmax=None, start_face=None, t_rtol=1e-12,
                    bary_tol=1e-10):
    r = om.trace(orig, dirs, tmax, start_face=start_face)
    bt, btt, bb = oracle.brute_closest_hit(points, om.tri_verts, orig, dirs, tmax, exclude=start_face)
    assert np.all(r["tri"] >= -1), np.unique(r["tri"])
    # generic rays (no vertex on the ray) never need the fallback: the walk itself
    # answers them
    assert np.all(r["steps"] >= 0), np.nonzero(r["steps"] < 0)[0][:10]
    same = r["tri"] == bt
    # ties between triangles sharing an edge may go either way; the brute force
    # then has a second hit at the same t
    if not np.all(same):
        bad = np.nonzero(~same)[0]
        for i in bad:
            assert r["tri"][i] >= 0 and bt[i] >= 0, (i, r["tri"][i], bt[i])
            assert abs(r["t"][i] - btt[i]) <= 1e-12
            # the oracle's triangle is also hit at that t
            tv = om.tri_verts[r["tri"][i]]
            P = points.astype(np.float64)
            A, B, Cc = P[tv[0]], P[tv[1]], P[tv[2]]
            h = orig[i].astype(np.float64) + btt[i] * dirs[i].astype(np.float64)
            w = np.linalg.lstsq(np.stack([B - A, Cc - A], 1), h - A, rcond=None)[0]
            assert w.min() > -1e-9 and w.sum() < 1 + 1e-9
    h = same & (bt >= 0)
    assert np.all(np.abs(r["t"][h] - btt[h]) <= t_rtol * np.abs(btt[h]))
    assert np.all(np.abs(r["bary"][h] - bb[h]) <= bary_tol)
    return r, same.mean()


def test_tiny_primary_vs_brute(tiny_mesh, tiny_oracle):
    o, d, _ = pinhole_rays((0.5, 0.5, 0.05), 64, 64, 60.0)
    r, frac = _check_vs_brute(tiny_oracle, tiny_mesh.points, o, d)
    assert frac == 1.0
    assert np.all(r["tri"] >= 0)          # the camera looks straight at the sphere


@pytest.mark.parametrize("n,jit,nsph,seed", [(4, 0.1, 2, 1), (8, 0.1, 5, 2), (8, 0.0, 3, 3),
                                             (6, 0.1, 1, 4)])
def test_random_rays_vs_brute(n, jit, nsph, seed):
    m = kuhn_mesh(n, jitter=jit, seed=seed, spheres=random_spheres(nsph, seed=seed, r_lo=0.1, r_hi=0.3))
    om = oracle.OracleMesh.from_kuhn(m)
    o, d = random_interior_rays(3000, seed)
    tm = np.random.default_rng(seed).uniform(0.05, 1.5, size=3000).astype(np.float32)
    tm[::3] = np.inf
    _check_vs_brute(om, m.points, o, d, tm)


def test_secondary_rays_vs_brute(tiny_mesh, tiny_oracle):
    """AO rays leaving from primary hits (start face given) against brute force
    with the start face excluded."""
    o, d, _ = pinhole_rays((0.5, 0.5, 0.05), 32, 32, 60.0)
    r = tiny_oracle.trace(o, d)
    hit = r["tri"] >= 0
    hp = o[hit].astype(np.float64) + r["t"][hit, None] * d[hit].astype(np.float64)
    nrm, _ = tri_geometry(tiny_mesh.points, tiny_oracle.tri_verts[r["tri"][hit]])
    ao, ad, atm, parent = ao_rays(hp, nrm, d[hit], k=8, seed=3, tmax=0.1)
    sf = r["tri"][hit][parent]
    _check_vs_brute(tiny_oracle, tiny_mesh.points, ao, ad, atm, start_face=sf, t_rtol=1e-9,
                    bary_tol=1e-8)


def _check_hit_tets(om, points, dirs, r):
    """Front/back tets of every hit: the two tets of the hit face, the front one
    on the side the ray comes from (its fourth vertex lies against the direction)."""
    hit = np.nonzero(r["tri"] >= 0)[0]
    P = np.asarray(points, np.float64)
    tv = om.tri_verts[r["tri"][hit]]
    A = P[tv[:, 0]]
    nf = np.cross(P[tv[:, 1]] - A, P[tv[:, 2]] - A)
    nd = np.einsum("ij,ij->i", nf, np.asarray(dirs, np.float64)[hit])
    pair = om.tri_tets[r["tri"][hit]]
    front, back = r["tets"][hit, 0], r["tets"][hit, 1]
    assert np.all(np.sort(np.stack([front, back], 1), 1) == np.sort(pair, 1))
    off = np.array([[v for v in om.tets[t] if v not in f][0] for t, f in zip(front, tv)])
    side = np.einsum("ij,ij->i", nf, P[off] - A)
    assert np.all(side * nd < 0)


def _fallback_vs_brute(om, points, o, d, tmax=None, start_face=None):
    """Rays traced with a cap of one step: every ray whose walk needs more takes the
    oracle's fallback.  Against brute force: the same id (both take the lowest id
    among hits within 1e-12 of the nearest), t to 1e-12 relative, weights to 1e-10."""
    r = om.trace(o, d, tmax, start_face=start_face, max_steps=1)
    fb = r["steps"] == -1
    assert fb.mean() > 0.5
    bt, btt, bb = oracle.brute_closest_hit(points, om.tri_verts, o, d, tmax, exclude=start_face)
    assert np.array_equal(r["tri"][fb], bt[fb])
    h = fb & (bt >= 0)
    assert h.sum() > 100
    assert np.all(np.abs(r["t"][h] - btt[h]) <= 1e-12 * np.abs(btt[h]))
    assert np.all(np.abs(r["bary"][h] - bb[h]) <= 1e-10)
    _check_hit_tets(om, points, d, r)
    return r


@pytest.mark.parametrize("kind", [1, 2])
def test_fallback_vs_brute_degenerate_rays(tiny_mesh, tiny_oracle, kind):
    """Rays aimed through mesh vertices (kind 1) and along tet edges (kind 2): many
    hit where several triangles meet, so the tie rule decides the id."""
    m = tiny_mesh
    o, d, k = precision_rays(m.points, m.tets, m.cflag, n=20000, seed=4)
    s = k == kind
    r = _fallback_vs_brute(tiny_oracle, m.points, o[s], d[s])
    # the fallback agrees with the walk wherever the walk finishes normally
    w = tiny_oracle.trace(o[s], d[s])
    ok = w["steps"] >= 0
    same = ok & (w["tri"] == r["tri"])
    assert same.sum() > 0.95 * ok.sum()
    assert np.array_equal(w["tets"][same], r["tets"][same])


@pytest.fixture(scope="module")
def degenerate_set(tiny_mesh, tiny_oracle):
    """The rays of the precision stress set (200,000 at seed 4) aimed through mesh
    vertices and along tet edges, their walk results and brute force."""
    m = tiny_mesh
    o, d, k = precision_rays(m.points, m.tets, m.cflag, n=200_000, seed=4)
    s = k >= 1
    o, d, k = o[s], d[s], k[s]
    w = tiny_oracle.trace(o, d)
    b = oracle.brute_closest_hit(m.points, tiny_oracle.tri_verts, o, d)
    return o, d, k, w, b


def test_degenerate_rays_hits_lie_on_the_ray(tiny_mesh, tiny_oracle, degenerate_set):
    """Every hit the oracle reports lies on its ray: the line meets the reported
    triangle (to 1e-9 of the scene extent) at the reported t > 0, and no hit comes
    before the closest one of the definition.  Rays that run along tet edges or
    through vertices are where the FP64 walk meets zero determinants; a walk that
    leaves its ray there must take the definition instead."""
    from oracle.compare import ray_triangle_gap
    o, d, k, w, (bt, btt, _) = degenerate_set
    h = np.nonzero(w["tri"] >= 0)[0]
    gap = ray_triangle_gap(tiny_mesh.points, tiny_oracle.tri_verts, w["tri"][h], o[h], d[h])
    assert gap.max() <= 1e-9, (gap.max(), h[np.argmax(gap)])
    assert np.all(w["t"][h] > 0)
    both = h[bt[h] >= 0]
    assert np.all(w["t"][both] >= btt[both] * (1 - 1e-9))
    # the degenerate rays do exercise the fallback (circling or leaving the ray)
    assert (w["steps"] == -1).sum() > 100


def test_degenerate_rays_vs_brute(tiny_mesh, tiny_oracle, degenerate_set):
    """Against the definition: the same triangle, except where the ray meets the
    surface at an edge or vertex (several triangles then contain the hit point, or
    the walk may pass between them); t to 1e-12 and weights to 1e-9 on identical
    hits."""
    o, d, k, w, (bt, btt, bb) = degenerate_set
    same = w["tri"] == bt
    assert same.mean() > 0.999
    P = tiny_mesh.points.astype(np.float64)
    mism = np.nonzero(~same)[0]
    hb = mism[bt[mism] >= 0]
    if hb.size:
        hp = o[hb].astype(np.float64) + btt[hb, None] * d[hb].astype(np.float64)
        tv = tiny_oracle.tri_verts[bt[hb]]
        A, B, Cc = P[tv[:, 0]], P[tv[:, 1]], P[tv[:, 2]]

        def seg(p, a, b):
            ab = b - a
            t = np.clip(np.einsum("ij,ij->i", p - a, ab) / np.einsum("ij,ij->i", ab, ab), 0, 1)
            return np.linalg.norm(p - (a + t[:, None] * ab), axis=1)

        edge = np.minimum(np.minimum(seg(hp, A, B), seg(hp, B, Cc)), seg(hp, Cc, A))
        assert edge.max() <= 1e-9, (edge.max(), hb[np.argmax(edge)])
    h = same & (bt >= 0)
    assert h.sum() > 1000
    assert np.all(np.abs(w["t"][h] - btt[h]) <= 1e-12 * np.abs(btt[h]) + 1e-12)
    assert np.all(np.abs(w["bary"][h] - bb[h]) <= 1e-9)


def test_fallback_vs_brute_secondary(tiny_mesh, tiny_oracle):
    """Secondary rays leaving hit faces, half of them into the sphere (every one of
    those hits its far side): the fallback must exclude the start face."""
    o, d, _ = pinhole_rays((0.5, 0.5, 0.05), 16, 16, 60.0)
    r0 = tiny_oracle.trace(o, d)
    hit = r0["tri"] >= 0
    hp = o[hit].astype(np.float64) + r0["t"][hit, None] * d[hit].astype(np.float64)
    nrm, _ = tri_geometry(tiny_mesh.points, tiny_oracle.tri_verts[r0["tri"][hit]])
    inward = np.where((np.arange(hit.sum()) % 2 == 0)[:, None], -d[hit], d[hit])
    ao, ad, atm, parent = ao_rays(hp, nrm, inward, k=8, seed=3, tmax=np.inf)
    sf = r0["tri"][hit][parent]
    r = _fallback_vs_brute(tiny_oracle, tiny_mesh.points, ao, ad, atm, start_face=sf)
    w = tiny_oracle.trace(ao, ad, atm, start_face=sf)
    assert np.array_equal(w["tri"], r["tri"])
    h = w["tri"] >= 0
    assert np.array_equal(w["tets"][h], r["tets"][h])


def test_fallback_ties_go_to_lowest_id():
    """Jitter-free grid, rays along +z whose x - y is a multiple of the cell size:
    each meets the surface exactly on the diagonal edge that two triangles of one
    cell face share (coordinates dyadic, so both triangles contain the point
    exactly).  The closest hit is then tied; the definition gives it the lower id."""
    m = kuhn_mesh(16, jitter=0.0)
    om = oracle.OracleMesh.from_kuhn(m)
    rng = np.random.default_rng(12)
    k = 2000
    a = np.round(rng.uniform(0.2, 0.8, k) * 2 ** 20) / 2 ** 20
    c = rng.integers(-3, 4, k) / 16.0
    o = np.stack([a, a - c, np.full(k, 0.03125)], 1).astype(np.float32)
    d = np.tile(np.array([[0, 0, 1]], np.float32), (k, 1))
    r = om.trace(o, d, max_steps=1)
    assert np.all(r["steps"] == -1)
    bt, btt, _ = oracle.brute_closest_hit(m.points, om.tri_verts, o, d)
    assert np.array_equal(r["tri"], bt)
    # the tie is real: with the reported triangle excluded, another is hit at the same t
    hit = np.nonzero(bt >= 0)[0][:300]
    t2, tt2, _ = oracle.brute_closest_hit(m.points, om.tri_verts, o[hit], d[hit], exclude=bt[hit])
    tied = (t2 >= 0) & (np.abs(tt2 - btt[hit]) <= 1e-12)
    assert tied.sum() > 100
    assert np.all(t2[tied] > bt[hit][tied])


def test_walk_hit_tets(tiny_mesh, tiny_oracle):
    """The walk's own front/back tets on the camera rays and random rays."""
    o, d, _ = pinhole_rays((0.5, 0.5, 0.05), 32, 32, 60.0)
    _check_hit_tets(tiny_oracle, tiny_mesh.points, d, tiny_oracle.trace(o, d))
    o, d = random_interior_rays(2000, 17)
    _check_hit_tets(tiny_oracle, tiny_mesh.points, d, tiny_oracle.trace(o, d))


# ---- closed forms on jitter-free grids ------------------------------------------

def _planes_crossed(o, h, n):
    """Hyperplanes x_i = k/n and x_i - x_j = k/n crossed strictly between o and h."""
    cnt = 0
    fs = [lambda x, i=i: x[..., i] for i in range(3)]
    fs += [lambda x, i=i, j=j: x[..., i] - x[..., j] for i, j in ((0, 1), (0, 2), (1, 2))]
    for f in fs:
        a, b = n * f(o), n * f(h)
        lo, hi = np.minimum(a, b), np.maximum(a, b)
        cnt = cnt + np.maximum(0, np.ceil(hi - 1e-7) - np.floor(lo + 1e-7) - 1).astype(int)
    return cnt


def test_step_count_closed_form():
    # n a power of two keeps every grid coordinate k/n exact in float32, so the
    # tet faces lie exactly on the planes counted below
    n = 8
    m = kuhn_mesh(n, jitter=0.0, spheres=[[0.5, 0.45, 0.55, 0.3], [0.2, 0.8, 0.3, 0.15]])
    om = oracle.OracleMesh.from_kuhn(m)
    o, d = random_interior_rays(4000, 21)
    r = om.trace(o, d)
    bt, btt, _ = oracle.brute_closest_hit(m.points, om.tri_verts, o, d)
    hit = bt >= 0
    assert hit.sum() > 800
    h = o[hit].astype(np.float64) + btt[hit, None] * d[hit].astype(np.float64)
    expect = _planes_crossed(o[hit].astype(np.float64), h, n)
    assert np.array_equal(r["steps"][hit], expect)


def test_axis_parallel_t_closed_form():
    n = 16
    m = kuhn_mesh(n, jitter=0.0)           # sphere r = 0.35 at the centre
    om = oracle.OracleMesh.from_kuhn(m)
    rng = np.random.default_rng(8)
    k = 400
    o = np.stack([rng.uniform(0.2, 0.8, k), rng.uniform(0.2, 0.8, k), rng.uniform(0.01, 0.1, k)], 1)
    o = o.astype(np.float32)
    d = np.tile(np.array([[0, 0, 1]], np.float32), (k, 1))
    r = om.trace(o, d)
    ci = np.floor(o[:, 0].astype(np.float64) * n).astype(int)
    cj = np.floor(o[:, 1].astype(np.float64) * n).astype(int)
    ck = np.floor(o[:, 2].astype(np.float64) * n).astype(int)
    for i in range(k):
        col = m.inside[ci[i], cj[i]]
        change = [z for z in range(ck[i], n - 1) if col[z] != col[z + 1]]
        if not change:
            assert r["tri"][i] == -1
            continue
        zhit = (change[0] + 1) / n
        assert r["tri"][i] >= 0
        assert abs(r["t"][i] - (zhit - float(o[i, 2]))) <= 1e-13


# ---- invariances of the definition -----------------------------------------------

def test_independent_of_source_tet(tiny_mesh, tiny_oracle):
    o, d = random_interior_rays(2000, 31)
    base = tiny_oracle.trace(o, d, source_tet=0)
    for src in (777, 12345, tiny_mesh.n_tets - 1):
        r = tiny_oracle.trace(o, d, source_tet=src)
        assert np.array_equal(r["tri"], base["tri"])
        h = base["tri"] >= 0
        assert np.array_equal(r["t"][h], base["t"][h])


def test_early_out_changes_nothing(tiny_mesh, tiny_oracle):
    o, d = random_interior_rays(3000, 41)
    tm = np.random.default_rng(1).uniform(0.0, 0.4, 3000).astype(np.float32)
    a = tiny_oracle.trace(o, d, tm, early_out=True)
    b = tiny_oracle.trace(o, d, tm, early_out=False)
    assert np.array_equal(a["tri"], b["tri"])
    h = a["tri"] >= 0
    assert np.array_equal(a["t"][h], b["t"][h])
    assert a["steps"].sum() < b["steps"].sum()


def test_locate_contains_point(tiny_mesh, tiny_oracle):
    rng = np.random.default_rng(3)
    x = rng.uniform(0.0, 1.0, size=(3000, 3)).astype(np.float32)
    t = tiny_oracle.locate(x)
    assert np.all(t >= 0)
    P = tiny_mesh.points.astype(np.float64)
    V = P[tiny_mesh.tets[t]]
    X = x.astype(np.float64)
    for j in range(4):   # x is on the inner side of every face (closed)
        f = [s for s in range(4) if s != j]
        A, B, Cc, W = V[:, f[0]], V[:, f[1]], V[:, f[2]], V[:, j]
        nrm = np.cross(B - A, Cc - A)
        sw = np.einsum("ij,ij->i", nrm, W - A)
        sx = np.einsum("ij,ij->i", nrm, X - A)
        assert np.all(sx * np.sign(sw) >= -1e-15)
    out = tiny_oracle.locate(np.array([[1.5, 0.5, 0.5], [-0.1, 0.2, 0.2]], np.float32))
    assert out.tolist() == [-1, -1]


def test_invalid_rays_and_start_tet(tiny_mesh, tiny_oracle):
    o = np.array([[0.5, 0.5, 0.05]] * 3 + [[2.0, 0.5, 0.5]], np.float32)
    d = np.array([[0, 0, 0], [np.nan, 0, 1], [0, 0, 1], [0, 0, 1]], np.float32)
    r = tiny_oracle.trace(o, d)
    assert r["tri"].tolist()[:2] == [-3, -3] and r["tri"][2] >= 0 and r["tri"][3] == -3
    # a caller-supplied start tet gives the same answer as location
    st = tiny_oracle.locate(o[2:3])
    r2 = tiny_oracle.trace(o[2:3], d[2:3], start_tet=st)
    assert r2["tri"][0] == r["tri"][2] and r2["t"][0] == r["t"][2]


def test_inconsistent_mesh_rejected():
    m = kuhn_mesh(4, jitter=0.0, spheres=[[0.5, 0.5, 0.5, 0.3]])
    cf = m.cflag.copy()
    t, j = np.argwhere(cf)[0]
    cf[t, j] = 0          # break the symmetry of one flag: the other side still has it
    with pytest.raises(ValueError):
        oracle.OracleMesh(m.points, m.tets, m.nbrs, cf)
