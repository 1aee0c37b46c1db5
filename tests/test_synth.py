"""Input generator checks: mesh invariants of the Kuhn-grid scenes and ray sets."""
import numpy as np
import pytest

from synth import kuhn_mesh, config_mesh, pinhole_rays, ao_rays, precision_rays
from synth.kuhn import tet_volumes6, random_spheres
from synth.rays import tile_order


def _face_table(tets):
    T = tets.shape[0]
    faces = np.sort(np.stack([np.delete(tets, j, axis=1) for j in range(4)], axis=1), axis=2)
    return faces.reshape(T * 4, 3)


@pytest.mark.parametrize("n,jit", [(1, 0.0), (2, 0.1), (4, 0.1), (7, 0.0), (8, 0.1)])
def test_kuhn_counts_and_links(n, jit):
    m = kuhn_mesh(n, jitter=jit, seed=3, spheres=random_spheres(3, seed=n))
    assert m.n_tets == 6 * n ** 3
    assert m.n_points == (n + 1) ** 3
    assert np.all(tet_volumes6(m.points, m.tets) > 0)
    # neighbours: found by face hashing, independently of the construction
    faces = _face_table(m.tets)
    key = (faces[:, 0].astype(np.int64) * m.n_points + faces[:, 1]) * m.n_points + faces[:, 2]
    order = np.argsort(key, kind="stable")
    ks = key[order]
    same = np.nonzero(ks[1:] == ks[:-1])[0]
    expect = np.full(m.n_tets * 4, -1, np.int64)
    a, b = order[same], order[same + 1]
    expect[a] = b // 4
    expect[b] = a // 4
    assert np.array_equal(expect.reshape(-1, 4), m.nbrs)
    # flags symmetric, never on the cube boundary
    fl = m.cflag.reshape(-1)
    assert np.array_equal(fl[a], fl[b])
    assert not np.any(fl[expect < 0])
    # Euler characteristic of a ball
    E = set()
    for i in range(4):
        for k in range(i + 1, 4):
            lo = np.minimum(m.tets[:, i], m.tets[:, k]).astype(np.int64)
            hi = np.maximum(m.tets[:, i], m.tets[:, k]).astype(np.int64)
            E.update((lo * m.n_points + hi).tolist())
    F = len(np.unique(key))
    assert m.n_points - len(E) + F - m.n_tets == 1


def test_tiny_config_counts(tiny_mesh):
    assert tiny_mesh.n_tets == 24576 and tiny_mesh.n_points == 4913
    # sphere r = 0.35 at the centre of a 16^3 grid: 576 inside/outside cell faces,
    # each split into two triangles
    assert tiny_mesh.n_constrained_faces() == 1152
    # jitter is +-0.1 cell and keeps volumes positive; the smallest 6*volume of a
    # Kuhn tet of side h is h^3, jitter shrinks it by well under half
    v = tet_volumes6(tiny_mesh.points, tiny_mesh.tets)
    assert v.min() > 0.4 / 16 ** 3


def test_jitter_only_moves_interior_vertices():
    m0 = kuhn_mesh(5, jitter=0.0)
    m1 = kuhn_mesh(5, jitter=0.1, seed=9)
    d = np.abs(m1.points - m0.points).max(axis=1)
    onb = np.any((m0.points == 0) | (m0.points == 1), axis=1)
    assert np.all(d[onb] == 0)
    assert np.all(d[~onb] > 0) and d.max() <= 0.1 / 5 + 1e-7


def test_pinhole_rays_shape_and_tiles():
    o, d, pix = pinhole_rays((0.5, 0.5, 0.05), 64, 64, 60.0)
    assert o.shape == (4096, 3) and d.shape == (4096, 3)
    assert np.allclose(np.linalg.norm(d, axis=1), 1, atol=1e-6)
    assert sorted(pix.tolist()) == list(range(4096))
    # first 64 rays form one 8x8 tile
    assert set((pix[:64] % 64).tolist()) == set(range(8))
    assert set((pix[:64] // 64).tolist()) == set(range(8))
    # horizontal FOV: the extreme columns are +-30 degrees off axis (minus half a pixel)
    row = d[np.argsort(pix)].reshape(64, 64, 3)[32]
    ang = np.degrees(np.arctan2(np.abs(row[:, 0]), row[:, 2]))
    assert 29.0 < ang.max() < 30.0
    assert np.array_equal(tile_order(3, 2, 1), np.arange(6))


def test_ao_rays_hemisphere():
    rng = np.random.default_rng(0)
    hp = rng.random((50, 3))
    nrm = rng.normal(size=(50, 3))
    din = rng.normal(size=(50, 3))
    o, d, tm, parent = ao_rays(hp, nrm, din, k=8, seed=1)
    assert o.shape == (400, 3) and np.all(tm == np.float32(0.1))
    n_side = -np.sign(np.einsum("ij,ij->i", nrm, din))[:, None] * nrm
    cosv = np.einsum("ij,ij->i", d.astype(np.float64), n_side[parent] / np.linalg.norm(n_side[parent], axis=1, keepdims=True))
    assert np.all(cosv > -1e-6)
    # cosine-weighted: E[cos] = 2/3
    assert abs(cosv.mean() - 2.0 / 3.0) < 0.05


def test_precision_rays_mix(tiny_mesh):
    o, d, kind = precision_rays(tiny_mesh.points, tiny_mesh.tets, tiny_mesh.cflag, n=2000, seed=4)
    assert (kind == 1).sum() == 200 and (kind == 2).sum() == 200
    assert np.allclose(np.linalg.norm(d, axis=1), 1, atol=1e-6)
    assert np.all((o >= 0) & (o <= 1))


def test_paper_config_spheres():
    sp = random_spheres(20, seed=2)
    assert sp.shape == (20, 4)
    assert np.all((sp[:, :3] >= 0.15) & (sp[:, :3] <= 0.85))
    assert np.all((sp[:, 3] >= 0.03) & (sp[:, 3] <= 0.12))
    # the camera at (0.5, 0.5, 0.02) is outside every sphere
    assert np.all(np.linalg.norm(sp[:, :3] - [0.5, 0.5, 0.02], axis=1) > sp[:, 3])


def test_batch_specs_ranges_and_seeding():
    from synth.batch import batch_specs, camera_rays, ao_from_hits
    a = batch_specs(count=64, seed=10)
    b = batch_specs(count=64, seed=10)
    assert [s["n"] for s in a] == [s["n"] for s in b]
    ns = np.array([s["n"] for s in a])
    rays = np.array([s["rays"] for s in a])
    assert ns.min() >= 8 and ns.max() <= 96 and len(set(ns)) > 20
    assert rays.min() >= 1000 and rays.max() <= 1_000_000
    for s in a:
        assert 1 <= len(s["spheres"]) <= 10
        assert np.all((s["eye"] > 0.0) & (s["eye"] < 1.0))
        assert abs(np.linalg.norm(s["forward"]) - 1.0) < 1e-12
    o, d = camera_rays(a[0])
    assert o.shape == ((a[0]["rays"] + 1) // 2, 3) and d.dtype == np.float32
    # AO rays: nothing hit -> empty; otherwise count rays leaving from hit faces
    z = ao_from_hits(None, None, o, d, np.full(len(o), -1, np.int32), np.zeros(len(o), np.float32), 10, 1)
    assert all(len(x) == 0 for x in z)


def test_served_secondary_rays_definition():
    """Host-side served rays: the PCG hash is a permutation of 32-bit values (on a
    2^20 sample: no collisions) and its unit numbers are uniform; shadow rays end
    at the light (t = 1); AO rays are unit, on the incoming side of the normal, and
    cosine-distributed (E[cos] = 2/3); pixels without a hit get a zero direction."""
    from synth.serve import pcg_hash, unit_floats, secondary_rays
    h = pcg_hash(np.arange(1 << 20, dtype=np.uint64))
    assert np.unique(h).size == 1 << 20
    u = unit_floats(h)
    assert u.min() >= 0.0 and u.max() < 1.0 and abs(u.mean() - 0.5) < 2e-3
    P = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0]], np.float32)
    tv = np.array([[0, 1, 2]])
    n = 20000
    rng = np.random.default_rng(1)
    o = np.c_[rng.uniform(0.05, 0.3, n), rng.uniform(0.05, 0.3, n), np.full(n, 1.0)].astype(np.float32)
    d = np.tile(np.array([[0, 0, -1]], np.float32), (n, 1))
    tri = np.zeros(n, np.int32)
    tri[::10] = -1
    t = np.ones(n)
    req = dict(kind="shadow", light=(0.5, 0.5, 3.0), ao_tmax=0.1, seed=5)
    so, sd, stm, ssf = secondary_rays(req, P, tv, o, d, tri, t)
    hit = tri >= 0
    assert np.allclose(so[hit] + sd[hit], [0.5, 0.5, 3.0], atol=1e-6) and np.all(stm[hit] == 1.0)
    assert np.all(sd[~hit] == 0) and np.all(ssf[~hit] == -1) and np.all(ssf[hit] == 0)
    ao, ad, atm, asf = secondary_rays(dict(req, kind="ao"), P, tv, o, d, tri, t)
    assert np.allclose(np.linalg.norm(ad[hit], axis=1), 1.0, atol=1e-6)
    cos = ad[hit, 2].astype(np.float64)      # the normal on the incoming side is +z
    assert cos.min() >= 0.0 and abs(cos.mean() - 2.0 / 3.0) < 5.0 * np.sqrt(1.0 / 18.0 / hit.sum())
    assert np.all(atm[hit] == np.float32(0.1)) and np.allclose(ao[hit, 2], 0.0)
