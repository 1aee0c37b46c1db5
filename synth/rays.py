"""Seeded ray sets: pinhole primary rays, cosine-weighted ambient-occlusion rays,
precision-stress rays and uniform random rays.

All rays are produced in float64 and rounded to float32, which is the input
precision of the traversal.  Nothing here traces a ray: secondary (AO) rays are
built from hit records that the caller supplies.
"""
from __future__ import annotations

import numpy as np


def _normalize(v):
    return v / np.linalg.norm(v, axis=-1, keepdims=True)


def tile_order(W: int, H: int, tile: int = 8) -> np.ndarray:
    """Row-major pixel index of each ray when pixels are emitted in ``tile x tile``
    blocks (blocks row-major, pixels row-major inside a block).  ``tile <= 1``
    gives plain row-major order."""
    if tile <= 1:
        return np.arange(W * H, dtype=np.int64)
    ty, tx, iy, ix = np.meshgrid(np.arange((H + tile - 1) // tile), np.arange((W + tile - 1) // tile),
                                 np.arange(tile), np.arange(tile), indexing="ij")
    py = (ty * tile + iy).ravel()
    px = (tx * tile + ix).ravel()
    keep = (py < H) & (px < W)
    return (py[keep] * W + px[keep]).astype(np.int64)


def pinhole_rays(eye, W: int, H: int, fov_h_deg: float = 60.0, forward=(0.0, 0.0, 1.0),
                 up=(0.0, 1.0, 0.0), tile: int = 8):
    """Primary rays of a pinhole camera, one per pixel centre.

    ``fov_h_deg`` is the horizontal field of view; pixel row 0 is the top of the
    image; image right is ``forward x up``.  Returns ``(orig, dir, pixel)`` with
    float32 [n, 3] origins (all equal to ``eye``), float32 unit directions, and
    the row-major pixel index of each ray (rays are emitted in tile order).
    """
    f = _normalize(np.asarray(forward, dtype=np.float64))
    r = _normalize(np.cross(f, np.asarray(up, dtype=np.float64)))
    u = np.cross(r, f)
    pix = tile_order(W, H, tile)
    px = (pix % W).astype(np.float64)
    py = (pix // W).astype(np.float64)
    th = np.tan(np.radians(fov_h_deg) / 2.0)
    sx = (2.0 * (px + 0.5) / W - 1.0) * th
    sy = (1.0 - 2.0 * (py + 0.5) / H) * th * (H / W)
    d = _normalize(f[None, :] + sx[:, None] * r[None, :] + sy[:, None] * u[None, :])
    orig = np.broadcast_to(np.asarray(eye, dtype=np.float64), d.shape).astype(np.float32)
    return np.ascontiguousarray(orig), d.astype(np.float32), pix


def _tangent_frame(n):
    """Unit tangents (t1, t2) orthogonal to unit normals n [m, 3]."""
    a = np.where(np.abs(n[:, :1]) < 0.9, np.array([[1.0, 0.0, 0.0]]), np.array([[0.0, 1.0, 0.0]]))
    t1 = _normalize(np.cross(a, n))
    t2 = np.cross(n, t1)
    return t1, t2


def ao_rays(hit_pos, normal, incoming_dir, k: int = 8, seed: int = 3, tmax: float = 0.1):
    """``k`` cosine-weighted hemisphere rays per hit (Malley's method: uniform disk
    sample lifted to the hemisphere).

    ``hit_pos``: float64 [m, 3] hit points; ``normal``: [m, 3] geometric normals of
    the hit triangles (any orientation); ``incoming_dir``: [m, 3] directions of the
    rays that produced the hits.  The hemisphere is on the side the incoming ray
    came from.  Returns ``(orig f32[m*k,3], dir f32[m*k,3], tmax f32[m*k],
    parent int64[m*k])``; ``parent`` indexes the hit each ray belongs to.
    """
    hit_pos = np.asarray(hit_pos, dtype=np.float64).reshape(-1, 3)
    m = hit_pos.shape[0]
    nrm = _normalize(np.asarray(normal, dtype=np.float64).reshape(-1, 3))
    din = np.asarray(incoming_dir, dtype=np.float64).reshape(-1, 3)
    flip = np.einsum("ij,ij->i", nrm, din) > 0.0
    nrm[flip] *= -1.0
    rng = np.random.default_rng(seed)
    u1 = rng.random((m, k))
    u2 = rng.random((m, k))
    rad = np.sqrt(u1)
    phi = 2.0 * np.pi * u2
    x, y, z = rad * np.cos(phi), rad * np.sin(phi), np.sqrt(np.maximum(0.0, 1.0 - u1))
    t1, t2 = _tangent_frame(nrm)
    d = (x[..., None] * t1[:, None, :] + y[..., None] * t2[:, None, :]
         + z[..., None] * nrm[:, None, :]).reshape(-1, 3)
    d = _normalize(d).astype(np.float32)
    orig = np.repeat(hit_pos.astype(np.float32), k, axis=0)
    parent = np.repeat(np.arange(m, dtype=np.int64), k)
    return orig, d, np.full(m * k, tmax, dtype=np.float32), parent


def tri_geometry(points, tri_vertices):
    """Geometric (unnormalised) normals and vertex positions of triangles given by
    vertex-id triples; float64.  Input preparation for :func:`ao_rays`."""
    P = np.asarray(points, dtype=np.float64)
    tv = np.asarray(tri_vertices, dtype=np.int64).reshape(-1, 3)
    a, b, c = P[tv[:, 0]], P[tv[:, 1]], P[tv[:, 2]]
    return np.cross(b - a, c - a), (a, b, c)


def random_interior_rays(n: int, seed: int, lo: float = 1e-3, hi: float = 1.0 - 1e-3):
    """Origins uniform in ``[lo, hi]^3`` and directions uniform on the sphere."""
    rng = np.random.default_rng(seed)
    o = rng.uniform(lo, hi, size=(n, 3))
    d = _normalize(rng.normal(size=(n, 3)))
    return o.astype(np.float32), d.astype(np.float32)


def surface_edges(tets, cflag, n_points):
    """Sorted int64 keys ``a * n_points + b`` (a < b) of edges of constrained faces."""
    t_idx, slot = np.nonzero(cflag)
    keys = []
    for drop in range(4):
        sel = slot == drop
        if not np.any(sel):
            continue
        f = np.delete(tets[t_idx[sel]], drop, axis=1).astype(np.int64)
        for a, b in ((0, 1), (1, 2), (0, 2)):
            lo = np.minimum(f[:, a], f[:, b])
            hi = np.maximum(f[:, a], f[:, b])
            keys.append(lo * n_points + hi)
    if not keys:
        return np.zeros(0, dtype=np.int64)
    return np.unique(np.concatenate(keys))


def precision_rays(points, tets, cflag, n: int = 2_000_000, seed: int = 4,
                   frac_vertex: float = 0.10, frac_edge: float = 0.10):
    """Precision-stress ray set.

    * ``frac_vertex``: origin uniform in the interior, direction aimed exactly (in
      float64) through a random mesh vertex, then rounded to float32;
    * ``frac_edge``: origin at ``A + s (B - A)``, ``s ~ U(0.1, 0.9)``, direction
      ``+-(B - A)/|B - A|`` along a random tet edge that is not an edge of a
      constrained face;
    * the rest: origin uniform in the interior, direction uniform on the sphere.

    Returns ``(orig f32[n,3], dir f32[n,3], kind int8[n])`` with kind 0 random,
    1 vertex, 2 edge.
    """
    rng = np.random.default_rng(seed)
    P = np.asarray(points, dtype=np.float64)
    nv = int(round(n * frac_vertex))
    ne = int(round(n * frac_edge))
    nr = n - nv - ne
    # random
    o_r = rng.uniform(1e-3, 1.0 - 1e-3, size=(nr, 3))
    d_r = _normalize(rng.normal(size=(nr, 3)))
    # through vertices
    o_v = rng.uniform(1e-3, 1.0 - 1e-3, size=(nv, 3))
    V = P[rng.integers(0, P.shape[0], size=nv)]
    d_v = V - o_v
    bad = np.linalg.norm(d_v, axis=1) == 0.0
    d_v[bad] = 1.0
    d_v = _normalize(d_v)
    # along non-surface edges
    surf = surface_edges(tets, cflag, P.shape[0])
    pairs = np.array([(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)])
    o_e = np.empty((0, 3))
    d_e = np.empty((0, 3))
    while o_e.shape[0] < ne:
        m = 2 * (ne - o_e.shape[0]) + 16
        t = rng.integers(0, tets.shape[0], size=m)
        pr = pairs[rng.integers(0, 6, size=m)]
        A = tets[t, pr[:, 0]].astype(np.int64)
        B = tets[t, pr[:, 1]].astype(np.int64)
        key = np.minimum(A, B) * P.shape[0] + np.maximum(A, B)
        ok = ~np.isin(key, surf)
        A, B = A[ok], B[ok]
        s = rng.uniform(0.1, 0.9, size=(A.shape[0], 1))
        sg = np.where(rng.random(A.shape[0]) < 0.5, -1.0, 1.0)[:, None]
        o_e = np.concatenate([o_e, P[A] + s * (P[B] - P[A])])
        d_e = np.concatenate([d_e, sg * _normalize(P[B] - P[A])])
    o_e, d_e = o_e[:ne], d_e[:ne]
    orig = np.concatenate([o_r, o_v, o_e]).astype(np.float32)
    dirs = np.concatenate([d_r, d_v, d_e]).astype(np.float32)
    kind = np.concatenate([np.zeros(nr, np.int8), np.ones(nv, np.int8), np.full(ne, 2, np.int8)])
    return orig, dirs, kind
