"""Brute-force closest hit in FP64 (TEST INFRASTRUCTURE ONLY).

Every ray is intersected with every constrained triangle using the Moller-Trumbore
ray/triangle test (Moller & Trumbore 1997) with inclusive edges; the smallest
``t`` in ``(0, tmax]`` wins.  This is the plain definition of what the tet walk
computes, so the walk oracle is pinned against it on meshes small enough for
an all-pairs test.
"""
from __future__ import annotations

import numpy as np


def brute_closest_hit(points, tri_verts, orig, dirs, tmax=None, exclude=None,
                      tie_eps: float = 1e-12, chunk_pairs: int = 4_000_000):
    """Closest hit of each ray over all triangles.

    ``tri_verts``: int [F, 3] vertex ids in ascending order (triangle id = row).
    ``exclude``: optional int [n] triangle id to ignore per ray (the face a
    secondary ray leaves from), -1 = none.
    Returns ``(tri, t, bary)``: tri -1 on a miss; bary = weights of the 2nd and
    3rd vertex.  Hits whose t is within ``tie_eps`` (absolute, the scene extent
    is 1) of the smallest go to the lowest triangle id.
    """
    P = np.asarray(points, dtype=np.float64)
    tv = np.asarray(tri_verts, dtype=np.int64).reshape(-1, 3)
    A, B, Cc = P[tv[:, 0]], P[tv[:, 1]], P[tv[:, 2]]
    e1, e2 = B - A, Cc - A
    o_all = np.asarray(orig, dtype=np.float64).reshape(-1, 3)
    d_all = np.asarray(dirs, dtype=np.float64).reshape(-1, 3)
    n = o_all.shape[0]
    F = tv.shape[0]
    tm_all = np.full(n, np.inf) if tmax is None else np.broadcast_to(
        np.asarray(tmax, dtype=np.float64), (n,))
    ex_all = np.full(n, -1, np.int64) if exclude is None else np.asarray(exclude, np.int64)
    tri = np.full(n, -1, np.int32)
    tout = np.full(n, np.nan)
    bary = np.full((n, 2), np.nan)
    if F == 0:
        return tri, tout, bary
    step = max(1, chunk_pairs // F)
    fid = np.arange(F)
    for s in range(0, n, step):
        o = o_all[s:s + step, None, :]
        d = d_all[s:s + step, None, :]
        pvec = np.cross(d, e2[None])
        det = np.einsum("nfk,fk->nf", pvec, e1)
        with np.errstate(divide="ignore", invalid="ignore"):
            inv = 1.0 / det
            sv = o - A[None]
            u = np.einsum("nfk,nfk->nf", sv, pvec) * inv
            qvec = np.cross(sv, e1[None])
            v = np.einsum("nfk,nfk->nf", np.broadcast_to(d, qvec.shape), qvec) * inv
            t = np.einsum("nfk,fk->nf", qvec, e2) * inv
            ok = (det != 0.0) & (u >= 0.0) & (v >= 0.0) & (u + v <= 1.0) & (t > 0.0)
        ok &= t <= tm_all[s:s + step, None]
        ok &= fid[None, :] != ex_all[s:s + step, None]
        tt = np.where(ok, t, np.inf)
        tmin = tt.min(axis=1)
        hit = np.isfinite(tmin)
        near = ok & (tt <= tmin[:, None] + tie_eps)
        first = np.argmax(near, axis=1)
        r = np.arange(tt.shape[0])
        tri[s:s + step] = np.where(hit, first, -1)
        tout[s:s + step] = np.where(hit, t[r, first], np.nan)
        bary[s:s + step, 0] = np.where(hit, u[r, first], np.nan)
        bary[s:s + step, 1] = np.where(hit, v[r, first], np.nan)
    return tri, tout, bary
