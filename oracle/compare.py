"""Parity check of traversal results against the oracle (TEST INFRASTRUCTURE ONLY).

Acceptance, per ray set:
  * identical triangle id (or the same miss/abort code) for >= 99.99% of rays;
  * every other ray is explained: its hit point (the oracle's, or the point
    where the ray meets the other side's triangle) lies within ``edge_tol``
    (relative to the scene extent) of an edge or vertex of the oracle's or the
    compared triangle -- several ids are then correct -- or, for a hit/miss
    disagreement, the hit's t is within ``tmax_rtol`` of tmax;
  * matched hits: |dt| / t <= ``t_rtol`` and |d bary| <= ``bary_tol``;
  * no step-cap (-2) or invalid (-3) code on rays the oracle traces normally.
"""
from __future__ import annotations

import numpy as np


def _seg_dist(p, a, b):
    """Distance from points p [m, 3] to segments ab [m, 3]."""
    ab = b - a
    den = np.einsum("ij,ij->i", ab, ab)
    s = np.clip(np.einsum("ij,ij->i", p - a, ab) / np.where(den > 0, den, 1.0), 0.0, 1.0)
    return np.linalg.norm(p - (a + s[:, None] * ab), axis=1)


def _edge_distance(P, tri_verts, tri, h):
    """Distance from points h [m, 3] to the nearest edge of triangles ``tri``."""
    tv = tri_verts[tri]
    A, B, Cc = P[tv[:, 0]], P[tv[:, 1]], P[tv[:, 2]]
    return np.minimum(np.minimum(_seg_dist(h, A, B), _seg_dist(h, B, Cc)), _seg_dist(h, Cc, A))


def _plane_point(P, tri_verts, tri, o, d):
    tv = tri_verts[tri]
    A, B, Cc = P[tv[:, 0]], P[tv[:, 1]], P[tv[:, 2]]
    n = np.cross(B - A, Cc - A)
    with np.errstate(divide="ignore", invalid="ignore"):
        t = np.einsum("ij,ij->i", n, A - o) / np.einsum("ij,ij->i", n, d)
    return o + t[:, None] * d


def _line_seg_dist(o, u, a, b):
    """Distance between the lines o + s*u (u unit, s free) and segments ab."""
    e = b - a
    w0 = o - a
    bb = np.einsum("ij,ij->i", u, e)
    cc = np.einsum("ij,ij->i", e, e)
    dd = np.einsum("ij,ij->i", u, w0)
    ee = np.einsum("ij,ij->i", e, w0)
    den = cc - bb * bb
    with np.errstate(divide="ignore", invalid="ignore"):
        v = np.where(den > 1e-300, (ee - bb * dd) / den, 0.0)
    v = np.clip(v, 0.0, 1.0)
    s = bb * v - dd
    return np.linalg.norm(w0 + s[:, None] * u - v[:, None] * e, axis=1)


def ray_triangle_gap(points, tri_verts, tri, orig, dirs):
    """How far the line of each ray passes from its reported triangle: 0 when it
    crosses the triangle, else the distance to the nearest edge (float64)."""
    P = np.asarray(points, dtype=np.float64)
    tv = np.asarray(tri_verts)[tri]
    A, B, Cc = P[tv[:, 0]], P[tv[:, 1]], P[tv[:, 2]]
    o = np.asarray(orig, dtype=np.float64).reshape(-1, 3)
    d = np.asarray(dirs, dtype=np.float64).reshape(-1, 3)
    u = d / np.linalg.norm(d, axis=1, keepdims=True)
    with np.errstate(divide="ignore", invalid="ignore"):
        # inside test of the plane point
        n = np.cross(B - A, Cc - A)
        t = np.einsum("ij,ij->i", n, A - o) / np.einsum("ij,ij->i", n, u)
        h = o + t[:, None] * u
        inside = np.ones(len(o), dtype=bool)
        for X, Y in ((A, B), (B, Cc), (Cc, A)):
            inside &= np.einsum("ij,ij->i", np.cross(Y - X, h - X), n) >= 0
        gap = np.minimum(np.minimum(_line_seg_dist(o, u, A, B), _line_seg_dist(o, u, B, Cc)),
                         _line_seg_dist(o, u, Cc, A))
    return np.where(inside & np.isfinite(t), 0.0, gap)


def compare(points, tri_verts, orig, dirs, ref, got, tmax=None, extent=1.0, edge_tol=1e-6,
            t_rtol=1e-5, bary_tol=1e-4, tmax_rtol=1e-6, min_identical=0.9999):
    """Compare ``got`` (numpy dict: tri, t, bary) with oracle results ``ref``.
    Returns a report dict with ``ok`` and the details."""
    P = np.asarray(points, dtype=np.float64)
    o = np.asarray(orig, dtype=np.float64).reshape(-1, 3)
    d = np.asarray(dirs, dtype=np.float64).reshape(-1, 3)
    n = o.shape[0]
    rt, gt = np.asarray(ref["tri"]), np.asarray(got["tri"])
    tm = np.full(n, np.inf) if tmax is None else np.broadcast_to(np.asarray(tmax, np.float64), (n,))
    same = rt == gt
    rep = {"n": n, "identical": int(same.sum()), "frac_identical": float(same.mean()) if n else 1.0}
    # codes the oracle does not produce on valid rays
    bad_code = (gt <= -2) & (rt > -2)
    rep["gpu_abort_or_invalid"] = int(bad_code.sum())
    mism = np.nonzero(~same)[0]
    explained = np.zeros(mism.shape[0], dtype=bool)
    tol = edge_tol * extent
    if mism.size:
        mo, md = o[mism], d[mism]
        r_hit, g_hit = rt[mism] >= 0, gt[mism] >= 0
        ref_h = mo + np.asarray(ref["t"])[mism][:, None] * md
        near = np.zeros(mism.size, dtype=bool)
        if r_hit.any():
            idx = np.nonzero(r_hit)[0]
            near[idx] |= _edge_distance(P, tri_verts, rt[mism][idx], ref_h[idx]) <= tol
        if g_hit.any():
            idx = np.nonzero(g_hit)[0]
            # the ray's point on the other triangle's plane, and on the oracle's
            gh = _plane_point(P, tri_verts, gt[mism][idx], mo[idx], md[idx])
            near[idx] |= _edge_distance(P, tri_verts, gt[mism][idx], gh) <= tol
            both = idx[r_hit[idx]]
            if both.size:
                near[both] |= _edge_distance(P, tri_verts, gt[mism][both], ref_h[both]) <= tol
        # hit/miss at tmax
        tm_m = tm[mism]
        with np.errstate(invalid="ignore"):
            rtm = r_hit & ~g_hit & (np.abs(np.asarray(ref["t"])[mism] - tm_m) <= tmax_rtol * tm_m)
            gtv = np.asarray(got["t"], dtype=np.float64)[mism]
            gtm = g_hit & ~r_hit & (np.abs(gtv - tm_m) <= tmax_rtol * tm_m)
        explained = (near | rtm | gtm) & ~bad_code[mism]
    rep["mismatches"] = int(mism.size)
    rep["unexplained"] = mism[~explained].tolist()[:50]
    rep["n_unexplained"] = int((~explained).sum())
    hit = same & (rt >= 0)
    with np.errstate(invalid="ignore", divide="ignore"):
        rel = np.abs(np.asarray(got["t"], np.float64)[hit] - np.asarray(ref["t"])[hit]) / np.abs(
            np.asarray(ref["t"])[hit])
        db = np.abs(np.asarray(got["bary"], np.float64)[hit] - np.asarray(ref["bary"])[hit])
    rep["max_t_rel"] = float(np.nanmax(rel)) if rel.size else 0.0
    rep["max_bary"] = float(np.nanmax(db)) if db.size else 0.0
    rep["t_bad"] = int((~(rel <= t_rtol)).sum())
    rep["bary_bad"] = int((~(db <= bary_tol)).any(axis=1).sum()) if db.size else 0
    rep["ok"] = bool(rep["frac_identical"] >= min_identical and rep["n_unexplained"] == 0
                     and rep["t_bad"] == 0 and rep["bary_bad"] == 0
                     and rep["gpu_abort_or_invalid"] == 0)
    return rep
