"""Parity check of traversal results against the oracle (TEST INFRASTRUCTURE ONLY).

Acceptance, per ray set:
  * identical triangle id (or the same miss/abort code) for >= 99.99% of rays;
  * every other ray is explained, by one of:
      - the oracle hit triangle R, and its FP64 hit point lies within ``edge_tol``
        (relative to the scene extent) of an edge or vertex of R or of the
        compared triangle G; G, if any, is not nearer along the ray than R (to
        ``t_rtol``) -- the ray meets an edge where several ids are correct, or
        grazes R's edge and goes on to G;
      - G is nearer than R (or the oracle misses), and the point where the ray
        meets G's plane lies within ``edge_tol`` of an edge or vertex of G -- the
        ray grazes G's edge, which the oracle passed;
      - a hit/miss disagreement whose hit has t within ``tmax_rtol`` of tmax;
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
            t_rtol=1e-5, bary_tol=1e-4, tmax_rtol=1e-6, min_identical=0.9999, t_atol=0.0):
    """Compare ``got`` (numpy dict: tri, t, bary) with oracle results ``ref``.
    Returns a report dict with ``ok`` and the details.  ``t_atol`` (scalar or per
    ray, default 0): an absolute allowance added to ``t_rtol * |t|`` on matched
    hits, for rays that are compared with the oracle's on slightly different
    inputs (secondary rays rebuilt from hits of other precision)."""
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
        rtv = np.asarray(ref["t"], np.float64)[mism]
        gtv = np.asarray(got["t"], np.float64)[mism]
        with np.errstate(invalid="ignore"):
            # the compared hit is nearer along the ray than the oracle's (or the oracle misses)
            g_nearer = g_hit & (~r_hit | (gtv < rtv * (1.0 - t_rtol)))
        if r_hit.any():
            # the oracle's FP64 hit point on an edge of its own triangle or of G
            idx = np.nonzero(r_hit & ~g_nearer)[0]
            if idx.size:
                e = _edge_distance(P, tri_verts, rt[mism][idx], ref_h[idx]) <= tol
                gi = g_hit[idx]
                if gi.any():
                    both = idx[gi]
                    e[gi] |= _edge_distance(P, tri_verts, gt[mism][both], ref_h[both]) <= tol
                near[idx] = e
        if g_nearer.any():
            # the ray grazes an edge of G, which the oracle passed
            idx = np.nonzero(g_nearer)[0]
            gh = _plane_point(P, tri_verts, gt[mism][idx], mo[idx], md[idx])
            near[idx] = _edge_distance(P, tri_verts, gt[mism][idx], gh) <= tol
        if g_hit.any():
            # whatever the case, G itself lies on the ray (its line passes within tol of
            # G's closed triangle) at the reported t
            idx = np.nonzero(g_hit)[0]
            gap = ray_triangle_gap(P, tri_verts, gt[mism][idx], mo[idx], md[idx])
            tv = np.asarray(tri_verts)[gt[mism][idx]]
            A, B, Cc = P[tv[:, 0]], P[tv[:, 1]], P[tv[:, 2]]
            nrm = np.cross(B - A, Cc - A)
            with np.errstate(invalid="ignore", divide="ignore"):
                tpl = np.einsum("ij,ij->i", nrm, A - mo[idx]) / np.einsum("ij,ij->i", nrm, md[idx])
                on_ray = (gap <= tol) & (np.abs(gtv[idx] - tpl) <= t_rtol * np.abs(tpl) + tol)
            near[idx] &= on_ray
        # hit/miss at tmax
        tm_m = tm[mism]
        with np.errstate(invalid="ignore"):
            fin = np.isfinite(tm_m)
            rtm = r_hit & ~g_hit & fin & (np.abs(rtv - tm_m) <= tmax_rtol * tm_m)
            gtm = g_hit & ~r_hit & fin & (np.abs(gtv - tm_m) <= tmax_rtol * tm_m)
            # a reported hit never lies beyond tmax
            near &= ~(g_hit & (gtv > tm_m * (1.0 + tmax_rtol)))
        explained = (near | rtm | gtm) & ~bad_code[mism]
    rep["mismatches"] = int(mism.size)
    rep["unexplained"] = mism[~explained].tolist()[:50]
    rep["n_unexplained"] = int((~explained).sum())
    hit = same & (rt >= 0)
    atol = np.broadcast_to(np.asarray(t_atol, np.float64), (n,))[hit]
    with np.errstate(invalid="ignore", divide="ignore"):
        rel = np.maximum(np.abs(np.asarray(got["t"], np.float64)[hit] - np.asarray(ref["t"])[hit]) - atol,
                         0.0) / np.abs(np.asarray(ref["t"])[hit])
        db = np.abs(np.asarray(got["bary"], np.float64)[hit] - np.asarray(ref["bary"])[hit])
    rep["max_t_rel"] = float(np.nanmax(rel)) if rel.size else 0.0
    rep["max_bary"] = float(np.nanmax(db)) if db.size else 0.0
    rep["t_bad"] = int((~(rel <= t_rtol)).sum())
    rep["bary_bad"] = int((~(db <= bary_tol)).any(axis=1).sum()) if db.size else 0
    rep["ok"] = bool(rep["frac_identical"] >= min_identical and rep["n_unexplained"] == 0
                     and rep["t_bad"] == 0 and rep["bary_bad"] == 0
                     and rep["gpu_abort_or_invalid"] == 0)
    return rep
