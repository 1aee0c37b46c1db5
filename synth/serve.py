"""Host-side rays of a served request, for checking served results.

A served request renders one image: a camera ray per pixel in 8x8-tile order,
and for shadow and ambient-occlusion requests one more ray per pixel from the
camera ray's hit (the hit records are supplied by the caller; nothing here
traces a ray).  This restates the request's ray definitions in float64 numpy:

* camera ray: :func:`synth.rays.pinhole_rays` (pixel centres, horizontal field
  of view, row 0 at the top, 8x8 tiles);
* shadow ray: from the hit point P towards the light L, direction L - P, tmax 1
  (the light sits at t = 1), start face = the hit triangle;
* AO ray: one cosine-weighted direction about the hit triangle's normal, on the
  side the camera ray came from (Malley's method: a uniform disk point lifted to
  the hemisphere; tangent frame from the axis least aligned with the normal),
  tmax = ``ao_tmax``, start face = the hit triangle.  Its two uniform numbers
  for ray i come from the counter-based PCG hash (Jarzynski and Olano, "Hash
  Functions for GPU Rendering", JCGT 9(3), 2020) as
  ``pcg(seed ^ pcg(2 i))`` and ``pcg(seed ^ pcg(2 i + 1))``, top 24 bits / 2^24;
* a pixel whose camera ray hit nothing gets a zero direction (an invalid ray).
"""
from __future__ import annotations

import numpy as np

from .rays import pinhole_rays, _tangent_frame

_M32 = np.uint64(0xFFFFFFFF)


def pcg_hash(v):
    """The PCG hash of uint32 values (array in, uint32 array out)."""
    v = np.asarray(v, dtype=np.uint64) & _M32
    state = (v * np.uint64(747796405) + np.uint64(2891336453)) & _M32
    shift = (state >> np.uint64(28)) + np.uint64(4)
    word = (((state >> shift) ^ state) * np.uint64(277803737)) & _M32
    return ((word >> np.uint64(22)) ^ word).astype(np.uint32)


def unit_floats(h):
    """Uniform numbers in [0, 1) from 32-bit hashes: the top 24 bits / 2^24."""
    return (np.asarray(h, np.uint32) >> np.uint32(8)).astype(np.float64) / 16777216.0


def camera_rays(req):
    o, d, _ = pinhole_rays(req["eye"], req["width"], req["height"], req["fov_h_deg"],
                           forward=req["forward"], up=req["up"], tile=8)
    return o, d


def secondary_rays(req, points, tri_verts, orig, dirs, tri, t):
    """The shadow or AO ray of every pixel from the camera rays (orig, dirs) and
    their hits (tri, t); ``tri_verts`` maps a triangle id to its vertex ids in
    ascending order.  Returns float32 origins and directions, float32 tmax and
    int32 start faces."""
    n = orig.shape[0]
    o = np.asarray(orig, np.float64)
    d = np.asarray(dirs, np.float64)
    hit = np.asarray(tri) >= 0
    h = o + np.where(hit, np.asarray(t, np.float64), 0.0)[:, None] * d
    nd = np.zeros((n, 3))
    tmax = np.zeros(n)
    sf = np.where(hit, tri, -1).astype(np.int32)
    if req["kind"] == "shadow":
        nd[hit] = np.asarray(req["light"], np.float64)[None, :] - h[hit]
        tmax[hit] = 1.0
    else:
        P = np.asarray(points, np.float64)
        tv = np.asarray(tri_verts)[np.asarray(tri)[hit]]
        A, B, C = P[tv[:, 0]], P[tv[:, 1]], P[tv[:, 2]]
        nrm = np.cross(B - A, C - A)
        nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
        nrm[np.einsum("ij,ij->i", nrm, d[hit]) > 0.0] *= -1.0
        t1, t2 = _tangent_frame(nrm)
        i = np.nonzero(hit)[0].astype(np.uint64)
        seed = np.uint64(int(req["seed"]) & 0xFFFFFFFF)
        u1 = unit_floats(pcg_hash(seed ^ pcg_hash(np.uint64(2) * i).astype(np.uint64)))
        u2 = unit_floats(pcg_hash(seed ^ pcg_hash(np.uint64(2) * i + np.uint64(1)).astype(np.uint64)))
        rad, phi = np.sqrt(u1), 2.0 * np.pi * u2
        nd[hit] = ((rad * np.cos(phi))[:, None] * t1 + (rad * np.sin(phi))[:, None] * t2
                   + np.sqrt(np.maximum(0.0, 1.0 - u1))[:, None] * nrm)
        tmax[hit] = float(np.float32(req["ao_tmax"]))
    orig1 = np.where(hit[:, None], h, o)
    return (orig1.astype(np.float32), nd.astype(np.float32), tmax.astype(np.float32), sf)
