"""Seeded many-mesh workloads: uneven meshes, each with its own surface and its
own batch of primary and ambient-occlusion rays.

* :func:`batch_specs` draws the meshes and ray budgets: grid resolution n
  log-uniform in [n_lo, n_hi] (6 n^3 tets), 1..10 spheres per mesh (centres
  U[0.2, 0.8]^3, radii U[0.08, 0.25]) from a seed of its own, and a ray count
  log-uniform in [rays_lo, rays_hi] of which half are primary rays of a
  pinhole camera at a uniform interior point, looking roughly at one of the
  spheres, and half ambient-occlusion rays from their hits.
* :func:`camera_rays` builds the primary half; :func:`ao_from_hits` the other
  half from hit records that the caller supplies (this module traces nothing).
"""
from __future__ import annotations

import math

import numpy as np

from .kuhn import kuhn_mesh, random_spheres
from .rays import ao_rays, pinhole_rays, tri_geometry


def batch_specs(count: int = 64, seed: int = 10, n_lo: int = 8, n_hi: int = 96,
                rays_lo: int = 1_000, rays_hi: int = 1_000_000, r_lo: float = 0.08,
                r_hi: float = 0.25):
    """Per-mesh recipe dicts: ``n``, ``mesh_seed``, ``spheres``, ``rays``, ``eye``,
    ``forward``, ``up``, ``ao_seed``.  Sphere radii are U[r_lo, r_hi] (large
    enough that the coarsest grids still hold cells inside a sphere)."""
    rng = np.random.default_rng(seed)
    specs = []
    for k in range(count):
        n = int(round(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
        n_sph = int(rng.integers(1, 11))
        rays = int(round(math.exp(rng.uniform(math.log(rays_lo), math.log(rays_hi)))))
        spheres = random_spheres(n_sph, seed=seed * 1000 + 500 + k, centre_lo=0.2, centre_hi=0.8,
                                 r_lo=r_lo, r_hi=r_hi)
        eye = rng.uniform(0.05, 0.95, size=3)
        # look at a random sphere's centre, give or take
        aim = spheres[rng.integers(0, n_sph), :3] - eye
        fwd = aim / max(np.linalg.norm(aim), 1e-9) + rng.normal(scale=0.3, size=3)
        fwd /= np.linalg.norm(fwd)
        up = np.array([0.0, 1.0, 0.0]) if abs(fwd[1]) < 0.9 else np.array([1.0, 0.0, 0.0])
        specs.append(dict(n=n, mesh_seed=seed * 1000 + k, spheres=spheres, rays=rays, eye=eye,
                          forward=fwd, up=up, ao_seed=seed * 1000 + 700 + k))
    return specs


def spec_mesh(spec):
    return kuhn_mesh(spec["n"], jitter=0.1, seed=spec["mesh_seed"], spheres=spec["spheres"])


def camera_rays(spec, count=None):
    """The primary half of a spec's rays: a square image of at least ``count``
    pixels (default half the budget), truncated to ``count`` rays in tile order."""
    count = (spec["rays"] + 1) // 2 if count is None else count
    side = max(1, int(math.ceil(math.sqrt(count))))
    o, d, _ = pinhole_rays(spec["eye"], side, side, 60.0, forward=spec["forward"], up=spec["up"])
    return np.ascontiguousarray(o[:count]), np.ascontiguousarray(d[:count])


def ao_from_hits(points, tri_vertices, orig, dirs, tri, t, count, seed, tmax=0.1):
    """``count`` ambient-occlusion rays from the hits among (orig, dirs, tri, t):
    8 per hit, the first ``count`` of them.  ``tri_vertices(ids)`` maps triangle
    ids to vertex-id triples.  Returns ``(orig, dir, tmax, start_face)``; empty
    arrays when nothing was hit."""
    hit = tri >= 0
    if count <= 0 or not hit.any():
        z3 = np.zeros((0, 3), np.float32)
        return z3, z3.copy(), np.zeros(0, np.float32), np.zeros(0, np.int32)
    o = orig[hit].astype(np.float64)
    d = dirs[hit].astype(np.float64)
    hp = o + t[hit, None].astype(np.float64) * d
    nrm, _ = tri_geometry(points, tri_vertices(tri[hit]))
    k = max(1, min(8, int(math.ceil(count / hit.sum()))))
    ao, ad, atm, parent = ao_rays(hp, nrm, d, k=k, seed=seed, tmax=tmax)
    sf = tri[hit][parent].astype(np.int32)
    return ao[:count], ad[:count], atm[:count], sf[:count]
