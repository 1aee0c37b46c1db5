"""Kuhn-grid constrained tetrahedral meshes (seeded, vectorised).

The paper evaluates on TetGen/TetWild tetrahedralisations of public scenes;
those meshes are not available here, so every workload is a synthetic stand-in
with the same structure the traversal sees: points + tets + per-face neighbour
links + per-face "constrained" flags (the scene triangles are a subset of the
tet faces, as in a constrained tetrahedralisation, paper Sec. "Tetrahedral Mesh
Representation").

Construction
------------
* vertices ``(i, j, k) / n`` for ``0 <= i, j, k <= n``; point id
  ``(i*(n+1) + j)*(n+1) + k``.  Interior vertices (``0 < i, j, k < n``) are
  jittered per coordinate by ``U(-jitter, jitter) / n`` (numpy PCG64, seeded).
* cell ``c = (ci, cj, ck)`` is split into the 6 Kuhn (Freudenthal) tets, one per
  axis permutation ``pi``: ``(c, c+e[pi0], c+e[pi0]+e[pi1], c+(1,1,1))``; tet id
  ``cell*6 + perm``.  Odd permutations get vertex slots 2 and 3 swapped so every
  tet has positive orientation.
* ``nbrs[t][j]`` is the tet across the face opposite vertex slot ``j`` (-1 on the
  cube boundary); these are derived from the grid structure, and a face-hashing
  check in the tests confirms them.
* ``cflag[t][j] = 1`` when that face separates a cell whose (unjittered) centre
  lies inside the sphere union from one that lies outside.  Cube-boundary faces
  are never constrained, so rays that leave the cube miss.
"""
from __future__ import annotations

import dataclasses
import numpy as np

# axis permutations, in a fixed order (perm index = position in this list)
PERMS = [(0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)]
_PERM_INDEX = {p: i for i, p in enumerate(PERMS)}
_PERM_ODD = np.array([0, 1, 1, 0, 0, 1], dtype=bool)


@dataclasses.dataclass
class KuhnMesh:
    n: int
    points: np.ndarray        # float32 [P, 3]
    tets: np.ndarray          # int32 [T, 4] vertex ids
    nbrs: np.ndarray          # int32 [T, 4] tet across the face opposite slot j, -1 = boundary
    cflag: np.ndarray         # uint8 [T, 4] 1 = that face is scene geometry
    inside: np.ndarray        # bool [n, n, n] cell classification
    spheres: np.ndarray       # float64 [S, 4] (cx, cy, cz, r)
    jitter: float
    seed: int

    @property
    def n_points(self) -> int:
        return int(self.points.shape[0])

    @property
    def n_tets(self) -> int:
        return int(self.tets.shape[0])

    def n_constrained_faces(self) -> int:
        """Number of distinct constrained triangles (each is flagged on both sides)."""
        c = self.cflag.astype(np.int64)
        interior = self.nbrs >= 0
        # a flagged face with two tets is counted twice, one on the boundary once
        return int((c * interior).sum() // 2 + (c * ~interior).sum())


def sphere_union(spheres):
    """Return an ``inside(x, y, z)`` predicate for a union of spheres (cx, cy, cz, r)."""
    sph = np.asarray(spheres, dtype=np.float64).reshape(-1, 4)

    def inside(x, y, z):
        res = np.zeros(np.broadcast(x, y, z).shape, dtype=bool)
        for cx, cy, cz, r in sph:
            res |= (x - cx) ** 2 + (y - cy) ** 2 + (z - cz) ** 2 < r * r
        return res

    return inside


def random_spheres(count, seed, centre_lo=0.15, centre_hi=0.85, r_lo=0.03, r_hi=0.12):
    """``count`` spheres with centres U[lo, hi]^3 and radii U[r_lo, r_hi]."""
    rng = np.random.default_rng(seed)
    c = rng.uniform(centre_lo, centre_hi, size=(count, 3))
    r = rng.uniform(r_lo, r_hi, size=(count, 1))
    return np.concatenate([c, r], axis=1)


def kuhn_mesh(n: int, jitter: float = 0.1, seed: int = 0, spheres=None) -> KuhnMesh:
    """Build the Kuhn-grid mesh of the unit cube at resolution ``n``.

    ``spheres``: array-like [S, 4]; default is one sphere of radius 0.35 at the
    cube centre.  ``jitter`` is in cell units (0.1 = +-0.1 cell).
    """
    if n < 1:
        raise ValueError("n must be >= 1")
    if spheres is None:
        spheres = [[0.5, 0.5, 0.5, 0.35]]
    spheres = np.asarray(spheres, dtype=np.float64).reshape(-1, 4)
    n1 = n + 1

    # ---- points -------------------------------------------------------------
    g = np.arange(n1, dtype=np.int64)
    I, J, K = np.meshgrid(g, g, g, indexing="ij")
    I, J, K = I.ravel(), J.ravel(), K.ravel()
    pts = np.stack([I, J, K], axis=1).astype(np.float64) / n
    if jitter > 0.0:
        rng = np.random.default_rng(seed)
        jit = rng.uniform(-jitter, jitter, size=pts.shape) / n
        interior = (I > 0) & (I < n) & (J > 0) & (J < n) & (K > 0) & (K < n)
        pts[interior] += jit[interior]
    points = pts.astype(np.float32)

    # ---- cells ----------------------------------------------------------------
    c = np.arange(n, dtype=np.int64)
    CI, CJ, CK = np.meshgrid(c, c, c, indexing="ij")
    CI, CJ, CK = CI.ravel(), CJ.ravel(), CK.ravel()
    ncell = n ** 3
    cell = np.arange(ncell, dtype=np.int64)
    cc = np.stack([CI, CJ, CK], axis=1)

    ctr = (cc.astype(np.float64) + 0.5) / n
    inside_cells = sphere_union(spheres)(ctr[:, 0], ctr[:, 1], ctr[:, 2])

    def pid(a):  # [m, 3] integer grid coords -> point ids
        return (a[:, 0] * n1 + a[:, 1]) * n1 + a[:, 2]

    def cell_id(a):
        return (a[:, 0] * n + a[:, 1]) * n + a[:, 2]

    T = 6 * ncell
    tets = np.empty((T, 4), dtype=np.int32)
    nbrs = np.empty((T, 4), dtype=np.int32)
    cflag = np.zeros((T, 4), dtype=np.uint8)
    eye = np.eye(3, dtype=np.int64)
    ones = np.ones(3, dtype=np.int64)

    for m, p in enumerate(PERMS):
        e0, e1, e2 = eye[p[0]], eye[p[1]], eye[p[2]]
        v = [pid(cc), pid(cc + e0), pid(cc + e0 + e1), pid(cc + ones)]
        tid = cell * 6 + m
        nb = np.empty((ncell, 4), dtype=np.int64)
        cf = np.zeros((ncell, 4), dtype=np.uint8)
        # slot 0: face (v1, v2, v3) lies on the cell face x[pi0] = c[pi0] + 1
        other = cc + e0
        ok = other[:, p[0]] < n
        oc = cell_id(np.where(ok[:, None], other, 0))
        nb[:, 0] = np.where(ok, oc * 6 + _PERM_INDEX[(p[1], p[2], p[0])], -1)
        cf[:, 0] = (ok & (inside_cells != inside_cells[oc])).astype(np.uint8)
        # slot 3: face (v0, v1, v2) lies on the cell face x[pi2] = c[pi2]
        other = cc - e2
        ok = other[:, p[2]] >= 0
        oc = cell_id(np.where(ok[:, None], other, 0))
        nb[:, 3] = np.where(ok, oc * 6 + _PERM_INDEX[(p[2], p[0], p[1])], -1)
        cf[:, 3] = (ok & (inside_cells != inside_cells[oc])).astype(np.uint8)
        # slots 1 and 2: faces inside the cell, shared with the permutations that
        # swap (pi0, pi1) and (pi1, pi2) respectively
        nb[:, 1] = cell * 6 + _PERM_INDEX[(p[1], p[0], p[2])]
        nb[:, 2] = cell * 6 + _PERM_INDEX[(p[0], p[2], p[1])]
        order = [0, 1, 3, 2] if _PERM_ODD[m] else [0, 1, 2, 3]
        tets[tid] = np.stack([v[s] for s in order], axis=1)
        nbrs[tid] = nb[:, order]
        cflag[tid] = cf[:, order]

    mesh = KuhnMesh(n=n, points=points, tets=tets, nbrs=nbrs, cflag=cflag,
                    inside=inside_cells.reshape(n, n, n), spheres=spheres,
                    jitter=float(jitter), seed=int(seed))
    vol = tet_volumes6(mesh.points, mesh.tets)
    if not np.all(vol > 0):
        raise RuntimeError("jitter produced a non-positive tet volume; lower the jitter")
    return mesh


def tet_volumes6(points, tets, chunk=1 << 21):
    """Six times the signed volume of every tet, in float64 (input check only)."""
    out = np.empty(tets.shape[0], dtype=np.float64)
    P = points.astype(np.float64)
    for s in range(0, tets.shape[0], chunk):
        t = tets[s:s + chunk]
        a = P[t[:, 0]]
        b, c, d = P[t[:, 1]] - a, P[t[:, 2]] - a, P[t[:, 3]] - a
        out[s:s + chunk] = np.einsum("ij,ij->i", b, np.cross(c, d))
    return out


# ---- the workloads --------------------------------------------------------------

def config_mesh(name: str) -> KuhnMesh:
    """Meshes of the named workloads.

    * ``tiny``: n = 16 (24,576 tets), jitter 0.1 cell seed 0, one sphere r = 0.35
      at the cube centre.
    * ``paper``: n = 128 (12,582,912 tets), jitter 0.1 cell seed 1, union of 20
      spheres (centres U[0.15, 0.85]^3, radii U[0.03, 0.12], seed 2).
    * ``paper160``: the same scene on a finer grid, n = 160 (24,576,000 tets, whose
      records and points no longer fit the GPU's 256 MB last-level cache).
    """
    if name == "tiny":
        return kuhn_mesh(16, jitter=0.1, seed=0)
    if name == "paper":
        return kuhn_mesh(128, jitter=0.1, seed=1, spheres=random_spheres(20, seed=2))
    if name == "paper160":
        return kuhn_mesh(160, jitter=0.1, seed=1, spheres=random_spheres(20, seed=2))
    raise KeyError(name)
