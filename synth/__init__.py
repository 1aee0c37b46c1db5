"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This package only builds inputs: Kuhn-grid tetrahedral meshes with sphere-union
surfaces (``kuhn``) and ray sets (``rays``).  It holds none of the traversal
arithmetic; both the CPU oracle and the HIP path consume what it produces.
"""
from .kuhn import KuhnMesh, kuhn_mesh, sphere_union, random_spheres, config_mesh
from .rays import (pinhole_rays, ao_rays, precision_rays, random_interior_rays,
                   tri_geometry)

__all__ = ["KuhnMesh", "kuhn_mesh", "sphere_union", "random_spheres", "config_mesh",
           "pinhole_rays", "ao_rays", "precision_rays", "random_interior_rays",
           "tri_geometry"]
