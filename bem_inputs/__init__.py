"""Seeded synthetic inputs shared by the product's tests/benchmark and the
oracle: triangle meshes and random index samples.  Holds none of the
method's arithmetic (no kernels, quadrature, trees or approximation).

Meshes (all closed, conforming, counter-clockwise seen from outside):

* ``octahedron_sphere(n)`` -- the unit sphere of Sec. 4: every face of the
  double pyramid |x|_1 = 1 is regularly subdivided into n^2 triangles and the
  vertices are projected onto |x|_2 = 1.  nt = 8 n^2, nv = 4 n^2 + 2.
* ``cube_surface(m)`` -- the surface of [-1,1]^3, each face cut into four
  triangles about its centre and each of those refined m x m (nt = 24 m^2).
* ``perturbed_sphere(seed)`` -- a radially perturbed octahedron sphere with
  radius 1 + a p(x), a ~ U[0, 0.2], p a seeded random polynomial of degree <= 4
  in the unit direction (the span of spherical harmonics of degree <= 4),
  scaled to max |p| = 1, and a log-uniform size in [512, 8192] triangles.
"""
from .meshes import (Mesh, cube_surface, octahedron_sphere, perturbed_sphere,
                     perturbed_sphere_batch)
from .samples import sample_pairs, sample_subset

__all__ = ["Mesh", "octahedron_sphere", "cube_surface", "perturbed_sphere",
           "perturbed_sphere_batch", "sample_pairs", "sample_subset"]
