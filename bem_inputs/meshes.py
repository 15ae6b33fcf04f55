"""Synthetic triangle meshes (see the package docstring)."""
from dataclasses import dataclass

import numpy as np


@dataclass
class Mesh:
    v: np.ndarray    # (nv, 3) float64 vertex coordinates
    tri: np.ndarray  # (nt, 3) int32 vertex ids, counter-clockwise from outside
    name: str = ""

    @property
    def nv(self):
        return self.v.shape[0]

    @property
    def nt(self):
        return self.tri.shape[0]


def _subdivide(corners, n, lattice_scale):
    """Regular n x n subdivision of the triangle with integer-lattice corners
    (3, 3) (coordinates times ``lattice_scale``).  Returns integer lattice
    points (k, 3) and local triangles (n^2, 3) oriented like the corners."""
    A, B, C = (np.asarray(c, dtype=np.int64) for c in corners)
    idx = {}
    pts = []

    def pid(i, j):
        key = (i, j)
        if key not in idx:
            idx[key] = len(pts)
            pts.append((n - i - j) * A + i * B + j * C)
        return idx[key]

    tris = []
    for i in range(n):
        for j in range(n - i):
            tris.append((pid(i, j), pid(i + 1, j), pid(i, j + 1)))
            if i + j <= n - 2:
                tris.append((pid(i + 1, j), pid(i + 1, j + 1), pid(i, j + 1)))
    return np.array(pts, dtype=np.int64), np.array(tris, dtype=np.int64)


def _merge(faces):
    """Merge per-face (lattice points, triangles) by exact lattice coordinate."""
    gid = {}
    verts = []
    tris = []
    for pts, ftri in faces:
        local = np.empty(len(pts), dtype=np.int64)
        for k, p in enumerate(map(tuple, pts)):
            if p not in gid:
                gid[p] = len(verts)
                verts.append(p)
            local[k] = gid[p]
        tris.append(local[ftri])
    return np.array(verts, dtype=np.float64), np.concatenate(tris).astype(np.int32)


def octahedron_sphere(n: int) -> Mesh:
    """Unit sphere from the n-fold regular subdivision of the octahedron."""
    if n < 1:
        raise ValueError("n >= 1")
    faces = []
    for sx in (1, -1):
        for sy in (1, -1):
            for sz in (1, -1):
                A = (sx, 0, 0)
                B = (0, sy, 0)
                C = (0, 0, sz)
                if sx * sy * sz < 0:  # keep the face counter-clockwise from outside
                    B, C = C, B
                faces.append(_subdivide((A, B, C), n, n))
    v, tri = _merge(faces)
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    return Mesh(v, tri, f"octahedron_sphere(n={n})")


def cube_surface(m: int) -> Mesh:
    """Surface of [-1,1]^3: each face cut into four triangles about its centre,
    each refined m x m; nt = 24 m^2 (m = 32 gives 24576)."""
    faces = []
    for axis in range(3):
        for s in (1, -1):
            c = np.zeros(3, dtype=np.int64)
            c[axis] = s
            u = np.zeros(3, dtype=np.int64)
            w = np.zeros(3, dtype=np.int64)
            u[(axis + 1) % 3] = 1
            w[(axis + 2) % 3] = 1
            # corners counter-clockwise seen from outside (normal s * e_axis)
            quad = [c + u + w, c - u + w, c - u - w, c + u - w]
            if s < 0:
                quad = quad[::-1]
            for k in range(4):
                faces.append(_subdivide((c, quad[k], quad[(k + 1) % 4]), m, m))
    v, tri = _merge(faces)
    v /= m
    return Mesh(v, tri, f"cube_surface(m={m})")


def _poly_features(d):
    """Monomials x^a y^b z^c, 1 <= a+b+c <= 4, of unit directions d (k,3)."""
    cols = []
    for a in range(5):
        for b in range(5 - a):
            for c in range(5 - a - b):
                if 1 <= a + b + c <= 4:
                    cols.append(d[:, 0] ** a * d[:, 1] ** b * d[:, 2] ** c)
    return np.stack(cols, axis=1)


def perturbed_sphere(seed: int, n_min: int = 8, n_max: int = 32) -> Mesh:
    """Radially perturbed octahedron sphere, seeded (PCG64 seed = ``seed``).

    Size: N log-uniform in [8 n_min^2, 8 n_max^2], n = round(sqrt(N/8)).
    Radius: 1 + a p(x^), a ~ U[0, 0.2], p random polynomial of degree 1..4 in
    the unit direction x^, scaled so that max |p| over the vertices is 1.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    N = np.exp(rng.uniform(np.log(8 * n_min ** 2), np.log(8 * n_max ** 2)))
    n = int(np.clip(round(np.sqrt(N / 8.0)), n_min, n_max))
    a = rng.uniform(0.0, 0.2)
    base = octahedron_sphere(n)
    F = _poly_features(base.v)
    coef = rng.standard_normal(F.shape[1])
    p = F @ coef
    p /= np.max(np.abs(p))
    v = base.v * (1.0 + a * p)[:, None]
    return Mesh(v, base.tri, f"perturbed_sphere(seed={seed}, n={n}, a={a:.4f})")


def perturbed_sphere_batch(count: int = 64, first_seed: int = 0):
    return [perturbed_sphere(first_seed + k) for k in range(count)]
