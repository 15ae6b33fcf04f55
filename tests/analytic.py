"""Independent closed forms and brute-force integrators used to pin the
oracle.  None of this calls the oracle's quadrature; it follows classical
formulas of potential theory:

* ``self_integral`` -- the closed form of int_T int_T 1/|x - y| over a flat
  triangle with sides a, b, c and area A:
      (4 A^2 / 3) [F(a,b,c) + F(b,c,a) + F(c,a,b)],
      F(a,b,c) = ln(((a + b)^2 - c^2) / (b^2 - (a - c)^2)) / a,
  which gives (3/4) s^3 ln 3 for the equilateral triangle of side s.
* ``triangle_potential`` -- int_T 1/|x - y| dy at any point x, the
  edge-by-edge formula of Wilton et al. (1984) / Graglia (1993).
* ``solid_angle`` -- the signed solid angle of a triangle seen from x
  (Van Oosterom & Strackee 1983); int_T d/dn(y) 1/|x - y| dy = -Omega(x)
  for the counter-clockwise (outward) normal.
* ``duffy_points`` -- a plain Duffy/Gauss rule on a triangle, optionally
  graded towards the collapsed vertex and towards the edge t = 0, for the
  outer integral of the brute-force pins.
"""
import numpy as np


def self_integral(p0, p1, p2):
    p0, p1, p2 = (np.asarray(p, dtype=float) for p in (p0, p1, p2))
    a = np.linalg.norm(p1 - p2)
    b = np.linalg.norm(p2 - p0)
    c = np.linalg.norm(p0 - p1)
    A = 0.5 * np.linalg.norm(np.cross(p1 - p0, p2 - p0))

    def F(a, b, c):
        return np.log(((a + b) ** 2 - c ** 2) / (b ** 2 - (a - c) ** 2)) / a

    return 4.0 * A * A / 3.0 * (F(a, b, c) + F(b, c, a) + F(c, a, b))


def triangle_potential(x, p):
    """int_T 1/|x - y| dy for points x (k,3) and triangle p (3,3)."""
    x = np.atleast_2d(np.asarray(x, dtype=float))
    p = np.asarray(p, dtype=float)
    n = np.cross(p[1] - p[0], p[2] - p[0])
    n /= np.linalg.norm(n)
    h = (x - p[0]) @ n                       # signed height
    rho = x - h[:, None] * n[None, :]        # projection onto the plane
    total = np.zeros(x.shape[0])
    for k in range(3):
        pm, pp = p[k], p[(k + 1) % 3]
        l = (pp - pm) / np.linalg.norm(pp - pm)
        u = np.cross(l, n)                   # outward in-plane edge normal
        t0 = (pm - rho) @ u
        sm = (pm - rho) @ l
        sp = (pp - rho) @ l
        Rm = np.linalg.norm(x - pm, axis=1)
        Rp = np.linalg.norm(x - pp, axis=1)
        R0sq = t0 ** 2 + h ** 2
        f = np.log((Rp + sp) / (Rm + sm))
        ah = np.abs(h)
        beta = (np.arctan2(t0 * sp, R0sq + ah * Rp) - np.arctan2(t0 * sm, R0sq + ah * Rm))
        total += t0 * f - ah * beta
    return total


def solid_angle(x, p):
    """Signed solid angle (Van Oosterom-Strackee) of triangle p from x (k,3)."""
    x = np.atleast_2d(np.asarray(x, dtype=float))
    a = p[0][None, :] - x
    b = p[1][None, :] - x
    c = p[2][None, :] - x
    la, lb, lc = (np.linalg.norm(q, axis=1) for q in (a, b, c))
    num = np.einsum("ij,ij->i", a, np.cross(b, c))
    den = (la * lb * lc + np.einsum("ij,ij->i", a, b) * lc
           + np.einsum("ij,ij->i", a, c) * lb + np.einsum("ij,ij->i", b, c) * la)
    return 2.0 * np.arctan2(num, den)


def gauss_legendre01(q):
    """numpy's Gauss-Legendre rule mapped to [0,1] (independent of the oracle)."""
    z, w = np.polynomial.legendre.leggauss(q)
    return 0.5 * (z + 1.0), 0.5 * w


def duffy_points(p, q, grade_vertex=1, grade_edge=1, composite=1):
    """Points (k,3) and weights (k,) integrating over triangle p, collapsing at
    p[0]: y = p0 + s (p1 - p0) + s t (p2 - p1).  ``grade_*`` substitutes
    s = u^g / t = v^g to cluster points near p[0] / the edge p0-p1;
    ``composite`` splits [0,1] in each variable into that many panels."""
    p = np.asarray(p, dtype=float)
    g, w = gauss_legendre01(q)
    edges = np.linspace(0.0, 1.0, composite + 1)
    u = np.concatenate([edges[k] + (edges[k + 1] - edges[k]) * g for k in range(composite)])
    wu = np.concatenate([(edges[k + 1] - edges[k]) * w for k in range(composite)])
    U, V = np.meshgrid(u, u, indexing="ij")
    WU, WV = np.meshgrid(wu, wu, indexing="ij")
    s = U ** grade_vertex
    ds = grade_vertex * U ** (grade_vertex - 1)
    t = V ** grade_edge
    dt = grade_edge * V ** (grade_edge - 1)
    sqrt_g = np.linalg.norm(np.cross(p[1] - p[0], p[2] - p[1]))
    pts = (p[0][None, :] + s.ravel()[:, None] * (p[1] - p[0])[None, :]
           + (s * t).ravel()[:, None] * (p[2] - p[1])[None, :])
    wts = (WU * WV * ds * dt * s).ravel() * sqrt_g
    return pts, wts
