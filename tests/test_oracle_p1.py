"""Pins of the oracle's piecewise-linear local matrices (Sec. 2.2, eq.
reference_integral with low-order polynomial bases).

* Partition of unity: the nine entries of a pair sum to its
  piecewise-constant entry (same points and weights), every class.
* Disjoint pairs against an independent numpy quadrature (a collapsed
  tensor rule with the collapse at another vertex, barycentric coordinates
  solved from the points), converging together at high order.
* Single-layer symmetry L^{ij} = (L^{ji})^T for disjoint, vertex-adjacent and
  identical pairs (to rounding), edge pairs to quadrature error.
* Mirror symmetries of symmetric configurations (an equilateral triangle, a
  rhombus of two equilateral triangles, two triangles meeting at a vertex
  symmetric under a reflection): equal entries at the exchanged vertices, at
  a high order -- a vertex assigned to the wrong shape function breaks them.
* Gauss's identity for piecewise linears: on a closed polyhedron the double
  layer rows sum to -1/2 int phi_v = -|star(v)| / 6, converging with q.
"""
import numpy as np

import oracle
from bem_inputs import octahedron_sphere


def test_partition_of_unity_all_classes():
    m = octahedron_sphere(4)
    rng = np.random.Generator(np.random.PCG64(1))
    rows = np.concatenate([np.arange(10), rng.integers(0, m.nt, 40)])
    cols = np.concatenate([np.arange(10), rng.integers(0, m.nt, 40)])
    # add edge and vertex neighbours of triangle 0
    t0 = set(m.tri[0])
    for t in range(m.nt):
        c = len(t0 & set(m.tri[t]))
        if c in (1, 2):
            rows = np.append(rows, 0)
            cols = np.append(cols, t)
    for kernel, kappa in ((0, 0.0), (1, 3.0)):
        for layer in (0, 1):
            L = oracle.p1_pairs(m.v, m.tri, rows, cols, kernel=kernel, layer=layer, kappa=kappa)
            P0 = oracle.entries(m.v, m.tri, rows, cols, kernel=kernel, layer=layer, kappa=kappa)
            scale = np.abs(P0).max()
            assert np.abs(L.sum(axis=(1, 2)) - P0).max() <= 1e-14 * scale


def _numpy_p1_disjoint(P, Q, kernel_fn, q):
    """Independent rule: each triangle collapsed at its last vertex,
    x = p2 + u (p0 - p2) + v (1 - u) (p1 - p2), Jacobian 2 A (1 - u); the
    barycentric coordinates are solved from the points."""
    g, w = np.polynomial.legendre.leggauss(q)
    g, w = (g + 1) / 2, w / 2

    def pts(T):
        A = 0.5 * np.linalg.norm(np.cross(T[1] - T[0], T[2] - T[0]))
        U, Vv = np.meshgrid(g, g, indexing="ij")
        W = np.outer(w, w) * 2 * A * (1 - U)
        X = T[2] + U[..., None] * (T[0] - T[2]) + (Vv * (1 - U))[..., None] * (T[1] - T[2])
        M = np.stack([T[0] - T[2], T[1] - T[2]], axis=1)  # 3 x 2
        lam01 = np.linalg.lstsq(M, (X.reshape(-1, 3) - T[2]).T, rcond=None)[0].T
        lam = np.column_stack([lam01, 1 - lam01.sum(axis=1)])
        return X.reshape(-1, 3), W.ravel(), lam

    X, WX, LX = pts(P)
    Y, WY, LY = pts(Q)
    K = kernel_fn(X[:, None, :], Y[None, :, :])
    return np.einsum("a,ak,ab,b,bl->kl", WX, LX, K, WY, LY)


def test_disjoint_pairs_against_independent_rule():
    m = octahedron_sphere(4)
    for i, j in ((0, 70), (3, 100), (17, 44)):
        assert oracle.shared_vertices(m.tri, i, j) == 0
        P, Q = m.v[m.tri[i]], m.v[m.tri[j]]
        nq = np.cross(Q[1] - Q[0], Q[2] - Q[0])
        nq /= np.linalg.norm(nq)

        def slp(x, y):
            return 1.0 / (4 * np.pi * np.linalg.norm(x - y, axis=-1))

        def dlp(x, y):
            d = x - y
            return (d @ nq) / (4 * np.pi * np.linalg.norm(d, axis=-1) ** 3)

        for layer, fn in ((0, slp), (1, dlp)):
            ref = _numpy_p1_disjoint(P, Q, fn, 14)
            got = oracle.p1_pairs(m.v, m.tri, [i], [j], layer=layer, q_reg=12)[0].real
            assert np.abs(got - ref).max() <= 1e-11 * np.abs(ref).max(), (i, j, layer)


def test_single_layer_symmetry():
    m = octahedron_sphere(4)
    t0 = set(m.tri[0])
    vert = next(t for t in range(m.nt) if len(t0 & set(m.tri[t])) == 1)
    edge = next(t for t in range(m.nt) if len(t0 & set(m.tri[t])) == 2)
    for j, tol in ((90, 1e-14), (vert, 1e-14), (0, 1e-14), (edge, 1e-4)):
        a = oracle.p1_pairs(m.v, m.tri, [0], [j])[0]
        b = oracle.p1_pairs(m.v, m.tri, [j], [0])[0]
        assert np.abs(a - b.T).max() <= tol * np.abs(a).max(), (j, tol)


def test_mirror_symmetric_configurations():
    s3 = np.sqrt(3.0)
    # equilateral triangle: every vertex alike
    v = np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [0.5, s3 / 2, 0.0]])
    L = oracle.p1_pairs(v, np.array([[0, 1, 2]]), [0], [0], q_sing=12)[0].real
    d, o = np.diag(L), L[~np.eye(3, dtype=bool)]
    assert np.ptp(d) <= 1e-9 * d.max() and np.ptp(o) <= 1e-9 * o.max()
    assert d.min() > o.max()  # a node's own hat function weighs most
    # rhombus A B C D, triangles (A, B, C) and (B, A, D), shared edge A B;
    # the reflection across C D exchanges A and B and keeps both triangles
    v = np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [0.5, s3 / 2, 0.0], [0.5, -s3 / 2, 0.0]])
    tri = np.array([[0, 1, 2], [1, 0, 3]])
    L = oracle.p1_pairs(v, tri, [0], [1], q_sing=12)[0].real  # rows (A, B, C), cols (B, A, D)
    A_, B_, C_ = 0, 1, 2
    Bc, Ac, Dc = 0, 1, 2
    pairs = [((A_, Ac), (B_, Bc)), ((A_, Bc), (B_, Ac)), ((C_, Ac), (C_, Bc)),
             ((A_, Dc), (B_, Dc))]
    for (k1, l1), (k2, l2) in pairs:
        assert abs(L[k1, l1] - L[k2, l2]) <= 1e-9 * np.abs(L).max(), ((k1, l1), (k2, l2))
    # two triangles meeting at O, symmetric under the reflection y -> -y
    v = np.array([[0.0, 0.0, 0.0], [1.0, 0.4, 0.0], [1.0, -0.4, 0.0],
                  [-1.0, 0.5, 0.3], [-1.0, -0.5, 0.3]])
    tri = np.array([[0, 1, 2], [0, 4, 3]])
    for layer in (0, 1):
        L = oracle.p1_pairs(v, tri, [0], [1], layer=layer, q_sing=12)[0].real  # (O, A1, A2) x (O, B2, B1)
        eq = [((1, 2), (2, 1)), ((1, 1), (2, 2)), ((0, 1), (0, 2)), ((1, 0), (2, 0))]
        for (k1, l1), (k2, l2) in eq:
            assert abs(L[k1, l1] - L[k2, l2]) <= 1e-9 * np.abs(L).max(), (layer, k1, l1)


def test_gauss_identity_piecewise_linear():
    m = octahedron_sphere(2)  # 32 triangles, 18 vertices
    area = 0.5 * np.linalg.norm(np.cross(m.v[m.tri[:, 1]] - m.v[m.tri[:, 0]],
                                         m.v[m.tri[:, 2]] - m.v[m.tri[:, 0]]), axis=1)
    star = np.zeros(m.v.shape[0])
    for t, t3 in enumerate(m.tri):
        star[t3] += area[t]
    verts = np.arange(m.v.shape[0])
    devs = []
    for q in (3, 4, 5):
        K = oracle.p1_block(m.v, m.tri, verts, verts, layer=1, q_reg=q, q_sing=q).real
        devs.append(np.abs(K.sum(axis=1) + star / 6).max() / (star.max() / 6))
    assert devs[-1] <= 1e-3 and devs[2] < devs[1] < devs[0], devs
