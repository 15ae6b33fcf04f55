"""Pins of the FP64 oracle against what the mathematics fixes.

Each test ties a part of the oracle to something other than itself:
exactness of the 1-D and triangle rules, polynomial reproduction by every
Sauter-Schwab region set, the closed-form self-integral, semi-analytic brute
force (triangle potential, solid angle), the Gauss identity for the double
layer, Helmholtz at kappa = 0, the smooth imaginary part of the Helmholtz
kernel, symmetry, and the single-layer potential of the unit sphere.
"""
import math

import numpy as np
import pytest

import analytic as an
import oracle
from bem_inputs import cube_surface, octahedron_sphere


def areas(v, tri):
    p = v[tri]
    return 0.5 * np.linalg.norm(np.cross(p[:, 1] - p[:, 0], p[:, 2] - p[:, 0]), axis=1)


def full_matrix(m, **op):
    n = m.nt
    R, C = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    return oracle.entries(m.v, m.tri, R.ravel(), C.ravel(), **op).reshape(n, n)


# ---------------------------------------------------------------- base rules
@pytest.mark.parametrize("q", [1, 2, 3, 4, 5, 6, 8, 12, 16, 24])
def test_gauss_legendre_exact_to_degree_2q_minus_1(q):
    x, w = oracle.gauss01(q)
    assert np.all(np.diff(x) > 0) and np.all(w > 0)
    for k in range(2 * q):
        assert abs(np.dot(w, x ** k) - 1.0 / (k + 1)) < 4e-16 * (k + 1)
    # and it is the same rule as numpy's (a library routine)
    xr, wr = an.gauss_legendre01(q)
    assert np.allclose(x, xr, rtol=0, atol=4e-16) and np.allclose(w, wr, rtol=0, atol=4e-16)


def test_tri7_exact_to_degree_5():
    b, w = oracle.tri7()
    assert abs(w.sum() - 1.0) < 1e-15 and np.allclose(b.sum(axis=1), 1.0)
    # reference triangle (0,0), (1,0), (0,1): int x^a y^b = a! b! / (a+b+2)!
    x = b[:, 1]
    y = b[:, 2]
    for a in range(6):
        for c in range(6 - a):
            exact = math.factorial(a) * math.factorial(c) / math.factorial(a + c + 2)
            got = 0.5 * np.dot(w, x ** a * y ** c)
            assert abs(got - exact) < 1e-16
    # degree 6 is not integrated exactly (the rule is degree 5, not more)
    assert abs(0.5 * np.dot(w, x ** 6) - math.factorial(6) / math.factorial(8)) > 1e-8


# ------------------------------------------------ Sauter-Schwab region sets
def ref_monomial(a, b):
    """int over {0 <= t <= s <= 1} of s^a t^b."""
    return 1.0 / ((b + 1) * (a + b + 2))


@pytest.mark.parametrize("case", [oracle.IDENTICAL, oracle.EDGE, oracle.VERTEX])
def test_ss_regions_reproduce_polynomials(case):
    pts, w = oracle.ss_rule(case, 6)
    # all points lie in the reference triangle pair
    assert np.all(pts[:, 1] <= pts[:, 0] + 1e-15) and np.all(pts[:, 3] <= pts[:, 2] + 1e-15)
    assert np.all(pts >= -1e-15) and np.all(pts <= 1 + 1e-15)
    for e in [(0, 0, 0, 0), (1, 0, 0, 0), (0, 1, 0, 0), (0, 0, 1, 0), (0, 0, 0, 1),
              (2, 0, 0, 0), (1, 1, 0, 0), (0, 0, 1, 1), (1, 0, 1, 0), (0, 1, 0, 1),
              (1, 0, 0, 1), (0, 2, 0, 0), (0, 0, 0, 2), (2, 1, 0, 1), (1, 1, 1, 1)]:
        f = pts[:, 0] ** e[0] * pts[:, 1] ** e[1] * pts[:, 2] ** e[2] * pts[:, 3] ** e[3]
        exact = ref_monomial(e[0], e[1]) * ref_monomial(e[2], e[3])
        assert abs(np.dot(w, f) - exact) < 1e-15, e


def test_ss_regions_are_a_partition_smooth_nonpolynomial():
    # a smooth non-polynomial integrand: the rules converge to the plain
    # tensor (Duffy) value, so no region is missing or counted twice
    def f(p):
        return np.exp(p[:, 0] - 0.5 * p[:, 1] + 0.3 * p[:, 2] * p[:, 3]) * np.cos(p[:, 3] - p[:, 1])

    g, w = an.gauss_legendre01(24)
    S, T = np.meshgrid(g, g, indexing="ij")
    WS, WT = np.meshgrid(w, w, indexing="ij")
    s, t, ws = S.ravel(), (S * T).ravel(), (WS * WT * S).ravel()
    A = np.stack([np.repeat(s, s.size), np.repeat(t, s.size), np.tile(s, s.size), np.tile(t, s.size)], 1)
    ref = np.dot(np.repeat(ws, ws.size) * np.tile(ws, ws.size), f(A))
    for case in (oracle.IDENTICAL, oracle.EDGE, oracle.VERTEX):
        pts, w2 = oracle.ss_rule(case, 8)
        assert abs(np.dot(w2, f(pts)) - ref) < 1e-13 * abs(ref)


# ---------------------------------------------- identical pairs: closed form
def test_closed_form_itself_pinned_by_semianalytic_integration():
    p = np.array([[0.1, -0.2, 0.05], [1.3, 0.1, -0.1], [0.4, 0.9, 0.3]])
    pts, w = an.duffy_points(p, 40, composite=4)
    semi = np.dot(w, an.triangle_potential(pts, p))
    assert abs(semi - an.self_integral(*p)) < 5e-8 * an.self_integral(*p)
    s = 0.7
    eq = np.array([[0, 0, 0], [s, 0, 0], [s / 2, s * math.sqrt(3) / 2, 0]])
    assert abs(an.self_integral(*eq) - 0.75 * s ** 3 * math.log(3)) < 1e-15


@pytest.mark.parametrize("tri_pts,q,tol", [
    ([[0, 0, 0], [1, 0, 0], [0.5, math.sqrt(3) / 2, 0]], 12, 1e-14),
    ([[0.1, -0.2, 0.05], [1.3, 0.1, -0.1], [0.4, 0.9, 0.3]], 16, 1e-14),
])
def test_identical_slp_matches_closed_form(tri_pts, q, tol):
    v = np.array(tri_pts, dtype=float)
    tri = np.array([[0, 1, 2]], dtype=np.int32)
    exact = an.self_integral(*v) / (4 * math.pi)
    got = oracle.entries(v, tri, [0], [0], q_sing=q)[0]
    assert abs(got.imag) == 0.0
    assert abs(got.real - exact) < tol * exact
    # and the error decreases with the order
    errs = [abs(oracle.entries(v, tri, [0], [0], q_sing=k)[0].real - exact) for k in (3, 5, 8)]
    assert errs[0] > errs[1] > errs[2]


# ------------------------------------ edge / vertex pairs: semi-analytic
def _semi(v, tri, i, j, layer):
    pi, pj = v[tri[i]], v[tri[j]]
    shared = [a for a in tri[i] if a in tri[j]]
    k = list(tri[i]).index(shared[0])
    pts, w = an.duffy_points(np.roll(pi, -k, axis=0), 40, composite=4)
    f = an.triangle_potential(pts, pj) if layer == oracle.SLP else -an.solid_angle(pts, pj)
    return np.dot(w, f) / (4 * math.pi)


@pytest.mark.parametrize("case,layer,tol", [
    (oracle.VERTEX, oracle.SLP, 1e-11), (oracle.VERTEX, oracle.DLP, 1e-10),
    (oracle.EDGE, oracle.SLP, 2e-8), (oracle.EDGE, oracle.DLP, 2e-8),
])
def test_adjacent_pairs_match_semianalytic_brute_force(case, layer, tol):
    m = octahedron_sphere(2)
    j = next(j for j in range(1, m.nt) if oracle.shared_vertices(m.tri, 0, j) == case)
    ref = _semi(m.v, m.tri, 0, j, layer)
    got = oracle.entries(m.v, m.tri, [0], [j], layer=layer, q_sing=10)[0].real
    assert abs(got - ref) < tol * abs(ref)
    # a wrong relabelling or map would not converge: coarse orders are farther
    coarse = oracle.entries(m.v, m.tri, [0], [j], layer=layer, q_sing=4)[0].real
    assert abs(coarse - ref) > abs(got - ref)


def test_regular_pairs_match_semianalytic_brute_force():
    m = octahedron_sphere(4)
    for j in (40, 77, 101):
        assert oracle.shared_vertices(m.tri, 0, j) == 0
        for layer in (oracle.SLP, oracle.DLP):
            pts, w = an.duffy_points(m.v[m.tri[0]], 30)
            pj = m.v[m.tri[j]]
            f = an.triangle_potential(pts, pj) if layer == oracle.SLP else -an.solid_angle(pts, pj)
            ref = np.dot(w, f) / (4 * math.pi)
            got = oracle.entries(m.v, m.tri, [0], [j], layer=layer, q_reg=8)[0].real
            assert abs(got - ref) < 1e-9 * abs(ref)
            tri7 = oracle.entries(m.v, m.tri, [0], [j], layer=layer, rule=oracle.RULE_TRI7)[0].real
            assert abs(tri7 - ref) < 1e-3 * abs(ref)


# ------------------------------------------------------- double layer
def test_gauss_identity_sphere_converges():
    m = octahedron_sphere(2)
    a = areas(m.v, m.tri)
    dev = []
    for q in (3, 4, 5, 6):
        K = full_matrix(m, layer=oracle.DLP, q_reg=q, q_sing=q).real
        dev.append(np.max(np.abs(K.sum(axis=1) + a / 2) / a))
    assert dev[-1] < 2e-6
    assert all(dev[k] > dev[k + 1] for k in range(3))


def test_gauss_identity_cube_and_coplanar_zeros():
    m = cube_surface(1)
    a = areas(m.v, m.tri)
    K = full_matrix(m, layer=oracle.DLP, q_reg=6, q_sing=6).real
    assert np.max(np.abs(K.sum(axis=1) + a / 2) / a) < 1e-3
    normals = np.cross(m.v[m.tri[:, 1]] - m.v[m.tri[:, 0]], m.v[m.tri[:, 2]] - m.v[m.tri[:, 0]])
    normals /= np.linalg.norm(normals, axis=1, keepdims=True)
    coplanar = np.abs(normals @ normals.T - 1) < 1e-12
    for i in range(m.nt):
        for j in range(m.nt):
            if coplanar[i, j] and abs(np.dot(m.v[m.tri[i, 0]] - m.v[m.tri[j, 0]], normals[j])) < 1e-14:
                assert K[i, j] == 0.0


def test_dlp_identical_is_zero():
    m = octahedron_sphere(3)
    d = oracle.entries(m.v, m.tri, np.arange(m.nt), np.arange(m.nt), layer=oracle.DLP, q_sing=5).real
    assert np.max(np.abs(d)) < 1e-16


# ------------------------------------------------------------ Helmholtz
def test_helmholtz_kappa_zero_equals_laplace():
    m = octahedron_sphere(2)
    for layer in (oracle.SLP, oracle.DLP):
        L = full_matrix(m, layer=layer, q_reg=3, q_sing=3)
        H = full_matrix(m, kernel=oracle.HELMHOLTZ, kappa=0.0, layer=layer, q_reg=3, q_sing=3)
        assert np.max(np.abs(H - L)) <= 1e-15 * np.max(np.abs(L))
        assert np.max(np.abs(H.imag)) == 0.0


def test_helmholtz_imag_part_is_smooth_and_matches_plain_duffy():
    # Im g = sin(kappa r) / (4 pi r) is smooth, so a plain high-order Duffy
    # rule on both triangles (kappa sinc(kappa r) where points coincide) must
    # agree with the Sauter-Schwab value for an identical pair.
    kappa = 8.0
    v = np.array([[0.0, 0.0, 0.0], [0.3, 0.05, 0.0], [0.1, 0.25, 0.02]])
    tri = np.array([[0, 1, 2]], dtype=np.int32)
    ss = oracle.entries(v, tri, [0], [0], kernel=oracle.HELMHOLTZ, kappa=kappa, q_sing=12)[0]
    pts, w = an.duffy_points(v, 16)
    d = np.linalg.norm(pts[:, None, :] - pts[None, :, :], axis=2)
    f = kappa * np.sinc(kappa * d / np.pi) / (4 * math.pi)
    plain = w @ f @ w
    assert abs(ss.imag - plain) < 1e-13 * abs(plain)
    # real part: (cos(kr) - 1)/r is continuous but kinked at r = 0, so the
    # plain rule converges only algebraically; the singular part is Laplace
    lap = oracle.entries(v, tri, [0], [0], q_sing=12)[0].real
    f2 = np.where(d > 0, (np.cos(kappa * d) - 1) / np.where(d > 0, d, 1), 0.0) / (4 * math.pi)
    assert abs(ss.real - (lap + w @ f2 @ w)) < 3e-4 * abs(ss.real)


# ------------------------------------------------------------ symmetry etc.
def test_slp_symmetry_by_pair_class():
    m = octahedron_sphere(3)
    V = full_matrix(m, q_reg=4, q_sing=5).real
    cls = np.array([[oracle.shared_vertices(m.tri, i, j) for j in range(m.nt)] for i in range(m.nt)])
    asym = np.abs(V - V.T) / np.max(np.abs(V))
    assert np.max(asym[cls != oracle.EDGE]) < 1e-15
    e = asym[cls == oracle.EDGE]
    assert np.max(e) < 1e-5 and np.max(e) > 0  # the edge rule is symmetric only to quadrature error


def test_unit_sphere_single_layer_potential():
    # int_S 1/(4 pi |x - y|) dy = 1 on the unit sphere, so row sums of V tend
    # to area(tau_i) as the mesh is refined (O(h^2) geometry error)
    err = []
    for n in (4, 8):
        m = octahedron_sphere(n)
        V = full_matrix(m, q_reg=3, q_sing=4).real
        a = areas(m.v, m.tri)
        err.append(np.max(np.abs(V.sum(axis=1) / a - 1)))
    assert err[1] < 0.01 and err[1] < err[0] / 3


def test_far_pairs_tend_to_midpoint_rule():
    m = octahedron_sphere(8)
    a = areas(m.v, m.tri)
    c = m.v[m.tri].mean(axis=1)
    i = 0
    far = np.argsort(-np.linalg.norm(c - c[i], axis=1))[:5]
    g = oracle.entries(m.v, m.tri, np.full(5, i), far, q_reg=4).real
    mid = a[i] * a[far] / (4 * math.pi * np.linalg.norm(c[far] - c[i], axis=1))
    assert np.max(np.abs(g - mid) / mid) < 1e-3


def test_invalid_arguments_rejected():
    m = octahedron_sphere(1)
    with pytest.raises(ValueError):
        oracle.entries(m.v, m.tri, [0], [m.nt])
    with pytest.raises(ValueError):
        oracle.entries(m.v, m.tri, [0], [0], q_sing=0)
