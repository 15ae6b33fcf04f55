"""Pins of the learned selector's oracle (network, Adam, inputs, targets,
decision rule) against facts that do not come from the oracle itself:
finite differences of the loss, the linear regime of a ReLU network, the
first Adam step, closed-form geometry and the convergence order of Gauss
rules."""
import numpy as np
import pytest

import oracle
from bem_inputs import octahedron_sphere
from oracle import mlp, selector


def _problem(n_out, n=37, seed=3):
    rng = np.random.Generator(np.random.PCG64(seed))
    p = mlp.init(n_out, seed, mu=rng.normal(size=8), sigma=rng.uniform(0.5, 2.0, size=8))
    x = rng.normal(size=(n, 8))
    t = rng.normal(size=(n, n_out))
    return p, x, t


@pytest.mark.parametrize("n_out", [6, 1])
def test_gradient_matches_central_differences(n_out):
    p, x, t = _problem(n_out)
    g, L = mlp.grad(p, x, t, n_out)
    assert L == pytest.approx(mlp.loss(p, x, t, n_out), rel=1e-14)
    rng = np.random.Generator(np.random.PCG64(9))
    idx = rng.choice(p.size, size=60, replace=False)
    h = 1e-6
    for k in idx:
        e = np.zeros_like(p)
        e[k] = h
        fd = (mlp.loss(p + e, x, t, n_out) - mlp.loss(p - e, x, t, n_out)) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(g[k])), k
    # mu and sigma are not trained
    assert np.all(g[:16] == 0.0)


def test_linear_regime_is_an_affine_map_with_least_squares_gradient():
    # positive weights and inputs keep every ReLU active: y = A z + c exactly,
    # and dL/db4 = 2/(n n_out) sum (y - t) (closed form)
    n_out = 3
    rng = np.random.Generator(np.random.PCG64(1))
    d = mlp.unpack(mlp.init(n_out, 2), n_out)
    for k in ("1", "2", "3", "4"):
        d["W" + k] = np.abs(d["W" + k]) * 0.1
        d["b" + k] = np.abs(rng.normal(size=d["b" + k].shape))
    p = mlp.pack(d, n_out)
    x = np.abs(rng.normal(size=(11, 8)))
    y, _ = mlp.forward(p, x, n_out)
    A = d["W4"] @ d["W3"] @ d["W2"] @ d["W1"]
    c = d["W4"] @ (d["W3"] @ (d["W2"] @ d["b1"] + d["b2"]) + d["b3"]) + d["b4"]
    assert np.allclose(y, x @ A.T + c, rtol=1e-13, atol=1e-13)
    t = rng.normal(size=y.shape)
    g, _ = mlp.grad(p, x, t, n_out)
    gd = mlp.unpack(g, n_out)
    assert np.allclose(gd["b4"], 2.0 * (y - t).sum(axis=0) / y.size, rtol=1e-13)


def test_first_adam_step_moves_each_parameter_by_lr_times_sign():
    rng = np.random.Generator(np.random.PCG64(4))
    p = rng.normal(size=50)
    g = rng.normal(size=50)
    p1, m, v = mlp.adam(p, g, np.zeros(50), np.zeros(50), 1, lr=0.01, eps=1e-12)
    assert np.allclose(p - p1, 0.01 * np.sign(g), rtol=1e-9)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_features_of_a_known_pair():
    # two unit right triangles in the plane z = 0, the second shifted by 5 in x
    v = np.array([[0, 0, 0], [1, 0, 0], [1, 1, 0], [5, 0, 0], [6, 0, 0], [6, 1, 0]], float)
    tri = np.array([[0, 1, 2], [3, 4, 5]], np.int32)
    f = selector.features(v, tri, [0], [1], layer=1, kappa=2.0)[0]
    D = np.sqrt(2.0)
    assert f[0] == pytest.approx(np.log(5.0 / D), rel=1e-15)
    assert f[1] == pytest.approx(np.sqrt(3) / 4 * 2.0 / 0.5, rel=1e-15)
    assert f[2] == pytest.approx(f[1], rel=1e-15)
    assert f[3] == 1.0 and f[6] == 1.0
    assert f[4] == pytest.approx(2.0 * D, rel=1e-15)
    assert f[5] == pytest.approx(np.log(1e-12), rel=1e-15)  # parallel normals: floor
    assert f[7] == pytest.approx(np.log(1e-8), rel=1e-15)   # in-plane separation: floor
    # tilt the second triangle out of the plane: |n_i - n_j|^2 = 2 (1 - cos a)
    a = 0.3
    v2 = v.copy()
    v2[5] = [6.0, np.cos(a), np.sin(a)]
    f2 = selector.features(v2, tri, [0], [1], layer=1, kappa=2.0)[0]
    assert f2[5] == pytest.approx(np.log(2 * (1 - np.cos(a))), rel=1e-13)


def test_features_are_invariant_under_similarity_maps():
    m = octahedron_sphere(6)
    rng = np.random.Generator(np.random.PCG64(7))
    rows = rng.integers(0, m.nt, 40)
    cols = rng.integers(0, m.nt, 40)
    ok = np.array([oracle.shared_vertices(m.tri, i, j) == 0 for i, j in zip(rows, cols)])
    rows, cols = rows[ok], cols[ok]
    Q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    if np.linalg.det(Q) < 0:
        Q[:, 0] *= -1
    v2 = 3.7 * m.v @ Q.T + np.array([1.0, -2.0, 0.5])
    f1 = selector.features(m.v, m.tri, rows, cols)
    f2 = selector.features(v2, m.tri, rows, cols)
    assert np.allclose(f1, f2, rtol=1e-12, atol=1e-12)
    equilateral = np.array([[0, 0, 0], [1, 0, 0], [0.5, np.sqrt(3) / 2, 0], [9, 0, 0],
                            [10, 0, 0], [9.5, np.sqrt(3) / 2, 0]])
    fe = selector.features(equilateral, np.array([[0, 1, 2], [3, 4, 5]]), [0], [1])[0]
    assert fe[1] == pytest.approx(1.0, rel=1e-14)


def test_targets_decay_like_a_gauss_rule_for_a_separated_pair():
    # the error of the q-point rule against order 8 falls by orders of
    # magnitude from q = 1 to q = 5 for a well-separated pair
    m = octahedron_sphere(8)
    t = selector.targets(m.v, m.tri, [0], [400])[0]
    assert np.all(np.diff(t[:5]) < -1.0), t
    assert t[0] < 0 and t[4] < -9


def test_decision_rule_is_monotone_and_falls_back():
    pred = np.array([[-3, -5, -9, -11, -13, -15],   # q = 3 passes, and 4 above it
                     [-3, -9, -6, -11, -13, -15],   # q = 2 passes but 3 fails: 4
                     [-3, -5, -6, -7, -13, -15],    # 4 fails: plain order 5
                     [-9, -9, -9, -9, -13, -15]])   # q_min = 2 bounds it
    q = selector.decide(pred, q_plain=5, tol=1e-8, margin=0.5)
    assert list(q) == [3, 4, 5, 2]
    q4 = selector.decide(pred, q_plain=4, tol=1e-8, margin=0.5)
    assert list(q4) == [3, 4, 4, 2]
