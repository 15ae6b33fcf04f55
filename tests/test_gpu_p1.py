"""Piecewise-linear (P1) bases on the GPU (through the C-ABI) against the
oracle.

* Local 3 x 3 matrices of triangle pairs of every class (disjoint, vertex,
  edge, identical), Laplace and Helmholtz, single and double layer, with the
  Duffy rule and with the seven-point rule for the disjoint pairs: within
  1e-12 of the oracle's, relative to the largest entry of each set.
* Dense blocks of the P1 Galerkin matrix (the local matrices summed over the
  triangles around each vertex pair) of the 512-triangle sphere: within
  1e-12 of the oracle's assembly; Gauss's identity for the double layer,
  rows summing to -|star(v)| / 6 up to quadrature error.
"""
import numpy as np
import pytest

import oracle
from bem_inputs import octahedron_sphere, sample_subset

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pk():
    import paper_1510_07244_amd as pk
    return pk


@pytest.fixture(scope="module")
def ctx(pk):
    c = pk.Context(0)
    yield c
    c.close()


def _pairs(m, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    rows = list(rng.integers(0, m.nt, 300))
    cols = list(rng.integers(0, m.nt, 300))
    for i in sample_subset(np.arange(m.nt), 20, seed=seed + 1):
        ti = set(m.tri[i])
        rows.append(i), cols.append(i)  # identical
        for j in range(m.nt):
            c = len(ti & set(m.tri[j]))
            if c in (1, 2):
                rows.append(i), cols.append(j)
    return np.array(rows, dtype=np.int32), np.array(cols, dtype=np.int32)


@pytest.mark.parametrize("kernel,kappa", [(0, 0.0), (1, 3.0)])
@pytest.mark.parametrize("layer", [0, 1])
@pytest.mark.parametrize("rule", [0, 1])
def test_p1_local_matrices(pk, ctx, kernel, kappa, layer, rule):
    import torch
    m = octahedron_sphere(8)
    rows, cols = _pairs(m, 3 + layer)
    mesh = pk.Mesh(torch.from_numpy(m.v), torch.from_numpy(m.tri))
    op = pk.make_op(kernel, layer, regular_rule=rule, q_regular=4, q_singular=4, kappa=kappa)
    dt = torch.complex128 if kernel else torch.float64
    out = torch.full((9 * rows.size,), float("nan"), dtype=dt, device="cuda")
    ctx.p1_pairs(mesh, op, torch.from_numpy(rows).cuda(), torch.from_numpy(cols).cuda(), out)
    ctx.check()
    got = out.cpu().numpy().reshape(-1, 3, 3)
    if rule == 0:
        ref = oracle.p1_pairs(m.v, m.tri, rows, cols, kernel=kernel, layer=layer, kappa=kappa,
                              q_reg=4, q_sing=4)
        ref = ref if kernel else ref.real
        assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()
        for c in range(4):  # every class present and matched
            sel = np.array([oracle.shared_vertices(m.tri, i, j) == c for i, j in zip(rows, cols)])
            assert sel.any()
            assert np.abs(got[sel] - ref[sel]).max() <= 1e-12 * np.abs(ref).max(), c
    else:
        # seven-point rule: partition of unity against the piecewise-constant
        # entries of the same rule
        p0 = oracle.entries(m.v, m.tri, rows, cols, kernel=kernel, layer=layer, kappa=kappa,
                            rule=1, q_reg=4, q_sing=4)
        p0 = p0 if kernel else p0.real
        assert np.abs(got.sum(axis=(1, 2)) - p0).max() <= 1e-12 * np.abs(p0).max()


@pytest.mark.parametrize("layer", [0, 1])
def test_p1_dense_blocks(pk, ctx, layer):
    import torch
    from paper_1510_07244_amd.p1 import p1_block
    m = octahedron_sphere(8)
    mesh = pk.Mesh(torch.from_numpy(m.v), torch.from_numpy(m.tri))
    op = pk.make_op(pk.LAPLACE, layer, q_regular=4, q_singular=4)
    nv = m.v.shape[0]
    rv = sample_subset(np.arange(nv), 37, seed=5)
    cv = sample_subset(np.arange(nv), 41, seed=6)
    got = p1_block(ctx, mesh, m.tri, op, rv, cv).cpu().numpy().reshape(cv.size, rv.size).T
    ctx.check()
    ref = oracle.p1_block(m.v, m.tri, rv, cv, layer=layer, q_reg=4, q_sing=4).real
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()
    if layer == 1:  # Gauss's identity over all columns
        every = np.arange(nv)
        K = p1_block(ctx, mesh, m.tri, op, every, every).cpu().numpy().reshape(nv, nv).T
        area = 0.5 * np.linalg.norm(np.cross(m.v[m.tri[:, 1]] - m.v[m.tri[:, 0]],
                                             m.v[m.tri[:, 2]] - m.v[m.tri[:, 0]]), axis=1)
        star = np.zeros(nv)
        for t, t3 in enumerate(m.tri):
            star[t3] += area[t]
        assert np.abs(K.sum(axis=1) + star / 6).max() <= 2e-4 * (star.max() / 6)
