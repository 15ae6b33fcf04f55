"""Pins of the oracle's cluster/block tree and Green quadrature matrices.

* The cluster tree partitions the index set, the block tree tiles I x J
  exactly once, admissible leaves satisfy the condition, near leaves touch
  a leaf cluster (Sec. 2.3).
* Green's representation formula with Gauss quadrature on the Green box
  (Sec. 2.3, eq. green_apx) reproduces admissible blocks of the single-layer
  matrix from the row matrix A_t and the column factors B_ts, and (with the
  Green box of the column cluster, normal derivatives in y) of the
  double-layer matrix, to Green-quadrature accuracy, for Laplace and for
  Helmholtz.  A dropped term, a wrong sign or a wrong normal fails these by
  orders of magnitude.
"""
import numpy as np
import pytest

import oracle
from bem_inputs import octahedron_sphere
from oracle import htree


@pytest.fixture(scope="module")
def sphere2048():
    m = octahedron_sphere(16)
    cl = htree.cluster_tree(m.v, m.tri, leaf=64)
    near, far = htree.block_tree(cl, eta=2.0)
    return m, cl, near, far


def test_cluster_tree_partitions(sphere2048):
    m, cl, _, _ = sphere2048
    assert np.array_equal(np.sort(cl[0].idx), np.arange(m.nt))
    tlo, thi = htree.tri_boxes(m.v, m.tri)
    for c in cl:
        assert np.all(tlo[c.idx] >= c.lo) and np.all(thi[c.idx] <= c.hi)
        if c.sons:
            joined = np.concatenate([cl[s].idx for s in c.sons])
            assert np.array_equal(np.sort(joined), np.sort(c.idx))
            assert len(set(cl[c.sons[0]].idx) & set(cl[c.sons[1]].idx)) == 0
        else:
            assert c.idx.size <= 64


def test_block_tree_tiles_matrix_once(sphere2048):
    m, cl, near, far = sphere2048
    cover = np.zeros((m.nt, m.nt), dtype=np.int32)
    for t, s in near + far:
        cover[np.ix_(cl[t].idx, cl[s].idx)] += 1
    assert np.all(cover == 1)
    for t, s in far:
        d = max(htree.box_diam(cl[t].lo, cl[t].hi), htree.box_diam(cl[s].lo, cl[s].hi))
        assert d <= 2.0 * htree.box_dist(cl[t].lo, cl[t].hi, cl[s].lo, cl[s].hi)
    for t, s in near:
        assert not cl[t].sons or not cl[s].sons


def test_config2_tree_sizes():
    # 8192-triangle sphere, leaf 64, eta = 2
    m = octahedron_sphere(32)
    cl = htree.cluster_tree(m.v, m.tri, leaf=64)
    near, far = htree.block_tree(cl, eta=2.0)
    leaves = [c for c in cl if not c.sons]
    assert len(cl) == 367 and len(leaves) == 184
    assert len(near) == 2400 and len(far) == 3760


def test_green_points_integrate_box_surface():
    lo = np.array([-0.3, 0.1, 0.2])
    hi = np.array([0.5, 0.4, 1.0])
    z, zn, zw = htree.green_points(lo, hi, 4)
    ext = hi - lo
    area = 2 * (ext[0] * ext[1] + ext[1] * ext[2] + ext[0] * ext[2])
    assert abs(zw.sum() - area) < 1e-14
    # divergence theorem: int <x, n> = 3 vol
    assert abs(np.dot(zw, np.einsum("ij,ij->i", z, zn)) - 3 * np.prod(ext)) < 1e-13
    assert np.allclose(np.abs(zn).sum(axis=1), 1.0)


def _admissible_pair(sphere2048, min_size=40):
    m, cl, near, far = sphere2048
    for t, s in far:
        if cl[t].idx.size >= min_size and cl[s].idx.size >= min_size and not cl[t].sons:
            return t, s
    raise AssertionError("no admissible leaf pair")


@pytest.mark.parametrize("kernel,kappa", [(oracle.LAPLACE, 0.0), (oracle.HELMHOLTZ, 4.0)])
def test_green_representation_reproduces_slp_block(sphere2048, kernel, kappa):
    m, cl, _, _ = sphere2048
    t, s = _admissible_pair(sphere2048)
    rows, cols = cl[t].idx, cl[s].idx
    lo, hi, delta = htree.green_box(cl[t])
    G = oracle.block(m.v, m.tri, rows, cols, kernel=kernel, kappa=kappa, q_reg=4)
    errs = []
    for qg in (4, 8, 12):
        z, zn, zw = htree.green_points(lo, hi, qg)
        nm = zw.size
        A = oracle.green_matrix(m.v, m.tri, rows, z, zn, zw, delta, kernel=kernel, kappa=kappa, side=0, q=4)
        M = oracle.green_matrix(m.v, m.tri, cols, z, zn, zw, delta, kernel=kernel, kappa=kappa, side=0, q=4)
        Ap, Am = A[:, :nm], A[:, nm:]
        Bp, Bm = M[:, nm:] / delta, M[:, :nm] / delta
        approx = Ap @ Bp.T - Am @ Bm.T
        errs.append(np.linalg.norm(approx - G) / np.linalg.norm(G))
        # the minus sign matters: a "+" would be far off
        wrong = Ap @ Bp.T + Am @ Bm.T
        assert np.linalg.norm(wrong - G) / np.linalg.norm(G) > 0.1
    # Green quadrature converges with its order (it is coarse at q_G = 4)
    assert errs[2] < 2e-4 and errs[2] < errs[1] / 5 < errs[0] / 25


@pytest.mark.parametrize("kernel,kappa", [(oracle.LAPLACE, 0.0), (oracle.HELMHOLTZ, 4.0)])
def test_green_representation_reproduces_dlp_block_from_column_side(sphere2048, kernel, kappa):
    # K_ij = int phi_i int d/dn(y) g(x,y) psi_j: Green's formula in y on the
    # box of the column cluster s, then d/dn(y):
    #   d/dn(y) g(x,y) ~ sum w [d/dn(y) g(y,z) d/dn(z) g(x,z) - d/dn(y)d/dn(z) g(y,z) g(x,z)]
    m, cl, _, _ = sphere2048
    t, s = _admissible_pair(sphere2048)
    rows, cols = cl[t].idx, cl[s].idx
    lo, hi, delta = htree.green_box(cl[s])
    K = oracle.block(m.v, m.tri, rows, cols, kernel=kernel, kappa=kappa, layer=oracle.DLP, q_reg=4)
    errs = []
    for qg in (4, 12):
        z, zn, zw = htree.green_points(lo, hi, qg)
        nm = zw.size
        A = oracle.green_matrix(m.v, m.tri, rows, z, zn, zw, delta, kernel=kernel, kappa=kappa, side=0, q=4)
        C = oracle.green_matrix(m.v, m.tri, cols, z, zn, zw, delta, kernel=kernel, kappa=kappa, side=1, q=4)
        approx = (A[:, nm:] / delta) @ C[:, :nm].T - A[:, :nm] @ (C[:, nm:] / delta).T
        errs.append(np.linalg.norm(approx - K) / np.linalg.norm(K))
    assert errs[1] < 2e-4 and errs[1] < errs[0] / 20
