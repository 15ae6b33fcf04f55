"""Host parts of the Green cross approximation (no GPU): Green boxes and
points against the oracle's, and the adaptive cross approximation against
what linear algebra fixes (exact rank recovery, interpolation property,
inverse of the pivot block, tie-breaking)."""
import numpy as np
import pytest

from bem_inputs import octahedron_sphere
from oracle import htree


def test_green_points_match_oracle():
    import paper_1510_07244_amd as pk
    m = octahedron_sphere(8)
    ct = pk.ClusterTree(m.v, m.tri)
    for qg in (1, 3, 4):
        z, zn, zw, delta = pk.green_points(ct.box, qg)
        for c in range(ct.n):
            lo, hi, dref = htree.green_box(htree.Cluster(idx=None, lo=ct.box[c, :3], hi=ct.box[c, 3:]))
            zr, znr, zwr = htree.green_points(lo, hi, qg)
            assert abs(delta[c] - dref) <= 1e-15 * dref
            assert np.allclose(z[c], zr, rtol=0, atol=4e-16)
            assert np.array_equal(zn[c], znr)
            assert np.allclose(zw[c], zwr, rtol=1e-14, atol=0)


@pytest.mark.parametrize("cplx", [False, True])
def test_aca_recovers_low_rank_and_interpolates(cplx):
    import paper_1510_07244_amd as pk
    rng = np.random.default_rng(4)
    mats, nrows = [], []
    for n, r in ((40, 5), (64, 12), (17, 17), (30, 1)):
        U = rng.standard_normal((n, r))
        W = rng.standard_normal((r, 24))
        if cplx:
            U = U + 1j * rng.standard_normal((n, r))
            W = W + 1j * rng.standard_normal((r, 24))
        mats.append((U @ W, r))
        nrows.append(n)
    off = np.zeros(len(mats), dtype=np.int64)
    off[1:] = np.cumsum([a.size for a, _ in mats])[:-1]
    packed = np.concatenate([a.T.ravel() for a, _ in mats])  # column-major
    flat = packed.view(np.float64) if cplx else packed
    rank, prow, pcol, pinv = pk.aca(flat, off, nrows, 24, 1e-12, 24, is_complex=cplx)
    for t, (A, r) in enumerate(mats):
        k = rank[t]
        assert k == r
        rows, cols = prow[t, :k], pcol[t, :k]
        assert len(set(rows)) == k and len(set(cols)) == k
        P = pinv[t].view(np.complex128) if cplx else pinv[t]
        P = P[:k * k].reshape(k, k).T  # column-major, leading dimension k
        assert np.allclose(P @ A[np.ix_(rows, cols)], np.eye(k), atol=1e-9)
        V = A[:, cols] @ P
        assert np.allclose(V[rows], np.eye(k), atol=1e-9)          # R_t V_t = I
        assert np.linalg.norm(V @ A[rows] - A) <= 1e-9 * np.linalg.norm(A)


def test_aca_first_pivot_and_ties():
    import paper_1510_07244_amd as pk
    A = np.array([[1.0, 3.0], [-3.0, 2.0], [0.5, 0.0]])  # |3| twice: row 0 col 1 wins (smallest row)
    flat = A.T.ravel()
    rank, prow, pcol, _ = pk.aca(flat, [0], [3], 2, 0.0, 2)
    assert prow[0, 0] == 0 and pcol[0, 0] == 1


def test_aca_rejects_bad_arguments():
    import paper_1510_07244_amd as pk
    with pytest.raises(pk.BemError):
        pk.aca(np.zeros(4), [0], [2], 2, -1.0, 2)


def test_aca_nan_columns_stay_in_bounds():
    # a column of NaN has no entry equal to its (NaN-ignoring) maximum: the
    # pivot search must stop at the column's end; an all-NaN matrix has rank 0
    import paper_1510_07244_amd as pk
    A = np.full((5, 4), np.nan)
    rank, _, _, _ = pk.aca(A.T.ravel().copy(), [0], [5], 4, 1e-12, 4)
    assert rank[0] == 0
    B = np.random.default_rng(0).standard_normal((8, 6))
    B[:, 2] = np.nan
    rank, _, pcol, _ = pk.aca(B.T.ravel().copy(), [0], [8], 6, 1e-12, 6)
    assert 0 < rank[0] <= 6 and 2 not in pcol[0, :rank[0]]


def test_rank_head_cluster_features():
    # the rank head's inputs from a host cluster tree (no GPU needed)
    import types
    import paper_1510_07244_amd as pk
    from paper_1510_07244_amd.selector import cluster_features
    from bem_inputs import octahedron_sphere
    m = octahedron_sphere(8)
    ct = pk.ClusterTree(m.v, m.tri, leaf=64)
    height = np.zeros(ct.n, dtype=np.int32)
    for c in range(ct.n - 1, -1, -1):
        s = ct.sons[c]
        if s[0] >= 0:
            height[c] = 1 + max(height[s[0]], height[s[1]])
    h = types.SimpleNamespace(ct=ct, height=height, kappa=0.0, eps=5e-8)
    X = cluster_features(h, 1)
    assert X.shape == (ct.n, 8) and X.dtype == np.float32
    assert np.isclose(X[0, 0], np.log2(m.nt))  # the root holds every triangle
    assert np.all((X[:, 2] <= 1) & (X[:, 3] <= X[:, 2] + 1e-7) & (X[:, 3] >= 0))
    assert np.all(X[:, 4] == height) and np.all(X[:, 5] == 0) and np.all(X[:, 6] == 1)
    assert np.allclose(X[:, 7], np.log10(5e-8))
    sons = ct.sons[0]
    assert X[sons[0], 0] < X[0, 0] and X[sons[0], 1] <= X[0, 1] + 1e-7


def test_cluster_features_follow_their_definition():
    """bem_cluster_features against the eight inputs written out here: log2
    of the triangle count, log10 of the box diagonal, middle and smallest box
    extent over the largest, height, kappa times the diagonal, side, log10 of
    the tolerance (a flat box and a one-triangle cluster included)."""
    import paper_1510_07244_amd as pk
    m = octahedron_sphere(8)
    ct = pk.ClusterTree(m.v, m.tri)
    height = np.zeros(ct.n, dtype=np.int32)
    for c in range(ct.n - 1, -1, -1):
        s = ct.sons[c]
        if s[0] >= 0:
            height[c] = 1 + max(height[s[0]], height[s[1]])
    box = ct.box.copy()
    begin, end = ct.begin.copy(), ct.end.copy()
    box[0, 2] = box[0, 5]  # a flat box
    end[1] = begin[1] + 1  # one triangle
    X = pk.cluster_features(box, begin, end, height, 3.0, 1, 5e-8)
    for c in range(ct.n):
        e = sorted(box[c, 3:] - box[c, :3])
        d = float(np.sqrt(sum(x * x for x in e)))
        ref = [np.log2(max(end[c] - begin[c], 1)), np.log10(d), e[1] / e[2], e[0] / e[2],
               height[c], 3.0 * d, 1.0, np.log10(5e-8)]
        assert np.allclose(X[c], np.float32(ref), rtol=1e-6, atol=1e-7), c
    assert X[0, 3] == 0.0 and X[1, 0] == 0.0
    with pytest.raises(pk.BemError):
        pk.cluster_features(box, begin, end, height, 3.0, 1, 0.0)


def test_block_lists_match_the_per_block_construction(monkeypatch):
    """h2._block_lists (index arithmetic over the whole list) against the
    lists built block by block: near field plain and mirrored (diagonal
    blocks their own mirror), coupling-like pivot lists plain and mirrored."""
    import paper_1510_07244_amd as pk
    from paper_1510_07244_amd import h2

    class Rec:
        def __init__(self, rp, ri, cp, ci, off, mirror=None):
            self.rp, self.ri, self.cp, self.ci = rp, ri, cp, ci
            self.off, self.mirror = off, mirror

    monkeypatch.setattr(h2, "Blocks", Rec)
    m = octahedron_sphere(16)
    ct = pk.ClusterTree(m.v, m.tri)
    near, far = pk.block_tree(ct, eta=2.0)
    size = (ct.end - ct.begin).astype(np.int64)
    start = ct.begin.astype(np.int64)
    rng = np.random.default_rng(7)
    piv = [np.sort(rng.choice(ct.idx(c), size=min(size[c], rng.integers(1, 9)), replace=False))
           for c in range(ct.n)]
    psize = np.array([p.size for p in piv], dtype=np.int64)
    pstart = np.concatenate([[0], np.cumsum(psize)[:-1]])
    pflat = np.concatenate(piv)

    def reference(pairs, lists, mirror, keep_diag):
        rows = [lists(t) for t, s in pairs]
        cols = [lists(s) for t, s in pairs]
        sizes = [len(r) * len(c) for r, c in zip(rows, cols)]
        off = np.concatenate([[0], np.cumsum(sizes)[:-1]])
        keep = [k for k, (t, s) in enumerate(pairs) if (t <= s if keep_diag else t < s)] \
            if mirror else list(range(len(pairs)))
        pos = {(int(t), int(s)): k for k, (t, s) in enumerate(pairs)}
        mo = [off[pos[(int(pairs[k][1]), int(pairs[k][0]))]] for k in keep] if mirror else None
        return ([r for k in keep for r in rows[k]], [len(rows[k]) for k in keep],
                [c for k in keep for c in cols[k]], [len(cols[k]) for k in keep],
                off[keep], mo, sum(sizes))

    for pairs, spec, lists, keep_diag in (
            (near, (ct.perm, start, size), ct.idx, True),
            (far, (pflat, pstart, psize), lambda c: piv[c], False)):
        for mirror in (False, True):
            b, total = h2._block_lists(pairs, spec, spec, mirror, keep_diag)
            ri, nr, ci, nc, off, mo, tot = reference(pairs, lists, mirror, keep_diag)
            assert total == tot
            assert np.array_equal(b.ri, ri) and np.array_equal(np.diff(b.rp), nr)
            assert np.array_equal(b.ci, ci) and np.array_equal(np.diff(b.cp), nc)
            assert np.array_equal(b.off, off)
            assert (b.mirror is None) == (mo is None)
            if mo is not None:
                assert np.array_equal(b.mirror, mo)
