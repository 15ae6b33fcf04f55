"""The learned rank head (per-cluster prediction of the cross approximation's
rank) and the rank caps it feeds into the basis setup (GPU).

* Trained on the finished setups of a 2048-triangle sphere, a cube surface
  and two perturbed spheres (both sides), it predicts the ranks of the
  held-out 8192-triangle sphere with a mean absolute error of a few ranks.
* Bases built with its caps are the plain bases bit for bit (the pivot
  search is redone without the bound wherever a cap is reached): same
  ranks, pivots and basis matrices.
"""
import numpy as np
import pytest

from bem_inputs import cube_surface, octahedron_sphere, perturbed_sphere

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pk():
    import torch
    import paper_1510_07244_amd as pk
    assert torch.cuda.is_available()
    return pk


@pytest.fixture(scope="module")
def ctx(pk):
    c = pk.Context(0)
    yield c
    c.close()


def _setup(pk, ctx, m):
    from paper_1510_07244_amd.h2 import H2Setup
    h = H2Setup(ctx, m.v, m.tri, kernel=pk.LAPLACE, q_regular=4, q_singular=4)
    return h, h.bases((0, 1))


def test_rank_head_predicts_and_caps_keep_the_bases(pk, ctx):
    from paper_1510_07244_amd.selector import RankHead, cluster_features
    train = [_setup(pk, ctx, m) for m in (octahedron_sphere(16), cube_surface(16),
                                          perturbed_sphere(101), perturbed_sphere(102))]
    head = RankHead(ctx, seed=3)
    X, R = RankHead.samples(train)
    losses = head.fit(X, R)
    assert losses[-1] < 0.5 * losses[0]
    h, (V, W) = _setup(pk, ctx, octahedron_sphere(32))
    err = []
    for B in (V, W):
        p = head.predict(cluster_features(h, B.side))
        err.append(np.abs(p - B.rank)[h.needed])
    err = np.concatenate(err)
    print(f"rank head on the held-out sphere: mean abs error {err.mean():.2f}, max {err.max():.1f}")
    assert err.mean() < 8.0
    caps = [head.caps(h, 0), head.caps(h, 1)]
    V2, W2 = h.bases((0, 1), rank_caps=caps)
    assert h.cap_stats["levels"] > 0
    for A, B in ((V, V2), (W, W2)):
        assert np.array_equal(A.rank, B.rank)
        assert all(np.array_equal(A.piv[c], B.piv[c]) for c in range(h.ct.n))
        for c in np.nonzero(h.needed)[0]:
            assert np.array_equal(A.vhat(c), B.vhat(c))


def test_caps_that_bind_fall_back_to_the_plain_search(pk, ctx):
    # caps far below the ranks: every level's bound is reached, every level
    # is searched again without it, and the bases are the plain ones
    h, (V, W) = _setup(pk, ctx, octahedron_sphere(16))
    caps = [np.full(h.ct.n, 5, dtype=np.int64), np.full(h.ct.n, 5, dtype=np.int64)]
    V2, W2 = h.bases((0, 1), rank_caps=caps)
    assert h.cap_stats["levels"] > 0
    assert h.cap_stats["fallbacks"] == h.cap_stats["levels"]
    for A, B in ((V, V2), (W, W2)):
        assert np.array_equal(A.rank, B.rank)
        for c in np.nonzero(h.needed)[0]:
            assert np.array_equal(A.piv[c], B.piv[c])
            assert np.array_equal(A.vhat(c), B.vhat(c))
