"""GPU parity of the one-pass near field of both layers
(bem_assemble_nearfield_both).

* Dense blocks of a 128-triangle sphere (a block on the diagonal larger than
  every sub-tile and a ragged one; Laplace and Helmholtz, several orders)
  against the oracle's single- and double-layer blocks at 1e-12.
* Mirrored near-field lists of the H2 block tree (one of each pair (t, s),
  (s, t) evaluated): every block of both outputs -- the evaluated ones and
  the transposes -- against the oracle on a seeded sample (all blocks of
  the 2048-triangle sphere's list are written; the 8192-triangle sphere is
  the benchmark's launch), and against the per-layer entry point on the
  whole list at 1e-13 of the largest entry (rounding order differs).
* Entries of pairs with a common vertex (Laplace and Helmholtz) equal those
  of the per-layer passes bit for bit.
* The mixed form (FP32 regular pairs, FP64 singular and near-singular ones)
  of the one-pass call: every sampled block of both outputs within 1e-6
  relative Frobenius error of the oracle, and within 1e-6 of the per-layer
  mixed passes on every block.
* Error paths: both outputs must differ; a
  mirrored per-layer list whose sub-tile has more singular pairs than its
  list holds (a non-manifold fan of triangles around one edge) is reported
  as BEM_EUNSUPPORTED, and the one-pass form assembles it.
"""
import numpy as np
import pytest

import oracle
from bem_inputs import octahedron_sphere, sample_subset

pytestmark = pytest.mark.gpu

TOL = 1e-12


def _close(got, ref, tol=TOL):
    got = np.asarray(got)
    ref = np.asarray(ref)
    assert np.all(np.isfinite(got))
    fro = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    ent = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
    assert fro <= tol and ent <= tol, (fro, ent)


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


def _kw(op, layer):
    return dict(kernel=op.kernel, layer=layer, kappa=op.kappa, rule=op.regular_rule,
                q_reg=op.q_regular, q_sing=op.q_singular)


def _both(pk, ctx, mesh, op, blocks, total):
    import torch
    dt = pk.out_dtype(op)
    s = torch.full((total,), float("nan"), dtype=dt, device="cuda")
    d = torch.full((total,), float("nan"), dtype=dt, device="cuda")
    ctx.assemble_nearfield_both(mesh, op, blocks, s, d)
    ctx.check()
    return s.cpu().numpy(), d.cpu().numpy()


def _split(res, rows, cols):
    outs, o = [], 0
    for r, c in zip(rows, cols):
        outs.append(res[o:o + len(r) * len(c)].reshape(len(c), len(r)).T)  # column-major
        o += len(r) * len(c)
    return outs


@pytest.mark.parametrize("kernel,kappa,q", [(0, 0.0, 4), (0, 0.0, 7), (0, 0.0, 2),
                                            (1, 4.0, 4), (1, 8.0, 5)])
def test_both_dense_small_sphere(pk, ctx, kernel, kappa, q):
    import torch
    m = octahedron_sphere(4)  # 128 triangles
    op = pk.make_op(kernel, pk.SLP, q_regular=q, q_singular=q, kappa=kappa)
    idx = np.arange(m.nt, dtype=np.int32)
    rows = [idx, idx[5:42]]
    cols = [idx, idx[17:100]]
    mesh = pk.Mesh(torch.from_numpy(m.v), torch.from_numpy(m.tri))
    blocks, total = pk.Blocks.from_lists(rows, cols)
    s, d = _both(pk, ctx, mesh, op, blocks, total)
    for layer, res in ((0, s), (1, d)):
        full = oracle.block(m.v, m.tri, idx, idx, **_kw(op, layer))
        ref = full if kernel == pk.HELMHOLTZ else full.real
        got = _split(res, rows, cols)
        _close(got[0], ref)
        _close(got[1], ref[np.ix_(rows[1], cols[1])])


@pytest.mark.parametrize("n,kernel,kappa,nsample", [(16, 0, 0.0, 16), (16, 1, 4.0, 10),
                                                    (32, 0, 0.0, 14)])
def test_both_mirrored_lists_against_oracle(pk, ctx, n, kernel, kappa, nsample):
    from paper_1510_07244_amd.h2 import H2Setup
    m = octahedron_sphere(n)
    h = H2Setup(ctx, m.v, m.tri, kernel=kernel, kappa=kappa, q_regular=4, q_singular=4)
    half, total = h.near_blocks(mirror=True)
    full, total2 = h.near_blocks()
    assert total2 == total and half.n < full.n
    op = h.op(pk.SLP)
    s, d = _both(pk, ctx, h.mesh, op, half, total)
    rows = [h.ct.idx(t) for t, _ in h.near]
    cols = [h.ct.idx(u) for _, u in h.near]
    gs, gd = _split(s, rows, cols), _split(d, rows, cols)
    # sample: evaluated blocks, mirrored blocks and diagonal ones
    up = [k for k, (t, u) in enumerate(h.near) if t < u]
    lo = [k for k, (t, u) in enumerate(h.near) if t > u]
    dg = [k for k, (t, u) in enumerate(h.near) if t == u]
    pick = set()
    for ks, seed in ((up, 3), (lo, 5), (dg, 7)):
        pick |= set(sample_subset(np.asarray(ks), min(nsample // 3 + 1, len(ks)), seed=seed).tolist())
    for k in sorted(pick):
        for layer, got in ((0, gs), (1, gd)):
            ref = oracle.block(m.v, m.tri, rows[k], cols[k], **_kw(op, layer))
            _close(got[k], ref if kernel == pk.HELMHOLTZ else ref.real)


@pytest.mark.parametrize("kernel,kappa", [(0, 0.0), (1, 4.0)])
def test_both_equals_per_layer_passes(pk, ctx, kernel, kappa):
    # the one-pass form on the mirrored list against the per-layer entry
    # point on the whole list: equal up to rounding on every entry
    import torch
    from paper_1510_07244_amd.h2 import H2Setup
    m = octahedron_sphere(16)
    h = H2Setup(ctx, m.v, m.tri, kernel=kernel, kappa=kappa, q_regular=4, q_singular=4)
    half, total = h.near_blocks(mirror=True)
    full, _ = h.near_blocks()
    s, d = _both(pk, ctx, h.mesh, h.op(pk.SLP), half, total)
    for layer, got in ((pk.SLP, s), (pk.DLP, d)):
        op = h.op(layer)
        ref = torch.full((total,), float("nan"), dtype=pk.out_dtype(op), device="cuda")
        ctx.assemble_nearfield(h.mesh, op, full, ref)
        ctx.check()
        ref = ref.cpu().numpy()
        assert np.all(np.isfinite(got))
        assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()


def test_both_unmirrored_equals_per_layer(pk, ctx):
    # without mirrors every entry of both outputs is written once; the
    # diagonal blocks' entries agree with the per-layer passes to rounding
    import torch
    m = octahedron_sphere(8)
    op = pk.make_op(pk.LAPLACE, pk.SLP, q_regular=4, q_singular=4)
    mesh = pk.Mesh(torch.from_numpy(m.v), torch.from_numpy(m.tri))
    idx = np.arange(m.nt, dtype=np.int32)
    blocks, total = pk.Blocks.from_lists([idx[:300], idx[300:]], [idx[:300], idx[:211]])
    s, d = _both(pk, ctx, mesh, op, blocks, total)
    for layer, got in ((pk.SLP, s), (pk.DLP, d)):
        ref = torch.full((total,), float("nan"), dtype=torch.float64, device="cuda")
        ctx.assemble_nearfield(mesh, pk.make_op(pk.LAPLACE, layer, q_regular=4, q_singular=4),
                               blocks, ref)
        ctx.check()
        ref = ref.cpu().numpy()
        assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()


def _shares_vertex(tr, tc):
    # (len(tr), len(tc)) counts of common vertices
    return (tr[:, None, :, None] == tc[None, :, None, :]).sum(axis=(2, 3))


@pytest.mark.parametrize("kernel,kappa", [(0, 0.0), (1, 4.0)])
def test_both_singular_entries_bitwise_per_layer(pk, ctx, kernel, kappa):
    # pairs with a common vertex: the one-pass form sums each layer with the
    # per-layer Sauter-Schwab loop's operands in its order (Helmholtz edge-
    # and vertex-adjacent pairs share one eta pass), so the entries are
    # equal bit for bit
    import torch
    m = octahedron_sphere(8)
    mesh = pk.Mesh(torch.from_numpy(m.v), torch.from_numpy(m.tri))
    idx = np.arange(m.nt, dtype=np.int32)
    rows, cols = [idx[:300], idx[300:]], [idx[:300], idx[:211]]
    blocks, total = pk.Blocks.from_lists(rows, cols)
    op = pk.make_op(kernel, pk.SLP, q_regular=4, q_singular=4, kappa=kappa)
    s, d = _both(pk, ctx, mesh, op, blocks, total)
    # column-major blocks: entry (i, j) of a block at i + rows * j
    common = np.concatenate([_shares_vertex(m.tri[r], m.tri[c]).T.ravel()
                             for r, c in zip(rows, cols)])
    assert all(np.count_nonzero(common == k) for k in (1, 2, 3))
    mask = common > 0
    for layer, got in ((pk.SLP, s), (pk.DLP, d)):
        ref = torch.full((total,), float("nan"), dtype=pk.out_dtype(op), device="cuda")
        ctx.assemble_nearfield(mesh, pk.make_op(kernel, layer, q_regular=4, q_singular=4,
                                                kappa=kappa), blocks, ref)
        ctx.check()
        ref = ref.cpu().numpy()
        assert np.all(np.isfinite(got[mask]))
        assert np.array_equal(got[mask], ref[mask]), (layer, np.abs(got - ref)[mask].max())


def test_both_error_paths(pk, ctx):
    import torch
    m = octahedron_sphere(4)
    mesh = pk.Mesh(torch.from_numpy(m.v), torch.from_numpy(m.tri))
    idx = np.arange(m.nt, dtype=np.int32)
    blocks, total = pk.Blocks.from_lists([idx], [idx])
    op = pk.make_op(pk.LAPLACE, pk.SLP, q_regular=4, q_singular=4)
    a = torch.zeros(total, dtype=torch.float64, device="cuda")
    b = torch.zeros(total, dtype=torch.float64, device="cuda")
    with pytest.raises(pk.BemError) as e:
        ctx.assemble_nearfield_both(mesh, op, blocks, a, a)
    assert e.value.code == pk.BEM_EINVAL
    with pytest.raises(ValueError):
        ctx.assemble_nearfield_both(mesh, op, blocks, a, b[:-1])
    assert not torch.any(a != 0) and not torch.any(b != 0)  # nothing written
    ctx.check()


def _book(n):
    """n triangles sharing the edge (v0, v1), fanned around it: every pair is
    edge-adjacent (a non-manifold mesh)."""
    ang = np.linspace(0.0, 2.0 * np.pi, n, endpoint=False) + 0.1
    v = np.zeros((n + 2, 3))
    v[1] = (1.0, 0.0, 0.0)
    v[2:, 0] = 0.5
    v[2:, 1] = np.cos(ang)
    v[2:, 2] = np.sin(ang)
    tri = np.array([[0, 1, 2 + k] for k in range(n)], dtype=np.int32)
    return v, tri


def test_mirrored_list_overflow_reported_and_one_pass_form_handles_it(pk, ctx):
    # a 64 x 64 block of edge-adjacent pairs: the per-layer single layer with
    # a mirror would list 8192 pairs in a 4096-slot list -> BEM_EUNSUPPORTED;
    # the one-pass form lists each pair once and matches the oracle
    import torch
    v, tri = _book(128)
    mesh = pk.Mesh(torch.from_numpy(v), torch.from_numpy(tri))
    rows = np.arange(64, dtype=np.int32)
    cols = np.arange(64, 128, dtype=np.int32)
    blocks = pk.Blocks(np.array([0, 64], np.int32), rows, np.array([0, 64], np.int32), cols,
                       np.array([0], np.int64), np.array([4096], np.int64))
    op = pk.make_op(pk.LAPLACE, pk.SLP, q_regular=3, q_singular=3)
    out = torch.full((8192,), float("nan"), dtype=torch.float64, device="cuda")
    ctx.assemble_nearfield(mesh, op, blocks, out)
    with pytest.raises(pk.BemError) as e:
        ctx.check()
    assert e.value.code == pk.BEM_EUNSUPPORTED
    s, d = _both(pk, ctx, mesh, op, blocks, 8192)
    S = s[:4096].reshape(64, 64).T  # column-major (rows x cols)
    Sm = s[4096:].reshape(64, 64).T  # transposed block (cols x rows)
    D, Dm = d[:4096].reshape(64, 64).T, d[4096:].reshape(64, 64).T
    r, c = rows[::9], cols[::9]
    for layer, blk, mir in ((0, S, Sm), (1, D, Dm)):
        ref = oracle.block(v, tri, r, c, **_kw(op, layer)).real
        _close(blk[np.ix_(r, c - 64)], ref)
        ref_t = oracle.block(v, tri, c, r, **_kw(op, layer)).real
        _close(mir[np.ix_(c - 64, r)], ref_t)


@pytest.mark.parametrize("n,kernel,kappa", [(32, 0, 0.0), (16, 1, 4.0)])
def test_both_mixed_form(pk, ctx, n, kernel, kappa):
    import torch
    from paper_1510_07244_amd.h2 import H2Setup
    m = octahedron_sphere(n)
    h = H2Setup(ctx, m.v, m.tri, kernel=kernel, kappa=kappa, q_regular=4, q_singular=4)
    half, total = h.near_blocks(mirror=True)
    full, _ = h.near_blocks()
    ops = []
    for layer in (pk.SLP, pk.DLP):
        op = h.op(layer)
        op.precision, op.near_singular_ratio = pk.MIXED, 0.5
        ops.append(op)
    s, d = _both(pk, ctx, h.mesh, ops[0], half, total)
    assert s.dtype == (np.complex64 if kernel else np.float32)
    rows = [h.ct.idx(t) for t, _ in h.near]
    cols = [h.ct.idx(u) for _, u in h.near]
    per_layer = []
    for op in ops:
        ref = torch.full((total,), float("nan"), dtype=pk.out_dtype(op), device="cuda")
        ctx.assemble_nearfield(h.mesh, op, full, ref)
        ctx.check()
        per_layer.append(_split(ref.cpu().numpy(), rows, cols))
    gs, gd = _split(s, rows, cols), _split(d, rows, cols)
    for got, ref in ((gs, per_layer[0]), (gd, per_layer[1])):
        for g, r in zip(got, ref):
            assert np.all(np.isfinite(g))
            assert np.linalg.norm(g - r) <= 1e-6 * np.linalg.norm(r)
    up = [k for k, (t, u) in enumerate(h.near) if t < u]
    lo = [k for k, (t, u) in enumerate(h.near) if t > u]
    dg = [k for k, (t, u) in enumerate(h.near) if t == u]
    pick = set()
    for ks, seed in ((up, 13), (lo, 17), (dg, 19)):
        pick |= set(sample_subset(np.asarray(ks), min(3, len(ks)), seed=seed).tolist())
    for k in sorted(pick):
        for layer, got in ((0, gs), (1, gd)):
            ref = oracle.block(m.v, m.tri, rows[k], cols[k], **_kw(ops[0], layer))
            ref = ref if kernel == pk.HELMHOLTZ else ref.real
            assert np.linalg.norm(got[k] - ref) <= 1e-6 * np.linalg.norm(ref)


def test_phases_on_four_streams_equal_one_stream_bitwise(pk, ctx):
    # the step's independent phases (bases, near field of both layers, SLP
    # and DLP coupling) on four streams, each through its own context, give
    # the same bits as on one stream: every entry is written once by the
    # same kernel, whatever else runs beside it
    import torch
    from paper_1510_07244_amd.h2 import H2Setup
    m = octahedron_sphere(16)
    h = H2Setup(ctx, m.v, m.tri, kernel=pk.LAPLACE, q_regular=4, q_singular=4)
    V, W = h.bases((0, 1))
    half, total = h.near_blocks(mirror=True)
    cs, n_cs = h.coupling_blocks(V, V, mirror=True)
    cd, n_cd = h.coupling_blocks(V, W)
    slp, dlp = h.op(pk.SLP), h.op(pk.DLP)
    f64 = dict(dtype=torch.float64, device="cuda")

    def run(ctxs, streams):
        o = [torch.full((n,), float("nan"), **f64) for n in (total, total, n_cs, n_cd)]
        c0, c1, c2, c3 = ctxs
        s0, s1, s2, s3 = streams
        c3.assemble_coupling(h.mesh, dlp, cd, o[3], s3)
        c2.assemble_coupling(h.mesh, slp, cs, o[2], s2)
        c1.assemble_nearfield_both(h.mesh, slp, half, o[0], o[1], s1)
        h.basis_replay(V, s0)
        h.basis_replay(W, s0)
        torch.cuda.synchronize()
        for c, s in zip(ctxs, streams):
            c.check(s)
        return [x.cpu().numpy() for x in o] + [V.replay.V.cpu().numpy(), W.replay.V.cpu().numpy()]

    main = torch.cuda.current_stream()
    one = run([ctx] * 4, [main] * 4)
    extra = [pk.Context(0) for _ in range(3)]
    try:
        four = run([ctx] + extra, [torch.cuda.Stream() for _ in range(4)])
    finally:
        for c in extra:
            c.close()
    for a, b in zip(one, four):
        assert np.all(np.isfinite(a))
        assert np.array_equal(a, b)


def test_both_empty_ragged_and_tri7(pk, ctx):
    import torch
    m = octahedron_sphere(4)
    mesh = pk.Mesh(torch.from_numpy(m.v), torch.from_numpy(m.tri))
    op = pk.make_op(pk.LAPLACE, pk.SLP, regular_rule=pk.RULE_TRI7, q_singular=3)
    # blocks without entries write nothing and succeed
    empty, total0 = pk.Blocks.from_lists([np.arange(0), np.arange(3)], [np.arange(4), np.arange(0)])
    z = torch.zeros(0, dtype=torch.float64, device="cuda")
    ctx.assemble_nearfield_both(mesh, op, empty, z, torch.zeros(0, dtype=torch.float64, device="cuda"))
    ctx.check()
    assert total0 == 0
    # blocks with no rows or no columns between ragged ones
    idx = np.arange(m.nt, dtype=np.int32)
    rows = [idx[3:70], idx[:0], idx[100:101], idx[7:128]]
    cols = [idx[50:128], idx[5:9], idx[:0], idx[0:1]]
    blocks, total = pk.Blocks.from_lists(rows, cols)
    s, d = _both(pk, ctx, mesh, op, blocks, total)
    for layer, res in ((0, s), (1, d)):
        got = _split(res, rows, cols)
        for g, r, c in zip(got, rows, cols):
            if r.size and c.size:
                _close(g, oracle.block(m.v, m.tri, r, c, **_kw(op, layer)).real)
