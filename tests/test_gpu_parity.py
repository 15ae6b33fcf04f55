"""GPU parity: the HIP path through the C-ABI against the FP64 oracle.

Tolerance (FP64 path): per compared set, ||G_gpu - G_oracle||_F <= 1e-12
||G_oracle||_F and max |G_gpu - G_oracle| <= 1e-12 max |G_oracle|.  Block
lists come from the oracle's own cluster / block tree; pivot lists are seeded
random subsets of admissible cluster pairs (no input comes from the HIP path).
The Helmholtz path at kappa = 0 reproduces the Laplace path (imaginary parts
exactly zero).
"""
import numpy as np
import pytest

import oracle
from bem_inputs import cube_surface, octahedron_sphere, sample_pairs, sample_subset
from oracle import htree

pytestmark = pytest.mark.gpu

TOL = 1e-12


def _close(got, ref, tol=TOL):
    got = np.asarray(got)
    ref = np.asarray(ref)
    fro = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    ent = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
    assert np.all(np.isfinite(got))
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


def _op_kw(op):
    return dict(kernel=op.kernel, layer=op.layer, kappa=op.kappa, rule=op.regular_rule,
                q_reg=op.q_regular, q_sing=op.q_singular)


def _assemble(pk, ctx, m, op, rows, cols, coupling=False):
    import torch
    mesh = pk.Mesh(torch.from_numpy(m.v), torch.from_numpy(m.tri))
    blocks, total = pk.Blocks.from_lists(rows, cols)
    out = torch.full((total,), float("nan"), dtype=pk.out_dtype(op), device="cuda")
    (ctx.assemble_coupling if coupling else ctx.assemble_nearfield)(mesh, op, blocks, out)
    ctx.check()
    res = out.cpu().numpy()
    outs, o = [], 0
    for r, c in zip(rows, cols):
        outs.append(res[o:o + len(r) * len(c)].reshape(len(c), len(r)).T)  # column-major
        o += len(r) * len(c)
    return outs


def _near_lists(m, leaf=64):
    cl = htree.cluster_tree(m.v, m.tri, leaf=leaf)
    near, far = htree.block_tree(cl, eta=2.0)
    return cl, near, far


# --------------------------------------------------------- dense workloads
def test_dense_sphere512_laplace_slp_tri7_ss3(pk, ctx):
    """512-triangle sphere, dense: 7-point rule regular, Sauter-Schwab order 3."""
    m = octahedron_sphere(8)
    op = pk.make_op(pk.LAPLACE, pk.SLP, regular_rule=pk.RULE_TRI7, q_regular=3, q_singular=3)
    cl, near, far = _near_lists(m)
    assert len(far) == 0 and len(near) == 64
    rows = [cl[t].idx for t, s in near]
    cols = [cl[s].idx for t, s in near]
    got = _assemble(pk, ctx, m, op, rows, cols)
    full = oracle.block(m.v, m.tri, np.arange(m.nt), np.arange(m.nt), **_op_kw(op))
    for g, r, c in zip(got, rows, cols):
        _close(g, full[np.ix_(r, c)].real)


@pytest.mark.parametrize("kernel,layer,kappa,q", [
    (0, 1, 0.0, 4), (1, 0, 2.0, 4), (1, 1, 4.0, 4), (1, 0, 8.0, 5), (1, 1, 8.0, 5),
    (0, 0, 0.0, 2), (0, 0, 0.0, 6), (0, 1, 0.0, 7), (0, 0, 0.0, 1),
])
def test_dense_small_sphere_all_kernels(pk, ctx, kernel, layer, kappa, q):
    m = octahedron_sphere(4)  # 128 triangles
    op = pk.make_op(kernel, layer, q_regular=q, q_singular=q, kappa=kappa)
    idx = np.arange(m.nt, dtype=np.int32)
    # one ragged block larger than every sub-tile, plus a small ragged one
    rows = [idx, idx[5:42]]
    cols = [idx, idx[17:100]]
    got = _assemble(pk, ctx, m, op, rows, cols)
    full = oracle.block(m.v, m.tri, idx, idx, **_op_kw(op))
    ref = full if kernel == pk.HELMHOLTZ else full.real
    _close(got[0], ref)
    _close(got[1], ref[np.ix_(rows[1], cols[1])])


def test_cube_dlp_coplanar_entries_are_zero(pk, ctx):
    m = cube_surface(2)
    op = pk.make_op(pk.LAPLACE, pk.DLP, q_regular=4, q_singular=4)
    idx = np.arange(m.nt, dtype=np.int32)
    got = _assemble(pk, ctx, m, op, [idx], [idx])[0]
    ref = oracle.block(m.v, m.tri, idx, idx, **_op_kw(op)).real
    assert np.all(np.isfinite(got))
    zero = ref == 0.0
    assert zero.sum() > 0
    assert np.max(np.abs(got[zero])) <= 1e-15 * np.max(np.abs(ref))
    _close(got, ref)


# --------------------------------------------------- full-size near field
@pytest.mark.parametrize("layer", [0, 1])
def test_sphere8192_nearfield_full_call_sampled(pk, ctx, layer):
    """All 2400 near blocks of the 8192-triangle sphere in one call (the
    benchmark's launch), checked on a seeded sample of blocks and on every
    singular pair class."""
    m = octahedron_sphere(32)
    op = pk.make_op(pk.LAPLACE, layer, q_regular=4, q_singular=4)
    cl, near, _ = _near_lists(m)
    rows = [cl[t].idx for t, s in near]
    cols = [cl[s].idx for t, s in near]
    got = _assemble(pk, ctx, m, op, rows, cols)
    pick = sample_subset(np.arange(len(near)), 24, seed=11)
    diag = [k for k, (t, s) in enumerate(near) if t == s][:4]
    for k in sorted(set(pick.tolist()) | set(diag)):
        ref = oracle.block(m.v, m.tri, rows[k], cols[k], **_op_kw(op)).real
        _close(got[k], ref)


def test_helmholtz_sphere_q5_blocks(pk, ctx):
    m = octahedron_sphere(16)
    op = pk.make_op(pk.HELMHOLTZ, pk.DLP, q_regular=5, q_singular=5, kappa=8.0)
    cl, near, _ = _near_lists(m)
    pick = [near[k] for k in sample_subset(np.arange(len(near)), 10, seed=3)]
    pick += [b for b in near if b[0] == b[1]][:2]
    rows = [cl[t].idx for t, s in pick]
    cols = [cl[s].idx for t, s in pick]
    got = _assemble(pk, ctx, m, op, rows, cols)
    for g, r, c in zip(got, rows, cols):
        _close(g, oracle.block(m.v, m.tri, r, c, **_op_kw(op)))


# ------------------------------------------------------------ coupling
def test_coupling_on_pivot_lists(pk, ctx):
    m = octahedron_sphere(32)
    op = pk.make_op(pk.LAPLACE, pk.SLP, q_regular=4, q_singular=4)
    cl, _, far = _near_lists(m)
    pick = sample_subset(np.arange(len(far)), 40, seed=5)
    rows, cols = [], []
    for n, k in enumerate(pick):
        t, s = far[k]
        rows.append(sample_subset(cl[t].idx, 7 + n % 30, seed=100 + n))
        cols.append(sample_subset(cl[s].idx, 5 + (3 * n) % 40, seed=200 + n))
    got = _assemble(pk, ctx, m, op, rows, cols, coupling=True)
    for g, r, c in zip(got, rows, cols):
        _close(g, oracle.block(m.v, m.tri, r, c, **_op_kw(op)).real)


@pytest.mark.parametrize("layer", [0, 1])
@pytest.mark.parametrize("precision", [0, 1])
def test_helmholtz_at_kappa_zero_is_laplace(pk, ctx, layer, precision):
    # the Helmholtz kernels at kappa = 0 reduce to the Laplace ones: the
    # Helmholtz path (its own sine and cosine, Sauter-Schwab xi sums by the
    # rule instead of moments) gives the Laplace path's entries up to
    # rounding, with imaginary parts exactly zero; near field (every pair
    # class) and coupling lists, plain and mixed
    m = octahedron_sphere(16)
    cl, near, far = _near_lists(m)
    lap = pk.make_op(pk.LAPLACE, layer, precision=precision, q_regular=4, q_singular=4,
                     near_singular_ratio=0.5 if precision else 0.0)
    hel = pk.make_op(pk.HELMHOLTZ, layer, precision=precision, q_regular=4, q_singular=4,
                     kappa=0.0, near_singular_ratio=0.5 if precision else 0.0)
    tol = 1e-5 if precision else 1e-13
    nrows = [cl[t].idx for t, s in near[:24]]
    ncols = [cl[s].idx for t, s in near[:24]]
    pick = sample_subset(np.arange(len(far)), 12, seed=7)
    crows = [sample_subset(cl[far[k][0]].idx, 20, seed=k) for k in pick]
    ccols = [sample_subset(cl[far[k][1]].idx, 30, seed=k + 1) for k in pick]
    for rows, cols, coupling in ((nrows, ncols, False), (crows, ccols, True)):
        a = _assemble(pk, ctx, m, lap, rows, cols, coupling=coupling)
        b = _assemble(pk, ctx, m, hel, rows, cols, coupling=coupling)
        for x, y in zip(a, b):
            assert np.all(y.imag == 0.0)
            _close(y.real, x, tol)


def test_coupling_rejects_adjacent_pairs(pk, ctx):
    import torch
    m = octahedron_sphere(4)
    op = pk.make_op(pk.LAPLACE, pk.SLP)
    mesh = pk.Mesh(torch.from_numpy(m.v), torch.from_numpy(m.tri))
    blocks, total = pk.Blocks.from_lists([np.arange(10)], [np.arange(10)])
    out = torch.zeros(total, dtype=torch.float64, device="cuda")
    ctx.assemble_coupling(mesh, op, blocks, out)
    with pytest.raises(pk.BemError) as e:
        ctx.check()
    assert e.value.code == pk.BEM_EINVAL
    ctx.check()  # the flag was cleared


# ------------------------------------------------------------ entries
@pytest.mark.parametrize("kernel,layer,kappa", [(0, 0, 0.0), (0, 1, 0.0), (1, 0, 4.0), (1, 1, 2.0)])
def test_eval_entries_random_and_singular(pk, ctx, kernel, layer, kappa):
    import torch
    m = octahedron_sphere(16)
    op = pk.make_op(kernel, layer, q_regular=4, q_singular=4, kappa=kappa)
    r, c = sample_pairs(m.nt, 3000, seed=21)
    # every singular class, on several rows
    extra_r, extra_c = [], []
    for i in (0, 17, 999):
        for j in range(m.nt):
            if oracle.shared_vertices(m.tri, i, j):
                extra_r.append(i)
                extra_c.append(j)
    r = np.concatenate([r, extra_r]).astype(np.int32)
    c = np.concatenate([c, extra_c]).astype(np.int32)
    mesh = pk.Mesh(torch.from_numpy(m.v), torch.from_numpy(m.tri))
    out = torch.zeros(r.size, dtype=pk.out_dtype(op), device="cuda")
    ctx.eval_entries(mesh, op, torch.from_numpy(r).cuda(), torch.from_numpy(c).cuda(), out)
    ctx.check()
    ref = oracle.entries(m.v, m.tri, r, c, **_op_kw(op))
    got = out.cpu().numpy()
    _close(got, ref if kernel == 1 else ref.real)
    # singular entries are large: check them on their own too
    k = r.size - len(extra_r)
    _close(got[k:], (ref if kernel == 1 else ref.real)[k:])


# ------------------------------------------------------ error handling
def test_invalid_indices_flagged_not_written(pk, ctx):
    import torch
    m = octahedron_sphere(4)
    op = pk.make_op()
    mesh = pk.Mesh(torch.from_numpy(m.v), torch.from_numpy(m.tri))
    blocks, total = pk.Blocks.from_lists([np.array([0, 1, m.nt])], [np.array([3, 4])])
    out = torch.zeros(total, dtype=torch.float64, device="cuda")
    ctx.assemble_nearfield(mesh, op, blocks, out)
    with pytest.raises(pk.BemError):
        ctx.check()
    # entry list with a bad index
    rows = torch.tensor([0, -1], dtype=torch.int32, device="cuda")
    cols = torch.tensor([1, 2], dtype=torch.int32, device="cuda")
    out2 = torch.zeros(2, dtype=torch.float64, device="cuda")
    ctx.eval_entries(mesh, op, rows, cols, out2)
    with pytest.raises(pk.BemError):
        ctx.check()
    # output too small for the block list: rejected on the device, nothing written
    blocks, total = pk.Blocks.from_lists([np.arange(8)], [np.arange(8)])
    small = torch.zeros(total - 1, dtype=torch.float64, device="cuda")
    ctx.assemble_nearfield(mesh, op, blocks, small)
    with pytest.raises(pk.BemError):
        ctx.check()
    assert torch.count_nonzero(small).item() == 0


def test_host_validation(pk, ctx):
    import torch
    m = octahedron_sphere(2)
    mesh = pk.Mesh(torch.from_numpy(m.v), torch.from_numpy(m.tri))
    blocks, total = pk.Blocks.from_lists([np.arange(4)], [np.arange(4)])
    out = torch.zeros(total, dtype=torch.float64, device="cuda")
    for bad in (pk.make_op(q_regular=0), pk.make_op(q_singular=13), pk.make_op(kernel=3),
                pk.make_op(kappa=float("nan"))):
        with pytest.raises(pk.BemError) as e:
            ctx.assemble_nearfield(mesh, bad, blocks, out)
        assert e.value.code == pk.BEM_EINVAL


def test_degenerate_triangle_flagged(pk, ctx):
    import torch
    v = np.array([[0, 0, 0], [1, 0, 0], [2, 0, 0], [0, 1, 0]], dtype=np.float64)
    tri = np.array([[0, 1, 2], [0, 1, 3]], dtype=np.int32)  # first has zero area
    mesh = pk.Mesh(torch.from_numpy(v), torch.from_numpy(tri))
    blocks, total = pk.Blocks.from_lists([np.arange(2)], [np.arange(2)])
    out = torch.zeros(total, dtype=torch.float64, device="cuda")
    ctx.assemble_nearfield(mesh, pk.make_op(), blocks, out)
    with pytest.raises(pk.BemError):
        ctx.check()


def test_empty_inputs(pk, ctx):
    import torch
    m = octahedron_sphere(2)
    mesh = pk.Mesh(torch.from_numpy(m.v), torch.from_numpy(m.tri))
    op = pk.make_op()
    blocks, total = pk.Blocks.from_lists([np.arange(0), np.arange(3)], [np.arange(5), np.arange(0)])
    assert total == 0
    out = torch.zeros(0, dtype=torch.float64, device="cuda")
    ctx.assemble_nearfield(mesh, op, blocks, out)
    empty = torch.zeros(0, dtype=torch.int32, device="cuda")
    ctx.eval_entries(mesh, op, empty, empty, out)
    ctx.check()


def test_bitwise_reproducible(pk, ctx):
    import torch
    m = octahedron_sphere(16)
    op = pk.make_op(pk.HELMHOLTZ, pk.SLP, kappa=4.0)
    cl, near, _ = _near_lists(m)
    rows = [cl[t].idx for t, s in near]
    cols = [cl[s].idx for t, s in near]
    a = _assemble(pk, ctx, m, op, rows, cols)
    b = _assemble(pk, ctx, m, op, rows, cols)
    for x, y in zip(a, b):
        assert np.array_equal(np.ascontiguousarray(x).view(np.uint8),
                              np.ascontiguousarray(y).view(np.uint8))
