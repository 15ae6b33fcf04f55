"""GPU tests of the learned form (order selector).

* Network kernels against the FP64 oracle: FP32 forward (1e-5), FP16 matrix
  core inference (3e-2 of the output range), mean-squared-error gradient
  (1e-4 relative, ragged sample count), Adam step (1e-6).
* Training samples (inputs 1e-6, targets 1e-3 in log10 units where the
  error is above rounding) against the oracle's inputs and targets.
* Order selection: the fused kernel equals stored inputs -> FP16 inference
  -> the decision rule taken in FP32, entry by entry.
* Per-entry order assembly: plain order everywhere = the plain kernel bit
  for bit; forced mixed orders = the oracle at each entry's order (1e-12).
* Gain: a selector trained on GPU-generated pairs keeps every sampled
  near-field block of the 8192-triangle sphere within 1e-6 relative
  Frobenius error of the plain-order oracle while spending fewer quadrature
  points than the plain rule.
"""
import numpy as np
import pytest

import oracle
from bem_inputs import octahedron_sphere, sample_subset
from oracle import htree, mlp, selector

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


def _dev(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    return t.to(device="cuda", dtype=dtype) if dtype else t.cuda()


def _problem(n_out, n, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    p = mlp.init(n_out, seed, mu=rng.normal(size=8) * 0.3, sigma=rng.uniform(0.5, 2.0, size=8))
    x = rng.normal(size=(n, 8))
    t = rng.normal(size=(n, n_out))
    return p.astype(np.float32), x.astype(np.float32), t.astype(np.float32)


@pytest.mark.parametrize("n_out", [6, 1])
def test_forward_fp32_and_fp16(pk, ctx, n_out):
    import torch
    p, x, _ = _problem(n_out, 1000, 5)
    ref, _ = mlp.forward(p.astype(np.float64), x.astype(np.float64), n_out)
    y = torch.empty((1000, n_out), dtype=torch.float32, device="cuda")
    ctx.mlp_forward(n_out, _dev(p), _dev(x), y, fp16=False)
    ctx.check()
    assert np.abs(y.cpu().numpy() - ref).max() <= 1e-5 * np.abs(ref).max()
    y.fill_(float("nan"))
    ctx.mlp_forward(n_out, _dev(p), _dev(x), y, fp16=True)
    ctx.check()
    err = np.abs(y.cpu().numpy() - ref).max()
    assert err <= 3e-2 * np.abs(ref).max(), err


@pytest.mark.parametrize("n_out,n", [(6, 1000), (6, 16), (1, 333)])
def test_gradient_matches_oracle(pk, ctx, n_out, n):
    import torch
    p, x, t = _problem(n_out, n, 11)
    g_ref, L_ref = mlp.grad(p.astype(np.float64), x.astype(np.float64), t.astype(np.float64), n_out)
    g = torch.full((p.size,), float("nan"), dtype=torch.float32, device="cuda")
    L = torch.zeros(1, dtype=torch.float32, device="cuda")
    ctx.mlp_grad(n_out, _dev(p), _dev(x), _dev(t), g, L)
    ctx.check()
    g = g.cpu().numpy()
    assert np.linalg.norm(g - g_ref) <= 1e-4 * np.linalg.norm(g_ref)
    assert float(L.cpu()) == pytest.approx(L_ref, rel=1e-5)
    # deterministic: a second call gives the same bits
    g2 = torch.empty_like(torch.from_numpy(g)).cuda()
    ctx.mlp_grad(n_out, _dev(p), _dev(x), _dev(t), g2, None)
    ctx.check()
    assert np.array_equal(g2.cpu().numpy().view(np.uint32), g.view(np.uint32))


def test_adam_matches_oracle(pk, ctx):
    rng = np.random.Generator(np.random.PCG64(2))
    p, g, m, v = (rng.normal(size=500).astype(np.float32) for _ in range(4))
    v = np.abs(v)
    P, M, V = _dev(p), _dev(m), _dev(v)
    ctx.mlp_adam(P, _dev(g), M, V, 7, 1e-3)
    ctx.check()
    p1, m1, v1 = mlp.adam(p.astype(np.float64), g.astype(np.float64), m.astype(np.float64),
                          v.astype(np.float64), 7, 1e-3)
    # FP32 against FP64: relative 1e-6 plus an absolute 1e-6 for values
    # that cancel to near zero (m = 0.9 m + 0.1 g)
    assert np.allclose(P.cpu().numpy(), p1, rtol=1e-6, atol=1e-6)
    assert np.allclose(M.cpu().numpy(), m1, rtol=1e-6, atol=1e-6)
    assert np.allclose(V.cpu().numpy(), v1, rtol=1e-6, atol=1e-6)


@pytest.mark.parametrize("kernel,layer,kappa", [(0, 0, 0.0), (0, 1, 0.0), (1, 1, 4.0)])
def test_samples_match_oracle(pk, ctx, kernel, layer, kappa):
    import torch
    from paper_1510_07244_amd.selector import near_pairs
    m = octahedron_sphere(16)
    r, c = near_pairs(m.v, m.tri, 300, seed=kernel * 10 + layer)
    op = pk.make_op(kernel, layer, kappa=kappa)
    mesh = pk.Mesh(torch.from_numpy(m.v), torch.from_numpy(m.tri))
    x = torch.empty((r.size, 8), dtype=torch.float32, device="cuda")
    t = torch.empty((r.size, 6), dtype=torch.float32, device="cuda")
    ctx.selector_samples(mesh, op, _dev(r), _dev(c), x, t)
    ctx.check()
    fx = selector.features(m.v, m.tri, r, c, layer=layer, kappa=kappa)
    assert np.allclose(x.cpu().numpy(), fx, rtol=1e-6, atol=1e-6)
    ft = selector.targets(m.v, m.tri, r, c, kernel=kernel, layer=layer, kappa=kappa)
    got = t.cpu().numpy()
    # where the error is well above the rounding of the order-8 sum (whose
    # summation order differs between the two sides)
    sel = ft > -10
    assert np.abs(got[sel] - ft[sel]).max() <= 2e-3
    assert np.all(got >= -16.0001) and np.all(np.isfinite(got))


def _near(pk, m, nblocks, seed):
    cl = htree.cluster_tree(m.v, m.tri, 64)
    near, _ = htree.block_tree(cl, 2.0)
    pick = [near[k] for k in sample_subset(np.arange(len(near)), nblocks, seed=seed)]
    pick += [b for b in near if b[0] == b[1]][:2]
    rows = [cl[t].idx for t, s in pick]
    cols = [cl[s].idx for t, s in pick]
    blocks, total = pk.Blocks.from_lists(rows, cols)
    return rows, cols, blocks, total


def test_select_orders_equals_inference_and_rule(pk, ctx):
    import torch
    m = octahedron_sphere(16)
    mesh = pk.Mesh(torch.from_numpy(m.v), torch.from_numpy(m.tri))
    rows, cols, blocks, total = _near(pk, m, 5, 3)
    # an untrained network with a spread of outputs around the threshold
    p, _, _ = _problem(6, 1, 21)
    p[16 + 64 * 8 + 64 + 2 * (64 * 64 + 64) + 64 * 6:] = -7.0  # output biases near log10 tol
    P = _dev(p)
    op = pk.make_op(pk.LAPLACE, pk.SLP, q_regular=4)
    orders = torch.full((total,), -1, dtype=torch.int8, device="cuda")
    ctx.select_orders(mesh, op, blocks, P, orders, 1e-7, 0.5, 2)
    ctx.check()
    got = orders.cpu().numpy()
    # the same pairs through stored inputs, FP16 inference and the rule in FP32
    R = np.concatenate([np.tile(r, len(c)) for r, c in zip(rows, cols)]).astype(np.int32)
    C = np.concatenate([np.repeat(c, len(r)) for r, c in zip(rows, cols)]).astype(np.int32)
    sing = np.array([oracle.shared_vertices(m.tri, i, j) > 0 for i, j in zip(R, C)])
    assert np.all(got[sing] == 0)
    reg = np.nonzero(~sing)[0]
    x = torch.empty((reg.size, 8), dtype=torch.float32, device="cuda")
    t = torch.empty((reg.size, 6), dtype=torch.float32, device="cuda")
    ctx.selector_samples(mesh, op, _dev(R[reg]), _dev(C[reg]), x, t)
    y = torch.empty((reg.size, 6), dtype=torch.float32, device="cuda")
    ctx.mlp_forward(6, P, x, y, fp16=True)
    ctx.check()
    pred = y.cpu().numpy()
    lt = np.float32(np.log10(1e-7))
    want = np.full(reg.size, 4)
    run = np.ones(reg.size, dtype=bool)
    for q in (3, 2):
        run &= (pred[:, q - 1] + np.float32(0.5)).astype(np.float32) <= lt
        want[run] = q
    assert np.array_equal(got[reg], want)
    assert len(set(want.tolist())) > 1  # the case exercises more than one order


def test_learned_kernel_plain_orders_bitwise(pk, ctx):
    import torch
    for kernel, layer, q, kappa in ((0, 0, 4, 0.0), (0, 1, 4, 0.0), (1, 0, 5, 4.0)):
        m = octahedron_sphere(16)
        mesh = pk.Mesh(torch.from_numpy(m.v), torch.from_numpy(m.tri))
        rows, cols, blocks, total = _near(pk, m, 4, 7)
        op = pk.make_op(kernel, layer, q_regular=q, q_singular=4, kappa=kappa)
        ref = torch.full((total,), float("nan"), dtype=pk.out_dtype(op), device="cuda")
        ctx.assemble_nearfield(mesh, op, blocks, ref)
        orders = torch.full((total,), q, dtype=torch.int8, device="cuda")
        out = torch.full_like(ref, float("nan"))
        ctx.assemble_nearfield_learned(mesh, op, blocks, orders, out)
        ctx.check()
        a = torch.view_as_real(out).cpu().numpy() if out.is_complex() else out.cpu().numpy()
        b = torch.view_as_real(ref).cpu().numpy() if ref.is_complex() else ref.cpu().numpy()
        assert np.array_equal(a.view(np.uint64), b.view(np.uint64)), (kernel, layer)


def test_learned_kernel_forced_orders_vs_oracle(pk, ctx):
    import torch
    m = octahedron_sphere(16)
    mesh = pk.Mesh(torch.from_numpy(m.v), torch.from_numpy(m.tri))
    rows, cols, blocks, total = _near(pk, m, 4, 9)
    rng = np.random.Generator(np.random.PCG64(3))
    q_map = rng.integers(2, 5, size=total).astype(np.int8)
    for layer in (0, 1):
        op = pk.make_op(pk.LAPLACE, layer, q_regular=4, q_singular=4)
        out = torch.full((total,), float("nan"), dtype=torch.float64, device="cuda")
        ctx.assemble_nearfield_learned(mesh, op, blocks, _dev(q_map), out)
        ctx.check()
        res = out.cpu().numpy()
        off = 0
        for r, c in zip(rows, cols):
            n = len(r) * len(c)
            got = res[off:off + n].reshape(len(c), len(r)).T
            qb = q_map[off:off + n].reshape(len(c), len(r)).T
            off += n
            want = np.zeros_like(got)
            for q in (2, 3, 4):
                blk = oracle.block(m.v, m.tri, r, c, layer=layer, q_reg=q, q_sing=4).real
                want[qb == q] = blk[qb == q]
            sing = np.array([[oracle.shared_vertices(m.tri, i, j) > 0 for j in c] for i in r])
            want[sing] = oracle.block(m.v, m.tri, r, c, layer=layer, q_reg=4, q_sing=4).real[sing]
            assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()


def test_invalid_order_is_flagged_and_left_unwritten(pk, ctx):
    import torch
    m = octahedron_sphere(8)
    mesh = pk.Mesh(torch.from_numpy(m.v), torch.from_numpy(m.tri))
    rows, cols, blocks, total = _near(pk, m, 1, 1)
    op = pk.make_op(pk.LAPLACE, pk.SLP, q_regular=4)
    orders = torch.full((total,), 4, dtype=torch.int8, device="cuda")
    orders[total // 2] = 7
    out = torch.zeros(total, dtype=torch.float64, device="cuda")
    ctx.assemble_nearfield_learned(mesh, op, blocks, orders, out)
    with pytest.raises(pk.BemError) as ei:
        ctx.check()
    assert ei.value.code == pk.BEM_EINVAL


def test_trained_selector_gain(pk, ctx):
    """Training on GPU-generated pairs, then the gain over the plain rule on
    the 8192-triangle sphere at the 1e-6 block bar."""
    import torch
    from paper_1510_07244_amd.selector import Selector, samples
    jobs = []
    for n, cnt in ((8, 20000), (16, 40000), (32, 60000)):
        m = octahedron_sphere(n)
        for layer in (0, 1):
            jobs.append((m.v, m.tri, pk.make_op(pk.LAPLACE, layer), cnt, 100 * n + layer))
    X, T = samples(ctx, jobs)
    sel = Selector(ctx, seed=1)
    sel.set_standardisation(X)
    losses = sel.fit(X, T, epochs=12, batch=2048, lr=2e-3, seed=2)
    assert losses[-1] < 0.2 * losses[0], losses
    m = octahedron_sphere(32)
    mesh = pk.Mesh(torch.from_numpy(m.v), torch.from_numpy(m.tri))
    rows, cols, blocks, total = _near(pk, m, 12, 5)
    saved_points = {1: 0, 4: 0}
    plain_points = 0
    for layer in (0, 1):
        op = pk.make_op(pk.LAPLACE, layer, q_regular=4, q_singular=4)
        refs = [oracle.block(m.v, m.tri, r, c, layer=layer, q_reg=4, q_sing=4).real
                for r, c in zip(rows, cols)]
        for group in (1, 4):  # entry by entry, and runs of four rows
            orders = sel.orders(mesh, op, blocks, total, tol=1e-7, margin=0.5, group=group)
            out = torch.full((total,), float("nan"), dtype=torch.float64, device="cuda")
            ctx.assemble_nearfield_learned(mesh, op, blocks, orders, out)
            ctx.check()
            q = orders.cpu().numpy().astype(np.int64)
            reg = q > 0
            if group == 1:
                plain_points += int(reg.sum()) * 4 ** 4
            saved_points[group] += int((4 ** 4 - q[reg] ** 4).sum())
            res = out.cpu().numpy()
            off = 0
            for (r, c), ref in zip(zip(rows, cols), refs):
                n = len(r) * len(c)
                got = res[off:off + n].reshape(len(c), len(r)).T
                qb = q[off:off + n].reshape(len(c), len(r)).T
                off += n
                err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
                assert err <= 1e-6, (layer, group, err)
                # a run of `group` rows (sub-tiles of 64 rows) of a column
                # shares one order among its pairs without a common vertex
                for r0 in range(0, len(r), group):
                    run = qb[r0:min(r0 + group, (r0 // 64 + 1) * 64)]
                    for col in run.T:
                        assert len(set(col[col > 0].tolist())) <= 1
    assert saved_points[1] >= 0.2 * plain_points, (saved_points, plain_points)
    assert saved_points[4] >= 0.1 * plain_points, (saved_points, plain_points)
    # outside the training range (these Laplace samples all have kappa D = 0)
    # the plain order is kept for every pair, whatever the network predicts
    oph = pk.make_op(pk.HELMHOLTZ, pk.SLP, q_regular=4, q_singular=4, kappa=30.0)
    guarded = sel.orders(mesh, oph, blocks, total, tol=1e-7, margin=0.5).cpu().numpy()
    free = sel.orders(mesh, oph, blocks, total, tol=1e-7, margin=0.5, guard=False).cpu().numpy()
    reg = guarded > 0
    assert np.array_equal(reg, free > 0)
    assert np.all(guarded[reg] == 4)
    # on the mesh the network was trained on, the guard changes only the
    # few pairs beyond the sampled extremes, and only by raising orders
    opl = pk.make_op(pk.LAPLACE, pk.DLP, q_regular=4, q_singular=4)
    a = sel.orders(mesh, opl, blocks, total, tol=1e-7, margin=0.5).cpu().numpy()
    b = sel.orders(mesh, opl, blocks, total, tol=1e-7, margin=0.5, guard=False).cpu().numpy()
    assert (a == b).mean() >= 0.99 and np.all(a >= b) and np.any(a[a > 0] < 4)


def test_mlp_save_load_resumes_training_bitwise(pk, ctx, tmp_path):
    """Training resumed from a saved file (parameters, Adam moments, step)
    equals training that was never interrupted, bit for bit; a file without
    moments refuses a request for them."""
    import torch
    rng = np.random.Generator(np.random.PCG64(17))
    n_out, n = 6, 1000
    X = torch.from_numpy(rng.standard_normal((n, 8)).astype(np.float32)).cuda()
    T = torch.from_numpy(rng.standard_normal((n, n_out)).astype(np.float32)).cuda()
    np_ = pk.mlp_params(n_out)
    P0 = torch.from_numpy((0.1 * rng.standard_normal(np_)).astype(np.float32)).cuda()
    P0[8:16] = 1.0
    rg = torch.from_numpy(np.concatenate([-np.ones(8), np.ones(8)]).astype(np.float32)).cuda()

    def steps(P, m, v, first, count):
        g = torch.zeros_like(P)
        for k in range(first, first + count):
            ctx.mlp_grad(n_out, P, X, T, g)
            ctx.mlp_adam(P, g, m, v, k, 1e-3)

    P, m, v = P0.clone(), torch.zeros_like(P0), torch.zeros_like(P0)
    steps(P, m, v, 1, 5)
    path = str(tmp_path / "net.bin")
    ctx.mlp_save(path, n_out, P, m, v, range=rg, step=5)
    steps(P, m, v, 6, 5)  # uninterrupted
    P2, m2, v2 = (torch.full_like(P0, float("nan")) for _ in range(3))
    rg2 = torch.full_like(rg, float("nan"))
    step = ctx.mlp_load(path, n_out, P2, m2, v2, range=rg2)
    assert step == 5 and torch.equal(rg2, rg)
    steps(P2, m2, v2, step + 1, 5)  # resumed
    torch.cuda.synchronize()
    for a, b in ((P, P2), (m, m2), (v, v2)):
        assert np.array_equal(a.cpu().numpy().view(np.uint32), b.cpu().numpy().view(np.uint32))
    bare = str(tmp_path / "bare.bin")
    ctx.mlp_save(bare, n_out, P)
    with pytest.raises(pk.BemError) as e:
        ctx.mlp_load(bare, n_out, P2, m2, v2)
    assert e.value.code == pk.BEM_EINVAL
    with pytest.raises(pk.BemError) as e:
        ctx.mlp_load(path, 1, P2)  # another n_out
    assert e.value.code == pk.BEM_EINVAL


def test_learned_coupling_keeps_h2_accuracy(pk, ctx):
    """Orders chosen per entry of the coupling blocks (pivot lists of the
    admissible blocks) by a network trained on near-field and admissible
    pairs: the H2 blocks V_t S W_s^T of the 8192-triangle sphere stay within
    1e-6 of the dense oracle, the coupling matrices within 1e-6 of the plain
    ones, with far fewer quadrature points."""
    import torch
    from h2util import FullBases, coupling_matrix, coupling_offsets
    from paper_1510_07244_amd.h2 import H2Setup
    from paper_1510_07244_amd.selector import Selector, samples
    jobs = []
    for n, cnt in ((8, 20000), (16, 40000), (32, 60000)):
        m = octahedron_sphere(n)
        for layer in (0, 1):
            jobs.append((m.v, m.tri, pk.make_op(pk.LAPLACE, layer), cnt, 100 * n + layer))
            if n > 8:  # the 512-triangle sphere has no admissible blocks
                jobs.append((m.v, m.tri, pk.make_op(pk.LAPLACE, layer), cnt // 2,
                             300 * n + layer, "far"))
    X, T = samples(ctx, jobs)
    sel = Selector(ctx, seed=1)
    sel.set_standardisation(X)
    sel.fit(X, T, epochs=12, batch=2048, lr=2e-3, seed=2)
    m = octahedron_sphere(32)
    h = H2Setup(ctx, m.v, m.tri)
    V, W = h.bases((0, 1))
    for layer, B in ((pk.SLP, V), (pk.DLP, W)):
        op = h.op(layer)
        blocks, total = h.coupling_blocks(V, B)
        plain = torch.empty(total, dtype=torch.float64, device="cuda")
        ctx.assemble_coupling(h.mesh, op, blocks, plain)
        orders = sel.orders(h.mesh, op, blocks, total, tol=1e-7, margin=0.5)
        learned = torch.full_like(plain, float("nan"))
        ctx.assemble_nearfield_learned(h.mesh, op, blocks, orders, learned)
        ctx.check()
        q = orders.cpu().numpy().astype(np.int64)
        assert q.min() >= 2 and q.max() <= 4
        saved = 1.0 - float((q ** 4).sum()) / (q.size * 4 ** 4)
        assert saved >= 0.5, saved  # admissible pairs are far apart
        P, L = plain.cpu().numpy(), learned.cpu().numpy()
        offs, _ = coupling_offsets(h, V, B)
        Vf, Bf = FullBases(h, V), FullBases(h, B)
        for k in sample_subset(np.arange(len(h.far)), 25, seed=7 + layer):
            t, s = h.far[k]
            kt, ks = V.piv[t].size, B.piv[s].size
            Sp = coupling_matrix(P, offs[k], kt, ks)
            Sl = coupling_matrix(L, offs[k], kt, ks)
            assert np.linalg.norm(Sl - Sp) <= 1e-6 * np.linalg.norm(Sp), (layer, k)
            ref = oracle.block(m.v, m.tri, h.ct.idx(t), h.ct.idx(s), layer=layer, q_reg=4,
                               q_sing=4).real
            err = np.linalg.norm(Vf(t) @ Sl @ Bf(s).T - ref) / np.linalg.norm(ref)
            assert err <= 1e-6, (layer, k, err)
