"""Products with the assembled H^2 matrices and the two boundary value
problems of Sec. 4, solved on the GPU (GPU tests, through the C-ABI).

* H^2 product (library grouped matrix-vector kernels): against the dense
  oracle matrix times the same seeded vector within 1e-6 (the H^2
  approximation error), Laplace SLP and DLP and Helmholtz; against the
  host evaluation of the same near-field blocks, coupling matrices and
  nested bases at 1e-12 (the kernels' arithmetic alone).  The product
  captured in a HIP graph replays the eager product bit for bit.
* Interior Dirichlet problem for the Laplace equation (Sec. 4): the Galerkin
  system V alpha = (1/2 M + K) beta for f1 = x1^2 - x3^2,
  f2 = g(x, (1.2, 1.2, 1.2)), f3 = g(x, (1, 0.25, 1)) on the octahedron
  spheres with 512, 2048 and 8192 triangles, solved by conjugate gradients:
  the Neumann data converge like O(h) to the exact ones (the error halves
  with h), and on the 512-triangle sphere the solution equals the dense
  oracle system's (numpy solve) within the H^2 and solver tolerances.  The
  solver with every step on the device (bem_cg_step, graph replays) takes
  the host-driven one's iterations to the same iterate.
* Exterior Dirichlet problem for the Helmholtz equation by the
  Brakhage-Werner formulation (Sec. 4): kappa = 3, eta = kappa, data
  f = g(x, (0, 0, 0.2)); (1/2 M + K - i eta V) w = (int f psi_i) by
  BiCGStab; the potential u = (D - i eta S) w at exterior points approaches
  f there as the mesh is refined.
"""
import numpy as np
import pytest

import oracle
from bem_inputs import octahedron_sphere, sample_subset
from h2util import FullBases, coupling_matrix, coupling_offsets

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


def _assembled(pk, ctx, m, kernel=0, kappa=0.0, q=4):
    """H2 setup of both layers as the step makes it: one-pass near field on
    the mirrored list, mirrored single-layer coupling, double-layer
    coupling; returns the setup and the two H2Matrix operators."""
    import torch
    from paper_1510_07244_amd.h2 import H2Setup
    from paper_1510_07244_amd.h2mv import H2Matrix
    h = H2Setup(ctx, m.v, m.tri, kernel=kernel, kappa=kappa, q_regular=q, q_singular=q)
    V, W = h.bases((0, 1))
    dt = torch.complex128 if kernel else torch.float64
    half, total = h.near_blocks(mirror=True)
    ns = torch.empty(total, dtype=dt, device="cuda")
    nd = torch.empty_like(ns)
    ctx.assemble_nearfield_both(h.mesh, h.op(pk.SLP), half, ns, nd)
    cs, n_cs = h.coupling_blocks(V, V, mirror=True)
    cd, n_cd = h.coupling_blocks(V, W)
    ss = torch.empty(n_cs, dtype=dt, device="cuda")
    sd = torch.empty(n_cd, dtype=dt, device="cuda")
    ctx.assemble_coupling(h.mesh, h.op(pk.SLP), cs, ss)
    ctx.assemble_coupling(h.mesh, h.op(pk.DLP), cd, sd)
    ctx.check()
    return h, H2Matrix(h, V, V, ns, ss), H2Matrix(h, V, W, nd, sd)


def _host_h2(h, M, near, coup):
    """The same H^2 product on the host, block by block (test reference of
    the kernels' arithmetic, from the same device data)."""
    Vf, Wf = FullBases(h, M.V), FullBases(h, M.W)
    nearh, couph = near.cpu().numpy(), coup.cpu().numpy()

    def mv(x):
        y = np.zeros_like(x)
        o = 0
        for t, s in h.near:
            r, c = h.ct.idx(t), h.ct.idx(s)
            G = nearh[o:o + r.size * c.size].reshape(c.size, r.size).T
            o += r.size * c.size
            y[r] += G @ x[c]
        offs, _ = coupling_offsets(h, M.V, M.W)
        for k, (t, s) in enumerate(h.far):
            S = coupling_matrix(couph, offs[k], M.V.piv[t].size, M.W.piv[s].size)
            y[h.ct.idx(t)] += Vf(t) @ (S @ (Wf(s).T @ x[h.ct.idx(s)]))
        return y
    return mv


@pytest.mark.parametrize("kernel,kappa", [(0, 0.0), (1, 4.0)])
def test_h2_matvec(pk, ctx, kernel, kappa):
    import torch
    m = octahedron_sphere(16)  # 2048 triangles: the dense oracle matrix is cheap
    h, Hv, Hk = _assembled(pk, ctx, m, kernel, kappa)
    rng = np.random.Generator(np.random.PCG64(4))
    x = rng.standard_normal(m.nt) + (1j * rng.standard_normal(m.nt) if kernel else 0)
    dt = torch.complex128 if kernel else torch.float64
    xd = torch.from_numpy(x).to(device="cuda", dtype=dt)
    every = np.arange(m.nt)
    for layer, H in ((0, Hv), (1, Hk)):
        y = torch.full_like(xd, float("nan"))
        H.matvec(xd, y)
        ctx.check()
        got = y.cpu().numpy()
        host = _host_h2(h, H, H.near, H.coupling)(x)
        assert np.linalg.norm(got - host) <= 1e-12 * np.linalg.norm(host), layer
        G = oracle.block(m.v, m.tri, every, every, kernel=kernel, kappa=kappa, layer=layer,
                         q_reg=4, q_sing=4)
        ref = G @ x
        ref = ref if kernel else ref.real
        assert np.linalg.norm(got - ref) <= 1e-6 * np.linalg.norm(ref), layer
        # accumulate mode adds to what y holds
        H.matvec(xd, y, accumulate=True)
        ctx.check()
        assert np.allclose(y.cpu().numpy(), 2 * got, rtol=0, atol=1e-13 * np.abs(got).max())


@pytest.mark.parametrize("kernel,kappa", [(0, 0.0), (1, 4.0)])
def test_h2_matvec_graph_replays_match_eager(pk, ctx, kernel, kappa):
    # the product captured in a HIP graph (near field on a second stream
    # inside the capture): every replay, with eager work and
    # synchronisations between replays, gives the eager product bit for bit
    import torch
    from paper_1510_07244_amd.h2mv import GraphedMatvec
    m = octahedron_sphere(16)
    h, Hv, Hk = _assembled(pk, ctx, m, kernel, kappa)
    rng = np.random.Generator(np.random.PCG64(9))
    x = rng.standard_normal(m.nt) + (1j * rng.standard_normal(m.nt) if kernel else 0)
    dt = torch.complex128 if kernel else torch.float64
    xd = torch.from_numpy(x).to(device="cuda", dtype=dt)
    view = (lambda t: torch.view_as_real(t).cpu().numpy()) if kernel else (lambda t: t.cpu().numpy())
    for H in (Hv, Hk):
        ref = torch.empty_like(xd)
        H.matvec(xd, ref)
        ctx.check()
        want = view(ref).view(np.uint64)
        G = GraphedMatvec(H)
        y = torch.empty_like(xd)
        for rep in range(4):
            y.fill_(float("nan"))  # eager work between replays
            torch.cuda.synchronize()
            G(xd, y)
            ctx.check()
            assert np.array_equal(view(y).view(np.uint64), want), rep
        assert len(G.graphs) == 1
        # another buffer pair gets its own graph; the first one still replays
        y2 = torch.empty_like(xd)
        G(xd, y2)
        G(xd, y)
        ctx.check()
        assert len(G.graphs) == 2
        assert np.array_equal(view(y2).view(np.uint64), want)
        assert np.array_equal(view(y).view(np.uint64), want)


def test_h2_matvec_sphere8192_deterministic(pk, ctx):
    # on the 8192-triangle sphere some inadmissible blocks have a father as
    # row cluster (the column cluster is a leaf): their rows overlap the
    # sons' blocks; the product stays reproducible bit for bit and equal to
    # the host evaluation of the same factors
    import torch
    m = octahedron_sphere(32)
    h, Hv, Hk = _assembled(pk, ctx, m)
    assert any(h.ct.sons[int(t), 0] >= 0 for t, s in h.near)  # such blocks exist
    rng = np.random.Generator(np.random.PCG64(6))
    x = rng.standard_normal(m.nt)
    xd = torch.from_numpy(x).cuda()
    for H in (Hv, Hk):
        y1, y2 = torch.empty_like(xd), torch.empty_like(xd)
        H.matvec(xd, y1)
        H.matvec(xd, y2)
        ctx.check()
        a, b = y1.cpu().numpy(), y2.cpu().numpy()
        assert np.array_equal(a.view(np.uint64), b.view(np.uint64))
        host = _host_h2(h, H, H.near, H.coupling)(x)
        assert np.linalg.norm(a - host) <= 1e-12 * np.linalg.norm(host)


def _laplace_data(m):
    """Dirichlet values at the triangle centroids and exact Neumann data at
    the centroids projected to the sphere (outward normal = position)."""
    c = m.v[m.tri].mean(axis=1)
    x = c / np.linalg.norm(c, axis=1)[:, None]
    out = []
    f1 = c[:, 0] ** 2 - c[:, 2] ** 2
    out.append((f1, 2 * x[:, 0] ** 2 - 2 * x[:, 2] ** 2))  # grad f1 . x
    for z in ((1.2, 1.2, 1.2), (1.0, 0.25, 1.0)):
        z = np.array(z)
        d = np.linalg.norm(c - z, axis=1)
        dx = x - z
        r = np.linalg.norm(dx, axis=1)
        out.append((1.0 / (4 * np.pi * d), -(dx * x).sum(axis=1) / (4 * np.pi * r ** 3)))
    return out


def test_laplace_dirichlet_neumann_converges(pk, ctx):
    import torch
    from paper_1510_07244_amd.h2mv import cg
    errs = []
    for n in (8, 16, 32):
        m = octahedron_sphere(n)
        h, Hv, Hk = _assembled(pk, ctx, m)
        area = 0.5 * np.linalg.norm(np.cross(m.v[m.tri[:, 1]] - m.v[m.tri[:, 0]],
                                             m.v[m.tri[:, 2]] - m.v[m.tri[:, 0]]), axis=1)
        e_n, sols = [], []
        for beta, dn in _laplace_data(m):
            bd = torch.from_numpy(beta).cuda()
            rhs = torch.empty_like(bd)
            Hk.matvec(bd, rhs)
            ctx.mass_apply(h.mesh, 0.5, bd, rhs)
            alpha = torch.zeros_like(bd)
            it, res = cg(ctx, Hv.matvec, rhs, alpha, tol=1e-10, maxit=500)
            ctx.check()
            assert res <= 1e-10, (n, it, res)
            a = alpha.cpu().numpy()
            sols.append((a, beta))
            e_n.append(np.sqrt((area * (a - dn) ** 2).sum() / (area * dn ** 2).sum()))
        errs.append(e_n)
        if n == 8:  # the dense oracle system of the same rules
            every = np.arange(m.nt)
            Vd = oracle.block(m.v, m.tri, every, every, layer=0, q_reg=4, q_sing=4).real
            Kd = oracle.block(m.v, m.tri, every, every, layer=1, q_reg=4, q_sing=4).real
            for a, beta in sols:
                ref = np.linalg.solve(Vd, 0.5 * area * beta + Kd @ beta)
                assert np.linalg.norm(a - ref) <= 1e-5 * np.linalg.norm(ref)
    errs = np.array(errs)  # rows: meshes 512, 2048, 8192; columns: f1, f2, f3
    print("Neumann L2 errors (rows 512/2048/8192 triangles; f1, f2, f3):\n", errs, flush=True)
    ratios = errs[:-1] / errs[1:]
    assert np.all(ratios >= 1.6), ratios  # O(h): halving h halves the error
    assert np.all(errs[-1] <= 0.05), errs[-1]


def test_cg_on_the_device_matches_host_cg(pk, ctx):
    # the conjugate gradients with every step on the device (one step
    # captured in a HIP graph, bem_cg_step keeping the scalars on the
    # device) take the host-driven solver's iterations to the same iterate,
    # also when the stopping test holds in the middle of a batch of replays
    import torch
    from paper_1510_07244_amd.h2mv import cg, cg_device
    m = octahedron_sphere(16)
    h, Hv, Hk = _assembled(pk, ctx, m)
    beta, _ = _laplace_data(m)[0]
    bd = torch.from_numpy(beta).cuda()
    rhs = torch.empty_like(bd)
    Hk.matvec(bd, rhs)
    ctx.mass_apply(h.mesh, 0.5, bd, rhs)
    for tol, check in ((1e-10, 8), (1e-6, 5), (1e-10, 1)):
        a_host = torch.zeros_like(bd)
        it_h, res_h = cg(ctx, Hv.matvec, rhs, a_host, tol=tol, maxit=500)
        a_dev = torch.zeros_like(bd)
        it_d, res_d = cg_device(ctx, Hv, rhs, a_dev, tol=tol, maxit=500, check=check)
        ctx.check()
        assert it_d == it_h, (tol, check, it_d, it_h)
        assert res_d <= tol and abs(res_d - res_h) <= 1e-3 * res_h
        x, y = a_dev.cpu().numpy(), a_host.cpu().numpy()
        assert np.linalg.norm(x - y) <= 1e-12 * np.linalg.norm(y)
    # the iteration limit stops it too
    a_dev = torch.zeros_like(bd)
    it_d, res_d = cg_device(ctx, Hv, rhs, a_dev, tol=1e-14, maxit=7, check=4)
    ctx.check()
    assert it_d == 7 and res_d > 1e-14


def test_helmholtz_brakhage_werner_exterior(pk, ctx):
    import torch
    from paper_1510_07244_amd.h2mv import PointIntegrals, bicgstab
    kappa, eta, z0 = 3.0, 3.0, np.array([0.0, 0.0, 0.2])
    rng = np.random.Generator(np.random.PCG64(8))
    d = rng.standard_normal((12, 3))
    pts = d / np.linalg.norm(d, axis=1)[:, None] * rng.uniform(1.5, 3.0, size=(12, 1))
    r = np.linalg.norm(pts - z0, axis=1)
    exact = np.exp(1j * kappa * r) / (4 * np.pi * r)
    errs = []
    for n in (8, 16, 32):
        m = octahedron_sphere(n)
        h, Hv, Hk = _assembled(pk, ctx, m, kernel=1, kappa=kappa)
        op = h.op(pk.SLP)
        src = PointIntegrals(ctx, h.mesh, op, 0, z0[None, :])
        b = torch.zeros(m.nt, dtype=torch.complex128, device="cuda")
        src.column(0, b)  # b_i = int_{tau_i} f

        tmp = torch.empty_like(b)

        def apply(wv, out):
            Hk.matvec(wv, out)
            Hv.matvec(wv, tmp)
            ctx.vec_axpby(-1j * eta, tmp, 1.0, out)
            ctx.mass_apply(h.mesh, 0.5, wv, out)

        w = torch.zeros_like(b)
        it, res = bicgstab(ctx, apply, b, w, tol=1e-9, maxit=500)
        ctx.check()
        assert res <= 1e-9, (n, it, res)
        u = torch.zeros(len(pts), dtype=torch.complex128, device="cuda")
        dl = PointIntegrals(ctx, h.mesh, op, 1, pts)
        sl = PointIntegrals(ctx, h.mesh, op, 0, pts)
        dl.apply(w, u)
        us = torch.zeros_like(u)
        sl.apply(w, us)
        ctx.vec_axpby(-1j * eta, us, 1.0, u)
        ctx.check()
        got = u.cpu().numpy()
        errs.append(np.abs(got - exact).max() / np.abs(exact).max())
        if n == 8:  # the same pipeline against the dense oracle system
            every = np.arange(m.nt)
            Vd = oracle.block(m.v, m.tri, every, every, kernel=1, kappa=kappa, layer=0,
                              q_reg=4, q_sing=4)
            Kd = oracle.block(m.v, m.tri, every, every, kernel=1, kappa=kappa, layer=1,
                              q_reg=4, q_sing=4)
            area = 0.5 * np.linalg.norm(np.cross(m.v[m.tri[:, 1]] - m.v[m.tri[:, 0]],
                                                 m.v[m.tri[:, 2]] - m.v[m.tri[:, 0]]), axis=1)
            wref = np.linalg.solve(np.diag(0.5 * area) + Kd - 1j * eta * Vd, b.cpu().numpy())
            assert np.linalg.norm(w.cpu().numpy() - wref) <= 1e-5 * np.linalg.norm(wref)
    print("Brakhage-Werner exterior errors (512/2048/8192 triangles):", errs, flush=True)
    assert errs[1] < errs[0] and errs[2] < errs[1], errs
    assert errs[2] <= 1e-2, errs


@pytest.mark.parametrize("cplx", [False, True])
@pytest.mark.parametrize("trans", [False, True])
def test_gemv_grouped_ragged_against_numpy(pk, ctx, cplx, trans):
    # the grouped product on its own, with group output lengths and block
    # input lengths from 1 to the maximum 512 (one and several chunks of 64
    # rows, ragged tails, groups of one block and of many), gathered inputs
    # and scattered outputs; against numpy in FP64 at 1e-12 (accumulation
    # into y included)
    import torch
    rng = np.random.Generator(np.random.PCG64(17 + 2 * cplx + trans))
    nx, ny = 3000, 6000
    ms = [1, 7, 64, 65, 100, 128, 129, 200, 300, 512, 33, 64]
    out_perm = rng.permutation(ny)
    groups, o = [], 0
    for g, m in enumerate(ms):
        nb = 1 if g % 3 == 0 else int(rng.integers(2, 6))
        blocks = []
        for _ in range(nb):
            n = int(rng.choice([1, 5, 16, 17, 63, 64, 80, 130, 257, 512]))
            inp = rng.choice(nx, size=n, replace=False).astype(np.int32)
            shape = (n, m) if trans else (m, n)
            A = rng.standard_normal(shape) + (1j * rng.standard_normal(shape) if cplx else 0)
            blocks.append((A, inp))
        groups.append((out_perm[o:o + m].astype(np.int32), blocks))
        o += m
    x = rng.standard_normal(nx) + (1j * rng.standard_normal(nx) if cplx else 0)
    y0 = rng.standard_normal(ny) + (1j * rng.standard_normal(ny) if cplx else 0)
    ref = y0.copy()
    grp_ptr, out_ptr, out_idx, in_ptr, in_idx, a_off, Aflat = [0], [0], [], [0], [], [], []
    off = 0
    for out, blocks in groups:
        acc = np.zeros(out.size, dtype=ref.dtype)
        for A, inp in blocks:
            acc += (A.T if trans else A) @ x[inp]
            a_off.append(off)
            Aflat.append(A.ravel(order="F"))
            off += A.size
            in_idx.append(inp)
            in_ptr.append(in_ptr[-1] + inp.size)
        ref[out] += acc
        out_idx.append(out)
        out_ptr.append(out_ptr[-1] + out.size)
        grp_ptr.append(len(a_off))
    dt = torch.complex128 if cplx else torch.float64
    i32 = lambda a: torch.from_numpy(np.asarray(a, dtype=np.int32)).cuda()
    A = torch.from_numpy(np.concatenate(Aflat)).to(device="cuda", dtype=dt)
    xd = torch.from_numpy(x).to(device="cuda", dtype=dt)
    yd = torch.from_numpy(y0).to(device="cuda", dtype=dt)
    ctx.gemv_grouped(trans, i32(grp_ptr), i32(out_ptr), i32(np.concatenate(out_idx)), i32(in_ptr),
                     i32(np.concatenate(in_idx)), torch.tensor(a_off, dtype=torch.int64).cuda(),
                     A, xd, yd)
    ctx.check()
    got = yd.cpu().numpy()
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()
