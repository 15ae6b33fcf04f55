"""GPU parity at the full sizes of the Helmholtz workloads, in the launch
configuration the bench uses (a mesh's whole near-field list in one call),
checked on sampled blocks against the oracle one block at a time.

* Near field of the sphere with 32768 triangles and of the cube surface with
  24576 triangles (leaf 64, eta 2), Sauter-Schwab and Duffy/Gauss order 5,
  kappa in {2, 4, 8}, single and double layer: plain FP64 within 1e-12
  relative per sampled block (Frobenius and largest entry); the mixed form
  (kappa 8) within 1e-6 relative Frobenius per block.
* H2 coupling of the 32768-triangle sphere for the Helmholtz double layer at
  kappa 8: sampled admissible blocks V S W^T within 1e-6 of the oracle's
  dense block.
"""
import numpy as np
import pytest

import oracle
from h2util import full_basis
from bem_inputs import cube_surface, octahedron_sphere, sample_subset
from oracle import htree

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


@pytest.fixture(scope="module", params=["sphere32768", "cube24576"])
def mesh_lists(request, pk):
    import torch
    m = octahedron_sphere(64) if request.param == "sphere32768" else cube_surface(32)
    cl = htree.cluster_tree(m.v, m.tri, 64)
    near, _ = htree.block_tree(cl, 2.0)
    rows = [cl[t].idx for t, s in near]
    cols = [cl[s].idx for t, s in near]
    blocks, total = pk.Blocks.from_lists(rows, cols)
    sizes = np.array([r.size * c.size for r, c in zip(rows, cols)], dtype=np.int64)
    offs = np.concatenate([[0], np.cumsum(sizes)[:-1]])
    # one block on the diagonal (identical, edge and vertex pairs) and one off it
    diag = [k for k, (t, s) in enumerate(near) if t == s]
    off_diag = [k for k, (t, s) in enumerate(near) if t != s]
    pick = [diag[len(diag) // 3], off_diag[int(sample_subset(np.arange(len(off_diag)), 1, seed=7)[0])]]
    mesh = pk.Mesh(torch.from_numpy(m.v), torch.from_numpy(m.tri))
    return dict(m=m, mesh=mesh, blocks=blocks, total=total, rows=rows, cols=cols, offs=offs,
                pick=pick)


def _sampled(pk, ctx, L, op):
    import torch
    out = torch.full((L["total"],), float("nan"), dtype=pk.out_dtype(op), device="cuda")
    ctx.assemble_nearfield(L["mesh"], op, L["blocks"], out)
    ctx.check()
    res = []
    for k in L["pick"]:
        r, c = L["rows"][k], L["cols"][k]
        o = int(L["offs"][k])
        g = out[o:o + r.size * c.size].cpu().numpy().reshape(c.size, r.size).T
        res.append((g, r, c))
    del out
    return res


def _kw(op):
    return dict(kernel=op.kernel, layer=op.layer, kappa=op.kappa, rule=op.regular_rule,
                q_reg=op.q_regular, q_sing=op.q_singular)


@pytest.mark.parametrize("kappa", [2.0, 4.0, 8.0])
@pytest.mark.parametrize("layer", [0, 1])
def test_helmholtz_nearfield_plain(pk, ctx, mesh_lists, kappa, layer):
    op = pk.make_op(pk.HELMHOLTZ, layer, q_regular=5, q_singular=5, kappa=kappa)
    for g, r, c in _sampled(pk, ctx, mesh_lists, op):
        ref = oracle.block(mesh_lists["m"].v, mesh_lists["m"].tri, r, c, **_kw(op))
        assert np.all(np.isfinite(g))
        fro = np.linalg.norm(g - ref) / np.linalg.norm(ref)
        ent = np.abs(g - ref).max() / np.abs(ref).max()
        assert fro <= 1e-12 and ent <= 1e-12, (fro, ent)


@pytest.mark.parametrize("layer", [0, 1])
def test_helmholtz_nearfield_mixed(pk, ctx, mesh_lists, layer):
    op = pk.make_op(pk.HELMHOLTZ, layer, precision=pk.MIXED, q_regular=5, q_singular=5,
                    kappa=8.0, near_singular_ratio=0.5)
    for g, r, c in _sampled(pk, ctx, mesh_lists, op):
        assert g.dtype == np.complex64
        ref = oracle.block(mesh_lists["m"].v, mesh_lists["m"].tri, r, c, **_kw(op))
        assert np.linalg.norm(g - ref) <= 1e-6 * np.linalg.norm(ref)


def test_helmholtz_h2_coupling_sphere32768(pk, ctx):
    import torch
    from paper_1510_07244_amd.h2 import H2Setup
    m = octahedron_sphere(64)
    h = H2Setup(ctx, m.v, m.tri, kernel=pk.HELMHOLTZ, kappa=8.0, q_regular=5, q_singular=5)
    V, W = h.bases((0, 1))
    blocks, total = h.coupling_blocks(V, W)
    op = h.op(pk.DLP)
    out = torch.full((total,), float("nan"), dtype=pk.out_dtype(op), device="cuda")
    ctx.assemble_coupling(h.mesh, op, blocks, out)
    ctx.check()
    sizes = np.array([V.piv[t].size * W.piv[s].size for t, s in h.far], dtype=np.int64)
    offs = np.concatenate([[0], np.cumsum(sizes)[:-1]])
    small = [k for k, (t, s) in enumerate(h.far)
             if h.ct.idx(t).size * h.ct.idx(s).size <= 128 * 128]
    for k in sample_subset(np.array(small), 6, seed=3):
        t, s = h.far[k]
        kt, ks = V.piv[t].size, W.piv[s].size
        S = out[int(offs[k]):int(offs[k]) + kt * ks].cpu().numpy().reshape(ks, kt).T
        approx = full_basis(h, V, t) @ S @ full_basis(h, W, s).T
        ref = oracle.block(m.v, m.tri, h.ct.idx(t), h.ct.idx(s), kernel=pk.HELMHOLTZ, kappa=8.0,
                           layer=pk.DLP, q_reg=5, q_sing=5)
        assert np.linalg.norm(approx - ref) <= 1e-6 * np.linalg.norm(ref)
