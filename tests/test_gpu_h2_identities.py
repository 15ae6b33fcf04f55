"""End-to-end checks of the assembled H^2 matrices against identities of the
operators (GPU; host matrix-vector products in FP64 numpy).

* Gauss's identity: on a closed polyhedral surface the double layer
  potential of the constant 1 is -1/2 at every point of a face, so the
  Galerkin rows sum to -|tau_i| / 2 exactly, up to quadrature and H^2
  approximation error.  Checked on the 8192-triangle sphere with the
  benchmark's pipeline: one-pass near field of both layers on the mirrored
  list, DLP coupling blocks, nested bases V (rows) and W (double-layer
  columns); K 1 = sum near blocks + sum_far V_t S_ts (W_s^T 1).
* The single layer of the constant 1 on the unit sphere is 1: the rows of
  V (mirrored near field and coupling) sum to |tau_i| up to the O(h^2)
  geometry error of the flat facets.
"""
import numpy as np
import pytest

from bem_inputs import octahedron_sphere
from h2util import FullBases

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


def _areas(m):
    e1 = m.v[m.tri[:, 1]] - m.v[m.tri[:, 0]]
    e2 = m.v[m.tri[:, 2]] - m.v[m.tri[:, 0]]
    return 0.5 * np.linalg.norm(np.cross(e1, e2), axis=1)


def _near_rowsum(h, res):
    y = np.zeros(h.tri.shape[0])
    o = 0
    for t, s in h.near:
        r, c = h.ct.idx(t), h.ct.idx(s)
        blk = res[o:o + r.size * c.size].reshape(c.size, r.size).T
        o += r.size * c.size
        np.add.at(y, r, blk.sum(axis=1))
    return y


def _far_rowsum(h, res, row_basis, col_basis):
    # y_t += V_t S_ts (W_s^T 1_s), with the full (expanded) nested bases
    y = np.zeros(h.tri.shape[0])
    vfull, wsum = {}, {}
    Vf, Wf = FullBases(h, row_basis), FullBases(h, col_basis)
    o = 0
    for t, s in h.far:
        t, s = int(t), int(s)
        kt, ks = row_basis.piv[t].size, col_basis.piv[s].size
        S = res[o:o + kt * ks].reshape(ks, kt).T
        o += kt * ks
        if t not in vfull:
            vfull[t] = Vf(t)
        if s not in wsum:
            wsum[s] = Wf(s).sum(axis=0)
        np.add.at(y, h.ct.idx(t), vfull[t] @ (S @ wsum[s]))
    return y


def test_h2_double_layer_gauss_identity_sphere8192(pk, ctx):
    import torch
    from paper_1510_07244_amd.h2 import H2Setup
    m = octahedron_sphere(32)
    h = H2Setup(ctx, m.v, m.tri, kernel=pk.LAPLACE, q_regular=4, q_singular=4)
    V, W = h.bases((0, 1))
    half, total = h.near_blocks(mirror=True)
    f64 = dict(dtype=torch.float64, device="cuda")
    s = torch.full((total,), float("nan"), **f64)
    d = torch.full((total,), float("nan"), **f64)
    ctx.assemble_nearfield_both(h.mesh, h.op(pk.SLP), half, s, d)
    cd, n_cd = h.coupling_blocks(V, W)
    cdo = torch.full((n_cd,), float("nan"), **f64)
    ctx.assemble_coupling(h.mesh, h.op(pk.DLP), cd, cdo)
    ctx.check()
    a = _areas(m)
    near = _near_rowsum(h, d.cpu().numpy())
    far = _far_rowsum(h, cdo.cpu().numpy(), V, W)
    dev = np.abs(near + far + a / 2) / a
    print(f"Gauss identity: max {dev.max():.3e}, median {np.median(dev):.3e}", flush=True)
    # the far field carries a real share of the row sum: the check sees it
    assert np.median(np.abs(far) / a) > 0.05
    assert dev.max() < 2e-4, (dev.max(), np.median(dev))


def test_h2_single_layer_row_sums_unit_sphere(pk, ctx):
    import torch
    from paper_1510_07244_amd.h2 import H2Setup
    m = octahedron_sphere(32)
    h = H2Setup(ctx, m.v, m.tri, kernel=pk.LAPLACE, q_regular=4, q_singular=4)
    (V,) = h.bases((0,))
    half, total = h.near_blocks(mirror=True)
    f64 = dict(dtype=torch.float64, device="cuda")
    s = torch.full((total,), float("nan"), **f64)
    ctx.assemble_nearfield(h.mesh, h.op(pk.SLP), half, s)
    cs, n_cs = h.coupling_blocks(V, V, mirror=True)
    cso = torch.full((n_cs,), float("nan"), **f64)
    ctx.assemble_coupling(h.mesh, h.op(pk.SLP), cs, cso)
    ctx.check()
    a = _areas(m)
    y = _near_rowsum(h, s.cpu().numpy()) + _far_rowsum(h, cso.cpu().numpy(), V, V)
    err = np.abs(y / a - 1)
    print(f"single-layer row sums: max {err.max():.3e}, median {np.median(err):.3e}", flush=True)
    assert err.max() < 5e-3, (err.max(), np.median(err))
