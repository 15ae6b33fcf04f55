"""Parity of the H^2 pipeline on its real shapes (GPU, through the C-ABI).

* Coupling blocks G[t~ x s~] (Sec. 2.3-2.4) on the pivot lists a real setup
  chooses -- the widest and tallest blocks (several column sub-tiles of the
  coupling kernel) and a seeded sample -- against the oracle's entries on
  the same pivot triangles, element by element at 1e-12 of the block:
  Laplace single layer (mirrored list, as the step assembles it) and double
  layer on the 8192-triangle sphere, Helmholtz double layer at kappa 8 on the
  32768-triangle sphere (q = 5); the mixed form within 1e-6 per block.
  The pivots are inputs, so the comparison is well defined (which pivots
  cross approximation picks is not pinned).
* The whole H^2 matrix of the 8192-triangle sphere (Laplace SLP and DLP):
  relative Frobenius error against the dense oracle matrix, globally and
  per block, within 1e-6 (near-field blocks from the one-pass kernel on the
  mirrored list, admissible blocks V_t S W_s^T).
* The Helmholtz workloads (32768-triangle sphere, 24576-triangle cube,
  kappa 2, 4, 8, q = 5): sampled admissible blocks of both layers within 1e-6,
  plain and (kappa 8) with mixed coupling blocks.
* The basis contraction V = A[:, tau] P of every level against the
  oracle's one-sum-per-entry product with the same P, each entry within
  1e-12 of sum_l |A_il| |P_lj| (transfer matrices with as many pivots as
  rows are the identity up to rounding, so their entries cancel), and P
  (the host inverse of the pivot block) against the oracle's Gauss-Jordan
  inverse, the rows t~ of V against the identity.
"""
import numpy as np
import pytest

import oracle
from bem_inputs import cube_surface, octahedron_sphere, sample_subset
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


def _assemble_coupling(pk, ctx, h, op, V, W, mirror):
    import torch
    blocks, total = h.coupling_blocks(V, W, mirror=mirror)
    out = torch.full((total,), float("nan"), dtype=pk.out_dtype(op), device="cuda")
    ctx.assemble_coupling(h.mesh, op, blocks, out)
    ctx.check()
    got = out.cpu().numpy()
    assert np.all(np.isfinite(got))  # every entry written
    return got


def _pick_blocks(h, V, W, n_wide, n_tall, n_rand, seed):
    """The widest and the tallest admissible blocks, and a seeded sample."""
    kt = np.array([V.piv[t].size for t, s in h.far])
    ks = np.array([W.piv[s].size for t, s in h.far])
    wide = np.argsort(-ks, kind="stable")[:n_wide]
    tall = np.argsort(-kt, kind="stable")[:n_tall]
    rand = sample_subset(np.arange(len(h.far)), n_rand, seed=seed)
    return sorted(set(wide.tolist()) | set(tall.tolist()) | set(rand.tolist())), kt, ks


def _close(g, ref, tol=1e-12, scale=None):
    if np.abs(ref).max() == 0.0:
        # a double-layer block of coplanar triangles (a cube face) vanishes
        # exactly: the computed one must be tiny against the operator's scale
        assert scale is not None and np.abs(g).max() <= tol * scale, np.abs(g).max()
        return
    fro = np.linalg.norm(g - ref) / np.linalg.norm(ref)
    ent = np.abs(g - ref).max() / np.abs(ref).max()
    assert fro <= tol and ent <= tol, (fro, ent)


# ------------------------------------------------------------ Laplace, 8192
@pytest.fixture(scope="module")
def lap8192(pk, ctx):
    import torch
    from paper_1510_07244_amd.h2 import H2Setup
    m = octahedron_sphere(32)
    h = H2Setup(ctx, m.v, m.tri, kernel=pk.LAPLACE, q_regular=4, q_singular=4)
    V, W = h.bases((0, 1))
    S = {pk.SLP: _assemble_coupling(pk, ctx, h, h.op(pk.SLP), V, V, True),
         pk.DLP: _assemble_coupling(pk, ctx, h, h.op(pk.DLP), V, W, False)}
    half, total = h.near_blocks(mirror=True)
    ns = torch.full((total,), float("nan"), dtype=torch.float64, device="cuda")
    nd = torch.full_like(ns, float("nan"))
    ctx.assemble_nearfield_both(h.mesh, h.op(pk.SLP), half, ns, nd)
    ctx.check()
    N = {pk.SLP: ns.cpu().numpy(), pk.DLP: nd.cpu().numpy()}
    return dict(m=m, h=h, V=V, W=W, S=S, N=N)


@pytest.mark.parametrize("layer", [0, 1])
def test_coupling_real_pivots_laplace(pk, lap8192, layer):
    L = lap8192
    m, h, V = L["m"], L["h"], L["V"]
    W = V if layer == pk.SLP else L["W"]
    offs, _ = coupling_offsets(h, V, W)
    pick, kt, ks = _pick_blocks(h, V, W, 10, 10, 24, seed=11 + layer)
    assert ks[pick].max() > 96 and kt[pick].max() > 96  # several sub-tiles per block
    for k in pick:
        t, s = h.far[k]
        g = coupling_matrix(L["S"][layer], offs[k], kt[k], ks[k])
        ref = oracle.block(m.v, m.tri, V.piv[t], W.piv[s], layer=layer, q_reg=4, q_sing=4).real
        _close(g, ref)


@pytest.mark.parametrize("layer", [0, 1])
def test_h2_global_error_sphere8192(pk, lap8192, layer):
    # || H - G ||_F / || G ||_F over the whole matrix, G the dense oracle
    # matrix at the plain orders, H the near-field blocks plus V_t S_ts W_s^T
    L = lap8192
    m, h, V = L["m"], L["h"], L["V"]
    W = V if layer == pk.SLP else L["W"]
    Vf, Wf = FullBases(h, V), FullBases(h, W)
    offs, _ = coupling_offsets(h, V, W)
    num = den = 0.0
    worst_far = worst_near = 0.0
    for k, (t, s) in enumerate(h.far):
        S = coupling_matrix(L["S"][layer], offs[k], V.piv[t].size, W.piv[s].size)
        approx = Vf(t) @ S @ Wf(s).T
        ref = oracle.block(m.v, m.tri, h.ct.idx(t), h.ct.idx(s), layer=layer, q_reg=4,
                           q_sing=4).real
        e, r = np.linalg.norm(approx - ref) ** 2, np.linalg.norm(ref) ** 2
        num, den = num + e, den + r
        worst_far = max(worst_far, np.sqrt(e / r))
    o = 0
    for t, s in h.near:
        r_, c_ = h.ct.idx(t), h.ct.idx(s)
        g = L["N"][layer][o:o + r_.size * c_.size].reshape(c_.size, r_.size).T
        o += r_.size * c_.size
        ref = oracle.block(m.v, m.tri, r_, c_, layer=layer, q_reg=4, q_sing=4).real
        e, r = np.linalg.norm(g - ref) ** 2, np.linalg.norm(ref) ** 2
        num, den = num + e, den + r
        worst_near = max(worst_near, np.sqrt(e / r))
    glob = np.sqrt(num / den)
    print(f"layer {layer}: global {glob:.3e}, worst admissible block {worst_far:.3e}, "
          f"worst near-field block {worst_near:.3e}", flush=True)
    assert glob <= 1e-6 and worst_far <= 1e-6, (glob, worst_far)
    assert worst_near <= 1e-12, worst_near


@pytest.mark.parametrize("side", [0, 1])
def test_contraction_against_oracle(pk, lap8192, side):
    _contraction_parity(lap8192["h"], lap8192["V"] if side == 0 else lap8192["W"], cplx=False)


def _contraction_parity(h, B, cplx, per_level=6):
    m2 = 2 * h.m
    for li, lv in enumerate(B.levels):
        A_h = lv.A.cpu().numpy()
        V_h = lv.V.cpu().numpy()
        pinv_h = lv.pinv.cpu().numpy()
        a_off = np.concatenate([[0], np.cumsum(lv.nrows_h.astype(np.int64) * m2)[:-1]])
        for p in sample_subset(np.arange(lv.cls.size), min(per_level, lv.cls.size), seed=li):
            c, n, k = int(lv.cls[p]), int(lv.nrows_h[p]), int(lv.rank_h[p])
            if k == 0:
                continue
            A = A_h[a_off[p]:a_off[p] + n * m2].reshape(m2, n).T
            tau = lv.pcol_h[p, :k]
            pf = pinv_h[p]
            P = (pf[:2 * k * k].view(np.complex128) if cplx else pf[:k * k]).reshape(k, k).T
            got = V_h[lv.v_off_h[p]:lv.v_off_h[p] + n * k].reshape(k, n).T
            ref = oracle.contract(A, tau, P)
            ref = ref if cplx else ref.real
            # a transfer matrix can be the identity up to rounding (as many
            # pivots as rows): its entries cancel, so each entry is compared
            # against the size of its terms, sum_l |A_il| |P_lj| (the bound
            # of a sum's rounding error), not against the result
            scale = np.abs(A[:, tau]) @ np.abs(P)
            assert np.all(np.abs(got - ref) <= 1e-12 * scale), (li, p)
            # the host inverse against the oracle's, relative to the pivot
            # block's conditioning; R_t V = I on the pivot rows
            pos = {int(x): q for q, x in enumerate(B.rows[c])}
            prow = np.array([pos[int(x)] for x in B.piv[c]], dtype=np.int32)
            M = A[np.ix_(prow, tau)]
            cond = np.linalg.cond(M)
            Po = oracle.inverse(M)
            assert np.linalg.norm(P - Po) <= 1e-13 * cond * np.linalg.norm(Po), (li, p, cond)
            assert np.abs(got[prow] - np.eye(k)).max() <= 1e-13 * cond, (li, p, cond)


# ------------------------------------------------------- Helmholtz, config 3
@pytest.fixture(scope="module", params=[("sphere32768", 2.0), ("sphere32768", 4.0),
                                        ("sphere32768", 8.0), ("cube24576", 2.0),
                                        ("cube24576", 4.0), ("cube24576", 8.0)],
                ids=lambda p: f"{p[0]}-k{p[1]:g}")
def helm(request, pk, ctx):
    from paper_1510_07244_amd.h2 import H2Setup
    name, kappa = request.param
    m = octahedron_sphere(64) if name == "sphere32768" else cube_surface(32)
    h = H2Setup(ctx, m.v, m.tri, kernel=pk.HELMHOLTZ, kappa=kappa, q_regular=5, q_singular=5)
    V, W = h.bases((0, 1))
    return dict(name=name, kappa=kappa, m=m, h=h, V=V, W=W)


@pytest.mark.parametrize("layer", [0, 1])
def test_helmholtz_h2_blocks(pk, ctx, helm, layer):
    m, h, V, kappa = helm["m"], helm["h"], helm["V"], helm["kappa"]
    W = V if layer == pk.SLP else helm["W"]
    forms = [("plain", h.op(layer))]
    if kappa == 8.0:
        op = h.op(layer)
        op.precision, op.near_singular_ratio = pk.MIXED, 0.5
        forms.append(("mixed", op))
    offs, _ = coupling_offsets(h, V, W)
    small = np.array([k for k, (t, s) in enumerate(h.far)
                      if h.ct.idx(t).size * h.ct.idx(s).size <= 128 * 128])
    pick = sample_subset(small, 6, seed=int(kappa) + 10 * layer)
    Vf, Wf = FullBases(h, V), FullBases(h, W)
    refs = {}
    for form, op in forms:
        S_all = _assemble_coupling(pk, ctx, h, op, V, W, layer == pk.SLP)
        scale = np.abs(S_all).max()  # the largest coupling entry of the operator
        for k in pick:
            t, s = h.far[k]
            S = coupling_matrix(S_all, offs[k], V.piv[t].size, W.piv[s].size).astype(np.complex128)
            if k not in refs:
                refs[k] = (oracle.block(m.v, m.tri, h.ct.idx(t), h.ct.idx(s), kernel=pk.HELMHOLTZ,
                                        kappa=kappa, layer=layer, q_reg=5, q_sing=5),
                           oracle.block(m.v, m.tri, V.piv[t], W.piv[s], kernel=pk.HELMHOLTZ,
                                        kappa=kappa, layer=layer, q_reg=5, q_sing=5))
            dense, coup = refs[k]
            if form == "plain":
                _close(S, coup, scale=scale)  # the coupling block itself at FP64 parity
            elif np.abs(coup).max() > 0:
                assert np.linalg.norm(S - coup) <= 1e-6 * np.linalg.norm(coup)
            else:
                assert np.abs(S).max() <= 1e-6 * scale
            approx = Vf(t) @ S @ Wf(s).T
            if np.abs(dense).max() == 0.0:  # coplanar double layer: exactly zero
                assert np.abs(approx).max() <= 1e-6 * scale, (form, k)
                continue
            err = np.linalg.norm(approx - dense) / np.linalg.norm(dense)
            assert err <= 1e-6, (form, k, err)


def test_coupling_real_pivots_helmholtz_dlp_k8(pk, ctx):
    from paper_1510_07244_amd.h2 import H2Setup
    m = octahedron_sphere(64)
    h = H2Setup(ctx, m.v, m.tri, kernel=pk.HELMHOLTZ, kappa=8.0, q_regular=5, q_singular=5)
    V, W = h.bases((0, 1))
    S_all = _assemble_coupling(pk, ctx, h, h.op(pk.DLP), V, W, False)
    offs, _ = coupling_offsets(h, V, W)
    pick, kt, ks = _pick_blocks(h, V, W, 8, 8, 12, seed=21)
    assert ks[pick].max() > 80
    for k in pick:
        t, s = h.far[k]
        g = coupling_matrix(S_all, offs[k], kt[k], ks[k])
        ref = oracle.block(m.v, m.tri, V.piv[t], W.piv[s], kernel=pk.HELMHOLTZ, kappa=8.0,
                           layer=pk.DLP, q_reg=5, q_sing=5)
        _close(g, ref)
    _contraction_parity(h, W, cplx=True, per_level=3)


def _complete_pivoting_order(M):
    """Row and column orders in which Gaussian elimination on M takes the
    largest remaining entry as each pivot (what the cross approximation's
    full pivoting gives the pivot block)."""
    R = np.array(M, dtype=np.complex128)
    rows, cols = list(range(M.shape[0])), list(range(M.shape[1]))
    orow, ocol = [], []
    for _ in range(M.shape[0]):
        sub = np.abs(R[np.ix_(rows, cols)])
        i, j = np.unravel_index(np.argmax(sub), sub.shape)
        r, c = rows[i], cols[j]
        R -= np.outer(R[:, c], R[r, :]) / R[r, c]
        orow.append(r), ocol.append(c)
        rows.remove(r), cols.remove(c)
    return np.array(orow), np.array(ocol)


@pytest.mark.parametrize("cplx", [False, True])
def test_pivot_inverse_against_oracle(pk, ctx, cplx):
    """bem_pivot_inverse on seeded matrices with pivot rows and columns
    scattered in a larger one (ragged ranks, k = 1, the largest rank of the
    register-resident kernel and one beyond it, a zero entry in the
    block), listed in complete-pivoting order as the cross approximation
    lists them, against the oracle's Gauss-Jordan inverse relative to the
    block's condition number.  A list whose first pivot is zero raises
    BEM_ENONFINITE."""
    import torch
    rng = np.random.Generator(np.random.PCG64(30 + cplx))
    # ranks up to 192 (real) / 128 (complex) take the register-resident
    # kernel, larger ones the one in global memory
    big = 200 if not cplx else 150
    acols, max_rank = 256, big
    shapes = [(40, 40), (57, 33), (9, 1), (64, 17), (30, 8), (big + 20, big),
              (192 if not cplx else 128, 192 if not cplx else 128)]
    A_list, prow, pcol = [], [], []
    for n, k in shapes:
        A = rng.standard_normal((n, acols)) + (1j * rng.standard_normal((n, acols)) if cplx else 0)
        pr = rng.choice(n, size=k, replace=False)
        pc = rng.choice(acols, size=k, replace=False)
        if k > 1:
            A[pr[0], pc[0]] = 0.0  # a zero in the block
        orow, ocol = _complete_pivoting_order(A[np.ix_(pr, pc)])
        A_list.append(A), prow.append(pr[orow]), pcol.append(pc[ocol])
    nrows = np.array([s[0] for s in shapes], dtype=np.int32)
    rank = np.array([s[1] for s in shapes], dtype=np.int32)
    a_off = np.concatenate([[0], np.cumsum(nrows * acols)[:-1]]).astype(np.int64)
    PR = np.zeros((len(shapes), max_rank), dtype=np.int32)
    PC = np.zeros((len(shapes), max_rank), dtype=np.int32)
    for t in range(len(shapes)):
        PR[t, :rank[t]], PC[t, :rank[t]] = prow[t], pcol[t]
    dt = torch.complex128 if cplx else torch.float64
    dev = lambda a, t: torch.as_tensor(np.ascontiguousarray(a)).to(device="cuda", dtype=t)
    A_dev = dev(np.concatenate([a.T.ravel() for a in A_list]), dt)
    f = 2 if cplx else 1
    pinv = torch.full((len(shapes), max_rank * max_rank * f), float("nan"), dtype=torch.float64,
                      device="cuda")
    ctx.pivot_inverse(cplx, dev(nrows, torch.int32), dev(rank, torch.int32), max_rank,
                      dev(PR, torch.int32), dev(PC, torch.int32), A_dev, dev(a_off, torch.int64),
                      acols, pinv)
    ctx.check()
    got_all = pinv.cpu().numpy()
    for t, (n, k) in enumerate(shapes):
        row = got_all[t, :k * k * f]
        P = (row.view(np.complex128) if cplx else row).reshape(k, k).T
        M = A_list[t][np.ix_(prow[t], pcol[t])]
        ref = oracle.inverse(M)
        ref = ref if cplx else ref.real
        cond = np.linalg.cond(M)
        assert np.linalg.norm(P - ref) <= 1e-13 * cond * np.linalg.norm(ref), (t, cond)
        assert np.abs(M @ P - np.eye(k)).max() <= 1e-13 * cond, t
    # a zero first pivot: the device flag, reported at the check
    t = 0
    zr = np.where(A_list[t] == 0.0)
    PR0, PC0 = PR.copy(), PC.copy()
    PR0[t, 0], PC0[t, 0] = zr[0][0], zr[1][0]
    PR0[t, 1:rank[t]] = [r for r in prow[t] if r != zr[0][0]][:rank[t] - 1]
    PC0[t, 1:rank[t]] = [c for c in pcol[t] if c != zr[1][0]][:rank[t] - 1]
    ctx.pivot_inverse(cplx, dev(nrows, torch.int32), dev(rank, torch.int32), max_rank,
                      dev(PR0, torch.int32), dev(PC0, torch.int32), A_dev,
                      dev(a_off, torch.int64), acols, pinv)
    with pytest.raises(pk.BemError) as err:
        ctx.check()
    assert err.value.code == pk.BEM_ENONFINITE
