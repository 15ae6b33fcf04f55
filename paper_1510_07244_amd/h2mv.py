"""Products with an assembled H^2 matrix (Sec. 2.3-2.4) and the Krylov
solvers of the experiments (Sec. 4), driving the C-ABI: every product and
vector operation is a library kernel; this module builds the index lists
once and orders the calls.

    H x = near field  +  V_t S_ts W_s^T x  over the admissible blocks,

evaluated as: near field y|_t += G_ts x|_s (grouped by row leaf), forward
transformation x^_s = W^_s^T x|_s (leaves) and W^_s^T (x^_s1, x^_s2)
(fathers, bottom-up), coupling y^_t += S_ts x^_s (grouped by row cluster),
backward transformation (fathers push V^_t y^_t to their sons' coefficients
top-down, leaves add V^_t y^_t to y|_t).
"""
import numpy as np

from . import HELMHOLTZ


def _dev(a, dtype):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def _on(stream):
    """Context making `stream` (a torch stream or a raw HIP stream handle)
    torch's current stream, so that the tensor operations around the library
    calls (zeroing, copies, scalar reads) are ordered with them."""
    import contextlib
    import torch
    if stream is None:
        return contextlib.nullcontext()
    if not isinstance(stream, torch.cuda.Stream):
        stream = torch.cuda.ExternalStream(int(stream))
    return torch.cuda.stream(stream)


class _Call:
    """Device index lists of one bem_gemv_grouped call."""

    def __init__(self, groups, trans, A, src, dst):
        """groups: list of (out_idx, [(a_off, in_idx), ...]); src / dst name
        the buffers read and written ('x', 'y', 'xh', 'yh').  The groups are
        listed by decreasing size (matrix entries), so that a launch with
        more groups than workgroup slots starts its largest ones first."""
        import torch
        size = lambda g: len(g[0]) * sum(len(inp) for _, inp in g[1])
        groups = sorted(groups, key=lambda g: -size(g))  # stable: ties keep their order
        grp_ptr, out_ptr, out_idx, in_ptr, in_idx, a_off = [0], [0], [], [0], [], []
        for out, blocks in groups:
            out_idx.append(np.asarray(out, dtype=np.int32))
            out_ptr.append(out_ptr[-1] + len(out))
            for off, inp in blocks:
                in_idx.append(np.asarray(inp, dtype=np.int32))
                in_ptr.append(in_ptr[-1] + len(inp))
                a_off.append(off)
            grp_ptr.append(len(a_off))
        cat = lambda xs: np.concatenate(xs) if xs else np.zeros(0, np.int32)
        self.grp_ptr = _dev(np.array(grp_ptr), torch.int32)
        self.out_ptr = _dev(np.array(out_ptr), torch.int32)
        self.out_idx = _dev(cat(out_idx), torch.int32)
        self.in_ptr = _dev(np.array(in_ptr), torch.int32)
        self.in_idx = _dev(cat(in_idx), torch.int32)
        self.a_off = _dev(np.array(a_off, dtype=np.int64), torch.int64)
        self.trans, self.A, self.src, self.dst = trans, A, src, dst


class H2Matrix:
    """An assembled H^2 matrix on the device, ready for products.

    h: the H2Setup; row_basis / col_basis: its ClusterBasis objects (the
    same object for a single layer); near: packed near-field output in the
    order of h.near (block (t, s) column-major, leading dimension |t|);
    coupling: packed coupling output in the order of h.far (block k_t x k_s).
    The tensors are referenced, not copied."""

    def __init__(self, h, row_basis, col_basis, near, coupling):
        import torch
        self.h, self.ctx = h, h.ctx
        self.n = int(h.tri.shape[0])
        self.cplx = h.kernel == HELMHOLTZ
        self.dtype = torch.complex128 if self.cplx else torch.float64
        ct = h.ct
        self.V, self.W = row_basis, col_basis
        # coefficient slots of each cluster in the buffers xh (column basis)
        # and yh (row basis)
        def slots(B):
            off = np.zeros(ct.n + 1, dtype=np.int64)
            off[1:] = np.cumsum(B.rank)
            return off
        self.cw, self.cv = slots(col_basis), slots(row_basis)
        self.xh = torch.zeros(int(self.cw[-1]), dtype=self.dtype, device="cuda")
        self.yh = torch.zeros(int(self.cv[-1]), dtype=self.dtype, device="cuda")
        rng = lambda off, c: np.arange(off[c], off[c] + (off[c + 1] - off[c]))
        # near field, grouped by row cluster; a block is inadmissible when
        # either cluster is a leaf, so a row cluster may be a father whose
        # triangles are its sons' too: one call per height of the row cluster
        # (clusters of one height are disjoint, so a call's groups never
        # share an output)
        rows = {}
        o = 0
        for t, s in h.near:
            t, s = int(t), int(s)
            rows.setdefault(t, []).append((o, ct.idx(s)))
            o += ct.idx(t).size * ct.idx(s).size
        by_height = {}
        for t, bl in rows.items():
            by_height.setdefault(int(h.height[t]), []).append((ct.idx(t), bl))
        self.near_calls = [_Call(g, False, near, "x", "y") for _, g in sorted(by_height.items())]
        # forward transformation of the column basis, level by level upwards
        fwd = []
        for lv in col_basis.levels:
            groups = []
            for p, c in enumerate(lv.cls):
                c = int(c)
                s0, s1 = ct.sons[c]
                inp = (col_basis.rows[c] if s0 < 0 else
                       np.concatenate([rng(self.cw, s0), rng(self.cw, s1)]))
                groups.append((rng(self.cw, c), [(int(lv.v_off_h[p]), inp)]))
            leaf = ct.sons[int(lv.cls[0]), 0] < 0
            fwd.append(_Call(groups, True, lv.V, "x" if leaf else "xh", "xh"))
        # coupling, grouped by row cluster
        cols = {}
        o = 0
        for t, s in h.far:
            t, s = int(t), int(s)
            cols.setdefault(t, []).append((o, rng(self.cw, s)))
            o += int(row_basis.rank[t]) * int(col_basis.rank[s])
        self.coupling_call = _Call([(rng(self.cv, t), bl) for t, bl in cols.items()], False,
                                   coupling, "xh", "yh")
        # backward transformation of the row basis, level by level downwards
        bwd = []
        for lv in reversed(row_basis.levels):
            groups = []
            for p, c in enumerate(lv.cls):
                c = int(c)
                s0, s1 = ct.sons[c]
                out = (row_basis.rows[c] if s0 < 0 else
                       np.concatenate([rng(self.cv, s0), rng(self.cv, s1)]))
                groups.append((out, [(int(lv.v_off_h[p]), rng(self.cv, c))]))
            leaf = ct.sons[int(lv.cls[0]), 0] < 0
            bwd.append(_Call(groups, False, lv.V, "yh", "y" if leaf else "yh"))
        self.fwd, self.bwd = fwd, bwd
        self.near, self.coupling = near, coupling
        for lv_list in (col_basis.levels, row_basis.levels):
            for lv in lv_list:  # one kind of cluster per level (heights)
                kinds = {bool(ct.sons[int(c), 0] < 0) for c in lv.cls}
                assert len(kinds) == 1

    def _run(self, call, bufs, stream):
        self.ctx.gemv_grouped(call.trans, call.grp_ptr, call.out_ptr, call.out_idx, call.in_ptr,
                              call.in_idx, call.a_off, call.A, bufs[call.src], bufs[call.dst],
                              stream=stream)

    def matvec(self, x, y, stream=None, accumulate=False):
        """y (+)= H x for device vectors of n entries, on `stream` (default:
        torch's current stream).  The near field runs on a second stream
        beside the chain forward transformation -> coupling -> backward
        transformation, which needs y only at its leaf level: that level
        waits for the near field, so y receives its terms in the same order
        as on one stream (bit for bit the same result)."""
        import torch
        with _on(stream):
            main = torch.cuda.current_stream()
            if getattr(self, "_side", None) is None:
                self._side = torch.cuda.Stream()
            side = self._side
            side.wait_stream(main)
            bufs = {"x": x, "y": y, "xh": self.xh, "yh": self.yh}
            with torch.cuda.stream(side):
                if not accumulate:
                    y.zero_()
                for c in self.near_calls:
                    self._run(c, bufs, None)
            self.xh.zero_()
            self.yh.zero_()
            for c in self.fwd:
                self._run(c, bufs, None)
            self._run(self.coupling_call, bufs, None)
            joined = False
            for c in self.bwd:
                if c.dst == "y" and not joined:
                    main.wait_stream(side)
                    joined = True
                self._run(c, bufs, None)
            if not joined:
                main.wait_stream(side)
        return y


class GraphedMatvec:
    """H.matvec captured in a HIP graph, one graph per pair of vector
    buffers: the first call with a pair runs the product once and captures
    it, later calls replay the graph (one launch for the whole product
    instead of one per kernel).  The graphs read and write the buffers they
    were captured with, so callers that keep their vectors in place (like
    cg and bicgstab) reuse them.  Usable wherever H.matvec is."""

    def __init__(self, H, accumulate=False):
        self.H, self.accumulate = H, accumulate
        self.graphs = {}

    def __call__(self, x, y, stream=None):
        import torch
        key = (x.data_ptr(), y.data_ptr(), x.numel(), y.numel(), x.dtype, y.dtype)
        with _on(stream):
            hit = self.graphs.get(key)
            if hit is None:
                self.H.matvec(x, y, accumulate=self.accumulate)  # eager, before capture
                g = torch.cuda.CUDAGraph()
                torch.cuda.current_stream().synchronize()
                with torch.cuda.graph(g):
                    self.H.matvec(x, y, accumulate=self.accumulate)
                self.graphs[key] = (g, x, y)  # keeps the buffers alive
                hit = self.graphs[key]
            hit[0].replay()
        return y


# ------------------------------------------------------------ Krylov solvers
class _Dot:
    def __init__(self, ctx):
        import torch
        self.ctx = ctx
        self.buf = torch.zeros(2, dtype=torch.float64, device="cuda")

    def __call__(self, x, y, conj=True, stream=None):
        self.ctx.vec_dot(x, y, self.buf, conj=conj, stream=stream)
        r, i = self.buf.cpu().numpy()
        return complex(r, i) if x.is_complex() else float(r)


def cg(ctx, apply, b, x, tol=1e-10, maxit=1000, stream=None):
    """Conjugate gradients (Hestenes-Stiefel, Sec. 4) for a symmetric
    positive definite operator `apply(p, q)` (q = A p), from the initial
    guess in x; stops when |r| <= tol |b|.  Returns (iterations, relative
    residual).  Vector updates and dot products are library kernels; the
    scalars come back to the host once per step.  Everything runs on
    `stream` (made torch's current stream, which `apply` is called on)."""
    with _on(stream):
        return _cg(ctx, apply, b, x, tol, maxit)


def _cg(ctx, apply, b, x, tol, maxit):
    import torch
    stream = None
    dot = _Dot(ctx)
    r = torch.empty_like(b)
    q = torch.empty_like(b)
    apply(x, q)
    r.copy_(b)
    ctx.vec_axpby(-1.0, q, 1.0, r, stream)  # r = b - A x
    p = r.clone()
    rr = dot(r, r)
    bb = dot(b, b)
    it = 0
    while it < maxit and rr > tol * tol * bb:
        apply(p, q)
        alpha = rr / dot(p, q)
        ctx.vec_axpby(alpha, p, 1.0, x, stream)
        ctx.vec_axpby(-alpha, q, 1.0, r, stream)
        rr_new = dot(r, r)
        ctx.vec_axpby(1.0, r, rr_new / rr, p, stream)  # p = r + beta p
        rr = rr_new
        it += 1
    return it, float(np.sqrt(rr / bb))


def cg_device(ctx, H, b, x, tol=1e-10, maxit=1000, check=8, stream=None):
    """Conjugate gradients for an assembled symmetric positive definite H^2
    matrix H (real) with every step on the device: one step -- the product
    q = H p, p.q and bem_cg_step -- is captured in a HIP graph and replayed
    `check` times between the host's reads of the stopping flag.  Steps
    after the stopping test holds change nothing (bem_cg_step stops
    updating), so the iterate and the count are those of `cg` with the same
    tolerance.  Returns (iterations, relative residual)."""
    import torch
    with _on(stream):
        r, q, p = torch.empty_like(b), torch.empty_like(b), torch.empty_like(b)
        st = torch.zeros(10, dtype=torch.float64, device="cuda")
        bb_buf = torch.zeros(2, dtype=torch.float64, device="cuda")
        H.matvec(x, q)
        r.copy_(b)
        ctx.vec_axpby(-1.0, q, 1.0, r)  # r = b - A x
        p.copy_(r)
        ctx.vec_dot(r, r, st[0:2])
        ctx.vec_dot(b, b, bb_buf)
        rr, bb = st[0].item(), bb_buf[0].item()
        thr = tol * tol * bb
        if not (rr > thr and maxit > 0):
            return 0, float(np.sqrt(rr / bb))
        st[6:10] = torch.tensor([thr, 1.0, 0.0, float(maxit)], dtype=torch.float64)
        g = torch.cuda.CUDAGraph()
        torch.cuda.current_stream().synchronize()
        with torch.cuda.graph(g):
            H.matvec(p, q)
            ctx.vec_dot(p, q, st[2:4])
            ctx.cg_step(st, x, r, p, q)
        while True:
            for _ in range(check):
                g.replay()
            active, it, rr = st[7].item(), st[8].item(), st[0].item()
            if active == 0.0:
                break
        return int(it), float(np.sqrt(rr / bb))


def bicgstab(ctx, apply, b, x, tol=1e-10, maxit=1000, stream=None):
    """BiCGStab (van der Vorst) for a general (complex) operator
    `apply(p, q)`; stops when |r| <= tol |b|.  Returns (iterations, relative
    residual).  Runs on `stream` like cg."""
    with _on(stream):
        return _bicgstab(ctx, apply, b, x, tol, maxit)


def _bicgstab(ctx, apply, b, x, tol, maxit):
    import torch
    stream = None
    dot = _Dot(ctx)
    r = torch.empty_like(b)
    v = torch.empty_like(b)
    t = torch.empty_like(b)
    apply(x, v)
    r.copy_(b)
    ctx.vec_axpby(-1.0, v, 1.0, r, stream)
    r0 = r.clone()
    p = torch.zeros_like(b)
    v.zero_()
    rho = alpha = omega = 1.0
    bb = abs(dot(b, b))
    rr = abs(dot(r, r))
    it = 0
    while it < maxit and rr > tol * tol * bb:
        rho_new = dot(r0, r)
        beta = (rho_new / rho) * (alpha / omega)
        # p = r + beta (p - omega v)
        ctx.vec_axpby(-omega, v, 1.0, p, stream)
        ctx.vec_axpby(1.0, r, beta, p, stream)
        apply(p, v)
        alpha = rho_new / dot(r0, v)
        ctx.vec_axpby(-alpha, v, 1.0, r, stream)  # r is now s
        apply(r, t)
        omega = dot(t, r) / dot(t, t)
        ctx.vec_axpby(alpha, p, 1.0, x, stream)
        ctx.vec_axpby(omega, r, 1.0, x, stream)
        ctx.vec_axpby(-omega, t, 1.0, r, stream)
        rho = rho_new
        rr = abs(dot(r, r))
        it += 1
    return it, float(np.sqrt(rr / bb))


# ------------------------------------------- layer potentials at given points
class PointIntegrals:
    """Integrals of the kernel over every triangle against a set of points
    z_p away from the surface, by the library's Green-matrix kernel with unit
    weights (Sec. 2.3, eq. green_matrix):
        side 0:  int_{tau_i} g(x, z_p) dx          (single layer)
        side 1:  int_{tau_i} d/dn(x) g(x, z_p) dx  (double layer, normal of tau_i)
    The triangles are taken in chunks of at most 512 (one Green "cluster"
    each).  `apply(w, u, c)` adds c sum_i w_i I_ip to u_p (potential of the
    density w), `column(p, b)` adds I_ip to b_i (load vector of g(., z_p))."""

    CHUNK = 512

    def __init__(self, ctx, mesh, op, side, points):
        import torch
        self.ctx = ctx
        nt = int(mesh.tri.shape[0])
        pts = np.ascontiguousarray(points, dtype=np.float64).reshape(-1, 3)
        self.m = m = pts.shape[0]
        if not 1 <= m <= 512:
            raise ValueError("1 .. 512 points")
        chunks = [np.arange(a, min(a + self.CHUNK, nt), dtype=np.int32)
                  for a in range(0, nt, self.CHUNK)]
        ncl = len(chunks)
        nrows = np.array([c.size for c in chunks], dtype=np.int64)
        rp = np.concatenate([[0], np.cumsum(nrows)]).astype(np.int32)
        self.a_off = np.concatenate([[0], np.cumsum(nrows * 2 * m)[:-1]]).astype(np.int64)
        zn = np.zeros((ncl, m, 3))
        zn[..., 2] = 1.0  # the columns used here do not depend on it
        cplx = op.kernel == HELMHOLTZ
        self.A = torch.empty(int(nrows.sum() * 2 * m),
                             dtype=torch.complex128 if cplx else torch.float64, device="cuda")
        keep = dict(rp=_dev(rp, torch.int32), idx=_dev(np.concatenate(chunks), torch.int32),
                    z=_dev(np.broadcast_to(pts, (ncl, m, 3)), torch.float64),
                    zn=_dev(zn, torch.float64), zw=_dev(np.ones((ncl, m)), torch.float64),
                    delta=_dev(np.ones(ncl), torch.float64), off=_dev(self.a_off, torch.int64))
        ctx.green_matrix(mesh, op, side, keep["rp"], keep["idx"], keep["z"], keep["zn"], keep["zw"],
                         keep["delta"], keep["off"], self.A, max_rows=self.CHUNK)
        self._keep = keep
        # u_p += sum_i w_i I_ip: one group (the points), one block per chunk
        self.pot = _Call([(np.arange(m), [(int(o), c) for o, c in zip(self.a_off, chunks)])],
                         True, self.A, "w", "u")
        # b_i += I_ip of one point p: a group per chunk, its column p times 1
        self.col = [_Call([(c, [(int(o) + p * c.size, [0])]) for o, c in zip(self.a_off, chunks)],
                          False, self.A, "one", "b") for p in range(m)]
        self.one = torch.ones(1, dtype=self.A.dtype, device="cuda")

    def apply(self, w, u, stream=None):
        c = self.pot
        self.ctx.gemv_grouped(c.trans, c.grp_ptr, c.out_ptr, c.out_idx, c.in_ptr, c.in_idx,
                              c.a_off, c.A, w, u, stream=stream)

    def column(self, p, b, stream=None):
        c = self.col[p]
        self.ctx.gemv_grouped(c.trans, c.grp_ptr, c.out_ptr, c.out_idx, c.in_ptr, c.in_idx,
                              c.a_off, c.A, self.one, b, stream=stream)
