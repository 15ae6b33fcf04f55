"""H^2-matrix setup by Green cross approximation (Sec. 2.3-2.4), driving the
C-ABI: cluster and block trees (host), Green boxes and points (host), Green
matrices (GPU), adaptive cross approximation (host), basis contraction (GPU
matrix cores), coupling and near-field blocks (GPU).  This module only
orders the calls and moves arrays; every numerical step is a library call.

The H^2 approximation of an admissible block is
    G|_{t x s} ~ V_t G|_{t~ x s~} W_s^T
with V_t the nested row basis (side-0 Green matrices) and W_s the column
basis: W = V for the single layer, side-1 Green matrices for the double layer.
Nested bases store for each cluster the matrix V^_c whose rows belong to the
triangles ``rows[c]`` (the cluster for a leaf, t^ = union of the sons' pivots
for a father); the full basis V_t = diag(V_t1, V_t2) V^_t is never formed.
"""
import time

import numpy as np

from . import (HELMHOLTZ, LAPLACE, SLP, DLP, Blocks, ClusterTree, Mesh, block_tree, green_points,
               aca, make_op)


def _dev(a, dtype):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


_PINNED = {}


def _pinned(nbytes):
    """A pinned host byte buffer of at least nbytes, kept for the process
    (pinned allocations are slow; every setup reuses this one)."""
    import torch
    buf = _PINNED.get("buf")
    if buf is None or buf.numel() < nbytes:
        buf = torch.empty(max(nbytes, 1 << 22), dtype=torch.uint8, pin_memory=True)
        _PINNED["buf"] = buf
    return buf


class _Stager:
    """Host-to-device uploads through a pinned staging buffer, copied
    asynchronously on the current stream (a synchronous copy from pageable
    memory would also wait for every kernel queued before it).  The staged
    bytes must stay untouched until the copies are done: reset() only after
    the stream has been synchronised."""

    def __init__(self):
        self.buf, self.pos = None, 0

    def reset(self):
        self.pos = 0

    def upload(self, *arrays):
        """Several host arrays (each (array, numpy dtype)) to the device, one
        copy per dtype; returns device tensors (shapes kept) in order."""
        import torch
        groups = {}
        for k, (a, dt) in enumerate(arrays):
            groups.setdefault(np.dtype(dt), []).append(k)
        out = [None] * len(arrays)
        for dt, ks in groups.items():
            arrs = [np.ascontiguousarray(arrays[k][0], dtype=dt) for k in ks]
            n = sum(a.size for a in arrs)
            nbytes = n * dt.itemsize
            start = (self.pos + 255) // 256 * 256
            if self.buf is None or start + nbytes > self.buf.numel():
                if self.buf is not None and self.pos > 0:
                    torch.cuda.current_stream().synchronize()  # earlier copies done
                start = 0
                if self.buf is None or nbytes > self.buf.numel():
                    self.buf = torch.empty(max(nbytes, 8 << 20), dtype=torch.uint8,
                                           pin_memory=True)
            host = self.buf[start:start + nbytes].view(torch.from_numpy(np.zeros(0, dt)).dtype)
            hn = host.numpy()
            o = 0
            for a in arrs:
                hn[o:o + a.size] = a.ravel()
                o += a.size
            dev = torch.empty(n, dtype=host.dtype, device="cuda")
            dev.copy_(host, non_blocking=True)
            self.pos = start + nbytes
            o = 0
            for k, a in zip(ks, arrs):
                out[k] = dev[o:o + a.size].view(a.shape)
                o += a.size
        return out


_STAGER = _Stager()


def _upload(*arrays):
    return _STAGER.upload(*arrays)


class LevelPlan:
    """Device inputs of one tree level of a basis construction (cached so that
    the GPU part can be replayed without the host pivot search)."""


class ClusterBasis:
    def __init__(self, side, ncl):
        self.side = side
        self.rows = [None] * ncl   # triangle ids of the rows of V^_c
        self.piv = [None] * ncl    # pivot triangles t~_c
        self.rank = np.zeros(ncl, dtype=np.int32)
        self.levels = []           # LevelPlan per height (needed clusters only)
        self.where = [None] * ncl  # (level index, position in level)

    def flat_pivots(self):
        """(flat, start, size): cluster c's pivot triangles are
        flat[start[c] : start[c] + size[c]] (empty for clusters without a
        basis)."""
        size = np.array([0 if p is None else p.size for p in self.piv], dtype=np.int64)
        start = np.zeros(size.size, dtype=np.int64)
        np.cumsum(size[:-1], out=start[1:])
        flat = np.concatenate([p for p in self.piv if p is not None and p.size]
                              or [np.zeros(0, np.int64)]).astype(np.int64)
        return flat, start, size

    def vhat(self, c):
        """V^_c as a host numpy array (n_c x k_c)."""
        li, p = self.where[c]
        lv = self.levels[li]
        n, k = lv.nrows_h[p], self.rank[c]
        o = lv.v_off_h[p]
        flat = lv.V.cpu().numpy()
        return flat[o:o + n * k].reshape(k, n).T


def _block_lists(pairs, rows, cols, mirror, keep_diag):
    """Blocks of the cluster pairs (t, s): rows / cols = (flat, start, size)
    give a cluster c's triangles flat[start[c] : start[c] + size[c]].
    Outputs back to back in list order (column-major blocks).  mirror: only
    the blocks with t < s (and t == s if keep_diag) are listed, each with the
    output offset of (s, t) as its mirror -- its own for t == s, the block
    being its own transpose.  Returns (Blocks, total entries)."""
    pairs = np.asarray(pairs, dtype=np.int64).reshape(-1, 2)
    t, s_ = pairs[:, 0], pairs[:, 1]
    nr, nc = rows[2][t], cols[2][s_]
    sizes = nr * nc
    off = np.zeros(pairs.shape[0], dtype=np.int64)
    if sizes.size:
        np.cumsum(sizes[:-1], out=off[1:])
    keep = np.arange(pairs.shape[0])
    mirror_off = None
    if mirror:
        keep = np.nonzero(t <= s_ if keep_diag else t < s_)[0]
        if not keep_diag and 2 * keep.size != pairs.shape[0]:
            raise ValueError("the admissible blocks are not symmetric")
        ncl = int(pairs.max()) + 1 if pairs.size else 1
        key = t * ncl + s_
        order = np.argsort(key, kind="stable")
        want = s_[keep] * ncl + t[keep]
        at = np.searchsorted(key[order], want)
        if np.any(at >= key.size) or np.any(key[order][np.minimum(at, key.size - 1)] != want):
            raise ValueError("a block (t, s) without its transpose (s, t)")
        mirror_off = off[order[at]]

    def gather(flat, start, size, ids):
        n = size[ids]
        ptr = np.zeros(ids.size + 1, dtype=np.int64)
        np.cumsum(n, out=ptr[1:])
        idx = np.arange(ptr[-1], dtype=np.int64) + np.repeat(start[ids] - ptr[:-1], n)
        return ptr.astype(np.int32), flat[idx].astype(np.int32)

    rp, ri = gather(*rows, t[keep])
    cp, ci = gather(*cols, s_[keep])
    return Blocks(rp, ri, cp, ci, off[keep], mirror_off), int(sizes.sum())


class H2Setup:
    # Cross-approximation tolerance 5e-8 with Green order 4 keeps every
    # sampled admissible block of the 8192-triangle sphere below 1e-6 relative
    # error for the single and the double layer (3e-7 does not for the latter).
    def __init__(self, ctx, v, tri, kernel=LAPLACE, kappa=0.0, q_regular=4, q_singular=4,
                 leaf=64, eta=2.0, qg=4, eps=5e-8):
        import torch
        self.ctx = ctx
        self.v = np.ascontiguousarray(v, dtype=np.float64)
        self.tri = np.ascontiguousarray(tri, dtype=np.int32)
        self.kernel, self.kappa = kernel, float(kappa)
        self.q_regular, self.q_singular = q_regular, q_singular
        self.qg, self.eps = qg, eps
        self.cplx = kernel == HELMHOLTZ
        self.adtype = torch.complex128 if self.cplx else torch.float64
        self.mesh = Mesh(torch.from_numpy(self.v), torch.from_numpy(self.tri))
        t0 = time.perf_counter()
        self.ct = ClusterTree(self.v, self.tri, leaf=leaf)
        near, far = block_tree(self.ct, eta=eta)
        # blocks in decreasing estimated cost (near field: blocks on the
        # diagonal carry the identical pairs, then by size; coupling: by the
        # clusters' sizes, which their ranks follow): the block kernel is
        # dispatched in list order, so the largest blocks start first and the
        # small ones fill the tail (longest-processing-time order)
        size = (self.ct.end - self.ct.begin).astype(np.int64)
        key = [(-(int(t) == int(s)), -int(size[t] * size[s])) for t, s in near]
        self.near = near[sorted(range(len(near)), key=lambda k: key[k])]
        fkey = [-int(size[t] * size[s]) for t, s in far]
        self.far = far[sorted(range(len(far)), key=lambda k: fkey[k])]
        self.t_tree = time.perf_counter() - t0
        # heights: leaves 0, fathers 1 + max(sons)
        n = self.ct.n
        self.height = np.zeros(n, dtype=np.int32)
        for c in range(n - 1, -1, -1):  # sons have larger numbers (pre-order)
            s = self.ct.sons[c]
            if s[0] >= 0:
                self.height[c] = 1 + max(self.height[s[0]], self.height[s[1]])
        # clusters that need a basis: those of an admissible block and all
        # their descendants (a father's nested basis is expressed through its
        # sons'); the clusters above the admissible part of the block tree
        # (the root and its first descendants) enter no product
        self.needed = np.zeros(n, dtype=bool)
        self.needed[np.asarray(far, dtype=np.int64).ravel()] = True
        for c in range(n):  # fathers before sons (pre-order)
            s = self.ct.sons[c]
            if s[0] >= 0 and self.needed[c]:
                self.needed[s] = True
        self.z, self.zn, self.zw, self.delta = green_points(self.ct.box, qg)
        self.m = self.zw.shape[1]

    def op(self, layer):
        return make_op(self.kernel, layer, q_regular=self.q_regular, q_singular=self.q_singular,
                       kappa=self.kappa)

    # ----------------------------------------------------------- bases
    def _host_copy(self, A):
        """A device tensor copied into the pinned host buffer (a numpy view,
        valid until the next call)."""
        nbytes = A.numel() * A.element_size()
        h = _pinned(nbytes)[:nbytes].view(A.dtype)
        h.copy_(A)
        return h.numpy()

    def basis(self, side):
        """Construct the nested cluster basis of one side, level by level."""
        return self.bases((side,))[0]

    def bases(self, sides=(0, 1), rank_caps=None, device_inverse=True):
        """Construct the nested cluster bases of several sides together, level
        by level (the clusters of self.needed only; the others keep rank 0 and
        no pivots): per level one Green-matrix launch per side into one buffer,
        one copy to the host, one pivot search over the clusters of every side
        (twice the clusters per call keep the host threads busy at the top
        levels), then one contraction launch per side.

        rank_caps (optional, one int array over the clusters per side, e.g.
        from the learned rank head): a level's pivot search is bounded by the
        largest cap of its clusters instead of min(rows, 2m), which sizes the
        pivot and inverse buffers; a level where some cluster reaches that
        bound is searched again without it, so the bases are the ones the
        plain search gives.  self.cap_stats counts levels and fallbacks.

        device_inverse: the host search returns pivots only and the pivot
        blocks are inverted on the device (bem_pivot_inverse), so no
        inverse is formed on or copied from the host; otherwise bem_aca
        forms them on the host.  self.bases_time splits the wall time into
        device work (Green matrices, and the previous level's inverses and
        contractions, waited for at the copy), the copy to the host and the
        host pivot search."""
        import torch
        ct, m = self.ct, self.m
        Bs = [ClusterBasis(side, ct.n) for side in sides]
        op = self.op(SLP)
        self.cap_stats = {"levels": 0, "fallbacks": 0}
        self.bases_time = {"device": 0.0, "copy": 0.0, "pivot_search": 0.0}
        for h in range(int(self.height.max()) + 1):
            cls = np.nonzero((self.height == h) & self.needed)[0]
            if cls.size == 0:
                continue
            lvs, nrows_all = [], []
            for B in Bs:
                lv = LevelPlan()
                lv.cls = cls
                rows = []
                for c in cls:
                    s = ct.sons[c]
                    r = ct.idx(c) if s[0] < 0 else np.concatenate([B.piv[s[0]], B.piv[s[1]]])
                    B.rows[c] = r.astype(np.int32)
                    rows.append(B.rows[c])
                lv.nrows_h = np.array([r.size for r in rows], dtype=np.int32)
                lv.row_idx_h = np.concatenate(rows)
                lvs.append(lv)
                nrows_all.append(lv.nrows_h)
            nrows_all = np.concatenate(nrows_all)
            a_all = np.zeros(nrows_all.size, dtype=np.int64)  # offsets into the level's buffer
            a_all[1:] = np.cumsum(nrows_all.astype(np.int64) * 2 * m)[:-1]
            A_all = torch.empty(int(nrows_all.astype(np.int64).sum() * 2 * m), dtype=self.adtype,
                                device="cuda")
            base = 0
            for B, lv in zip(Bs, lvs):
                nrows = lv.nrows_h
                rp = np.zeros(cls.size + 1, dtype=np.int32)
                rp[1:] = np.cumsum(nrows)
                a_off = np.zeros(cls.size, dtype=np.int64)
                a_off[1:] = np.cumsum(nrows.astype(np.int64) * 2 * m)[:-1]
                size = int(nrows.astype(np.int64).sum() * 2 * m)
                (lv.row_ptr, lv.row_idx, lv.z, lv.zn, lv.zw, lv.delta, lv.a_off) = _upload(
                    (rp, np.int32), (lv.row_idx_h, np.int32), (self.z[cls], np.float64),
                    (self.zn[cls], np.float64), (self.zw[cls], np.float64),
                    (self.delta[cls], np.float64), (a_off, np.int64))
                lv.A = A_all[base:base + size]
                lv.max_rows = int(nrows.max())
                self.ctx.green_matrix(self.mesh, op, B.side, lv.row_ptr, lv.row_idx, lv.z, lv.zn,
                                      lv.zw, lv.delta, lv.a_off, lv.A, max_rows=lv.max_rows)
                base += size
            t0 = time.perf_counter()
            self.ctx.check()
            _STAGER.reset()  # the stream is idle: staged uploads are done
            t1 = time.perf_counter()
            A_h = self._host_copy(A_all)
            Af = A_h.view(np.float64) if self.cplx else A_h
            t2 = time.perf_counter()
            max_rank = int(min(nrows_all.max(), 2 * m))
            host_inv = not device_inverse
            if rank_caps is not None:
                cap = max(int(np.max(rank_caps[si][cls])) for si in range(len(Bs)))
                bound = max(1, min(max_rank, cap))
                rank_all, prow, pcol, pinv = aca(Af, a_all, nrows_all, 2 * m, self.eps, bound,
                                                 is_complex=self.cplx, inverse=host_inv)
                self.cap_stats["levels"] += 1
                if bound < max_rank and int(rank_all.max()) >= bound:  # the bound may have cut
                    self.cap_stats["fallbacks"] += 1
                    rank_all, prow, pcol, pinv = aca(Af, a_all, nrows_all, 2 * m, self.eps,
                                                     max_rank, is_complex=self.cplx,
                                                     inverse=host_inv)
                else:
                    max_rank = bound
            else:
                rank_all, prow, pcol, pinv = aca(Af, a_all, nrows_all, 2 * m, self.eps, max_rank,
                                                 is_complex=self.cplx, inverse=host_inv)
            t3 = time.perf_counter()
            self.bases_time["device"] += t1 - t0
            self.bases_time["copy"] += t2 - t1
            self.bases_time["pivot_search"] += t3 - t2
            for si, (B, lv) in enumerate(zip(Bs, lvs)):
                sl = slice(si * cls.size, (si + 1) * cls.size)
                nrows, rank = lv.nrows_h, rank_all[sl]
                for p, c in enumerate(cls):
                    k = rank[p]
                    B.rank[c] = k
                    B.piv[c] = B.rows[c][prow[sl][p, :k]]
                    B.where[c] = (len(B.levels), p)
                v_off = np.zeros(cls.size, dtype=np.int64)
                v_off[1:] = np.cumsum(nrows.astype(np.int64) * rank)[:-1]
                lv.v_off_h = v_off
                lv.rank_h, lv.pcol_h, lv.prow_h = rank, pcol[sl], prow[sl]
                lv.nrows, lv.rank, lv.piv_cols, lv.piv_rows, lv.v_off = _upload(
                    (nrows, np.int32), (rank, np.int32), (pcol[sl], np.int32),
                    (prow[sl], np.int32), (v_off, np.int64))
                lv.max_rank = max_rank
                if device_inverse:
                    lv.pinv = torch.empty((cls.size, max_rank * max_rank * (2 if self.cplx else 1)),
                                          dtype=torch.float64, device="cuda")
                    self.ctx.pivot_inverse(self.cplx, lv.nrows, lv.rank, max_rank, lv.piv_rows,
                                           lv.piv_cols, lv.A, lv.a_off, 2 * m, lv.pinv)
                else:
                    lv.pinv = _dev(pinv[sl], torch.float64)
                lv.V = torch.empty(int((nrows.astype(np.int64) * rank).sum()), dtype=self.adtype,
                                   device="cuda")
                self.ctx.basis_contract(self.cplx, lv.nrows, lv.rank, max_rank, lv.piv_cols,
                                        lv.pinv, lv.A, lv.a_off, 2 * m, lv.V, lv.v_off,
                                        max_rows=lv.max_rows)
                B.levels.append(lv)
        t0 = time.perf_counter()
        self.ctx.check()
        self.bases_time["device"] += time.perf_counter() - t0
        for B in Bs:
            B.replay = None  # built by the first basis_replay
        return Bs

    def _replay_plan(self, B):
        """Inputs of all levels concatenated (level by level), so that a replay
        is one Green-matrix launch and one contraction launch: with the pivots
        fixed, no level depends on another's results.  The levels' A and V
        become views of the combined buffers."""
        import torch
        Ls, m2 = B.levels, 2 * self.m
        rp = LevelPlan()
        cls = np.concatenate([lv.cls for lv in Ls])
        nrows = np.concatenate([lv.nrows_h for lv in Ls]).astype(np.int64)
        ptr = np.zeros(cls.size + 1, dtype=np.int32)
        ptr[1:] = np.cumsum(nrows)
        a_off = np.zeros(cls.size, dtype=np.int64)
        a_off[1:] = np.cumsum(nrows * m2)[:-1]
        rank = np.concatenate([lv.rank_h for lv in Ls]).astype(np.int32)
        v_off = np.zeros(cls.size, dtype=np.int64)
        v_off[1:] = np.cumsum(nrows * rank)[:-1]
        K = max(lv.max_rank for lv in Ls)
        f = 2 if self.cplx else 1
        pcol = np.zeros((cls.size, K), dtype=np.int32)
        pinv_d = torch.zeros((cls.size, K * K * f), dtype=torch.float64, device="cuda")
        i = 0
        for lv in Ls:
            n_l = lv.cls.size
            for p in range(n_l):
                k = int(lv.rank_h[p])
                pcol[i + p, :k] = lv.pcol_h[p, :k]
            # each inverse occupies the first k^2 entries of its slot
            w = lv.max_rank * lv.max_rank * f
            pinv_d[i:i + n_l, :w].copy_(lv.pinv.view(n_l, -1)[:, :w])
            i += n_l
        rp.ncl = int(cls.size)
        rp.row_ptr = _dev(ptr, torch.int32)
        rp.row_idx = _dev(np.concatenate([lv.row_idx_h for lv in Ls]), torch.int32)
        rp.z, rp.zn = _dev(self.z[cls], torch.float64), _dev(self.zn[cls], torch.float64)
        rp.zw, rp.delta = _dev(self.zw[cls], torch.float64), _dev(self.delta[cls], torch.float64)
        rp.a_off, rp.v_off = _dev(a_off, torch.int64), _dev(v_off, torch.int64)
        rp.nrows, rp.rank = _dev(nrows, torch.int32), _dev(rank, torch.int32)
        rp.piv_cols, rp.pinv, rp.max_rank = _dev(pcol, torch.int32), pinv_d, K
        rp.max_rows = int(nrows.max())
        rp.A = torch.empty(int((nrows * m2).sum()), dtype=self.adtype, device="cuda")
        rp.V = torch.empty(int((nrows * rank).sum()), dtype=self.adtype, device="cuda")
        ao = vo = 0
        for lv in Ls:
            na, nv = lv.A.numel(), lv.V.numel()
            rp.A[ao:ao + na].copy_(lv.A)
            rp.V[vo:vo + nv].copy_(lv.V)
            lv.A, lv.V = rp.A[ao:ao + na], rp.V[vo:vo + nv]
            ao, vo = ao + na, vo + nv
        return rp

    def basis_replay(self, B, stream=None):
        """Enqueue the GPU part of a basis construction again (Green matrices
        and contractions of every level, one launch each) with the pivots and
        inverses already chosen."""
        if B.replay is None:
            B.replay = self._replay_plan(B)
        rp = B.replay
        self.ctx.green_matrix(self.mesh, self.op(SLP), B.side, rp.row_ptr, rp.row_idx, rp.z, rp.zn,
                              rp.zw, rp.delta, rp.a_off, rp.A, max_rows=rp.max_rows, stream=stream)
        self.ctx.basis_contract(self.cplx, rp.nrows, rp.rank, rp.max_rank, rp.piv_cols, rp.pinv,
                                rp.A, rp.a_off, 2 * self.m, rp.V, rp.v_off, max_rows=rp.max_rows,
                                stream=stream)

    # ----------------------------------------------------------- blocks
    def near_blocks(self, mirror=False):
        """Triangle lists of the inadmissible blocks, outputs back to back in
        the order of self.near.  mirror (a single layer): of each pair (t, s),
        (s, t) with t != s only t < s is evaluated, the other written as its
        transpose (edge-adjacent entries evaluated as (j, i)); a block (t, t)
        is its own mirror: its entries with row >= column are evaluated and
        written transposed too."""
        ct = self.ct
        size = (ct.end - ct.begin).astype(np.int64)
        start = ct.begin.astype(np.int64)
        return _block_lists(self.near, (ct.perm, start, size), (ct.perm, start, size), mirror,
                            keep_diag=True)

    def coupling_blocks(self, row_basis, col_basis, mirror=False):
        """Pivot lists of the admissible blocks, outputs back to back in the
        order of self.far.  mirror (a single layer with one basis for rows and
        columns): of each pair (t, s), (s, t) only the block with t < s is
        evaluated and the other is written as its transpose."""
        if mirror and row_basis is not col_basis:
            raise ValueError("mirrored coupling blocks need one basis for rows and columns")
        return _block_lists(self.far, row_basis.flat_pivots(), col_basis.flat_pivots(), mirror,
                            keep_diag=False)
