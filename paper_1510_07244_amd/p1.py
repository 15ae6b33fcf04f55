"""Galerkin matrices of piecewise-linear (P1) bases (Sec. 2.2, eq.
reference_integral with low-order polynomial basis functions), driving the
C-ABI: the 3 x 3 local matrices of the triangle pairs (bem_p1_pairs) and
their sums over the triangles around each vertex pair (bem_p1_gather).
This module only builds index lists (the triangles around each vertex) and
orders the calls.
"""
import numpy as np


def vertex_stars(tri, vertices):
    """For the given vertices: the triangles around each (CSR: ptr, triangle
    ids, the vertex's position 0..2 in each), and the sorted set of those
    triangles with the star entries renumbered into it."""
    tri = np.asarray(tri)
    vertices = np.asarray(vertices, dtype=np.int64)
    want = np.zeros(int(tri.max()) + 1 if tri.size else 0, dtype=bool)
    want[vertices] = True
    t_ids, locs, verts = [], [], []
    for k in range(3):
        hit = np.nonzero(want[tri[:, k]])[0]
        t_ids.append(hit)
        locs.append(np.full(hit.size, k))
        verts.append(tri[hit, k])
    t_ids, locs, verts = np.concatenate(t_ids), np.concatenate(locs), np.concatenate(verts)
    tset = np.unique(t_ids)
    where = {int(v): i for i, v in enumerate(vertices)}
    order = np.lexsort((t_ids, np.array([where[int(v)] for v in verts], dtype=np.int64)))
    owner = np.array([where[int(v)] for v in verts], dtype=np.int64)[order]
    ptr = np.zeros(vertices.size + 1, dtype=np.int32)
    np.add.at(ptr, owner + 1, 1)
    ptr = np.cumsum(ptr).astype(np.int32)
    local = np.searchsorted(tset, t_ids[order]).astype(np.int32)
    return ptr, local, locs[order].astype(np.int32), tset.astype(np.int32)


def p1_block(ctx, mesh, tri, op, row_vertices, col_vertices, stream=None):
    """Dense block (len(row_vertices) x len(col_vertices), a column-major
    device tensor flattened) of the P1 Galerkin matrix of `op`: entry (v, w)
    sums the local matrices of every triangle around v against every
    triangle around w.  mesh: the device Mesh; tri: its host triangles."""
    import torch
    rp, rt, rl, rset = vertex_stars(tri, row_vertices)
    cp, ct, cl, cset = vertex_stars(tri, col_vertices)
    R, C = np.meshgrid(rset, cset, indexing="ij")
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32)).cuda()
    cplx = op.kernel == 1
    dt = torch.complex128 if cplx else torch.float64
    local = torch.empty(9 * R.size, dtype=dt, device="cuda")
    ctx.p1_pairs(mesh, op, dev(R.ravel()), dev(C.ravel()), local, stream)
    out = torch.empty(len(row_vertices) * len(col_vertices), dtype=dt, device="cuda")
    ctx.p1_gather(dev(rp), dev(rt), dev(rl), dev(cp), dev(ct), dev(cl), rset.size, cset.size,
                  local, out, stream)
    return out
