"""Oracle cluster tree, block tree and Green quadrature points (plain numpy).

TEST INFRASTRUCTURE ONLY.  Written from Sec. 2.3 of the paper:

* cluster tree by geometric subdivision (Sec. 2.3, cluster trees): a cluster
  with more than ``leaf`` triangles is split at the midpoint of the longest
  side of the bounding box of its triangle centroids; a centroid exactly on
  the midpoint goes to the first son; ties between equally long sides go to
  the lowest axis.  Clusters are numbered in depth-first pre-order.
* bounding boxes B_t are unions of the triangles' vertex boxes (Sec. 2.3,
  admissibility);
* block tree from (root, root): a block is an admissible leaf when
  max(diam B_t, diam B_s) <= eta dist(B_t, B_s) (Euclidean box diagonal and
  box-to-box distance), an inadmissible (near-field) leaf when t or s is a
  leaf cluster, and otherwise has the sons sons(t) x sons(s);
* the Green box omega_t is B_t grown by delta_t / 2 on every side, with
  delta_t = diam B_t, so dist(B_t, boundary of omega_t) = delta_t / 2
  (Sec. 2.3, Green boxes); its six faces carry q_G x q_G Gauss points each,
  in face order (-x, +x, -y, +y, -z, +z), then the first tangential axis
  (lower axis index), then the second; weights are the tensor Gauss weights
  times the face area, normals are the outward face normals.
"""
from dataclasses import dataclass, field

import numpy as np

from . import gauss01


@dataclass
class Cluster:
    idx: np.ndarray            # triangle ids, in order
    lo: np.ndarray             # bounding box B_t
    hi: np.ndarray
    sons: list = field(default_factory=list)
    level: int = 0


def tri_boxes(v, tri):
    p = v[tri]  # (nt, 3, 3)
    return p.min(axis=1), p.max(axis=1)


def centroids(v, tri):
    p = v[tri]
    return (p[:, 0, :] + p[:, 1, :] + p[:, 2, :]) / 3.0


def cluster_tree(v, tri, leaf=64):
    """Depth-first pre-order list of Cluster objects; element 0 is the root."""
    tlo, thi = tri_boxes(v, tri)
    cen = centroids(v, tri)
    out = []

    def make(idx, level):
        c = Cluster(idx=idx, lo=tlo[idx].min(axis=0), hi=thi[idx].max(axis=0), level=level)
        me = len(out)
        out.append(c)
        if idx.size > leaf:
            clo = cen[idx].min(axis=0)
            chi = cen[idx].max(axis=0)
            ext = chi - clo
            axis = 0
            for a in (1, 2):
                if ext[a] > ext[axis]:
                    axis = a
            mid = (clo[axis] + chi[axis]) / 2.0
            left = cen[idx, axis] <= mid
            if left.all() or (~left).all():
                return me
            s1 = make(idx[left], level + 1)
            s2 = make(idx[~left], level + 1)
            c.sons = [s1, s2]
        return me

    make(np.arange(tri.shape[0], dtype=np.int32), 0)
    return out


def box_diam(lo, hi):
    return float(np.sqrt(np.sum((hi - lo) ** 2)))


def box_dist(lo1, hi1, lo2, hi2):
    gap = np.maximum(0.0, np.maximum(lo2 - hi1, lo1 - hi2))
    return float(np.sqrt(np.sum(gap ** 2)))


def block_tree(clusters, eta=2.0):
    """Lists (near, far) of (t, s) cluster-index pairs in depth-first order."""
    near, far = [], []

    def rec(t, s):
        ct, cs = clusters[t], clusters[s]
        dmax = max(box_diam(ct.lo, ct.hi), box_diam(cs.lo, cs.hi))
        if dmax <= eta * box_dist(ct.lo, ct.hi, cs.lo, cs.hi):
            far.append((t, s))
        elif not ct.sons or not cs.sons:
            near.append((t, s))
        else:
            for t2 in ct.sons:
                for s2 in cs.sons:
                    rec(t2, s2)

    rec(0, 0)
    return near, far


def green_box(c: Cluster):
    """(lo, hi, delta) of omega_t."""
    delta = box_diam(c.lo, c.hi)
    return c.lo - delta / 2.0, c.hi + delta / 2.0, delta


def green_points(lo, hi, qg):
    """Points (6 qg^2, 3), outward normals (6 qg^2, 3), weights (6 qg^2,)."""
    gx, gw = gauss01(qg)
    z, zn, zw = [], [], []
    for axis in range(3):
        u, w = [a for a in range(3) if a != axis]
        area = (hi[u] - lo[u]) * (hi[w] - lo[w])
        for side, val in ((-1.0, lo[axis]), (1.0, hi[axis])):
            for a in range(qg):
                for b in range(qg):
                    p = np.zeros(3)
                    p[axis] = val
                    p[u] = lo[u] + gx[a] * (hi[u] - lo[u])
                    p[w] = lo[w] + gx[b] * (hi[w] - lo[w])
                    nrm = np.zeros(3)
                    nrm[axis] = side
                    z.append(p)
                    zn.append(nrm)
                    zw.append(gw[a] * gw[b] * area)
    return np.array(z), np.array(zn), np.array(zw)
