"""Plain FP64 oracle of the learned order selector's inputs, targets and
decision rule.

TEST INFRASTRUCTURE ONLY (like the rest of ``oracle``).

For a regular (vertex-disjoint) pair (tau_i, tau_j) with centroids c_i, c_j,
areas |tau|, longest edges d and unit normals n (from the mesh order):

    D   = max(d_i, d_j),  r = |c_i - c_j|
    x0  = ln(r / D)
    x1  = sqrt(3)/4 d_i^2 / |tau_i|          (1 for an equilateral triangle)
    x2  = sqrt(3)/4 d_j^2 / |tau_j|
    x3  = min(|tau_i|, |tau_j|) / max(|tau_i|, |tau_j|)
    x4  = kappa D                            (0 for Laplace)
    x5  = ln max(|n_i - n_j|^2, 1e-12)       (= ln 2(1 - cos angle))
    x6  = 0 single layer, 1 double layer
    x7  = ln max(|<c_i - c_j, n_j>| / r, 1e-8)

(the logarithms resolve nearly parallel normals and nearly in-plane
separations, where the double layer's entries are small and its rules'
relative errors large).

Targets, for q = 1 .. 6 (the Duffy/Gauss rule of Sec. 2.2 with q Gauss
points per coordinate; q^4 points per pair) against the same rule at
q_ref = 8:

    e_q = log10( max(|G_q - G_ref| / max(|G_ref|, 1e-3 s), 1e-16) ),
    s   = |tau_i| |tau_j| / (4 pi r)

(a floor relative to the size s of a single-layer entry keeps pairs whose
double-layer entry vanishes, such as coplanar ones, finite).

Decision: the smallest order q in [q_min, q_plain - 1] such that the
predicted error plus a margin is at most log10(tol) at q and at every order
between q and q_plain - 1; the plain order q_plain when q_plain - 1 already
fails (the plain rule is the fallback).
"""
import numpy as np

from . import entries, LAPLACE, SLP, RULE_DUFFY

Q_OUT = 6    # outputs: predicted e_q for q = 1 .. 6
Q_REF = 8


def _tri_geometry(v, tri):
    p = v[tri]                                   # (nt, 3, 3)
    c = p.mean(axis=1)
    e = np.stack([p[:, 1] - p[:, 0], p[:, 2] - p[:, 1], p[:, 0] - p[:, 2]], axis=1)
    d = np.sqrt((e ** 2).sum(-1)).max(axis=1)
    cr = np.cross(p[:, 1] - p[:, 0], p[:, 2] - p[:, 0])
    area = 0.5 * np.sqrt((cr ** 2).sum(-1))
    n = cr / (2.0 * area)[:, None]
    return c, d, area, n


def features(v, tri, rows, cols, layer=SLP, kappa=0.0):
    """(n, 8) FP64 inputs of the pairs (rows[k], cols[k])."""
    v = np.asarray(v, dtype=np.float64)
    tri = np.asarray(tri)
    rows, cols = np.asarray(rows), np.asarray(cols)
    c, d, area, n = _tri_geometry(v, tri)
    D = np.maximum(d[rows], d[cols])
    sep = c[rows] - c[cols]
    r = np.sqrt((sep ** 2).sum(-1))
    f = np.empty((rows.size, 8))
    f[:, 0] = np.log(r / D)
    f[:, 1] = np.sqrt(3.0) / 4.0 * d[rows] ** 2 / area[rows]
    f[:, 2] = np.sqrt(3.0) / 4.0 * d[cols] ** 2 / area[cols]
    f[:, 3] = np.minimum(area[rows], area[cols]) / np.maximum(area[rows], area[cols])
    f[:, 4] = kappa * D
    f[:, 5] = np.log(np.maximum(((n[rows] - n[cols]) ** 2).sum(-1), 1e-12))
    f[:, 6] = float(layer)
    f[:, 7] = np.log(np.maximum(np.abs((sep * n[cols]).sum(-1)) / r, 1e-8))
    return f


def targets(v, tri, rows, cols, kernel=LAPLACE, layer=SLP, kappa=0.0):
    """(n, 6) FP64 targets e_q, q = 1 .. 6."""
    v = np.asarray(v, dtype=np.float64)
    rows, cols = np.asarray(rows, dtype=np.int32), np.asarray(cols, dtype=np.int32)
    c, d, area, n = _tri_geometry(v, np.asarray(tri))
    r = np.sqrt(((c[rows] - c[cols]) ** 2).sum(-1))
    s = area[rows] * area[cols] / (4.0 * np.pi * r)
    kw = dict(kernel=kernel, layer=layer, kappa=kappa, rule=RULE_DUFFY, q_sing=4)
    ref = entries(v, tri, rows, cols, q_reg=Q_REF, **kw)
    den = np.maximum(np.abs(ref), 1e-3 * s)
    out = np.empty((rows.size, Q_OUT))
    for q in range(1, Q_OUT + 1):
        g = entries(v, tri, rows, cols, q_reg=q, **kw)
        out[:, q - 1] = np.log10(np.maximum(np.abs(g - ref) / den, 1e-16))
    return out


def decide(pred, q_plain, tol, margin, q_min=2):
    """Orders (int) from predicted errors pred (n, 6)."""
    pred = np.asarray(pred)
    out = np.full(pred.shape[0], q_plain, dtype=np.int64)
    lt = np.log10(tol)
    ok = np.ones(pred.shape[0], dtype=bool)
    for q in range(q_plain - 1, q_min - 1, -1):
        ok &= pred[:, q - 1] + margin <= lt
        out[ok] = q
    return out
