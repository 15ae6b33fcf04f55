"""Host helpers of the H^2 accuracy tests (test code, not part of the
library): the full cluster bases expanded from the nested ones, and the
H^2 approximation of an admissible block.

Nested bases (Sec. 2.4) store for each father t only the transfer matrix
V^_t, whose rows belong to the union of the sons' pivots; the full basis is
V_t = diag(V_t1, V_t2) V^_t, rows ordered like the cluster's triangles.
"""
import numpy as np


class FullBases:
    """Full bases V_t of one nested basis, expanded on the host (cached)."""

    def __init__(self, h, B):
        self.h, self.B = h, B
        self.cache = {}
        self.flat = {}  # level index -> host copy of that level's V

    def _vhat(self, c):
        li, p = self.B.where[c]
        if li not in self.flat:
            self.flat[li] = self.B.levels[li].V.cpu().numpy()
        lv = self.B.levels[li]
        n, k = int(lv.nrows_h[p]), int(self.B.rank[c])
        o = int(lv.v_off_h[p])
        return self.flat[li][o:o + n * k].reshape(k, n).T

    def __call__(self, c):
        c = int(c)
        if c not in self.cache:
            s = self.h.ct.sons[c]
            if s[0] < 0:
                self.cache[c] = self._vhat(c)
            else:
                V1, V2 = self(s[0]), self(s[1])
                D = np.zeros((V1.shape[0] + V2.shape[0], V1.shape[1] + V2.shape[1]),
                             dtype=V1.dtype)
                D[:V1.shape[0], :V1.shape[1]] = V1
                D[V1.shape[0]:, V1.shape[1]:] = V2
                self.cache[c] = D @ self._vhat(c)
        return self.cache[c]


def full_basis(h, B, c):
    """V_c of the nested basis B (one-off; use FullBases for many clusters)."""
    return FullBases(h, B)(c)


def coupling_offsets(h, V, W):
    """Output offsets of the admissible blocks in the order of h.far."""
    sizes = np.array([V.piv[t].size * W.piv[s].size for t, s in h.far], dtype=np.int64)
    return np.concatenate([[0], np.cumsum(sizes)[:-1]]), sizes


def coupling_matrix(flat, off, kt, ks):
    """Block k of a packed coupling output as a kt x ks array."""
    return flat[off:off + kt * ks].reshape(ks, kt).T
