// Host-side H^2 structure: cluster tree by geometric bisection and block tree
// with the standard admissibility condition (Sec. 2.3).  Plain host code; it
// is adaptive and cheap next to the quadrature.
#include <algorithm>
#include <cmath>
#include <vector>

#include "bem_internal.h"

namespace {

struct Box {
  double lo[3], hi[3];
};

double diam(const Box &b) {
  double s = 0;
  for (int k = 0; k < 3; ++k) s += (b.hi[k] - b.lo[k]) * (b.hi[k] - b.lo[k]);
  return std::sqrt(s);
}

double dist(const Box &a, const Box &b) {
  double s = 0;
  for (int k = 0; k < 3; ++k) {
    const double g = std::max(0.0, std::max(b.lo[k] - a.hi[k], a.lo[k] - b.hi[k]));
    s += g * g;
  }
  return std::sqrt(s);
}

struct TreeBuilder {
  const double *v;
  const int32_t *tri;
  int32_t leaf;
  std::vector<double> cen;   // [nt][3] triangle centroids
  std::vector<Box> tbox;     // per triangle
  std::vector<int32_t> perm;
  std::vector<int32_t> begin, end, son0, son1, level;
  std::vector<Box> box;

  int make(int32_t b, int32_t e, int32_t lev) {
    const int me = (int)begin.size();
    Box bb;
    for (int k = 0; k < 3; ++k) bb.lo[k] = INFINITY, bb.hi[k] = -INFINITY;
    for (int32_t p = b; p < e; ++p)
      for (int k = 0; k < 3; ++k) {
        bb.lo[k] = std::min(bb.lo[k], tbox[perm[p]].lo[k]);
        bb.hi[k] = std::max(bb.hi[k], tbox[perm[p]].hi[k]);
      }
    begin.push_back(b);
    end.push_back(e);
    son0.push_back(-1);
    son1.push_back(-1);
    level.push_back(lev);
    box.push_back(bb);
    if (e - b <= leaf) return me;
    // split at the midpoint of the longest side of the centroid box; a
    // centroid on the midpoint goes to the first son; ties between sides go
    // to the lowest axis
    double clo[3] = {INFINITY, INFINITY, INFINITY}, chi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int32_t p = b; p < e; ++p)
      for (int k = 0; k < 3; ++k) {
        clo[k] = std::min(clo[k], cen[3 * (size_t)perm[p] + k]);
        chi[k] = std::max(chi[k], cen[3 * (size_t)perm[p] + k]);
      }
    int axis = 0;
    for (int k = 1; k < 3; ++k)
      if (chi[k] - clo[k] > chi[axis] - clo[axis]) axis = k;
    const double mid = (clo[axis] + chi[axis]) / 2.0;
    // stable partition keeps the original order inside each son
    auto first = perm.begin() + b, last = perm.begin() + e;
    auto cut = std::stable_partition(
        first, last, [&](int32_t t) { return cen[3 * (size_t)t + axis] <= mid; });
    const int32_t m = (int32_t)(cut - perm.begin());
    if (m == b || m == e) return me;  // cannot split (coincident centroids)
    const int s0 = make(b, m, lev + 1);
    const int s1 = make(m, e, lev + 1);
    son0[me] = s0;
    son1[me] = s1;
    return me;
  }
};

}  // namespace

extern "C" {

int bem_cluster_tree(const double *v, int32_t nv, const int32_t *tri, int32_t nt, int32_t leaf,
                     int32_t max_clusters, int32_t *perm, int32_t *ncl, int32_t *cl_begin,
                     int32_t *cl_end, int32_t *cl_son, int32_t *cl_level, double *cl_box) {
  if (!v || !tri || nv <= 0 || nt <= 0 || leaf < 1 || max_clusters < 1 || !perm || !ncl ||
      !cl_begin || !cl_end || !cl_son || !cl_level || !cl_box)
    return BEM_EINVAL;
  for (int64_t k = 0; k < 3 * (int64_t)nt; ++k)
    if (tri[k] < 0 || tri[k] >= nv) return BEM_EINVAL;
  try {
    TreeBuilder tb;
    tb.v = v;
    tb.tri = tri;
    tb.leaf = leaf;
    tb.cen.resize(3 * (size_t)nt);
    tb.tbox.resize(nt);
    tb.perm.resize(nt);
    for (int32_t i = 0; i < nt; ++i) {
      const double *p0 = v + 3 * (size_t)tri[3 * (size_t)i];
      const double *p1 = v + 3 * (size_t)tri[3 * (size_t)i + 1];
      const double *p2 = v + 3 * (size_t)tri[3 * (size_t)i + 2];
      for (int k = 0; k < 3; ++k) {
        tb.cen[3 * (size_t)i + k] = (p0[k] + p1[k] + p2[k]) / 3.0;
        tb.tbox[i].lo[k] = std::min(p0[k], std::min(p1[k], p2[k]));
        tb.tbox[i].hi[k] = std::max(p0[k], std::max(p1[k], p2[k]));
      }
      tb.perm[i] = i;
    }
    tb.make(0, nt, 0);
    const int32_t n = (int32_t)tb.begin.size();
    if (n > max_clusters) return BEM_EINVAL;
    std::copy(tb.perm.begin(), tb.perm.end(), perm);
    for (int32_t c = 0; c < n; ++c) {
      cl_begin[c] = tb.begin[c];
      cl_end[c] = tb.end[c];
      cl_son[2 * c] = tb.son0[c];
      cl_son[2 * c + 1] = tb.son1[c];
      cl_level[c] = tb.level[c];
      for (int k = 0; k < 3; ++k) {
        cl_box[6 * (size_t)c + k] = tb.box[c].lo[k];
        cl_box[6 * (size_t)c + 3 + k] = tb.box[c].hi[k];
      }
    }
    *ncl = n;
  } catch (...) {
    return BEM_ENOMEM;
  }
  return BEM_OK;
}

int bem_block_tree(int32_t ncl, const int32_t *cl_son, const double *cl_box, double eta,
                   int32_t max_blocks, int32_t *near_ts, int32_t *nnear, int32_t *far_ts,
                   int32_t *nfar) {
  if (ncl < 1 || !cl_son || !cl_box || !(eta > 0) || max_blocks < 0 || !near_ts || !nnear ||
      !far_ts || !nfar)
    return BEM_EINVAL;
  for (int32_t c = 0; c < ncl; ++c)
    for (int k = 0; k < 2; ++k)
      if (cl_son[2 * c + k] >= ncl || cl_son[2 * c + k] < -1 || cl_son[2 * c + k] == c)
        return BEM_EINVAL;
  std::vector<Box> box(ncl);
  for (int32_t c = 0; c < ncl; ++c)
    for (int k = 0; k < 3; ++k) box[c].lo[k] = cl_box[6 * (size_t)c + k], box[c].hi[k] = cl_box[6 * (size_t)c + 3 + k];
  int32_t nn = 0, nf = 0;
  bool overflow = false;
  // explicit stack in the order of the recursive definition
  std::vector<std::pair<int32_t, int32_t>> st;
  st.emplace_back(0, 0);
  size_t guard = 0;
  while (!st.empty()) {
    if (++guard > (size_t)4 * ncl * (size_t)ncl + 16) return BEM_EINVAL;  // cyclic sons
    const auto [t, s] = st.back();
    st.pop_back();
    const double dm = std::max(diam(box[t]), diam(box[s]));
    if (dm <= eta * dist(box[t], box[s])) {
      if (nf < max_blocks) far_ts[2 * nf] = t, far_ts[2 * nf + 1] = s; else overflow = true;
      ++nf;
    } else if (cl_son[2 * t] < 0 || cl_son[2 * s] < 0) {
      if (nn < max_blocks) near_ts[2 * nn] = t, near_ts[2 * nn + 1] = s; else overflow = true;
      ++nn;
    } else {
      // push in reverse so that (t1,s1), (t1,s2), (t2,s1), (t2,s2) pop in order
      for (int a = 1; a >= 0; --a)
        for (int b = 1; b >= 0; --b) st.emplace_back(cl_son[2 * t + a], cl_son[2 * s + b]);
    }
  }
  *nnear = nn;
  *nfar = nf;
  return overflow ? BEM_EINVAL : BEM_OK;
}

}  // extern "C"
