// Block assembly kernels (gfx950, wave64).  One sub-tile (up to 64 x 64
// entries of one block G[t x s]; up to 128 x 96 for a plain coupling block)
// is processed by one workgroup: regular pairs one entry per lane, the rest
// (singular pairs; near-singular pairs in the mixed form) grouped by class in
// LDS and done one pair per lane in FP64.
//   k_blocks      one workgroup per block, looping over its sub-tiles (one
//                 layer, or the single and the double layer in one pass);
//   k_persistent  a fixed grid of workgroups popping sub-tiles of many
//                 blocks (of many meshes) from a cost-sorted global queue.
// Both call the same sub-tile code, so their results are bitwise equal.
#include <hip/hip_runtime.h>

#include "bem_block_core.h"

namespace bem {
namespace {

using namespace blk;

// The thread's index, read through an empty asm statement: values derived
// from it (lane, strides of the staging loops, LDS offsets) are then formed
// where they are used instead of being hoisted to the kernel's entry and
// held, or spilled, across the sub-tile loops (the block kernels drop 30 to
// 50 registers and their scratch spills this way).
__device__ __forceinline__ int thread_id() {
  int t = __builtin_amdgcn_workitem_id_x();
  asm volatile("" : "+v"(t));
  return t;
}

struct BlockHdr {
  int64_t rp0, cp0, nr, nc, off;
  int64_t moff;       // transposed copy (coupling of a single layer), -1: none
  bool diag;          // its own mirror (moff == off): a block on the diagonal,
                      // only its entries with row >= column are evaluated
  double cx, cy, cz;  // block-local origin: first vertex of the first row triangle
};

// Validates block b of a block list; false (and the flag) if its ranges or
// output slot are invalid.  Uniform across the workgroup.
__device__ __forceinline__ bool block_header(const BlockArgs &a, int b, BlockHdr *h) {
  const int64_t rp0 = a.row_ptr[b], rp1 = a.row_ptr[b + 1];
  const int64_t cp0 = a.col_ptr[b], cp1 = a.col_ptr[b + 1];
  const int64_t off = a.out_off[b];
  bool ok = rp0 >= 0 && rp0 <= rp1 && rp1 <= a.row_len && cp0 >= 0 && cp0 <= cp1 &&
            cp1 <= a.col_len && off >= 0 && off <= a.out_len;
  const int64_t nr = rp1 - rp0, nc = cp1 - cp0;
  ok = ok && (nr == 0 || nc <= (a.out_len - off) / nr);
  int i0 = 0;
  if (ok && nr > 0 && nc > 0) {
    i0 = a.row_idx[rp0];
    ok = i0 >= 0 && i0 < a.nt;
  }
  if (!ok) {
    if (thread_id() == 0) atomicOr(a.flags, FLAG_EINVAL);
    return false;
  }
  h->rp0 = rp0;
  h->cp0 = cp0;
  h->nr = nr;
  h->nc = nc;
  h->off = off;
  h->moff = a.mirror_off ? a.mirror_off[b] : -1;
  h->diag = h->moff >= 0 && h->moff == off && nr == nc;
  if (h->moff >= 0 && nr > 0 && !h->diag &&
      (h->moff == off || h->moff > a.out_len || nc > (a.out_len - h->moff) / nr)) {
    if (thread_id() == 0) atomicOr(a.flags, FLAG_EINVAL);  // onto itself, or does not fit
    h->moff = -1;
  }
  if (nr > 0 && nc > 0) {
    h->cx = a.geo[G_V0X * a.ldg + i0];
    h->cy = a.geo[G_V0Y * a.ldg + i0];
    h->cz = a.geo[G_V0Z * a.ldg + i0];
  }
  return true;
}

// The quadrature rule into LDS (padded with zero weights to nqp points).
__device__ __forceinline__ void load_rule(const BlockArgs &a, const Lds &l) {
  const int nqp = a.nq_pad, nq = a.nq;
  for (int k = thread_id(); k < nqp; k += kThreads) {
    const bool real = k < nq;
    l.rule[k] = real ? a.rule[k] : 0.0;
    l.rule[nqp + k] = real ? a.rule[nq + k] : 0.0;
    l.rule[2 * nqp + k] = real ? a.rule[2 * nq + k] : 0.0;
  }
}

// Phase A of a sub-tile (rows r0 .. r0 + tr, columns c0 .. c0 + tc): reset
// the counters, then triangle ids (validated), vertex ids, row geometry in
// block-local coordinates and column normals (and boxes in the mixed form).
// Starts with a barrier (the previous sub-tile is done with the LDS) and ends
// with one; false (uniformly, flag raised) if a triangle id is invalid.
template <bool MIXED>
__device__ bool stage_tile(const BlockArgs &a, const Lds &l, const BlockHdr &h, int64_t r0,
                           int64_t c0, int tr, int tc) {
  const int tid = thread_id(), TR = a.tr, TC = a.tc;
  const int64_t L = a.ldg;
  const double cx = h.cx, cy = h.cy, cz = h.cz;
  __syncthreads();
  if (tid < 16) l.ccount[tid] = 0, l.cursor[tid] = 0;
  if (tid == 0) *l.count = 0, *l.bad = 0, *l.rcount = 0;
  __syncthreads();
  for (int k = tid; k < tr + tc; k += kThreads) {
    const bool isrow = k < tr;
    const int id = isrow ? a.row_idx[h.rp0 + r0 + k] : a.col_idx[h.cp0 + c0 + (k - tr)];
    if (id < 0 || id >= a.nt) {
      *l.bad = 1;
      continue;
    }
    if (isrow) {
      l.rid[k] = id;
      for (int m = 0; m < 3; ++m) l.rv[m * TR + k] = a.tri[3 * (int64_t)id + m];
      l.rg[0 * TR + k] = 2.0 * (a.geo[G_V0X * L + id] - cx);
      l.rg[1 * TR + k] = 2.0 * (a.geo[G_V0Y * L + id] - cy);
      l.rg[2 * TR + k] = 2.0 * (a.geo[G_V0Z * L + id] - cz);
      for (int m = 0; m < 6; ++m) l.rg[(3 + m) * TR + k] = 2.0 * a.geo[(G_E1X + m) * L + id];
      l.rg[9 * TR + k] = a.geo[G_SG * L + id];
      if (l.rn) {
        l.rn[k] = a.geo[G_NX * L + id];
        l.rn[TR + k] = a.geo[G_NY * L + id];
        l.rn[2 * TR + k] = a.geo[G_NZ * L + id];
      }
      if constexpr (MIXED)
        for (int m = 0; m < 6; ++m) l.rb[m * TR + k] = a.geo[(G_LOX + m) * L + id];
    } else {
      const int cl = k - tr;
      l.cid[cl] = id;
      for (int m = 0; m < 3; ++m) l.cv[m * TC + cl] = a.tri[3 * (int64_t)id + m];
      l.cn[cl] = a.geo[G_NX * L + id];
      l.cn[TC + cl] = a.geo[G_NY * L + id];
      l.cn[2 * TC + cl] = a.geo[G_NZ * L + id];
      if constexpr (MIXED) {
        l.cg[cl] = 2.0 * (a.geo[G_V0X * L + id] - cx);
        l.cg[TC + cl] = 2.0 * (a.geo[G_V0Y * L + id] - cy);
        l.cg[2 * TC + cl] = 2.0 * (a.geo[G_V0Z * L + id] - cz);
        for (int m = 0; m < 6; ++m) l.cb[m * TC + cl] = a.geo[(G_LOX + m) * L + id];
      }
    }
  }
  __syncthreads();
  if (*l.bad) {
    if (tid == 0) atomicOr(a.flags, FLAG_EINVAL);
    return false;
  }
  return true;
}

// Phase B: the column quadrature points of the rule in l.rule (nq points
// padded to nqp with zero weights), then a barrier.
template <bool MIXED>
__device__ void stage_columns(const BlockArgs &a, const Lds &l, const BlockHdr &h, int tc, int nq,
                              int nqp) {
  const int TC = a.tc;
  const int64_t L = a.ldg;
  const double cx = h.cx, cy = h.cy, cz = h.cz;
  for (int k = thread_id(); k < tc * nqp; k += kThreads) {
    const int cl = k % tc, q = k / tc;
    const int id = l.cid[cl];
    const bool real = q < nq;
    const double s = l.rule[q], t = l.rule[nqp + q];
    const double W = l.rule[2 * nqp + q] * a.geo[G_SG * L + id];  // 0 for padding
    if constexpr (!MIXED) {
      double P0 = -kPad, P1 = -kPad, P2 = -kPad;  // padding: far away
      if (real) {
        P0 = 2.0 * fma(s, a.geo[G_E1X * L + id], fma(t, a.geo[G_E2X * L + id], a.geo[G_V0X * L + id] - cx));
        P1 = 2.0 * fma(s, a.geo[G_E1Y * L + id], fma(t, a.geo[G_E2Y * L + id], a.geo[G_V0Y * L + id] - cy));
        P2 = 2.0 * fma(s, a.geo[G_E1Z * L + id], fma(t, a.geo[G_E2Z * L + id], a.geo[G_V0Z * L + id] - cz));
      }
      double *y = l.ys + 6 * ((int64_t)q * TC + cl);
      y[0] = -2.0 * P0;
      y[1] = -2.0 * P1;
      y[2] = -2.0 * P2;
      y[3] = fma(P0, P0, fma(P1, P1, P2 * P2));
      y[4] = W;
      y[5] = fma(P0, l.cn[cl], fma(P1, l.cn[TC + cl], P2 * l.cn[2 * TC + cl]));
    } else {
      // local to the column triangle: Y = 2 (s e1 + t e2); padding far away
      double P0 = -kPad, P1 = -kPad, P2 = -kPad;
      if (real) {
        P0 = 2.0 * fma(s, a.geo[G_E1X * L + id], t * a.geo[G_E2X * L + id]);
        P1 = 2.0 * fma(s, a.geo[G_E1Y * L + id], t * a.geo[G_E2Y * L + id]);
        P2 = 2.0 * fma(s, a.geo[G_E1Z * L + id], t * a.geo[G_E2Z * L + id]);
      }
      float *y = reinterpret_cast<float *>(l.ys) + 8 * ((int64_t)q * TC + cl);
      y[0] = (float)P0;
      y[1] = (float)P1;
      y[2] = (float)P2;
      y[3] = (float)W;
      y[4] = (float)fma(P0, l.cn[cl], fma(P1, l.cn[TC + cl], P2 * l.cn[2 * TC + cl]));
      y[5] = y[6] = y[7] = 0.0f;
    }
  }
  __syncthreads();
}

// Phase D: the listed pairs (front of l.list, *l.count of them) grouped by
// class (identical, edge, vertex, near-singular) into l.sorted, each group
// padded to a multiple of 64 with kNoPair so that every wave-sized chunk
// holds one class.  Expects a barrier after the listing; ends with one
// unless nothing is listed.
struct Groups {
  int seg[4];  // start of the group of class c
  int total;   // padded length
};

__device__ __forceinline__ Groups group_listed(const Lds &l) {
  const int tid = thread_id();
  const int ns = *l.count;
  Groups g;
  const int n3 = (l.ccount[3] + 63) & ~63, n2 = (l.ccount[2] + 63) & ~63,
            n1 = (l.ccount[1] + 63) & ~63, n0 = (l.ccount[0] + 63) & ~63;
  g.seg[0] = n3 + n2 + n1;
  g.seg[1] = n3 + n2;
  g.seg[2] = n3;
  g.seg[3] = 0;
  g.total = n3 + n2 + n1 + n0;
  if (ns == 0) return g;  // uniform
  for (int k = tid; k < g.total; k += kThreads) l.sorted[k] = kNoPair;
  __syncthreads();
  for (int k = tid; k < ns; k += kThreads) {
    const uint16_t code = l.list[k];
    const int cls = (code >> 12) & 3;
    l.sorted[g.seg[cls] + atomicAdd(&l.cursor[cls], 1)] = code;
  }
  __syncthreads();
  return g;
}

// Phase E for one wave-sized chunk of the grouped list (chunk start pos):
// one pair per lane in FP64.
template <int KERNEL, int LAYER, bool MIXED>
__device__ __forceinline__ void singular_chunk(const BlockArgs &a, const Lds &l,
                                               const BlockHdr &h, int64_t r0, int64_t c0,
                                               const Groups &gr, int pos) {
  const int lane = thread_id() & (kWave - 1);
  const int cls = pos < gr.seg[2] ? CLS_IDENTICAL
                  : pos < gr.seg[1] ? CLS_EDGE
                  : pos < gr.seg[0] ? CLS_VERTEX : kNearSingular;
  const uint16_t code = l.sorted[pos + lane];
  const bool active = code != kNoPair;
  const bool swapped = active && (code & kSwapped);
  const int rl = code & 63, cl = (code >> 6) & 63;
  // a swapped code is the mirror block's entry: the pair (j, i) to (c, r)
  const int64_t dst = swapped ? h.moff + (c0 + cl) + h.nc * (r0 + rl)
                              : h.off + (r0 + rl) + h.nr * (c0 + cl);
  const int64_t mdst = h.moff >= 0 && !swapped && cls != CLS_EDGE
                           ? h.moff + (c0 + cl) + h.nc * (r0 + rl) : -1;
  if (cls == kNearSingular) {
    if (active) {
      const Acc<KERNEL> v = regular_pair_fp64<KERNEL, LAYER>(a.geo, a.ldg, a.rule, a.nq, a.kappa,
                                                             l.rid[rl], l.cid[cl]);
      store_as<KERNEL, MIXED>(a.out, dst, v, a.flags);
      if (mdst >= 0) store_as<KERNEL, MIXED>(a.out, mdst, v, a.flags);
    }
    return;
  }
  PairGeo g;
  bool have = false;
  if (active)
    have = pair_geometry(a.v, a.tri, a.nv, a.geo, a.ldg, swapped ? l.cid[cl] : l.rid[rl],
                         swapped ? l.rid[rl] : l.cid[cl], cls, a.flags, &g);
  if (!have) {  // idle lane: harmless finite geometry, result discarded
    for (int c = 0; c < 3; ++c)
      g.E1i[c] = c == 0, g.E2i[c] = c == 1, g.E1j[c] = -(c == 2), g.E2j[c] = 0, g.n[c] = 0;
    g.scale = 0.0;
  }
  const Acc<KERNEL> v = ss_pair_lane<KERNEL, LAYER>(g, a.ss, cls, a.kappa);
  if (have) {
    store_as<KERNEL, MIXED>(a.out, dst, v, a.flags);
    if (mdst >= 0) store_as<KERNEL, MIXED>(a.out, mdst, v, a.flags);
  }
}

// Phase E of the one-pass form (both layers, in FP64): the pair (i, j) of a
// listed code in both layers and, if the block has a mirror, the transposed
// pair (j, i): its double layer evaluated as (j, i), its single layer copied
// (vertex and near-singular pairs: equal up to rounding) or evaluated as
// (j, i) (edge pairs: that rule is not symmetric).  The class is uniform
// across the chunk.
template <int KERNEL, bool MIXED>
__device__ __forceinline__ void singular_chunk_both(const BlockArgs &a, const Lds &l,
                                                    const BlockHdr &h, int64_t r0, int64_t c0,
                                                    const Groups &gr, int pos) {
  const int lane = thread_id() & (kWave - 1);
  const int cls = pos < gr.seg[2] ? CLS_IDENTICAL
                  : pos < gr.seg[1] ? CLS_EDGE
                  : pos < gr.seg[0] ? CLS_VERTEX : kNearSingular;
  const uint16_t code = l.sorted[pos + lane];
  const bool active = code != kNoPair;
  const int rl = code & 63, cl = (code >> 6) & 63;
  const int64_t dst = h.off + (r0 + rl) + h.nr * (c0 + cl);
  const int64_t mdst = h.moff + (c0 + cl) + h.nc * (r0 + rl);
  if (cls == kNearSingular) {  // mixed form: a regular pair summed in FP64
    if (!active) return;
    const int i = l.rid[rl], j = l.cid[cl];
    const Acc<KERNEL> vs = regular_pair_fp64<KERNEL, BEM_SLP>(a.geo, a.ldg, a.rule, a.nq, a.kappa, i, j);
    const Acc<KERNEL> vd = regular_pair_fp64<KERNEL, BEM_DLP>(a.geo, a.ldg, a.rule, a.nq, a.kappa, i, j);
    store_as<KERNEL, MIXED>(a.out, dst, vs, a.flags);
    store_as<KERNEL, MIXED>(a.out2, dst, vd, a.flags);
    if (h.moff >= 0) {
      const Acc<KERNEL> md = regular_pair_fp64<KERNEL, BEM_DLP>(a.geo, a.ldg, a.rule, a.nq, a.kappa, j, i);
      store_as<KERNEL, MIXED>(a.out, mdst, vs, a.flags);
      store_as<KERNEL, MIXED>(a.out2, mdst, md, a.flags);
    }
    return;
  }
  auto idle = [](PairGeo *g) {  // harmless finite geometry, result discarded
    for (int c = 0; c < 3; ++c)
      g->E1i[c] = c == 0, g->E2i[c] = c == 1, g->E1j[c] = -(c == 2), g->E2j[c] = 0, g->n[c] = 0;
    g->scale = 0.0;
  };
  PairGeo g;
  bool have = false;
  if (active)
    have = pair_geometry(a.v, a.tri, a.nv, a.geo, a.ldg, l.rid[rl], l.cid[cl], cls, a.flags, &g);
  if (!have) idle(&g);
  // a Helmholtz pair with an edge or a vertex in common takes both layers
  // from one pass over its eta points (uniform branch: the class is the
  // wave's)
  const bool fuse = KERNEL == BEM_HELMHOLTZ && cls != CLS_IDENTICAL;
  Acc<KERNEL> vs, vd;
  if constexpr (KERNEL == BEM_HELMHOLTZ) {
    if (fuse) ss_pair_lane_both(g, a.ss, cls, a.kappa, &vs, &vd);
  }
  if (!fuse) {
    vs = ss_pair_lane<KERNEL, BEM_SLP>(g, a.ss, cls, a.kappa);
    vd = ss_pair_lane<KERNEL, BEM_DLP>(g, a.ss, cls, a.kappa);
  }
  if (have) {
    store_as<KERNEL, MIXED>(a.out, dst, vs, a.flags);
    store_as<KERNEL, MIXED>(a.out2, dst, vd, a.flags);
  }
  // uniform: no mirror, or an identical pair of a diagonal block (its own
  // transpose, already written)
  if (h.moff < 0 || (h.diag && cls == CLS_IDENTICAL)) return;
  have = false;
  if (active)
    have = pair_geometry(a.v, a.tri, a.nv, a.geo, a.ldg, l.cid[cl], l.rid[rl], cls, a.flags, &g);
  if (!have) idle(&g);
  Acc<KERNEL> ms = vs, md;
  if constexpr (KERNEL == BEM_HELMHOLTZ) {
    if (cls == CLS_EDGE) ss_pair_lane_both(g, a.ss, cls, a.kappa, &ms, &md);
  }
  if (KERNEL != BEM_HELMHOLTZ || cls != CLS_EDGE) {
    md = ss_pair_lane<KERNEL, BEM_DLP>(g, a.ss, cls, a.kappa);
    if (cls == CLS_EDGE) ms = ss_pair_lane<KERNEL, BEM_SLP>(g, a.ss, cls, a.kappa);
  }
  if (have) {
    store_as<KERNEL, MIXED>(a.out, mdst, ms, a.flags);
    store_as<KERNEL, MIXED>(a.out2, mdst, md, a.flags);
  }
}

// Whether entry (rl, cl) of the staged sub-tile goes to the FP64 pass:
// a common vertex (cls > 0), or in the mixed form a near-singular pair
// (bounding boxes closer than ratio * the larger box diagonal).
template <bool MIXED>
__device__ __forceinline__ bool fp64_pair(const Lds &l, int TR, int TC, int rl, int cl,
                                          double ratio, int *cls_out) {
  const int cls = shared_vertex_count(l.rv[rl], l.rv[TR + rl], l.rv[2 * TR + rl], l.cv[cl],
                                      l.cv[TC + cl], l.cv[2 * TC + cl]);
  *cls_out = cls;
  bool fp64 = cls != 0;
  if constexpr (MIXED) {
    if (!fp64 && ratio > 0.0) {
      double gap2 = 0.0, di = 0.0, dj = 0.0;
      for (int m = 0; m < 3; ++m) {
        const double rlo = l.rb[m * TR + rl], rhi = l.rb[(3 + m) * TR + rl];
        const double clo = l.cb[m * TC + cl], chi = l.cb[(3 + m) * TC + cl];
        const double g = fmax(0.0, fmax(clo - rhi, rlo - chi));
        gap2 = fma(g, g, gap2);
        di = fma(rhi - rlo, rhi - rlo, di);
        dj = fma(chi - clo, chi - clo, dj);
      }
      fp64 = gap2 < ratio * ratio * fmax(di, dj);
    }
  }
  return fp64;
}

// Entry e of the lower triangle (row >= column) of an n x n tile, columns
// in turn: column c holds rows c .. n - 1 and starts at S(c) = c n - c (c -
// 1) / 2; the FP32 estimate of c is corrected to the exact one.
__device__ __forceinline__ void lower_entry(int e, int n, int *rl, int *cl) {
  const float b = 2.0f * n + 1.0f;
  int c = (int)((b - sqrtf(fmaxf(b * b - 8.0f * e, 0.0f))) * 0.5f);
  c = max(0, min(c, n - 1));
  while (c > 0 && c * n - c * (c - 1) / 2 > e) --c;
  while (c + 1 < n && (c + 1) * n - (c + 1) * c / 2 <= e) ++c;
  *cl = c;
  *rl = c + (e - (c * n - c * (c - 1) / 2));
}

// One sub-tile: rows r0 .. r0 + TR, columns c0 .. c0 + TC of the block
// (LAYER = kBoth: the single layer to a.out and the double layer to a.out2).
// After staging, the pairs of the FP64 pass are listed and grouped by class;
// then every wave takes work from one counter -- first the FP64 chunks
// (heaviest), then the regular entries 64 at a time in column-major order
// (lanes of a chunk share a column, so column points are broadcast reads)
// -- until both are done, so the FP64 work is spread over the waves instead
// of ending the sub-tile.  Returns early (uniformly) if a triangle id is
// invalid.
template <int KERNEL, int LAYER, int XC, bool MIXED>
__device__ void subtile(const BlockArgs &a, const Lds &l, const BlockHdr &h, int64_t r0,
                        int64_t c0, int coupling) {
  const int tid = thread_id(), lane = tid & (kWave - 1);
  const int nqp = a.nq_pad, TR = a.tr, TC = a.tc;
  const int64_t nr = h.nr, off = h.off;
  const double kq = 0.25 * a.kappa;
  const double scale = (LAYER == BEM_DLP ? 0.5 : 1.0) * kInv4Pi;
  const double ratio = a.near_ratio;
  const int tr = (int)min((int64_t)TR, h.nr - r0), tc = (int)min((int64_t)TC, h.nc - c0);
  // a diagonal block evaluates its entries with row >= column only (the
  // rest are their transposes): a sub-tile wholly above the diagonal is
  // skipped, a square one on it enumerates its lower triangle
  if (h.diag && r0 + tr - 1 < c0) return;  // uniform
  const bool lower = h.diag && r0 == c0 && tr == tc;
  const bool upper_skip = h.diag && !lower;
  if (!stage_tile<MIXED>(a, l, h, r0, c0, tr, tc)) return;
  stage_columns<MIXED>(a, l, h, tc, a.nq, nqp);
  // phase C: list the pairs of the FP64 pass
  for (int e = tid; e < tr * tc; e += kThreads) {
    const int rl = e % tr, cl = e / tr;
    if (h.diag && r0 + rl < c0 + cl) continue;
    int cls;
    if (!fp64_pair<MIXED>(l, TR, TC, rl, cl, ratio, &cls)) continue;
    if (coupling && cls) {
      atomicOr(a.flags, FLAG_EINVAL);
    } else {
      // an edge-adjacent pair of a mirrored block is listed twice: the
      // mirror's entry is evaluated as (j, i)
      const bool twice = LAYER != kBoth && h.moff >= 0 && cls == CLS_EDGE;
      const uint16_t code = (uint16_t)(rl | (cl << 6) | (cls << 12));
      const int n = twice ? 2 : 1;
      const int slot = atomicAdd(l.count, n);
      if (slot + n <= TR * TC) {  // else the sub-tile fails below
        l.list[slot] = code;
        if (twice) l.list[slot + 1] = code | kSwapped;
      }
      atomicAdd(&l.ccount[cls], n);
    }
  }
  __syncthreads();
  if (*l.count > TR * TC) {  // uniform: more listed pairs than list slots
    if (tid == 0) atomicOr(a.flags, FLAG_LIST);
    return;
  }
  const Groups gr = group_listed(l);
  const int nreg = lower ? tr * (tr + 1) / 2 : tr * tc;
  const int nsc = gr.total / kWave, nrc = (nreg + kWave - 1) / kWave;
  for (;;) {
    int c = 0;
    if (lane == 0) c = atomicAdd(l.rcount, 1);
    c = __shfl(c, 0, kWave);
    if (c >= nsc + nrc) break;
    if (c < nsc) {
      if constexpr (LAYER == kBoth) {
        singular_chunk_both<KERNEL, MIXED>(a, l, h, r0, c0, gr, c * kWave);
      } else {
        singular_chunk<KERNEL, LAYER, MIXED>(a, l, h, r0, c0, gr, c * kWave);
      }
      continue;
    }
    const int e = (c - nsc) * kWave + lane;
    if (e >= nreg) continue;
    int rl, cl;
    if (lower) {
      lower_entry(e, tr, &rl, &cl);
    } else {
      rl = e % tr, cl = e / tr;
      if (upper_skip && r0 + rl < c0 + cl) continue;
    }
    int cls;
    if (fp64_pair<MIXED>(l, TR, TC, rl, cl, ratio, &cls)) continue;
    if constexpr (LAYER == kBoth) {
      Acc<KERNEL> vs, vd, vm;
      if constexpr (!MIXED) {
        regular_entry_both<KERNEL, XC>(l, TR, TC, nqp, rl, cl, kq, &vs, &vd, &vm);
      } else {
        regular_entry_both_f32<KERNEL, XC>(l, TR, TC, nqp, rl, cl, a.kappa, &vs, &vd, &vm);
      }
      const double fs = kInv4Pi, fd = 0.5 * kInv4Pi;
      vs.re *= fs;
      vd.re *= fd;
      vm.re *= fd;
      if constexpr (KERNEL == BEM_HELMHOLTZ) vs.im *= fs, vd.im *= fd, vm.im *= fd;
      const int64_t dst = off + (r0 + rl) + nr * (c0 + cl);
      store_as<KERNEL, MIXED>(a.out, dst, vs, a.flags);
      store_as<KERNEL, MIXED>(a.out2, dst, vd, a.flags);
      if (h.moff >= 0) {
        const int64_t mdst = h.moff + (c0 + cl) + h.nc * (r0 + rl);
        store_as<KERNEL, MIXED>(a.out, mdst, vs, a.flags);
        store_as<KERNEL, MIXED>(a.out2, mdst, vm, a.flags);
      }
      continue;
    }
    Acc<KERNEL> v;
    if constexpr (!MIXED) {
      v = regular_entry<KERNEL, LAYER, XC>(l, TR, TC, nqp, rl, cl, kq);
    } else {
      v = regular_entry_f32<KERNEL, LAYER, XC>(l, TR, TC, nqp, rl, cl, a.kappa);
    }
    v.re *= scale;
    if constexpr (KERNEL == BEM_HELMHOLTZ) v.im *= scale;
    store_as<KERNEL, MIXED>(a.out, off + (r0 + rl) + nr * (c0 + cl), v, a.flags);
    if (h.moff >= 0) store_as<KERNEL, MIXED>(a.out, h.moff + (c0 + cl) + h.nc * (r0 + rl), v, a.flags);
  }
}

// x-points per register chunk of the learned kernel for order q (q = 2 .. 6);
// equal to rule_chunk(q * q), so that an order map holding the plain order
// everywhere reproduces the plain kernel bit for bit.
__host__ __device__ constexpr int learned_xc(int kernel, int q) {
  return q == 2 ? 4 : q == 3 ? 9 : q == 4 ? (kernel == BEM_LAPLACE ? 8 : 4)
         : q == 5 ? 5 : (kernel == BEM_LAPLACE ? 9 : 4);
}

template <int KERNEL, int LAYER>
__device__ __forceinline__ Acc<KERNEL> regular_entry_q(int q, const Lds &l, int TR, int TC,
                                                       int nqp, int rl, int cl, double kq) {
  switch (q) {
    case 2: return regular_entry<KERNEL, LAYER, learned_xc(KERNEL, 2)>(l, TR, TC, nqp, rl, cl, kq);
    case 3: return regular_entry<KERNEL, LAYER, learned_xc(KERNEL, 3)>(l, TR, TC, nqp, rl, cl, kq);
    case 4: return regular_entry<KERNEL, LAYER, learned_xc(KERNEL, 4)>(l, TR, TC, nqp, rl, cl, kq);
    case 5: return regular_entry<KERNEL, LAYER, learned_xc(KERNEL, 5)>(l, TR, TC, nqp, rl, cl, kq);
    default: return regular_entry<KERNEL, LAYER, learned_xc(KERNEL, 6)>(l, TR, TC, nqp, rl, cl, kq);
  }
}

// Sub-tile of the learned form (plain FP64): every regular entry takes the
// Duffy/Gauss order of the order map (2 .. q_max); the entries are grouped by
// order (each group padded to a multiple of 64, one order per wave-sized
// chunk) and each order's column points are staged in turn.  Singular pairs
// as in the plain kernel.
template <int KERNEL, int LAYER>
__device__ void subtile_learned(const BlockArgs &a, const OrderRules &o, const Lds &l,
                                const BlockHdr &h, int64_t r0, int64_t c0) {
  const int tid = thread_id(), lane = tid & (kWave - 1);
  const int TR = a.tr, TC = a.tc;
  const int64_t nr = h.nr, off = h.off;
  const double kq = 0.25 * a.kappa;
  const double scale = (LAYER == BEM_DLP ? 0.5 : 1.0) * kInv4Pi;
  const int tr = (int)min((int64_t)TR, h.nr - r0), tc = (int)min((int64_t)TC, h.nc - c0);
  const int cap = TR * TC;
  if (!stage_tile<false>(a, l, h, r0, c0, tr, tc)) return;
  // classify: singular pairs to the front of the list, regular ones (with
  // their order) to the back
  for (int e = tid; e < tr * tc; e += kThreads) {
    const int rl = e % tr, cl = e / tr;
    const int cls = shared_vertex_count(l.rv[rl], l.rv[TR + rl], l.rv[2 * TR + rl], l.cv[cl],
                                        l.cv[TC + cl], l.cv[2 * TC + cl]);
    if (cls) {
      l.list[atomicAdd(l.count, 1)] = (uint16_t)(rl | (cl << 6) | (cls << 12));
      atomicAdd(&l.ccount[cls], 1);
      continue;
    }
    const int q = o.orders[off + (r0 + rl) + nr * (c0 + cl)];
    if (q < 2 || q > o.q_max) {
      atomicOr(a.flags, FLAG_EINVAL);
      continue;
    }
    l.list[cap - 1 - atomicAdd(l.rcount, 1)] = (uint16_t)(rl | (cl << 6) | (q << 12));
    atomicAdd(&l.ccount[8 + q], 1);
  }
  __syncthreads();
  // the singular pairs grouped by class at the front of sorted[], then the
  // regular ones by order (each group padded to a multiple of 64)
  const Groups gr = group_listed(l);
  const int nreg = *l.rcount;
  int seg[7];
  int total = gr.total;
  for (int q = o.q_max; q >= 2; --q) {
    seg[q] = total;
    total += (l.ccount[8 + q] + 63) & ~63;
  }
  for (int k = gr.total + tid; k < total; k += kThreads) l.sorted[k] = kNoPair;
  __syncthreads();
  for (int k = tid; k < nreg; k += kThreads) {
    const uint16_t code = l.list[cap - 1 - k];
    const int q = code >> 12;
    l.sorted[seg[q] + atomicAdd(&l.cursor[8 + q], 1)] = code;
  }
  // one phase per order present (its column points staged), the singular
  // chunks joining the first phase; the waves take chunks from a counter
  int nsc = gr.total / kWave;
  for (int q = o.q_max; q >= 1; --q) {
    const int n = q >= 2 ? l.ccount[8 + q] : 0;
    if (n == 0 && !(q == 1 && nsc > 0)) continue;  // q = 1: singular chunks alone
    if (tid == 0) l.cursor[15] = 0;
    const int xc = q >= 2 ? learned_xc(KERNEL, q) : 1;
    const int nq = q >= 2 ? o.nq[q] : 0, nqp = (nq + xc - 1) / xc * xc;
    if (n > 0) {
      for (int k = tid; k < nqp; k += kThreads) {
        const bool real = k < nq;
        l.rule[k] = real ? o.rule[q][k] : 0.0;
        l.rule[nqp + k] = real ? o.rule[q][nq + k] : 0.0;
        l.rule[2 * nqp + k] = real ? o.rule[q][2 * nq + k] : 0.0;
      }
    }
    __syncthreads();  // sorted[], the counter and the rule are in place
    if (n > 0) stage_columns<false>(a, l, h, tc, nq, nqp);
    const int nrc = ((n + 63) & ~63) / kWave;
    for (;;) {
      int c = 0;
      if (lane == 0) c = atomicAdd(&l.cursor[15], 1);
      c = __shfl(c, 0, kWave);
      if (c >= nsc + nrc) break;
      if (c < nsc) {
        singular_chunk<KERNEL, LAYER, false>(a, l, h, r0, c0, gr, c * kWave);
        continue;
      }
      const uint16_t code = l.sorted[seg[q] + (c - nsc) * kWave + lane];
      if (code == kNoPair) continue;
      const int rl = code & 63, cl = (code >> 6) & 63;
      Acc<KERNEL> v = regular_entry_q<KERNEL, LAYER>(q, l, TR, TC, nqp, rl, cl, kq);
      v.re *= scale;
      if constexpr (KERNEL == BEM_HELMHOLTZ) v.im *= scale;
      store_as<KERNEL, false>(a.out, off + (r0 + rl) + nr * (c0 + cl), v, a.flags);
    }
    nsc = 0;
    __syncthreads();  // before the next order's points and counter replace these
  }
}

template <int KERNEL, int LAYER>
__global__ __launch_bounds__(kThreads, 2) void k_blocks_learned(const BlockArgs a,
                                                                const OrderRules o) {
  extern __shared__ __align__(16) double lds_raw[];  // 16-byte aligned: ds_read_b128 of points
  BlockHdr h;
  if (!block_header(a, blockIdx.x, &h) || h.nr == 0 || h.nc == 0) return;
  const Lds l = carve<false>(lds_raw, a.nq_pad, a.tr, a.tc);
  for (int64_t r0 = 0; r0 < h.nr; r0 += a.tr)
    for (int64_t c0 = 0; c0 < h.nc; c0 += a.tc) subtile_learned<KERNEL, LAYER>(a, o, l, h, r0, c0);
}

template <int KERNEL, int LAYER, int XC, bool MIXED>
__global__ __launch_bounds__(kThreads, 2) void k_blocks(const BlockArgs a, const int coupling) {
  extern __shared__ __align__(16) double lds_raw[];  // 16-byte aligned: ds_read_b128 of points
  BlockHdr h;
  if (!block_header(a, blockIdx.x, &h) || h.nr == 0 || h.nc == 0) return;
  const Lds l = carve<MIXED>(lds_raw, a.nq_pad, a.tr, a.tc, LAYER == kBoth);
  load_rule(a, l);
  for (int64_t r0 = 0; r0 < h.nr; r0 += a.tr)
    for (int64_t c0 = 0; c0 < h.nc; c0 += a.tc)
      subtile<KERNEL, LAYER, XC, MIXED>(a, l, h, r0, c0, coupling);
}

// Persistent form: every workgroup pops work items (batch, block, r0, c0) --
// one sub-tile, or the whole block when r0 = c0 = -1 -- from a queue sorted by
// decreasing cost until it is empty; every batch shares the operator's kernel,
// precision and rules and has its own mesh, blocks, layer (single, double or
// both in one pass), sub-tile shape and output.
// Copy of a read-only struct at a wave-uniform address by scalar loads.
template <class T>
__device__ __forceinline__ T uniform_copy(const T *p) {
  static_assert(sizeof(T) % 4 == 0, "dword-sized struct");
  typedef const uint32_t __attribute__((address_space(4))) *cword_t;
  T v;
  const cword_t src = (cword_t)p;
  uint32_t *dst = reinterpret_cast<uint32_t *>(&v);
#pragma unroll
  for (int k = 0; k < (int)(sizeof(T) / 4); ++k) dst[k] = src[k];
  return v;
}

// One work item of batch entry d.x in the layer LAYER: the argument and
// header checks, the LDS layout of the entry's sub-tile shape (the rule,
// shared by every entry, loaded again where that layout moves it; no wave
// reads the LDS between the queue's barriers and the first barrier of the
// sub-tile's staging), then the sub-tile or the whole block.  Each layer has
// its own copy, so that nothing but the queue state is live across the
// choice of layer.
template <int KERNEL, int LAYER, int XC, bool MIXED>
__device__ __forceinline__ void persistent_item(const BlockArgs *__restrict__ batches, int4 d, int cp,
                                                double *lds_raw, int *carved) {
  // the entry's arguments are read where used (scalar loads from read-only
  // memory, which the compiler may repeat instead of holding or spilling
  // them across the sub-tile loops)
  const BlockArgs &a = batches[d.x];
  if (d.y < 0 || d.y >= a.nblocks) {
    if (thread_id() == 0) atomicOr(a.flags, FLAG_EINVAL);
    return;
  }
  BlockHdr h;
  if (!block_header(a, d.y, &h) || h.nr == 0 || h.nc == 0) return;
  const bool whole = d.z == -1 && d.w == -1;
  if (!whole && (d.z >= h.nr || d.w >= h.nc || d.z < 0 || d.w < 0)) {
    if (thread_id() == 0) atomicOr(a.flags, FLAG_EINVAL);
    return;
  }
  const Lds l = carve<MIXED>(lds_raw, a.nq_pad, a.tr, a.tc, LAYER == kBoth);
  const int shape = a.tr | (a.tc << 10);
  if (shape != *carved) {
    load_rule(a, l);
    *carved = shape;
  }
  if (whole) {  // the whole block, sub-tile by sub-tile
    for (int64_t r0 = 0; r0 < h.nr; r0 += a.tr)
      for (int64_t c0 = 0; c0 < h.nc; c0 += a.tc) subtile<KERNEL, LAYER, XC, MIXED>(a, l, h, r0, c0, cp);
  } else {
    subtile<KERNEL, LAYER, XC, MIXED>(a, l, h, d.z, d.w, cp);
  }
}

template <int KERNEL, int XC, bool MIXED>
__global__ __launch_bounds__(kThreads, 2) void k_persistent(const BlockArgs *__restrict__ batches,
                                                            const int32_t *mode,
                                                            const int4 *tiles, int32_t ntiles,
                                                            int32_t nbatch, int32_t *counter) {
  extern __shared__ __align__(16) double lds_raw[];  // 16-byte aligned: ds_read_b128 of points
  __shared__ int s_tile;
  // the queue and the batch arguments are read-only here: their loads have
  // wave-uniform addresses and are scalar, as the per-block kernel's
  // argument loads
  typedef const int32_t __attribute__((address_space(4))) *cint_t;
  int carved = -1;  // sub-tile shape whose LDS layout holds the rule, -1: none yet
  for (;;) {
    __syncthreads();  // everyone has read s_tile and left the previous tile
    if (thread_id() == 0) s_tile = atomicAdd(counter, 1);
    __syncthreads();
    const int t = __builtin_amdgcn_readfirstlane(s_tile);
    if (t >= ntiles) break;  // the counter only grows: every workgroup exits
    const int4 d = uniform_copy(tiles + t);
    const int md = d.x >= 0 && d.x < nbatch ? ((cint_t)mode)[d.x] : -1;
    const int cp = md & 1, layer = md >> 1;
    if (layer == BEM_SLP) {
      persistent_item<KERNEL, BEM_SLP, XC, MIXED>(batches, d, cp, lds_raw, &carved);
    } else if (layer == BEM_DLP) {
      persistent_item<KERNEL, BEM_DLP, XC, MIXED>(batches, d, cp, lds_raw, &carved);
    } else if (layer == kBoth) {
      persistent_item<KERNEL, kBoth, XC, MIXED>(batches, d, cp, lds_raw, &carved);
    } else if (thread_id() == 0) {  // batch index or mode out of range
      atomicOr(batches->flags, FLAG_EINVAL);
    }
  }
}

__global__ void k_reset_counter(int32_t *counter) { *counter = 0; }

template <int KERNEL, int LAYER, bool MIXED>
hipError_t launch_klm(bool coupling, const BlockArgs &a, size_t lds, hipStream_t s) {
  const dim3 grid(a.nblocks), block(kThreads);
  const int cp = coupling ? 1 : 0;
  switch (rule_chunk(a.nq, KERNEL)) {
    case 4: hipLaunchKernelGGL((k_blocks<KERNEL, LAYER, 4, MIXED>), grid, block, lds, s, a, cp); break;
    case 5: hipLaunchKernelGGL((k_blocks<KERNEL, LAYER, 5, MIXED>), grid, block, lds, s, a, cp); break;
    case 7: hipLaunchKernelGGL((k_blocks<KERNEL, LAYER, 7, MIXED>), grid, block, lds, s, a, cp); break;
    case 8: hipLaunchKernelGGL((k_blocks<KERNEL, LAYER, 8, MIXED>), grid, block, lds, s, a, cp); break;
    default: hipLaunchKernelGGL((k_blocks<KERNEL, LAYER, 9, MIXED>), grid, block, lds, s, a, cp); break;
  }
  return hipGetLastError();
}

template <int KERNEL, bool MIXED>
hipError_t launch_pers(int xc, const PersistentArgs &p, size_t lds, hipStream_t s) {
  const dim3 grid(p.grid), block(kThreads);
  switch (xc) {
#define BEM_PERS(X)                                                                     \
  hipLaunchKernelGGL((k_persistent<KERNEL, X, MIXED>), grid, block, lds, s, p.batches, \
                     p.mode, p.tiles, p.ntiles, p.nbatch, p.counter)
    case 4: BEM_PERS(4); break;
    case 5: BEM_PERS(5); break;
    case 7: BEM_PERS(7); break;
    case 8: BEM_PERS(8); break;
    case 9: BEM_PERS(9); break;
    default: return hipErrorInvalidValue;
#undef BEM_PERS
  }
  return hipGetLastError();
}

template <int KERNEL, bool MIXED>
hipError_t launch_both(const BlockArgs &a, size_t lds, hipStream_t s) {
  const dim3 grid(a.nblocks), block(kThreads);
  switch (rule_chunk(a.nq, KERNEL)) {
    case 4: hipLaunchKernelGGL((k_blocks<KERNEL, kBoth, 4, MIXED>), grid, block, lds, s, a, 0); break;
    case 5: hipLaunchKernelGGL((k_blocks<KERNEL, kBoth, 5, MIXED>), grid, block, lds, s, a, 0); break;
    case 7: hipLaunchKernelGGL((k_blocks<KERNEL, kBoth, 7, MIXED>), grid, block, lds, s, a, 0); break;
    case 8: hipLaunchKernelGGL((k_blocks<KERNEL, kBoth, 8, MIXED>), grid, block, lds, s, a, 0); break;
    default: hipLaunchKernelGGL((k_blocks<KERNEL, kBoth, 9, MIXED>), grid, block, lds, s, a, 0); break;
  }
  return hipGetLastError();
}

template <int KERNEL, int LAYER>
hipError_t launch_kl(bool coupling, bool mixed, const BlockArgs &a, size_t lds, hipStream_t s) {
  return mixed ? launch_klm<KERNEL, LAYER, true>(coupling, a, lds, s)
               : launch_klm<KERNEL, LAYER, false>(coupling, a, lds, s);
}

}  // namespace

// x-points per register chunk: the largest supported divisor of nq that keeps
// the kernel within 256 registers (two waves per SIMD), else 4 with padding.
int rule_chunk(int nq, int kernel) {
  static const int lap[] = {8, 9, 7, 5, 4};
  static const int hel[] = {4, 5, 7, 9, 8};  // sine/cosine chains need more registers
  for (int xc : (kernel == BEM_LAPLACE ? lap : hel))
    if (nq % xc == 0) return xc;
  return 4;
}

// LDS of a sub-tile; without the pair lists (coupling launches: every pair is
// regular, phase C only flags, and the lists sit past the allocation unread).
size_t block_lds_bytes(int nq_pad, int tr, int tc, bool mixed, bool lists, bool both) {
  size_t dbl = (size_t)blk::ypoint_doubles(mixed) * nq_pad * tc + 10 * (size_t)tr +
               3 * (size_t)nq_pad + 3 * (size_t)tc + (both ? 3 * (size_t)tr : 0);
  if (mixed) dbl += 3 * (size_t)tc + 6 * (size_t)tr + 6 * (size_t)tc;
  const size_t ints = (size_t)4 * tr + 4 * (size_t)tc + 36;
  return dbl * 8 + ints * 4 + (lists ? (size_t)2 * (2 * (size_t)tr * tc + blk::kSortPad) : 0);
}

// Largest sub-tile within the LDS budget.  Near-field sub-tiles carry the
// pair lists, whose entries pack row and column in 6 bits each (at most
// 64 x 64); so do mixed-precision coupling sub-tiles (their near-singular
// pairs go to the FP64 pass through the lists).  Plain coupling sub-tiles
// have no lists and take up to 128 rows and 96 columns, so that most coupling
// blocks (ranks up to ~100) are one sub-tile.
bool block_tile_shape(int nq_pad, bool mixed, size_t lds_budget, int *tr, int *tc,
                      size_t *lds_bytes, bool coupling, bool both) {
  static const int near_shapes[][2] = {{64, 64}, {64, 32}, {64, 16}, {64, 8}, {32, 8}, {16, 8},
                                       {8, 8}};
  static const int coupling_shapes[][2] = {{128, 96}, {128, 80}, {96, 80}, {128, 64}, {64, 64},
                                           {64, 32}, {64, 16}, {64, 8}, {32, 8}, {16, 8}, {8, 8}};
  const bool lists = !coupling || mixed;
  auto try_list = [&](const int(*shapes)[2], int n) {
    for (int k = 0; k < n; ++k) {
      const size_t bytes = block_lds_bytes(nq_pad, shapes[k][0], shapes[k][1], mixed, lists, both);
      if (bytes <= lds_budget) {
        *tr = shapes[k][0];
        *tc = shapes[k][1];
        *lds_bytes = bytes;
        return true;
      }
    }
    return false;
  };
  return lists ? try_list(near_shapes, 7) : try_list(coupling_shapes, 11);
}

hipError_t launch_blocks(int kernel, int layer, bool coupling, bool mixed, const BlockArgs &a,
                         size_t lds, hipStream_t s) {
  if (a.nblocks == 0) return hipSuccess;
  if (kernel == BEM_LAPLACE)
    return layer == BEM_SLP ? launch_kl<BEM_LAPLACE, BEM_SLP>(coupling, mixed, a, lds, s)
                            : launch_kl<BEM_LAPLACE, BEM_DLP>(coupling, mixed, a, lds, s);
  return layer == BEM_SLP ? launch_kl<BEM_HELMHOLTZ, BEM_SLP>(coupling, mixed, a, lds, s)
                          : launch_kl<BEM_HELMHOLTZ, BEM_DLP>(coupling, mixed, a, lds, s);
}

hipError_t launch_blocks_both(int kernel, bool mixed, const BlockArgs &a, size_t lds,
                              hipStream_t s) {
  if (a.nblocks == 0) return hipSuccess;
  if (kernel == BEM_LAPLACE)
    return mixed ? launch_both<BEM_LAPLACE, true>(a, lds, s) : launch_both<BEM_LAPLACE, false>(a, lds, s);
  return mixed ? launch_both<BEM_HELMHOLTZ, true>(a, lds, s) : launch_both<BEM_HELMHOLTZ, false>(a, lds, s);
}

int learned_chunk(int q, int kernel) { return learned_xc(kernel, q); }

hipError_t launch_blocks_learned(int kernel, int layer, const BlockArgs &a, const OrderRules &o,
                                 size_t lds, hipStream_t s) {
  if (a.nblocks == 0) return hipSuccess;
  const dim3 grid(a.nblocks), block(kThreads);
  if (kernel == BEM_LAPLACE) {
    if (layer == BEM_SLP) hipLaunchKernelGGL((k_blocks_learned<BEM_LAPLACE, BEM_SLP>), grid, block, lds, s, a, o);
    else hipLaunchKernelGGL((k_blocks_learned<BEM_LAPLACE, BEM_DLP>), grid, block, lds, s, a, o);
  } else {
    if (layer == BEM_SLP) hipLaunchKernelGGL((k_blocks_learned<BEM_HELMHOLTZ, BEM_SLP>), grid, block, lds, s, a, o);
    else hipLaunchKernelGGL((k_blocks_learned<BEM_HELMHOLTZ, BEM_DLP>), grid, block, lds, s, a, o);
  }
  return hipGetLastError();
}

hipError_t launch_reset_counter(int32_t *counter, hipStream_t s) {
  hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3(1), 0, s, counter);
  return hipGetLastError();
}

hipError_t launch_persistent(int kernel, bool mixed, int xc, const PersistentArgs &p, size_t lds,
                             hipStream_t s) {
  if (p.ntiles == 0 || p.grid == 0) return hipSuccess;
  if (kernel == BEM_LAPLACE)
    return mixed ? launch_pers<BEM_LAPLACE, true>(xc, p, lds, s)
                 : launch_pers<BEM_LAPLACE, false>(xc, p, lds, s);
  return mixed ? launch_pers<BEM_HELMHOLTZ, true>(xc, p, lds, s)
               : launch_pers<BEM_HELMHOLTZ, false>(xc, p, lds, s);
}

}  // namespace bem
