// Batched assembly in one persistent launch: the plan (host copy of the
// block structure, cost-sorted sub-tile queue, per-mesh geometry, launch
// configuration chosen by timing candidates, HIP graph) and its replay.
//
// Sec. 3 splits the blocks of a matrix into work lists of bounded size that
// worker threads hand to the GPU one by one (Algorithms add_block,
// assemble_gpu, schedule_tasks).  On one MI355X a single launch can hold the
// whole batch: the lists become one device queue of sub-tiles, popped by a
// fixed grid of workgroups (k_persistent), ordered by decreasing estimated
// cost so that the last pops are the cheapest (longest-processing-time
// order) and no compute unit idles behind one large block.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <new>
#include <sstream>
#include <string>
#include <tuple>
#include <vector>

#include "bem_internal.h"

using namespace bem;

struct bem_plan {
  bem_ctx *ctx = nullptr;  // null once the context is destroyed
  int device = 0;
  int kernel = 0;
  bool mixed = false;
  int32_t nq = 0;
  size_t lds = 0;
  bem_tune cfg{};
  int32_t nbatch = 0;
  int64_t ntiles = 0;
  // device memory owned by the plan
  double *geo = nullptr;
  BlockArgs *dbatch = nullptr;
  int32_t *dmode = nullptr;  // per batch: coupling flag | layer << 1
  int4 *dtiles = nullptr;
  int32_t *counter = nullptr;
  // distinct meshes and their geometry slices
  std::vector<bem_mesh> meshes;
  std::vector<int64_t> geo_off, geo_ld;
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

struct HostBatch {
  int mesh = 0;  // index into bem_plan::meshes
  int coupling = 0;
  int layer = 0;  // BEM_SLP, BEM_DLP or kLayerBoth
  bem_blocks blocks{};
  void *out = nullptr, *out2 = nullptr;
  int64_t out_len = 0;
  std::vector<int32_t> row_ptr, col_ptr, row_idx, col_idx;
  std::vector<int64_t> out_off;
};

constexpr int kLayerBoth = 2;  // both layers in one pass (the kernels' layer value)

template <class T>
hipError_t d2h(std::vector<T> *dst, const T *src, int64_t n) {
  dst->assign((size_t)std::max<int64_t>(n, 0), T{});
  if (n <= 0) return hipSuccess;
  return hipMemcpy(dst->data(), src, (size_t)n * sizeof(T), hipMemcpyDeviceToHost);
}

// Estimated cost of one sub-tile in regular point-pair units of the single
// layer: regular entries use nqp^2 point pairs; a pair with k common
// vertices has 2, 5 or 6 regions of q_s^3 eta points (k = 1, 2, 3), each
// about twice a regular point pair's work and summed one pair per lane:
// 8 k q_s^3 (measured on the near field of the 8192-triangle sphere, the
// singular pass takes about 1/6 of the launch for 1/40 of its flops).  The
// other layers scale the regular part by their issue slots per point pair
// over the single layer's (Laplace 12 : 14 : 16 for single, double, both in
// one pass; Helmholtz, with the sine and cosine, about 36 : 41 : 46) and the
// singular part by the Sauter-Schwab evaluations per pair (1, 1, 2.5: both
// layers of (i, j), the double layer of (j, i)).
struct CostModel {
  int nqp = 0, qs = 0;
  double reg_w = 1.0, sing_w = 1.0;
  std::vector<int32_t> vcount;  // per vertex: rows of the tile touching it
};

void layer_weights(int kernel, int layer, double *reg_w, double *sing_w) {
  static const double lap[3] = {1.0, 14.0 / 12.0, 16.0 / 12.0};
  static const double hel[3] = {1.0, 41.0 / 36.0, 46.0 / 36.0};
  *reg_w = (kernel == BEM_LAPLACE ? lap : hel)[layer];
  *sing_w = layer == kLayerBoth ? 2.5 : 1.0;
}

double tile_cost(CostModel &cm, const HostBatch &hb, const std::vector<int32_t> &tri,
                 int64_t rp0, int64_t cp0, int64_t r0, int64_t c0, int tr, int tc) {
  const double reg = cm.reg_w * (double)tr * tc * cm.nqp * cm.nqp;
  if (hb.coupling) return reg;
  for (int k = 0; k < tr; ++k)
    for (int m = 0; m < 3; ++m) ++cm.vcount[tri[3 * (size_t)hb.row_idx[rp0 + r0 + k] + m]];
  int64_t shared = 0;
  for (int k = 0; k < tc; ++k)
    for (int m = 0; m < 3; ++m) shared += cm.vcount[tri[3 * (size_t)hb.col_idx[cp0 + c0 + k] + m]];
  for (int k = 0; k < tr; ++k)
    for (int m = 0; m < 3; ++m) cm.vcount[tri[3 * (size_t)hb.row_idx[rp0 + r0 + k] + m]] = 0;
  return reg + cm.sing_w * 8.0 * (double)shared * cm.qs * cm.qs * cm.qs;
}

// Work items (batch, block, first row, first column) -- every sub-tile, or
// with whole = true every block as (batch, block, -1, -1) with the sum of its
// sub-tiles' costs -- sorted by decreasing cost; ties keep the natural order.
// shapes[e]: sub-tile rows and columns of batch entry e.
std::vector<int4> build_tiles(const std::vector<HostBatch> &hbs,
                              const std::vector<std::vector<int32_t>> &tris,
                              const std::vector<bem_mesh> &meshes,
                              const std::vector<std::pair<int, int>> &shapes, int kernel, int nqp,
                              int qs, bool whole) {
  std::vector<int4> tiles;
  std::vector<double> cost;
  for (size_t e = 0; e < hbs.size(); ++e) {
    const HostBatch &hb = hbs[e];
    const int tr = shapes[e].first, tc = shapes[e].second;
    CostModel cm;
    cm.nqp = nqp;
    cm.qs = qs;
    layer_weights(kernel, hb.layer, &cm.reg_w, &cm.sing_w);
    if (!hb.coupling) cm.vcount.assign((size_t)meshes[hb.mesh].nv, 0);
    for (int32_t b = 0; b < hb.blocks.n; ++b) {
      const int64_t rp0 = hb.row_ptr[b], cp0 = hb.col_ptr[b];
      const int64_t nr = hb.row_ptr[b + 1] - rp0, nc = hb.col_ptr[b + 1] - cp0;
      if (nr == 0 || nc == 0) continue;
      double sum = 0.0;
      for (int64_t r0 = 0; r0 < nr; r0 += tr)
        for (int64_t c0 = 0; c0 < nc; c0 += tc) {
          const int etr = (int)std::min<int64_t>(tr, nr - r0), etc = (int)std::min<int64_t>(tc, nc - c0);
          const double c = tile_cost(cm, hb, tris[hb.mesh], rp0, cp0, r0, c0, etr, etc);
          if (whole) {
            sum += c;
          } else {
            tiles.push_back(make_int4((int)e, b, (int)r0, (int)c0));
            cost.push_back(c);
          }
        }
      if (whole) {
        tiles.push_back(make_int4((int)e, b, -1, -1));
        cost.push_back(sum);
      }
    }
  }
  std::vector<size_t> order(tiles.size());
  for (size_t k = 0; k < order.size(); ++k) order[k] = k;
  std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t b) { return cost[a] > cost[b]; });
  std::vector<int4> sorted(tiles.size());
  for (size_t k = 0; k < order.size(); ++k) sorted[k] = tiles[order[k]];
  return sorted;
}

// Host-side validation of one block list (the kernels check again).
int validate(bem_ctx *ctx, const HostBatch &hb, const bem_mesh &m, int e) {
  const bem_blocks &b = hb.blocks;
  char msg[160];
  for (int32_t k = 0; k < b.n; ++k) {
    const int64_t rp0 = hb.row_ptr[k], rp1 = hb.row_ptr[k + 1];
    const int64_t cp0 = hb.col_ptr[k], cp1 = hb.col_ptr[k + 1];
    const int64_t off = hb.out_off[k];
    bool ok = rp0 >= 0 && rp0 <= rp1 && rp1 <= b.row_len && cp0 >= 0 && cp0 <= cp1 &&
              cp1 <= b.col_len && off >= 0 && off <= hb.out_len;
    const int64_t nr = rp1 - rp0, nc = cp1 - cp0;
    ok = ok && (nr == 0 || nc <= (hb.out_len - off) / nr);
    ok = ok && nr < (int64_t)1 << 30 && nc < (int64_t)1 << 30;
    if (!ok) {
      std::snprintf(msg, sizeof msg, "batch %d block %d: row/column range or output slot invalid", e, k);
      return fail(ctx, BEM_EINVAL, msg);
    }
  }
  for (const auto *ids : {&hb.row_idx, &hb.col_idx})
    for (int32_t id : *ids)
      if (id < 0 || id >= m.nt) {
        std::snprintf(msg, sizeof msg, "batch %d: triangle id %d out of range", e, id);
        return fail(ctx, BEM_EINVAL, msg);
      }
  return BEM_OK;
}

// ---------------------------------------------------------------- tuning cache
// One JSON object per line:
//   {"key": "...", "grid": G, "tile_rows": R, "tile_cols": C, "x_chunk": X,
//    "granularity": 1 (blocks) or 2 (sub-tiles), "ms": T}
bool json_int(const std::string &line, const char *field, long *v) {
  const std::string pat = std::string("\"") + field + "\":";
  const size_t p = line.find(pat);
  if (p == std::string::npos) return false;
  char *end = nullptr;
  *v = std::strtol(line.c_str() + p + pat.size(), &end, 10);
  return end != line.c_str() + p + pat.size();
}

bool cache_lookup(const char *path, const std::string &key, bem_tune *t) {
  if (!path) return false;
  std::ifstream f(path);
  if (!f) return false;
  const std::string kpat = "\"key\": \"" + key + "\"";
  std::string line;
  bool found = false;
  while (std::getline(f, line)) {  // the last matching line wins
    if (line.find(kpat) == std::string::npos) continue;
    long g, r, c, x, w;
    if (json_int(line, "grid", &g) && json_int(line, "tile_rows", &r) &&
        json_int(line, "tile_cols", &c) && json_int(line, "x_chunk", &x) &&
        json_int(line, "granularity", &w)) {
      t->grid = (int32_t)g;
      t->tile_rows = (int32_t)r;
      t->tile_cols = (int32_t)c;
      t->x_chunk = (int32_t)x;
      t->granularity = (int32_t)w;
      found = true;
    }
  }
  return found;
}

void cache_store(const char *path, const std::string &key, const bem_tune &t) {
  if (!path) return;
  std::ofstream f(path, std::ios::app);
  if (!f) return;
  f << "{\"key\": \"" << key << "\", \"grid\": " << t.grid << ", \"tile_rows\": " << t.tile_rows
    << ", \"tile_cols\": " << t.tile_cols << ", \"x_chunk\": " << t.x_chunk
    << ", \"granularity\": " << t.granularity << ", \"ms\": " << t.tuned_ms << "}\n";
}

bool valid_chunk(int x) { return x == 4 || x == 5 || x == 7 || x == 8 || x == 9; }

// Device resources of a plan; idempotent.
void release(bem_plan *p) {
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  if (p->cap) (void)hipStreamDestroy(p->cap);
  for (void *m : {(void *)p->geo, (void *)p->dbatch, (void *)p->dmode, (void *)p->dtiles,
                  (void *)p->counter})
    if (m) (void)hipFree(m);
  p->exec = nullptr;
  p->graph = nullptr;
  p->cap = nullptr;
  p->geo = nullptr;
  p->dbatch = nullptr;
  p->dmode = nullptr;
  p->dtiles = nullptr;
  p->counter = nullptr;
}

struct Candidate {
  int grid, tr, tc, xc;
  bool whole;    // queue whole blocks instead of sub-tiles
  int ctr, ctc;  // sub-tile of the plain coupling lists (0: none in the batch)
};

}  // namespace

void bem::detach_plans(bem_ctx *ctx) {
  for (bem_plan *p : ctx->plans) {
    release(p);
    p->ctx = nullptr;
  }
  ctx->plans.clear();
}

extern "C" {

int bem_plan_batched(bem_ctx *ctx, const bem_op *op, int32_t nbatch, const bem_batch *batches,
                     bem_tune *tune, const char *cache_path, void *stream, bem_plan **plan_out) {
  if (!ctx) return BEM_EINVAL;
  if (!plan_out) return fail(ctx, BEM_EINVAL, "plan is NULL");
  *plan_out = nullptr;
  int rc;
  if ((rc = check_op(ctx, op))) return rc;
  if (nbatch < 0 || (nbatch > 0 && !batches)) return fail(ctx, BEM_EINVAL, "batches is NULL");
  bem_tune want{};
  if (tune) want = *tune;
  if (want.grid < 0 || want.tile_rows < 0 || want.tile_rows > 64 || want.tile_cols < 0 ||
      want.tile_cols > 64 || (want.x_chunk && !valid_chunk(want.x_chunk)) ||
      (want.autotune != 0 && want.autotune != 1) || want.granularity < 0 ||
      want.granularity > 2 || want.reserved[0] || want.reserved[1])
    return fail(ctx, BEM_EINVAL, "tune: grid >= 0, tiles in [0, 64], x_chunk in {0,4,5,7,8,9}, "
                                 "autotune 0/1, granularity 0..2, reserved 0");
  DeviceGuard guard(ctx->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  bem_plan *p = new (std::nothrow) bem_plan;
  if (!p) return fail(ctx, BEM_ENOMEM, "host allocation failed");
  p->ctx = ctx;
  p->device = ctx->device;
  p->kernel = op->kernel;
  p->mixed = op->precision == BEM_MIXED;
  p->nbatch = nbatch;
  auto bail = [&](int code) {
    release(p);
    delete p;
    return code;
  };
  std::vector<HostBatch> hbs;
  std::vector<std::vector<int32_t>> tris;
  const bem::DevRules *rules = nullptr;
  try {
    hipError_t e = hipStreamSynchronize(s);  // the caller's writes of the index arrays
    if (e != hipSuccess) return bail(hip_fail(ctx, e, "hipStreamSynchronize"));
    hbs.resize((size_t)nbatch);
    for (int32_t k = 0; k < nbatch; ++k) {
      const bem_batch &bt = batches[k];
      HostBatch &hb = hbs[k];
      if ((rc = check_mesh(ctx, bt.mesh)) || (rc = check_blocks(ctx, bt.blocks, bt.out, bt.out_len)))
        return bail(rc);
      if ((bt.coupling != 0 && bt.coupling != 1) || bt.layers < BEM_BATCH_OP_LAYER ||
          bt.layers > BEM_BATCH_BOTH)
        return bail(fail(ctx, BEM_EINVAL, "bem_batch.coupling must be 0/1, layers 0..3"));
      hb.layer = bt.layers == BEM_BATCH_OP_LAYER ? op->layer
                 : bt.layers == BEM_BATCH_SLP    ? BEM_SLP
                 : bt.layers == BEM_BATCH_DLP    ? BEM_DLP
                                                 : kLayerBoth;
      if (hb.layer == kLayerBoth) {
        if (bt.coupling)
          return bail(fail(ctx, BEM_EINVAL, "BEM_BATCH_BOTH is for near-field lists only"));
        if (bt.out_len > 0 && (!bt.out2 || bt.out2 == bt.out))
          return bail(fail(ctx, BEM_EINVAL, "BEM_BATCH_BOTH: out2 is NULL or the same buffer as out"));
      } else if (bt.out2) {
        return bail(fail(ctx, BEM_EINVAL, "bem_batch.out2 is for BEM_BATCH_BOTH only"));
      }
      if (bt.blocks->mirror_off && hb.layer == BEM_DLP)
        return bail(fail(ctx, BEM_EINVAL, "mirror_off is for single layers and BEM_BATCH_BOTH"));
      if (bt.blocks->n > 0 && bt.mesh->nt == 0)
        return bail(fail(ctx, BEM_EINVAL, "blocks given for an empty mesh"));
      hb.coupling = bt.coupling;
      hb.blocks = *bt.blocks;
      hb.out = bt.out;
      hb.out2 = bt.out2;
      hb.out_len = bt.out_len;
      // meshes with identical descriptors share a geometry slice
      int mi = -1;
      for (size_t q = 0; q < p->meshes.size(); ++q) {
        const bem_mesh &m = p->meshes[q];
        if (m.v == bt.mesh->v && m.tri == bt.mesh->tri && m.nv == bt.mesh->nv && m.nt == bt.mesh->nt)
          mi = (int)q;
      }
      if (mi < 0) {
        mi = (int)p->meshes.size();
        p->meshes.push_back(*bt.mesh);
        tris.emplace_back();
        if ((e = d2h(&tris.back(), bt.mesh->tri, 3 * (int64_t)bt.mesh->nt)) != hipSuccess)
          return bail(hip_fail(ctx, e, "reading mesh triangles"));
        for (int32_t vid : tris.back())
          if (vid < 0 || vid >= bt.mesh->nv)
            return bail(fail(ctx, BEM_EINVAL, "mesh vertex id out of range"));
      }
      hb.mesh = mi;
      const bem_blocks &b = *bt.blocks;
      if (b.n > 0) {
        if ((e = d2h(&hb.row_ptr, b.row_ptr, (int64_t)b.n + 1)) != hipSuccess ||
            (e = d2h(&hb.col_ptr, b.col_ptr, (int64_t)b.n + 1)) != hipSuccess ||
            (e = d2h(&hb.out_off, b.out_off, (int64_t)b.n)) != hipSuccess ||
            (e = d2h(&hb.row_idx, b.row_idx, b.row_len)) != hipSuccess ||
            (e = d2h(&hb.col_idx, b.col_idx, b.col_len)) != hipSuccess)
          return bail(hip_fail(ctx, e, "reading block lists"));
        if ((rc = validate(ctx, hb, p->meshes[mi], k))) return bail(rc);
      }
    }
    if ((rc = get_rules(ctx, op, &rules))) return bail(rc);
    p->nq = rules->nq;
    // geometry slices
    int64_t total = 0;
    for (const bem_mesh &m : p->meshes) {
      const int64_t ld = std::max<int64_t>(((int64_t)m.nt + 63) / 64 * 64, 64);
      p->geo_off.push_back(total);
      p->geo_ld.push_back(ld);
      total += (int64_t)GEO_NF * ld;
    }
    if (total > 0 && (e = dev_malloc((void **)&p->geo, (size_t)total * sizeof(double))) != hipSuccess)
      return bail(hip_fail(ctx, e, "hipMalloc(plan geometry)"));
    if ((e = dev_malloc((void **)&p->counter, 256)) != hipSuccess ||
        (e = dev_malloc((void **)&p->dmode, sizeof(int32_t) * std::max(nbatch, 1))) != hipSuccess ||
        (e = dev_malloc((void **)&p->dbatch, sizeof(BlockArgs) * std::max(nbatch, 1))) != hipSuccess)
      return bail(hip_fail(ctx, e, "hipMalloc(plan)"));
    for (size_t q = 0; q < p->meshes.size(); ++q)
      if ((e = launch_geometry(p->meshes[q], p->geo + p->geo_off[q], p->geo_ld[q], ctx->flags, s)) !=
          hipSuccess)
        return bail(hip_fail(ctx, e, "geometry kernel launch"));
    std::vector<int32_t> hmode((size_t)std::max(nbatch, 1), 0);
    for (int32_t k = 0; k < nbatch; ++k) hmode[k] = hbs[k].coupling | hbs[k].layer << 1;
    if ((e = hipMemcpy(p->dmode, hmode.data(), hmode.size() * sizeof(int32_t),
                       hipMemcpyHostToDevice)) != hipSuccess)
      return bail(hip_fail(ctx, e, "hipMemcpy(batch modes)"));
  } catch (const std::bad_alloc &) {
    return bail(fail(ctx, BEM_ENOMEM, "host allocation failed"));
  }

  // ---- candidates
  int ncu = 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, ctx->device) != hipSuccess ||
      ncu <= 0)
    ncu = 256;
  const int def_xc = rule_chunk(p->nq, p->kernel);
  std::vector<int> xcs;
  if (want.x_chunk) {
    xcs.push_back(want.x_chunk);
  } else {
    xcs.push_back(def_xc);
    if (want.autotune)
      for (int x : {8, 9, 7, 5, 4})
        if (x != def_xc && p->nq % x == 0) xcs.push_back(x);
  }
  // sub-tiles: the lists with pair lists (near field; all in the mixed form)
  // take the candidate's shape, plain coupling lists the coupling kernel's
  bool any_lists = false, any_plain_coupling = false;
  for (const HostBatch &hb : hbs) {
    if (hb.coupling && !p->mixed) any_plain_coupling = true;
    else any_lists = true;
  }
  auto has_lists = [&](const HostBatch &hb) { return !hb.coupling || p->mixed; };
  auto make_cand = [&](int grid, int tr, int tc, int xc, bool whole) {
    Candidate c{grid, tr, tc, xc, whole, 0, 0};
    if (any_plain_coupling) {
      const int nqp = (p->nq + xc - 1) / xc * xc;
      size_t lds;
      if (!block_tile_shape(nqp, false, ctx->lds_budget, &c.ctr, &c.ctc, &lds, true, false))
        c.ctr = c.ctc = 0;
    }
    return c;
  };
  auto shapes_of = [&](const Candidate &c) {
    std::vector<std::pair<int, int>> sh(hbs.size());
    for (size_t k = 0; k < hbs.size(); ++k)
      sh[k] = has_lists(hbs[k]) ? std::make_pair(c.tr, c.tc) : std::make_pair(c.ctr, c.ctc);
    return sh;
  };
  // LDS of the launch: the largest layout of its batch entries (0: no entry)
  auto plan_lds = [&](const Candidate &c) -> size_t {
    const int nqp = (p->nq + c.xc - 1) / c.xc * c.xc;
    size_t m = 0;
    for (const HostBatch &hb : hbs) {
      const bool l = has_lists(hb);
      m = std::max(m, block_lds_bytes(nqp, l ? c.tr : c.ctr, l ? c.tc : c.ctc, p->mixed, l,
                                      hb.layer == kLayerBoth));
    }
    return m;
  };
  auto fits = [&](const Candidate &c) {
    return (!any_plain_coupling || c.ctr > 0) && plan_lds(c) <= ctx->lds_budget;
  };
  bool any_both = false;
  for (const HostBatch &hb : hbs) any_both = any_both || hb.layer == kLayerBoth;
  std::vector<Candidate> cands;
  for (int xc : xcs) {
    const int nqp = (p->nq + xc - 1) / xc * xc;
    std::vector<std::pair<int, int>> shapes;
    if (want.tile_rows && want.tile_cols) {
      shapes.push_back({want.tile_rows, want.tile_cols});
    } else {
      int tr, tc;
      size_t lds;
      if (block_tile_shape(nqp, p->mixed, ctx->lds_budget, &tr, &tc, &lds, false, any_both))
        shapes.push_back({want.tile_rows ? want.tile_rows : tr, want.tile_cols ? want.tile_cols : tc});
      if (want.autotune && any_lists)
        for (auto sh : {std::make_pair(64, 32), std::make_pair(32, 32), std::make_pair(32, 64)}) {
          if (want.tile_rows) sh.first = want.tile_rows;
          if (want.tile_cols) sh.second = want.tile_cols;
          if (std::find(shapes.begin(), shapes.end(), sh) == shapes.end()) shapes.push_back(sh);
        }
    }
    std::vector<int> grids;
    if (want.grid) {
      grids.push_back(want.grid);
    } else {
      grids.push_back(2 * ncu);
      if (want.autotune) grids.insert(grids.end(), {ncu, 3 * ncu / 2});
    }
    for (auto sh : shapes) {
      for (int g : grids) {
        for (int whole = 1; whole >= 0; --whole) {
          const bool take = whole ? want.granularity != 2
                                  : want.granularity == 2 || (want.granularity == 0 && want.autotune);
          if (!take) continue;
          const Candidate c = make_cand(g, sh.first, sh.second, xc, whole == 1);
          if (fits(c)) cands.push_back(c);
        }
      }
    }
  }
  if (cands.empty())
    return bail(fail(ctx, BEM_EUNSUPPORTED, "no sub-tile shape fits the LDS budget"));

  // ---- per-candidate device state
  // queues depend on the sub-tile shapes and granularity, not on the chunk
  std::map<std::tuple<int, int, bool, int, int>, std::vector<int4>> tile_sets;
  auto tiles_for = [&](const Candidate &c) -> const std::vector<int4> & {
    auto key = std::make_tuple(c.tr, c.tc, c.whole, c.ctr, c.ctc);
    auto it = tile_sets.find(key);
    if (it == tile_sets.end()) {
      const int nqp = (p->nq + def_xc - 1) / def_xc * def_xc;
      it = tile_sets.emplace(key, build_tiles(hbs, tris, p->meshes, shapes_of(c), p->kernel, nqp,
                                              op->q_singular, c.whole)).first;
    }
    return it->second;
  };
  size_t tiles_cap = 0;
  auto stage = [&](const Candidate &c, PersistentArgs *pa) -> int {
    const std::vector<int4> &tl = tiles_for(c);
    hipError_t e;
    if (tl.size() > tiles_cap) {
      if (p->dtiles) (void)hipFree(p->dtiles);
      p->dtiles = nullptr;
      tiles_cap = 0;
      if ((e = dev_malloc((void **)&p->dtiles, tl.size() * sizeof(int4))) != hipSuccess)
        return hip_fail(ctx, e, "hipMalloc(tile queue)");
      tiles_cap = tl.size();
    }
    if (!tl.empty() &&
        (e = hipMemcpy(p->dtiles, tl.data(), tl.size() * sizeof(int4), hipMemcpyHostToDevice)) !=
            hipSuccess)
      return hip_fail(ctx, e, "hipMemcpy(tile queue)");
    std::vector<BlockArgs> ha((size_t)std::max(nbatch, 1));
    const std::vector<std::pair<int, int>> sh = shapes_of(c);
    for (int32_t k = 0; k < nbatch; ++k) {
      const HostBatch &hb = hbs[k];
      const bem_mesh &m = p->meshes[hb.mesh];
      BlockArgs &a = ha[k];
      a = BlockArgs{};
      a.v = m.v;
      a.tri = m.tri;
      a.nv = m.nv;
      a.nt = m.nt;
      a.geo = p->geo ? p->geo + p->geo_off[hb.mesh] : nullptr;
      a.ldg = p->geo_ld[hb.mesh];
      a.nblocks = hb.blocks.n;
      a.row_ptr = hb.blocks.row_ptr;
      a.row_idx = hb.blocks.row_idx;
      a.col_ptr = hb.blocks.col_ptr;
      a.col_idx = hb.blocks.col_idx;
      a.row_len = hb.blocks.row_len;
      a.col_len = hb.blocks.col_len;
      a.out_off = hb.blocks.out_off;
      a.mirror_off = hb.blocks.mirror_off;
      a.out = hb.out;
      a.out2 = hb.out2;
      a.out_len = hb.out_len;
      a.rule = rules->tri;
      a.nq = rules->nq;
      a.nq_pad = (rules->nq + c.xc - 1) / c.xc * c.xc;
      a.tr = sh[k].first;
      a.tc = sh[k].second;
      for (int q = 0; q < 4; ++q) a.ss.eta[q] = rules->ss[q], a.ss.np[q] = rules->np[q];
      a.ss.xi = rules->xi;
      a.ss.q = rules->nxi;
      a.kappa = op->kernel == BEM_HELMHOLTZ ? op->kappa : 0.0;
      a.near_ratio = op->near_singular_ratio;
      a.flags = ctx->flags;
    }
    if (nbatch > 0 &&
        (e = hipMemcpy(p->dbatch, ha.data(), sizeof(BlockArgs) * nbatch, hipMemcpyHostToDevice)) !=
            hipSuccess)
      return hip_fail(ctx, e, "hipMemcpy(batch arguments)");
    pa->batches = p->dbatch;
    pa->mode = p->dmode;
    pa->tiles = p->dtiles;
    pa->ntiles = (int32_t)tl.size();
    pa->nbatch = nbatch;
    pa->counter = p->counter;
    pa->grid = (int32_t)std::min<int64_t>(c.grid, std::max<int64_t>((int64_t)tl.size(), 1));
    p->ntiles = (int64_t)tl.size();
    p->lds = plan_lds(c);
    return BEM_OK;
  };
  auto enqueue = [&](const PersistentArgs &pa, int xc, hipStream_t st) -> hipError_t {
    hipError_t e = launch_reset_counter(p->counter, st);
    if (e == hipSuccess) e = launch_persistent(p->kernel, p->mixed, xc, pa, p->lds, st);
    return e;
  };

  // ---- choose: cache, else time the candidates (or take the only one)
  int64_t entries = 0, tri_total = 0, ncoup = 0, nlayer[3] = {0, 0, 0};
  for (const HostBatch &hb : hbs) {
    for (int32_t b = 0; b < hb.blocks.n; ++b)
      entries += (int64_t)(hb.row_ptr[b + 1] - hb.row_ptr[b]) * (hb.col_ptr[b + 1] - hb.col_ptr[b]);
    ncoup += hb.coupling;
    ++nlayer[hb.layer];
  }
  for (const bem_mesh &m : p->meshes) tri_total += m.nt;
  char arch[64] = "gfx";
  {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, ctx->device) == hipSuccess)
      std::snprintf(arch, sizeof arch, "%s", prop.gcnArchName);
  }
  std::ostringstream ks;
  ks << arch << "/cu" << ncu << "/k" << op->kernel << "l" << nlayer[0] << "," << nlayer[1] << ","
     << nlayer[2] << "p" << op->precision
     << "r" << op->regular_rule << "q" << op->q_regular << "s" << op->q_singular << "/b" << nbatch
     << "c" << ncoup << "t" << tri_total << "e" << entries << "/fix" << want.grid << ","
     << want.tile_rows << "," << want.tile_cols << "," << want.x_chunk << "," << want.granularity;
  const std::string key = ks.str();
  Candidate best = cands[0];
  double best_ms = 0.0;
  bem_tune cached{};
  bool hit = want.autotune && cache_lookup(cache_path, key, &cached);
  if (hit) {
    const int nqp = valid_chunk(cached.x_chunk) ? (p->nq + cached.x_chunk - 1) / cached.x_chunk * cached.x_chunk : 0;
    hit = nqp > 0 && p->nq % cached.x_chunk == 0 && cached.grid > 0 && cached.tile_rows >= 1 &&
          cached.tile_rows <= 64 && cached.tile_cols >= 1 && cached.tile_cols <= 64;
    hit = hit && (cached.granularity == 1 || cached.granularity == 2) &&
          (want.granularity == 0 || want.granularity == cached.granularity);
    if (hit) {
      const Candidate c = make_cand(cached.grid, cached.tile_rows, cached.tile_cols,
                                    cached.x_chunk, cached.granularity == 1);
      hit = fits(c);
      if (hit) best = c;
    }
  }
  if (!hit && want.autotune && cands.size() > 1) {
    // successive halving: every candidate timed once (after one warm-up
    // launch of the first), then the fastest quarter (at least two) three
    // times more; the best of a candidate's launches decides
    hipEvent_t t0, t1;
    if (hipEventCreate(&t0) != hipSuccess || hipEventCreate(&t1) != hipSuccess)
      return bail(fail(ctx, BEM_EDEVICE, "hipEventCreate"));
    auto timed = [&](const Candidate &c, int reps, bool warm, float *best_of) -> int {
      PersistentArgs pa{};
      int r0 = stage(c, &pa);
      if (r0) return r0;
      hipError_t e = warm ? enqueue(pa, c.xc, s) : hipSuccess;
      float ms = 0.f, mn = 1e30f;
      for (int r = 0; r < reps && e == hipSuccess; ++r) {
        e = hipEventRecord(t0, s);
        if (e == hipSuccess) e = enqueue(pa, c.xc, s);
        if (e == hipSuccess) e = hipEventRecord(t1, s);
        if (e == hipSuccess) e = hipEventSynchronize(t1);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, t0, t1);
        mn = std::min(mn, ms);
      }
      if (e != hipSuccess) return hip_fail(ctx, e, "autotune launch");
      *best_of = mn;
      return BEM_OK;
    };
    std::vector<std::pair<float, size_t>> round1;
    for (size_t k = 0; k < cands.size(); ++k) {
      float ms = 0.f;
      if ((rc = timed(cands[k], 1, k == 0, &ms))) {
        (void)hipEventDestroy(t0);
        (void)hipEventDestroy(t1);
        return bail(rc);
      }
      round1.push_back({ms, k});
    }
    std::sort(round1.begin(), round1.end());
    const size_t keep = std::max<size_t>(2, (cands.size() + 3) / 4);
    double bms = 1e300;
    for (size_t i = 0; i < std::min(keep, round1.size()); ++i) {
      const Candidate &c = cands[round1[i].second];
      float ms = 0.f;
      if ((rc = timed(c, 3, false, &ms))) {
        (void)hipEventDestroy(t0);
        (void)hipEventDestroy(t1);
        return bail(rc);
      }
      ms = std::min(ms, round1[i].first);
      if (ms < bms) bms = ms, best = c;
    }
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1);
    best_ms = bms;
  }
  p->cfg.grid = best.grid;
  p->cfg.tile_rows = best.tr;
  p->cfg.tile_cols = best.tc;
  p->cfg.x_chunk = best.xc;
  p->cfg.granularity = best.whole ? 1 : 2;
  p->cfg.autotune = want.autotune;
  p->cfg.tuned_ms = best_ms;
  if (want.autotune && !hit && best_ms > 0) cache_store(cache_path, key, p->cfg);

  // ---- final state and graph: reset counter, geometry, persistent kernel
  PersistentArgs pa{};
  if ((rc = stage(best, &pa))) return bail(rc);
  hipError_t e = hipStreamSynchronize(s);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking);
  if (e != hipSuccess) return bail(hip_fail(ctx, e, "plan stream"));
  e = hipStreamBeginCapture(p->cap, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return bail(hip_fail(ctx, e, "hipStreamBeginCapture"));
  hipError_t le = launch_reset_counter(p->counter, p->cap);
  for (size_t q = 0; q < p->meshes.size() && le == hipSuccess; ++q)
    le = launch_geometry(p->meshes[q], p->geo + p->geo_off[q], p->geo_ld[q], ctx->flags, p->cap);
  if (le == hipSuccess)
    le = launch_persistent(p->kernel, p->mixed, best.xc, pa, p->lds, p->cap);
  e = hipStreamEndCapture(p->cap, &p->graph);
  if (le != hipSuccess) return bail(hip_fail(ctx, le, "kernel launch under capture"));
  if (e != hipSuccess) return bail(hip_fail(ctx, e, "hipStreamEndCapture"));
  e = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0);
  if (e != hipSuccess) return bail(hip_fail(ctx, e, "hipGraphInstantiate"));
  if (tune) *tune = p->cfg;
  ctx->plans.insert(p);
  *plan_out = p;
  return BEM_OK;
}

int bem_run_batched(bem_plan *plan, void *stream) {
  if (!plan || !plan->ctx) return BEM_EINVAL;  // null, or its context is gone
  DeviceGuard guard(plan->ctx->device);
  const hipError_t e = hipGraphLaunch(plan->exec, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(plan->ctx, e, "hipGraphLaunch");
  return BEM_OK;
}

int64_t bem_plan_tiles(const bem_plan *plan) { return plan ? plan->ntiles : 0; }

int bem_autotune(bem_ctx *ctx, const bem_op *op, int32_t nbatch, const bem_batch *batches,
                 bem_tune *tune, const char *cache_path, void *stream) {
  if (!ctx) return BEM_EINVAL;
  if (!tune) return fail(ctx, BEM_EINVAL, "tune is NULL");
  bem_tune t = *tune;
  t.autotune = 1;
  bem_plan *plan = nullptr;
  const int rc = bem_plan_batched(ctx, op, nbatch, batches, &t, cache_path, stream, &plan);
  if (rc) return rc;
  bem_plan_destroy(plan);
  *tune = t;
  return BEM_OK;
}

void bem_plan_destroy(bem_plan *plan) {
  if (!plan) return;
  if (plan->ctx) plan->ctx->plans.erase(plan);
  {
    DeviceGuard guard(plan->device);
    (void)hipDeviceSynchronize();
    release(plan);
  }
  delete plan;
}

}  // extern "C"
