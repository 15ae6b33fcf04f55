// C-ABI entry points: argument validation, context state (flags, scratch,
// quadrature tables) and kernel launches.  See include/bem.h.
#include <hip/hip_runtime.h>

#include <cstdlib>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>

#include "bem_internal.h"

namespace bem {

int fail(bem_ctx *ctx, int code, const std::string &msg) {
  if (ctx) ctx->err = msg;
  return code;
}

// Device allocation of the library's own buffers.  The environment variable
// BEM_FAULT_INJECT=alloc makes it fail as an exhausted device would (read at
// every call), so that callers can test their handling of BEM_ENOMEM.
hipError_t dev_malloc(void **p, size_t bytes) {
  const char *f = std::getenv("BEM_FAULT_INJECT");
  if (f && std::strcmp(f, "alloc") == 0) {
    *p = nullptr;
    return hipErrorOutOfMemory;
  }
  return hipMalloc(p, bytes);
}

int hip_fail(bem_ctx *ctx, hipError_t e, const char *where) {
  return fail(ctx, e == hipErrorOutOfMemory ? BEM_ENOMEM : BEM_EDEVICE,
              std::string(where) + ": " + hipGetErrorString(e));
}

int check_op(bem_ctx *ctx, const bem_op *op) {
  if (!op) return fail(ctx, BEM_EINVAL, "op is NULL");
  if (op->kernel != BEM_LAPLACE && op->kernel != BEM_HELMHOLTZ)
    return fail(ctx, BEM_EINVAL, "op.kernel must be BEM_LAPLACE or BEM_HELMHOLTZ");
  if (op->layer != BEM_SLP && op->layer != BEM_DLP)
    return fail(ctx, BEM_EINVAL, "op.layer must be BEM_SLP or BEM_DLP");
  if (op->precision != BEM_PLAIN_FP64 && op->precision != BEM_MIXED)
    return fail(ctx, BEM_EINVAL, "op.precision must be BEM_PLAIN_FP64 or BEM_MIXED");
  if (op->regular_rule != BEM_RULE_DUFFY && op->regular_rule != BEM_RULE_TRI7)
    return fail(ctx, BEM_EINVAL, "op.regular_rule must be BEM_RULE_DUFFY or BEM_RULE_TRI7");
  if (op->q_regular < 1 || op->q_regular > BEM_MAX_ORDER || op->q_singular < 1 ||
      op->q_singular > BEM_MAX_ORDER)
    return fail(ctx, BEM_EINVAL, "quadrature orders must be in [1, BEM_MAX_ORDER]");
  if (!std::isfinite(op->kappa) || !std::isfinite(op->near_singular_ratio) ||
      op->near_singular_ratio < 0)
    return fail(ctx, BEM_EINVAL, "op.kappa / op.near_singular_ratio must be finite (ratio >= 0)");
  for (int k = 0; k < 4; ++k)
    if (op->reserved[k]) return fail(ctx, BEM_EINVAL, "op.reserved must be zero");
  return BEM_OK;
}

int check_mesh(bem_ctx *ctx, const bem_mesh *m) {
  if (!m) return fail(ctx, BEM_EINVAL, "mesh is NULL");
  if (m->nv < 0 || m->nt < 0) return fail(ctx, BEM_EINVAL, "mesh sizes must be >= 0");
  if (m->nt > 0 && (!m->v || !m->tri || m->nv == 0))
    return fail(ctx, BEM_EINVAL, "mesh arrays are NULL");
  return BEM_OK;
}

int check_blocks(bem_ctx *ctx, const bem_blocks *b, const void *out, int64_t out_len) {
  if (!b) return fail(ctx, BEM_EINVAL, "blocks is NULL");
  if (b->n < 0 || b->row_len < 0 || b->col_len < 0 || out_len < 0)
    return fail(ctx, BEM_EINVAL, "negative size");
  if (b->n > 0 && (!b->row_ptr || !b->col_ptr || !b->out_off))
    return fail(ctx, BEM_EINVAL, "block arrays are NULL");
  if ((b->row_len > 0 && !b->row_idx) || (b->col_len > 0 && !b->col_idx))
    return fail(ctx, BEM_EINVAL, "row_idx / col_idx is NULL");
  if (out_len > 0 && !out) return fail(ctx, BEM_EINVAL, "out is NULL");
  return BEM_OK;
}

// Geometry scratch of at least nt triangles; grows (after a device sync).
int ensure_geo(bem_ctx *ctx, int32_t nt, int64_t *ldg) {
  const int64_t ld = ((int64_t)nt + 63) / 64 * 64;
  const size_t need = (size_t)bem::GEO_NF * (size_t)(ld > 0 ? ld : 64);
  if (need > ctx->geo_cap) {
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail(ctx, e, "hipDeviceSynchronize");
    if (ctx->geo) (void)hipFree(ctx->geo);
    ctx->geo = nullptr;
    ctx->geo_cap = 0;
    e = dev_malloc((void **)&ctx->geo, need * sizeof(double));
    if (e != hipSuccess) return hip_fail(ctx, e, "hipMalloc(geometry)");
    ctx->geo_cap = need;
  }
  *ldg = ld > 0 ? ld : 64;
  return BEM_OK;
}

// Device quadrature tables for (rule, q_regular, q_singular), built once.
int get_rules(bem_ctx *ctx, const bem_op *op, const bem::DevRules **out) {
  const int qr = op->regular_rule == BEM_RULE_TRI7 ? 0 : op->q_regular;
  const auto key = std::make_tuple(op->regular_rule, qr, op->q_singular);
  auto it = ctx->rules.find(key);
  if (it != ctx->rules.end()) {
    *out = &it->second;
    return BEM_OK;
  }
  bem::DevRules d;
  // the tables of a failed build are released (nothing is kept half-built)
  struct Release {
    bem::DevRules *d;
    ~Release() {
      if (!d) return;
      for (void *m : {(void *)d->tri, (void *)d->xi, (void *)d->ss[0], (void *)d->ss[1],
                      (void *)d->ss[2], (void *)d->ss[3]})
        if (m) (void)hipFree(m);
    }
  } release{&d};
  try {
    const bem::TriRule tr = bem::triangle_rule(op->regular_rule, op->q_regular);
    d.nq = (int)tr.s.size();
    std::vector<double> h;
    h.insert(h.end(), tr.s.begin(), tr.s.end());
    h.insert(h.end(), tr.t.begin(), tr.t.end());
    h.insert(h.end(), tr.w.begin(), tr.w.end());
    hipError_t e = dev_malloc((void **)&d.tri, h.size() * sizeof(double));
    if (e != hipSuccess) return hip_fail(ctx, e, "hipMalloc(rule)");
    e = hipMemcpy(d.tri, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(ctx, e, "hipMemcpy(rule)");
    {
      const bem::XiRule xr = bem::xi_rule(op->q_singular);
      const int q = op->q_singular;
      // [xi_a | w_a xi_a^2 | w_a xi_a | M1 = sum w xi, M2 = sum w xi^2]
      std::vector<double> hx(3 * q + 2, 0.0);
      double m1 = 0, m2 = 0;
      for (int k = 0; k < q; ++k) {
        hx[k] = xr.x[k];
        hx[q + k] = xr.w3[k] / xr.x[k];
        hx[2 * q + k] = xr.w3[k] / (xr.x[k] * xr.x[k]);
        m1 += hx[2 * q + k];
        m2 += hx[q + k];
      }
      hx[3 * q] = m1;
      hx[3 * q + 1] = m2;
      d.nxi = q;
      e = dev_malloc((void **)&d.xi, hx.size() * sizeof(double));
      if (e != hipSuccess) return hip_fail(ctx, e, "hipMalloc(xi rule)");
      e = hipMemcpy(d.xi, hx.data(), hx.size() * sizeof(double), hipMemcpyHostToDevice);
      if (e != hipSuccess) return hip_fail(ctx, e, "hipMemcpy(xi rule)");
    }
    for (int cls = 0; cls <= 3; ++cls) {
      const bem::SSRule r = cls ? bem::ss_rule(cls, op->q_singular)
                                : bem::ss_rule_identical_symmetric(op->q_singular);
      d.np[cls] = (int)r.w.size();
      std::vector<double> hs;
      for (const auto *vec : {&r.xs, &r.xt, &r.ys, &r.yt, &r.w}) hs.insert(hs.end(), vec->begin(), vec->end());
      e = dev_malloc((void **)&d.ss[cls], hs.size() * sizeof(double));
      if (e != hipSuccess) return hip_fail(ctx, e, "hipMalloc(ss rule)");
      e = hipMemcpy(d.ss[cls], hs.data(), hs.size() * sizeof(double), hipMemcpyHostToDevice);
      if (e != hipSuccess) return hip_fail(ctx, e, "hipMemcpy(ss rule)");
    }
  } catch (const std::bad_alloc &) {
    return fail(ctx, BEM_ENOMEM, "host allocation failed");
  } catch (const std::exception &ex) {
    return fail(ctx, BEM_EINVAL, ex.what());
  }
  auto ins = ctx->rules.emplace(key, d);
  release.d = nullptr;  // kept by the context
  *out = &ins.first->second;
  return BEM_OK;
}

// both: the near field of both layers in one pass (out: single layer, out2:
// double layer; op->layer is validated but not used).
// noalloc: geometry in the library's fixed array, quadrature tables only if
// the context already holds them (no allocation of any kind).
int assemble_blocks(bem_ctx *ctx, const bem_mesh *mesh, const bem_op *op,
                    const bem_blocks *blocks, void *out, int64_t out_len, void *stream,
                    bool coupling, bool both = false, void *out2 = nullptr,
                    bool noalloc = false) {
  if (!ctx) return BEM_EINVAL;
  int rc;
  if ((rc = check_mesh(ctx, mesh)) || (rc = check_op(ctx, op)) ||
      (rc = check_blocks(ctx, blocks, out, out_len)))
    return rc;
  if (blocks->mirror_off && !both && op->layer != BEM_SLP)
    return fail(ctx, BEM_EINVAL, "mirror_off is for single layers only");
  if (blocks->n == 0) return BEM_OK;
  if (mesh->nt == 0) return fail(ctx, BEM_EINVAL, "blocks given for an empty mesh");
  DeviceGuard g(ctx->device);
  int64_t ldg;
  const bem::DevRules *rules;
  double *geo = ctx->geo;
  if (noalloc) {
    if (mesh->nt > BEM_NOALLOC_MAX_TRI)
      return fail(ctx, BEM_EINVAL, "mesh larger than BEM_NOALLOC_MAX_TRI triangles");
    if (!ctx->noalloc_geo) return fail(ctx, BEM_EDEVICE, "no fixed geometry array on this device");
    const int qr = op->regular_rule == BEM_RULE_TRI7 ? 0 : op->q_regular;
    const auto it = ctx->rules.find(std::make_tuple(op->regular_rule, qr, op->q_singular));
    if (it == ctx->rules.end())
      return fail(ctx, BEM_EINVAL,
                  "quadrature tables of these orders are not built on this context (make one "
                  "call of another entry point with the same rule and orders first)");
    rules = &it->second;
    geo = ctx->noalloc_geo;
    ldg = ((int64_t)mesh->nt + 63) / 64 * 64;
  } else {
    if ((rc = ensure_geo(ctx, mesh->nt, &ldg)) || (rc = get_rules(ctx, op, &rules))) return rc;
    geo = ctx->geo;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = bem::launch_geometry(*mesh, geo, ldg, ctx->flags, s);
  if (e != hipSuccess) return hip_fail(ctx, e, "geometry kernel launch");
  bem::BlockArgs a{};
  a.v = mesh->v;
  a.tri = mesh->tri;
  a.nv = mesh->nv;
  a.nt = mesh->nt;
  a.geo = geo;
  a.ldg = ldg;
  a.nblocks = blocks->n;
  a.row_ptr = blocks->row_ptr;
  a.row_idx = blocks->row_idx;
  a.col_ptr = blocks->col_ptr;
  a.col_idx = blocks->col_idx;
  a.row_len = blocks->row_len;
  a.col_len = blocks->col_len;
  a.out_off = blocks->out_off;
  a.mirror_off = blocks->mirror_off;
  a.out = out;
  a.out2 = out2;
  a.out_len = out_len;
  a.rule = rules->tri;
  a.nq = rules->nq;
  const int xc = bem::rule_chunk(rules->nq, op->kernel);
  a.nq_pad = (rules->nq + xc - 1) / xc * xc;
  size_t lds;
  const bool mixed = op->precision == BEM_MIXED;
  if (!bem::block_tile_shape(a.nq_pad, mixed, ctx->lds_budget, &a.tr, &a.tc, &lds, coupling,
                             both))
    return fail(ctx, BEM_EUNSUPPORTED, "quadrature order too high for the LDS budget");
  a.near_ratio = op->near_singular_ratio;
  for (int c = 0; c < 4; ++c) a.ss.eta[c] = rules->ss[c], a.ss.np[c] = rules->np[c];
  a.ss.xi = rules->xi;
  a.ss.q = rules->nxi;
  a.kappa = op->kernel == BEM_HELMHOLTZ ? op->kappa : 0.0;
  a.flags = ctx->flags;
  e = both ? bem::launch_blocks_both(op->kernel, mixed, a, lds, s)
           : bem::launch_blocks(op->kernel, op->layer, coupling, mixed, a, lds, s);
  if (e != hipSuccess) return hip_fail(ctx, e, "block kernel launch");
  return BEM_OK;
}

}  // namespace bem

using namespace bem;

extern "C" {

int bem_create(bem_ctx **out, int device) {
  if (!out) return BEM_EINVAL;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || n <= 0) return BEM_EDEVICE;
  if (device < 0 || device >= n) return BEM_EINVAL;
  bem_ctx *ctx = new (std::nothrow) bem_ctx;
  if (!ctx) return BEM_ENOMEM;
  ctx->device = device;
  DeviceGuard g(device);
  int lds_max = 0;
  if (hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, device) ==
          hipSuccess &&
      lds_max >= 64 * 1024)
    ctx->lds_budget = std::min<size_t>((size_t)lds_max, 80 * 1024);  // keep 2 workgroups per CU
  hipError_t e = hipMalloc(&ctx->flags, 256);
  if (e == hipSuccess) e = hipMemset(ctx->flags, 0, 256);
  // the fixed array of the allocation-free entry point (address per device)
  if (e == hipSuccess) e = bem::noalloc_scratch(device, &ctx->noalloc_geo);
  if (e == hipSuccess) e = hipMalloc(&ctx->dot_part, bem::dot_scratch_doubles() * sizeof(double));
  if (e != hipSuccess) {
    if (ctx->flags) (void)hipFree(ctx->flags);
    if (ctx->dot_part) (void)hipFree(ctx->dot_part);
    delete ctx;
    return e == hipErrorOutOfMemory ? BEM_ENOMEM : BEM_EDEVICE;
  }
  *out = ctx;
  return BEM_OK;
}

void bem_destroy(bem_ctx *ctx) {
  if (!ctx) return;
  {
    DeviceGuard g(ctx->device);
    (void)hipDeviceSynchronize();
    bem::detach_plans(ctx);
    for (auto &kv : ctx->rules) {
      (void)hipFree(kv.second.tri);
      if (kv.second.xi) (void)hipFree(kv.second.xi);
      for (int c = 0; c < 4; ++c)
        if (kv.second.ss[c]) (void)hipFree(kv.second.ss[c]);
    }
    if (ctx->geo) (void)hipFree(ctx->geo);
    if (ctx->mlp_scratch) (void)hipFree(ctx->mlp_scratch);
    if (ctx->sel_scratch) (void)hipFree(ctx->sel_scratch);
    if (ctx->flags) (void)hipFree(ctx->flags);
    if (ctx->dot_part) (void)hipFree(ctx->dot_part);
  }
  delete ctx;
}

const char *bem_last_error(const bem_ctx *ctx) { return ctx ? ctx->err.c_str() : "no context"; }

int bem_check(bem_ctx *ctx, void *stream) {
  if (!ctx) return BEM_EINVAL;
  DeviceGuard g(ctx->device);
  hipError_t e = hipStreamSynchronize(static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(ctx, e, "hipStreamSynchronize");
  unsigned f = 0;
  e = hipMemcpy(&f, ctx->flags, sizeof f, hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipMemset(ctx->flags, 0, sizeof f);
  if (e != hipSuccess) return hip_fail(ctx, e, "reading device flags");
  if (f & bem::FLAG_EINVAL) return fail(ctx, BEM_EINVAL, "invalid index or degenerate triangle seen on the device");
  if (f & bem::FLAG_NONFINITE) return fail(ctx, BEM_ENONFINITE, "non-finite entry computed");
  if (f & bem::FLAG_LIST)
    return fail(ctx, BEM_EUNSUPPORTED,
                "a sub-tile has more singular pairs than its list holds (edges shared by many "
                "triangles in a mirrored block); assemble that block without mirror_off");
  return BEM_OK;
}

int bem_assemble_nearfield(bem_ctx *ctx, const bem_mesh *mesh, const bem_op *op,
                           const bem_blocks *blocks, void *out, int64_t out_len, void *stream) {
  return assemble_blocks(ctx, mesh, op, blocks, out, out_len, stream, false);
}

int bem_assemble_nearfield_noalloc(bem_ctx *ctx, const bem_mesh *mesh, const bem_op *op,
                                   const bem_blocks *blocks, void *out, int64_t out_len,
                                   void *stream) {
  return assemble_blocks(ctx, mesh, op, blocks, out, out_len, stream, false, false, nullptr,
                         true);
}

int bem_assemble_coupling(bem_ctx *ctx, const bem_mesh *mesh, const bem_op *op,
                          const bem_blocks *pivots, void *out, int64_t out_len, void *stream) {
  return assemble_blocks(ctx, mesh, op, pivots, out, out_len, stream, true);
}

int bem_assemble_nearfield_both(bem_ctx *ctx, const bem_mesh *mesh, const bem_op *op,
                                const bem_blocks *blocks, void *out_slp, void *out_dlp,
                                int64_t out_len, void *stream) {
  if (!ctx) return BEM_EINVAL;
  if (out_len > 0 && (!out_dlp || out_dlp == out_slp))
    return fail(ctx, BEM_EINVAL, "out_dlp is NULL or the same buffer as out_slp");
  return assemble_blocks(ctx, mesh, op, blocks, out_slp, out_len, stream, false, true, out_dlp);
}

int bem_green_matrix(bem_ctx *ctx, const bem_mesh *mesh, const bem_op *op, int32_t side,
                     int32_t ncl, const int32_t *row_ptr, const int32_t *row_idx, int64_t row_len,
                     int32_t m, const double *z, const double *zn, const double *zw,
                     const double *delta, const int64_t *out_off, void *out, int64_t out_len,
                     int32_t max_rows, void *stream) {
  if (!ctx) return BEM_EINVAL;
  int rc;
  if ((rc = check_mesh(ctx, mesh)) || (rc = check_op(ctx, op))) return rc;
  if (side != 0 && side != 1) return fail(ctx, BEM_EINVAL, "side must be 0 or 1");
  if (ncl < 0 || m < 0 || row_len < 0 || out_len < 0) return fail(ctx, BEM_EINVAL, "negative size");
  if (ncl == 0) return BEM_OK;
  if (!row_ptr || (row_len > 0 && !row_idx) || (m > 0 && (!z || !zn || !zw)) || !delta ||
      !out_off || (out_len > 0 && !out))
    return fail(ctx, BEM_EINVAL, "NULL array");
  if (mesh->nt == 0) return fail(ctx, BEM_EINVAL, "empty mesh");
  DeviceGuard g(ctx->device);
  bem_op duffy = *op;  // Green matrices always use the Duffy rule of order q_regular
  duffy.regular_rule = BEM_RULE_DUFFY;
  int64_t ldg;
  const bem::DevRules *rules;
  if ((rc = ensure_geo(ctx, mesh->nt, &ldg)) || (rc = get_rules(ctx, &duffy, &rules))) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = bem::launch_geometry(*mesh, ctx->geo, ldg, ctx->flags, s);
  if (e != hipSuccess) return hip_fail(ctx, e, "geometry kernel launch");
  bem::GreenArgs a{};
  a.geo = ctx->geo;
  a.ldg = ldg;
  a.nt = mesh->nt;
  a.ncl = ncl;
  a.row_ptr = row_ptr;
  a.row_idx = row_idx;
  a.row_len = row_len;
  a.m = m;
  a.z = z;
  a.zn = zn;
  a.zw = zw;
  a.delta = delta;
  a.out_off = out_off;
  a.out = out;
  a.out_len = out_len;
  a.rule = rules->tri;
  a.nq = rules->nq;
  a.kappa = op->kernel == BEM_HELMHOLTZ ? op->kappa : 0.0;
  a.flags = ctx->flags;
  // workgroups per cluster from the row-count hint (any hint is correct)
  const int64_t per = ((int64_t)std::max(max_rows, 1) * ((m + 3) / 4) + 255) / 256;  // 4 points a thread
  e = bem::launch_green(op->kernel, side, a, (int)std::min<int64_t>(per, 64), s);
  if (e != hipSuccess) return hip_fail(ctx, e, "green kernel launch");
  return BEM_OK;
}

int bem_basis_contract(bem_ctx *ctx, int32_t is_complex, int32_t nmat, const int32_t *nrows,
                       const int32_t *rank, int32_t max_rank, const int32_t *piv_cols,
                       const double *pinv, const void *A, const int64_t *a_off, int32_t acols,
                       int64_t a_len, void *V, const int64_t *v_off, int64_t v_len,
                       int32_t max_rows, void *stream) {
  if (!ctx) return BEM_EINVAL;
  if (nmat < 0 || max_rank < 1 || acols < 0 || a_len < 0 || v_len < 0)
    return fail(ctx, BEM_EINVAL, "invalid size");
  if (nmat == 0) return BEM_OK;
  if (!nrows || !rank || !piv_cols || !pinv || !a_off || !v_off || (a_len > 0 && !A) ||
      (v_len > 0 && !V))
    return fail(ctx, BEM_EINVAL, "NULL array");
  DeviceGuard g(ctx->device);
  bem::ContractArgs a{};
  a.nmat = nmat;
  a.nrows = nrows;
  a.rank = rank;
  a.piv_cols = piv_cols;
  a.max_rank = max_rank;
  a.pinv = pinv;
  a.A = A;
  a.a_off = a_off;
  a.acols = acols;
  a.a_len = a_len;
  a.V = V;
  a.v_off = v_off;
  a.v_len = v_len;
  a.flags = ctx->flags;
  // workgroups per matrix (four 16 x 16 tiles each) from the row-count hint
  const int64_t tiles = (int64_t)((std::max(max_rows, 1) + 15) / 16) * ((max_rank + 15) / 16);
  hipError_t e = bem::launch_contract(is_complex != 0, a, (int)std::min<int64_t>((tiles + 3) / 4, 64),
                                      static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(ctx, e, "contraction kernel launch");
  return BEM_OK;
}

int bem_pivot_inverse(bem_ctx *ctx, int32_t is_complex, int32_t nmat, const int32_t *nrows,
                      const int32_t *rank, int32_t max_rank, const int32_t *piv_rows,
                      const int32_t *piv_cols, const void *A, const int64_t *a_off,
                      int32_t acols, int64_t a_len, double *pinv, void *stream) {
  if (!ctx) return BEM_EINVAL;
  if (nmat < 0 || max_rank < 1 || max_rank > 512 || acols < 0 || a_len < 0)
    return fail(ctx, BEM_EINVAL, "invalid size (max_rank in [1, 512])");
  if (nmat == 0) return BEM_OK;
  if (!nrows || !rank || !piv_rows || !piv_cols || !a_off || !pinv || (a_len > 0 && !A))
    return fail(ctx, BEM_EINVAL, "NULL array");
  DeviceGuard g(ctx->device);
  bem::PivInvArgs a{};
  a.nmat = nmat;
  a.nrows = nrows;
  a.rank = rank;
  a.piv_rows = piv_rows;
  a.piv_cols = piv_cols;
  a.max_rank = max_rank;
  a.A = A;
  a.a_off = a_off;
  a.acols = acols;
  a.a_len = a_len;
  a.pinv = pinv;
  a.flags = ctx->flags;
  hipError_t e = bem::launch_pivot_inverse(is_complex != 0, a, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(ctx, e, "pivot inverse launch");
  return BEM_OK;
}

int bem_eval_entries(bem_ctx *ctx, const bem_mesh *mesh, const bem_op *op, int64_t n,
                     const int32_t *rows, const int32_t *cols, void *out, void *stream) {
  if (!ctx) return BEM_EINVAL;
  int rc;
  if ((rc = check_mesh(ctx, mesh)) || (rc = check_op(ctx, op))) return rc;
  if (n < 0) return fail(ctx, BEM_EINVAL, "n < 0");
  if (n == 0) return BEM_OK;
  if (!rows || !cols || !out) return fail(ctx, BEM_EINVAL, "rows / cols / out is NULL");
  if (mesh->nt == 0) return fail(ctx, BEM_EINVAL, "entries requested on an empty mesh");
  DeviceGuard g(ctx->device);
  int64_t ldg;
  const bem::DevRules *rules;
  if ((rc = ensure_geo(ctx, mesh->nt, &ldg)) || (rc = get_rules(ctx, op, &rules))) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = bem::launch_geometry(*mesh, ctx->geo, ldg, ctx->flags, s);
  if (e != hipSuccess) return hip_fail(ctx, e, "geometry kernel launch");
  bem::EntryArgs a{};
  a.v = mesh->v;
  a.tri = mesh->tri;
  a.nv = mesh->nv;
  a.nt = mesh->nt;
  a.geo = ctx->geo;
  a.ldg = ldg;
  a.n = n;
  a.rows = rows;
  a.cols = cols;
  a.out = out;
  a.rule = rules->tri;
  a.nq = rules->nq;
  for (int c = 0; c < 4; ++c) a.ss.eta[c] = rules->ss[c], a.ss.np[c] = rules->np[c];
  a.ss.xi = rules->xi;
  a.ss.q = rules->nxi;
  a.kappa = op->kernel == BEM_HELMHOLTZ ? op->kappa : 0.0;
  a.flags = ctx->flags;
  e = bem::launch_entries(op->kernel, op->layer, op->precision == BEM_MIXED, a, s);
  if (e != hipSuccess) return hip_fail(ctx, e, "entry kernel launch");
  return BEM_OK;
}

int bem_gemv_grouped(bem_ctx *ctx, int32_t is_complex, int32_t trans, int32_t ngroups,
                     const int32_t *grp_ptr, const int32_t *out_ptr, const int32_t *out_idx,
                     int64_t out_len, int32_t nblocks, const int32_t *in_ptr,
                     const int32_t *in_idx, int64_t in_len, const int64_t *a_off, const void *A,
                     int64_t a_len, const void *x, int64_t x_len, void *y, int64_t y_len,
                     void *stream) {
  if (!ctx) return BEM_EINVAL;
  if (ngroups < 0 || nblocks < 0 || out_len < 0 || in_len < 0 || a_len < 0 || x_len < 0 ||
      y_len < 0)
    return fail(ctx, BEM_EINVAL, "negative size");
  if (ngroups == 0) return BEM_OK;
  if (!grp_ptr || !out_ptr || (out_len > 0 && !out_idx) || (nblocks > 0 && (!in_ptr || !a_off)) ||
      (in_len > 0 && !in_idx) || (a_len > 0 && !A) || (x_len > 0 && !x) || (y_len > 0 && !y))
    return fail(ctx, BEM_EINVAL, "NULL array");
  DeviceGuard g(ctx->device);
  bem::GemvArgs a{};
  a.ngroups = ngroups;
  a.nblocks = nblocks;
  a.grp_ptr = grp_ptr;
  a.out_ptr = out_ptr;
  a.out_idx = out_idx;
  a.out_len = out_len;
  a.in_ptr = in_ptr;
  a.in_idx = in_idx;
  a.in_len = in_len;
  a.a_off = a_off;
  a.A = A;
  a.a_len = a_len;
  a.x = x;
  a.x_len = x_len;
  a.y = y;
  a.y_len = y_len;
  a.flags = ctx->flags;
  hipError_t e = bem::launch_gemv(is_complex != 0, trans != 0, a, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(ctx, e, "gemv kernel launch");
  return BEM_OK;
}

int bem_vec_dot(bem_ctx *ctx, int32_t is_complex, int32_t conj, int64_t n, const void *x,
                const void *y, double *out, void *stream) {
  if (!ctx) return BEM_EINVAL;
  if (n < 0 || !out || (n > 0 && (!x || !y))) return fail(ctx, BEM_EINVAL, "bad size or NULL array");
  DeviceGuard g(ctx->device);
  hipError_t e = bem::launch_dot(is_complex != 0, conj != 0, n, static_cast<const double *>(x),
                                 static_cast<const double *>(y), ctx->dot_part, out,
                                 static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(ctx, e, "dot kernel launch");
  return BEM_OK;
}

int bem_vec_axpby(bem_ctx *ctx, int32_t is_complex, int64_t n, double ar, double ai,
                  const void *x, double br, double bi, void *y, void *stream) {
  if (!ctx) return BEM_EINVAL;
  if (n < 0 || (n > 0 && (!x || !y))) return fail(ctx, BEM_EINVAL, "bad size or NULL array");
  DeviceGuard g(ctx->device);
  hipError_t e = bem::launch_axpby(is_complex != 0, n, ar, ai, static_cast<const double *>(x), br,
                                   bi, static_cast<double *>(y), static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(ctx, e, "axpby kernel launch");
  return BEM_OK;
}

int bem_cg_step(bem_ctx *ctx, int64_t n, double *state, void *x, void *r, void *p,
                const void *q, void *stream) {
  if (!ctx) return BEM_EINVAL;
  if (n < 0 || !state || (n > 0 && (!x || !r || !p || !q)))
    return fail(ctx, BEM_EINVAL, "bad size or NULL array");
  DeviceGuard g(ctx->device);
  hipError_t e = bem::launch_cg_step(n, state, static_cast<double *>(x), static_cast<double *>(r),
                                     static_cast<double *>(p), static_cast<const double *>(q),
                                     ctx->dot_part, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(ctx, e, "conjugate-gradient kernel launch");
  return BEM_OK;
}

int bem_mass_apply(bem_ctx *ctx, const bem_mesh *mesh, int32_t is_complex, double cr, double ci,
                   const void *x, void *y, void *stream) {
  if (!ctx) return BEM_EINVAL;
  int rc;
  if ((rc = check_mesh(ctx, mesh))) return rc;
  if (mesh->nt == 0) return BEM_OK;
  if (!x || !y) return fail(ctx, BEM_EINVAL, "NULL array");
  DeviceGuard g(ctx->device);
  int64_t ldg;
  if ((rc = ensure_geo(ctx, mesh->nt, &ldg))) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = bem::launch_geometry(*mesh, ctx->geo, ldg, ctx->flags, s);
  if (e == hipSuccess)
    e = bem::launch_mass(is_complex != 0, mesh->nt, ctx->geo, ldg, cr, ci,
                         static_cast<const double *>(x), static_cast<double *>(y), s);
  if (e != hipSuccess) return hip_fail(ctx, e, "mass kernel launch");
  return BEM_OK;
}

int bem_p1_pairs(bem_ctx *ctx, const bem_mesh *mesh, const bem_op *op, int64_t n,
                 const int32_t *rows, const int32_t *cols, void *out, void *stream) {
  if (!ctx) return BEM_EINVAL;
  int rc;
  if ((rc = check_mesh(ctx, mesh)) || (rc = check_op(ctx, op))) return rc;
  if (op->precision != BEM_PLAIN_FP64)
    return fail(ctx, BEM_EUNSUPPORTED, "piecewise-linear pairs are plain FP64");
  if (n < 0) return fail(ctx, BEM_EINVAL, "n < 0");
  if (n == 0) return BEM_OK;
  if (!rows || !cols || !out) return fail(ctx, BEM_EINVAL, "rows / cols / out is NULL");
  if (mesh->nt == 0) return fail(ctx, BEM_EINVAL, "pairs requested on an empty mesh");
  DeviceGuard g(ctx->device);
  int64_t ldg;
  const bem::DevRules *rules;
  if ((rc = ensure_geo(ctx, mesh->nt, &ldg)) || (rc = get_rules(ctx, op, &rules))) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = bem::launch_geometry(*mesh, ctx->geo, ldg, ctx->flags, s);
  if (e != hipSuccess) return hip_fail(ctx, e, "geometry kernel launch");
  bem::P1Args a{};
  a.v = mesh->v;
  a.tri = mesh->tri;
  a.nv = mesh->nv;
  a.nt = mesh->nt;
  a.geo = ctx->geo;
  a.ldg = ldg;
  a.n = n;
  a.rows = rows;
  a.cols = cols;
  a.out = out;
  a.rule = rules->tri;
  a.nq = rules->nq;
  for (int c = 0; c < 4; ++c) a.ss.eta[c] = rules->ss[c], a.ss.np[c] = rules->np[c];
  a.ss.xi = rules->xi;
  a.ss.q = rules->nxi;
  a.kappa = op->kernel == BEM_HELMHOLTZ ? op->kappa : 0.0;
  a.flags = ctx->flags;
  e = bem::launch_p1_pairs(op->kernel, op->layer, a, s);
  if (e != hipSuccess) return hip_fail(ctx, e, "P1 pair kernel launch");
  return BEM_OK;
}

int bem_p1_gather(bem_ctx *ctx, int32_t is_complex, int32_t nrv, const int32_t *rs_ptr,
                  const int32_t *rs_tri, const int32_t *rs_loc, int64_t rs_len, int32_t ncv,
                  const int32_t *cs_ptr, const int32_t *cs_tri, const int32_t *cs_loc,
                  int64_t cs_len, int32_t ntr, int32_t ntc, const void *local, void *out,
                  void *stream) {
  if (!ctx) return BEM_EINVAL;
  if (nrv < 0 || ncv < 0 || ntr < 0 || ntc < 0 || rs_len < 0 || cs_len < 0)
    return fail(ctx, BEM_EINVAL, "negative size");
  if ((int64_t)nrv * ncv == 0) return BEM_OK;
  if (!rs_ptr || !cs_ptr || (rs_len > 0 && (!rs_tri || !rs_loc)) ||
      (cs_len > 0 && (!cs_tri || !cs_loc)) || !out || ((int64_t)ntr * ntc > 0 && !local))
    return fail(ctx, BEM_EINVAL, "NULL array");
  DeviceGuard g(ctx->device);
  bem::P1GatherArgs a{};
  a.nrv = nrv;
  a.ncv = ncv;
  a.ntr = ntr;
  a.ntc = ntc;
  a.rs_ptr = rs_ptr;
  a.rs_tri = rs_tri;
  a.rs_loc = rs_loc;
  a.rs_len = rs_len;
  a.cs_ptr = cs_ptr;
  a.cs_tri = cs_tri;
  a.cs_loc = cs_loc;
  a.cs_len = cs_len;
  a.local = local;
  a.out = out;
  a.flags = ctx->flags;
  hipError_t e = bem::launch_p1_gather(is_complex != 0, a, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(ctx, e, "P1 gather launch");
  return BEM_OK;
}

}  // extern "C"
