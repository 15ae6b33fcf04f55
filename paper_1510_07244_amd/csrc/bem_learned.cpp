// C-ABI of the learned form: the order selector's network (FP32 training,
// FP16 inference), its training samples, order selection over near-field
// blocks and the near-field assembly with per-entry orders.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "bem_internal.h"

using namespace bem;

namespace {

int grow_mlp_scratch(bem_ctx *ctx, size_t floats) {
  if (floats <= ctx->mlp_cap) return BEM_OK;
  hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) return hip_fail(ctx, e, "hipDeviceSynchronize");
  if (ctx->mlp_scratch) (void)hipFree(ctx->mlp_scratch);
  ctx->mlp_scratch = nullptr;
  ctx->mlp_cap = 0;
  e = hipMalloc(&ctx->mlp_scratch, floats * sizeof(float));
  if (e != hipSuccess) return hip_fail(ctx, e, "hipMalloc(network scratch)");
  ctx->mlp_cap = floats;
  return BEM_OK;
}

int grow_sel_scratch(bem_ctx *ctx, size_t bytes) {
  if (bytes <= ctx->sel_cap) return BEM_OK;
  hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) return hip_fail(ctx, e, "hipDeviceSynchronize");
  if (ctx->sel_scratch) (void)hipFree(ctx->sel_scratch);
  ctx->sel_scratch = nullptr;
  ctx->sel_cap = 0;
  e = hipMalloc(&ctx->sel_scratch, bytes);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipMalloc(selector scratch)");
  ctx->sel_cap = bytes;
  return BEM_OK;
}

size_t packed_pad() { return (mlp_packed_bytes() + 255) / 256 * 256; }

// Duffy rules of orders 1 .. max (index = order) for an operator.
int order_rules(bem_ctx *ctx, const bem_op *op, int qmax, const DevRules **r) {
  for (int q = 1; q <= qmax; ++q) {
    bem_op o = *op;
    o.regular_rule = BEM_RULE_DUFFY;
    o.q_regular = q;
    int rc = get_rules(ctx, &o, &r[q]);
    if (rc) return rc;
  }
  return BEM_OK;
}

int block_list_args(bem_ctx *ctx, const bem_mesh *mesh, const bem_op *op, const bem_blocks *b,
                    const void *out, int64_t out_len) {
  int rc;
  if ((rc = check_mesh(ctx, mesh)) || (rc = check_op(ctx, op)) ||
      (rc = check_blocks(ctx, b, out, out_len)))
    return rc;
  if (b->n > 0 && mesh->nt == 0) return fail(ctx, BEM_EINVAL, "blocks given for an empty mesh");
  if (b->mirror_off) return fail(ctx, BEM_EINVAL, "mirror_off is not supported by the learned form");
  return BEM_OK;
}

}  // namespace

extern "C" {

int bem_mlp_params(int32_t n_out) {
  if (n_out < 1 || n_out > 16) return BEM_EINVAL;
  return mlp_params(n_out);
}

int bem_mlp_forward(bem_ctx *ctx, int32_t n_out, int32_t fp16, const float *params, int64_t n,
                    const float *x, float *y, void *stream) {
  if (!ctx) return BEM_EINVAL;
  if (n_out < 1 || n_out > 16 || (fp16 != 0 && fp16 != 1) || n < 0)
    return fail(ctx, BEM_EINVAL, "n_out in [1, 16], fp16 0/1, n >= 0");
  if (n == 0) return BEM_OK;
  if (!params || !x || !y) return fail(ctx, BEM_EINVAL, "NULL array");
  DeviceGuard g(ctx->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e;
  if (fp16) {
    int rc = grow_sel_scratch(ctx, packed_pad());
    if (rc) return rc;
    if ((e = launch_pack_net(n_out, params, ctx->sel_scratch, s)) != hipSuccess)
      return hip_fail(ctx, e, "network packing launch");
  }
  e = launch_mlp_forward(fp16 == 1, n_out, params, ctx->sel_scratch, n, x, y, s);
  if (e != hipSuccess) return hip_fail(ctx, e, "network forward launch");
  return BEM_OK;
}

int bem_mlp_grad(bem_ctx *ctx, int32_t n_out, const float *params, int64_t n, const float *x,
                 const float *t, float *grad, float *loss, void *stream) {
  if (!ctx) return BEM_EINVAL;
  if (n_out < 1 || n_out > 16 || n < 1) return fail(ctx, BEM_EINVAL, "n_out in [1, 16], n >= 1");
  if (!params || !x || !t || !grad) return fail(ctx, BEM_EINVAL, "NULL array");
  if (n > ((int64_t)1 << 31) * 16) return fail(ctx, BEM_EINVAL, "n too large");
  DeviceGuard g(ctx->device);
  const size_t need = mlp_grad_scratch_floats(n_out, n);
  int rc = grow_mlp_scratch(ctx, need);
  if (rc) return rc;
  const int64_t nwg = (n + 15) / 16;
  float *part = ctx->mlp_scratch, *lpart = ctx->mlp_scratch + (size_t)nwg * mlp_params(n_out);
  hipError_t e = launch_mlp_grad(n_out, params, n, x, t, part, lpart, grad, loss,
                                 static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(ctx, e, "network gradient launch");
  return BEM_OK;
}

int bem_mlp_adam(bem_ctx *ctx, int64_t np, float *params, const float *grad, float *m, float *v,
                 int32_t step, float lr, float beta1, float beta2, float eps, void *stream) {
  if (!ctx) return BEM_EINVAL;
  if (np < 0 || step < 1 || !(lr >= 0) || !(beta1 >= 0 && beta1 < 1) || !(beta2 >= 0 && beta2 < 1) ||
      !(eps > 0))
    return fail(ctx, BEM_EINVAL, "Adam: np >= 0, step >= 1, lr >= 0, betas in [0, 1), eps > 0");
  if (np == 0) return BEM_OK;
  if (!params || !grad || !m || !v) return fail(ctx, BEM_EINVAL, "NULL array");
  DeviceGuard g(ctx->device);
  const float c1 = (float)(1.0 / (1.0 - std::pow((double)beta1, step)));
  const float c2 = (float)(1.0 / (1.0 - std::pow((double)beta2, step)));
  hipError_t e = launch_mlp_adam(np, params, grad, m, v, lr, beta1, beta2, eps, c1, c2,
                                 static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(ctx, e, "Adam launch");
  return BEM_OK;
}

int bem_selector_samples(bem_ctx *ctx, const bem_mesh *mesh, const bem_op *op, int64_t n,
                         const int32_t *rows, const int32_t *cols, float *x, float *t,
                         void *stream) {
  if (!ctx) return BEM_EINVAL;
  int rc;
  if ((rc = check_mesh(ctx, mesh)) || (rc = check_op(ctx, op))) return rc;
  if (op->precision != BEM_PLAIN_FP64)
    return fail(ctx, BEM_EUNSUPPORTED, "selector samples use the plain FP64 rules");
  if (n < 0) return fail(ctx, BEM_EINVAL, "n < 0");
  if (n == 0) return BEM_OK;
  if (!rows || !cols || !x || !t) return fail(ctx, BEM_EINVAL, "NULL array");
  if (mesh->nt == 0) return fail(ctx, BEM_EINVAL, "empty mesh");
  DeviceGuard g(ctx->device);
  const DevRules *r[kSelQ + 1];
  const DevRules *ref;
  bem_op o8 = *op;
  o8.regular_rule = BEM_RULE_DUFFY;
  o8.q_regular = 8;
  int64_t ldg;
  if ((rc = order_rules(ctx, op, kSelQ, r)) || (rc = get_rules(ctx, &o8, &ref)) ||
      (rc = ensure_geo(ctx, mesh->nt, &ldg)))
    return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = launch_geometry(*mesh, ctx->geo, ldg, ctx->flags, s);
  if (e != hipSuccess) return hip_fail(ctx, e, "geometry kernel launch");
  SampleArgs a{};
  a.tri = mesh->tri;
  a.nt = mesh->nt;
  a.geo = ctx->geo;
  a.ldg = ldg;
  a.n = n;
  a.rows = rows;
  a.cols = cols;
  a.x = x;
  a.t = t;
  for (int q = 1; q <= kSelQ; ++q) a.rule[q - 1] = r[q]->tri, a.nq[q - 1] = r[q]->nq;
  a.rule[kSelQ] = ref->tri;
  a.nq[kSelQ] = ref->nq;
  a.kappa = op->kernel == BEM_HELMHOLTZ ? op->kappa : 0.0;
  a.flags = ctx->flags;
  e = launch_selector_samples(op->kernel, op->layer, a, s);
  if (e != hipSuccess) return hip_fail(ctx, e, "selector samples launch");
  return BEM_OK;
}

int bem_select_orders(bem_ctx *ctx, const bem_mesh *mesh, const bem_op *op,
                      const bem_blocks *blocks, const float *params, const float *range,
                      double tol, double margin, int32_t q_min, int32_t group,
                      int8_t *orders, int64_t orders_len, void *stream) {
  if (!ctx) return BEM_EINVAL;
  int rc;
  if ((rc = block_list_args(ctx, mesh, op, blocks, orders, orders_len))) return rc;
  if (op->regular_rule != BEM_RULE_DUFFY || op->q_regular < 2 || op->q_regular > kSelQ)
    return fail(ctx, BEM_EUNSUPPORTED, "order selection needs the Duffy rule with q_regular in [2, 6]");
  if (!(tol > 0) || !std::isfinite(tol) || !std::isfinite(margin) || q_min < 2 ||
      q_min > op->q_regular)
    return fail(ctx, BEM_EINVAL, "tol > 0, finite margin, q_min in [2, q_regular]");
  if (!params) return fail(ctx, BEM_EINVAL, "params is NULL");
  if (group < 1 || group > 8) return fail(ctx, BEM_EINVAL, "group in [1, 8]");
  if (blocks->n == 0) return BEM_OK;
  DeviceGuard g(ctx->device);
  int64_t ldg;
  const int64_t ldt = ((int64_t)mesh->nt + 63) / 64 * 64;
  if ((rc = ensure_geo(ctx, mesh->nt, &ldg)) ||
      (rc = grow_sel_scratch(ctx, packed_pad() + (size_t)ldt * (6 * sizeof(double) + 3 * sizeof(float)))))
    return rc;
  char *base = static_cast<char *>(ctx->sel_scratch);
  double *tin_c = reinterpret_cast<double *>(base + packed_pad());
  double *tin_n = tin_c + 3 * ldt;
  float *tin_f = reinterpret_cast<float *>(tin_n + 3 * ldt);
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = launch_geometry(*mesh, ctx->geo, ldg, ctx->flags, s);
  if (e == hipSuccess) e = launch_tri_inputs(ctx->geo, ldg, mesh->nt, tin_c, tin_n, tin_f, ldt, s);
  if (e == hipSuccess) e = launch_pack_net(kSelQ, params, base, s);
  if (e != hipSuccess) return hip_fail(ctx, e, "geometry / selector input launch");
  int ncu = 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, ctx->device) != hipSuccess ||
      ncu <= 0)
    ncu = 256;
  SelectArgs a{};
  a.tri = mesh->tri;
  a.nt = mesh->nt;
  a.geo = ctx->geo;
  a.ldg = ldg;
  a.nblocks = blocks->n;
  a.row_ptr = blocks->row_ptr;
  a.row_idx = blocks->row_idx;
  a.col_ptr = blocks->col_ptr;
  a.col_idx = blocks->col_idx;
  a.row_len = blocks->row_len;
  a.col_len = blocks->col_len;
  a.out_off = blocks->out_off;
  a.orders = orders;
  a.out_len = orders_len;
  a.net = base;
  a.tin_c = tin_c;
  a.tin_n = tin_n;
  a.tin_f = tin_f;
  a.ldt = ldt;
  a.range = range;
  a.layer = op->layer;
  a.q_plain = op->q_regular;
  a.q_min = q_min;
  a.group = group;
  a.margin = (float)margin;
  a.log_tol = (float)std::log10(tol);
  a.kappa = op->kernel == BEM_HELMHOLTZ ? op->kappa : 0.0;
  a.flags = ctx->flags;
  e = launch_select_orders(a, 4 * ncu, s);
  if (e != hipSuccess) return hip_fail(ctx, e, "order selection launch");
  return BEM_OK;
}

int bem_assemble_nearfield_learned(bem_ctx *ctx, const bem_mesh *mesh, const bem_op *op,
                                   const bem_blocks *blocks, const int8_t *orders, void *out,
                                   int64_t out_len, void *stream) {
  if (!ctx) return BEM_EINVAL;
  int rc;
  if ((rc = block_list_args(ctx, mesh, op, blocks, out, out_len))) return rc;
  if (op->precision != BEM_PLAIN_FP64 || op->regular_rule != BEM_RULE_DUFFY ||
      op->q_regular < 2 || op->q_regular > kSelQ)
    return fail(ctx, BEM_EUNSUPPORTED,
                "per-entry orders need plain FP64, the Duffy rule and q_regular in [2, 6]");
  if (out_len > 0 && !orders) return fail(ctx, BEM_EINVAL, "orders is NULL");
  if (blocks->n == 0) return BEM_OK;
  DeviceGuard g(ctx->device);
  const DevRules *r[BEM_MAX_ORDER + 1] = {};
  int64_t ldg;
  if ((rc = order_rules(ctx, op, op->q_regular, r)) || (rc = ensure_geo(ctx, mesh->nt, &ldg)))
    return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = launch_geometry(*mesh, ctx->geo, ldg, ctx->flags, s);
  if (e != hipSuccess) return hip_fail(ctx, e, "geometry kernel launch");
  OrderRules o{};
  for (int q = 2; q <= op->q_regular; ++q) o.rule[q] = r[q]->tri, o.nq[q] = r[q]->nq;
  o.orders = orders;
  o.q_max = op->q_regular;
  const DevRules *plain = r[op->q_regular];
  BlockArgs a{};
  a.v = mesh->v;
  a.tri = mesh->tri;
  a.nv = mesh->nv;
  a.nt = mesh->nt;
  a.geo = ctx->geo;
  a.ldg = ldg;
  a.nblocks = blocks->n;
  a.row_ptr = blocks->row_ptr;
  a.row_idx = blocks->row_idx;
  a.col_ptr = blocks->col_ptr;
  a.col_idx = blocks->col_idx;
  a.row_len = blocks->row_len;
  a.col_len = blocks->col_len;
  a.out_off = blocks->out_off;
  a.out = out;
  a.out_len = out_len;
  a.rule = plain->tri;
  a.nq = plain->nq;
  // LDS sized for the largest order (q^2 points are a multiple of its chunk)
  const int xc = learned_chunk(op->q_regular, op->kernel);
  a.nq_pad = (plain->nq + xc - 1) / xc * xc;
  size_t lds;
  if (!block_tile_shape(a.nq_pad, false, ctx->lds_budget, &a.tr, &a.tc, &lds))
    return fail(ctx, BEM_EUNSUPPORTED, "quadrature order too high for the LDS budget");
  for (int c = 0; c < 4; ++c) a.ss.eta[c] = plain->ss[c], a.ss.np[c] = plain->np[c];
  a.ss.xi = plain->xi;
  a.ss.q = plain->nxi;
  a.kappa = op->kernel == BEM_HELMHOLTZ ? op->kappa : 0.0;
  a.flags = ctx->flags;
  e = launch_blocks_learned(op->kernel, op->layer, a, o, lds, s);
  if (e != hipSuccess) return hip_fail(ctx, e, "learned block kernel launch");
  return BEM_OK;
}

// Network file: 8-byte tag, int32 n_out, step, contents (1 Adam moments, 2
// training range), reserved, then FP32 parameters [, m, v] [, range].
namespace {
constexpr char kMlpTag[8] = {'B', 'E', 'M', 'M', 'L', 'P', '0', '1'};
enum { MLP_MOMENTS = 1, MLP_RANGE = 2 };
}  // namespace

int bem_mlp_save(bem_ctx *ctx, const char *path, int32_t n_out, const float *params,
                 const float *m, const float *v, const float *range, int32_t step, void *stream) {
  if (!ctx) return BEM_EINVAL;
  const int np = mlp_params(n_out);
  if (np < 0) return fail(ctx, BEM_EINVAL, "n_out must be in [1, 16]");
  if (!path || !params || (!m) != (!v) || step < 0)
    return fail(ctx, BEM_EINVAL, "path / params NULL, m and v not both given, or step < 0");
  DeviceGuard g(ctx->device);
  hipError_t e = hipStreamSynchronize(static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(ctx, e, "hipStreamSynchronize");
  const int32_t contents = (m ? MLP_MOMENTS : 0) | (range ? MLP_RANGE : 0);
  std::vector<float> h((size_t)np * (m ? 3 : 1) + (range ? 16 : 0));
  e = hipMemcpy(h.data(), params, np * sizeof(float), hipMemcpyDeviceToHost);
  if (e == hipSuccess && m) e = hipMemcpy(h.data() + np, m, np * sizeof(float), hipMemcpyDeviceToHost);
  if (e == hipSuccess && m) e = hipMemcpy(h.data() + 2 * np, v, np * sizeof(float), hipMemcpyDeviceToHost);
  if (e == hipSuccess && range)
    e = hipMemcpy(h.data() + (size_t)np * (m ? 3 : 1), range, 16 * sizeof(float), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(ctx, e, "reading the network");
  FILE *f = std::fopen(path, "wb");
  if (!f) return fail(ctx, BEM_EINVAL, std::string("cannot open ") + path + " for writing");
  const int32_t head[4] = {n_out, step, contents, 0};
  bool ok = std::fwrite(kMlpTag, 1, 8, f) == 8 && std::fwrite(head, sizeof head, 1, f) == 1 &&
            std::fwrite(h.data(), sizeof(float), h.size(), f) == h.size();
  ok = (std::fclose(f) == 0) && ok;
  if (!ok) return fail(ctx, BEM_EINVAL, std::string("writing ") + path + " failed");
  return BEM_OK;
}

int bem_mlp_load(bem_ctx *ctx, const char *path, int32_t n_out, float *params, float *m, float *v,
                 float *range, int32_t *step, void *stream) {
  if (!ctx) return BEM_EINVAL;
  const int np = mlp_params(n_out);
  if (np < 0) return fail(ctx, BEM_EINVAL, "n_out must be in [1, 16]");
  if (!path || !params || (!m) != (!v))
    return fail(ctx, BEM_EINVAL, "path / params NULL, or m and v not both given");
  FILE *f = std::fopen(path, "rb");
  if (!f) return fail(ctx, BEM_EINVAL, std::string("cannot open ") + path);
  char tag[8];
  int32_t head[4];
  bool ok = std::fread(tag, 1, 8, f) == 8 && std::memcmp(tag, kMlpTag, 8) == 0 &&
            std::fread(head, sizeof head, 1, f) == 1;
  const int32_t contents = ok ? head[2] : 0;
  ok = ok && head[0] == n_out && head[1] >= 0 && (contents & ~(MLP_MOMENTS | MLP_RANGE)) == 0;
  ok = ok && (!m || (contents & MLP_MOMENTS)) && (!range || (contents & MLP_RANGE));
  std::vector<float> h;
  if (ok) {
    h.resize((size_t)np * ((contents & MLP_MOMENTS) ? 3 : 1) + ((contents & MLP_RANGE) ? 16 : 0));
    ok = std::fread(h.data(), sizeof(float), h.size(), f) == h.size() &&
         std::fgetc(f) == EOF;  // nothing after the declared contents
  }
  std::fclose(f);
  if (!ok)
    return fail(ctx, BEM_EINVAL, std::string(path) + ": not a network file of this n_out, "
                                 "truncated, or without the requested moments / range");
  DeviceGuard g(ctx->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = hipMemcpyAsync(params, h.data(), np * sizeof(float), hipMemcpyHostToDevice, s);
  if (e == hipSuccess && m)
    e = hipMemcpyAsync(m, h.data() + np, np * sizeof(float), hipMemcpyHostToDevice, s);
  if (e == hipSuccess && m)
    e = hipMemcpyAsync(v, h.data() + 2 * (size_t)np, np * sizeof(float), hipMemcpyHostToDevice, s);
  if (e == hipSuccess && range)
    e = hipMemcpyAsync(range, h.data() + (size_t)np * ((contents & MLP_MOMENTS) ? 3 : 1),
                       16 * sizeof(float), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);  // h is released on return
  if (e != hipSuccess) return hip_fail(ctx, e, "writing the network to the device");
  if (step) *step = head[1];
  return BEM_OK;
}

int bem_cluster_features(int32_t n, const double *box, const int32_t *begin, const int32_t *end,
                         const int32_t *height, double kappa, int32_t side, double eps,
                         float *out) {
  if (n < 0 || !(eps > 0.0) || (n > 0 && (!box || !begin || !end || !height || !out)))
    return BEM_EINVAL;
  const double leps = std::log10(eps);
  for (int32_t c = 0; c < n; ++c) {
    double ext[3], d2 = 0.0;
    for (int k = 0; k < 3; ++k) {
      ext[k] = box[6 * (int64_t)c + 3 + k] - box[6 * (int64_t)c + k];
      d2 += ext[k] * ext[k];
    }
    std::sort(ext, ext + 3);
    const double big = std::max(ext[2], 1e-300), diam = std::sqrt(d2);
    float *x = out + 8 * (int64_t)c;
    x[0] = (float)std::log2((double)std::max(end[c] - begin[c], 1));
    x[1] = (float)std::log10(std::max(diam, 1e-300));
    x[2] = (float)(ext[1] / big);
    x[3] = (float)(ext[0] / big);
    x[4] = (float)height[c];
    x[5] = (float)(kappa * diam);
    x[6] = (float)side;
    x[7] = (float)leps;
  }
  return BEM_OK;
}

}  // extern "C"
