// Internal declarations of the MI355X BEM assembly library (not installed).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <set>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/bem.h"

namespace bem {

// --------------------------------------------------------------- quadrature
// q-point Gauss-Legendre rule on [0,1], nodes increasing.
void gauss_legendre01(int q, double *x, double *w);

// Points of a rule on one flat triangle in the coordinates of the affine map
// Phi(s,t) = v0 + s (v1 - v0) + t (v2 - v1), such that
//   int_tau f ~ sqrt(g) * sum_k w[k] f(Phi(s[k], t[k])).
struct TriRule {
  std::vector<double> s, t, w;
};
TriRule triangle_rule(int rule, int q);

// Sauter-Schwab rule of one singular class, factored as (x^, y^) = xi g(eta):
// per region and (eta1, eta2, eta3) Gauss triple the map g at xi = 1
// (xs, xt, ys, yt) and the weight w_b w_c w_d J(eta) / xi^3; the xi nodes and
// weights w_a xi_a^3 are in XiRule.
struct SSRule {
  std::vector<double> xs, xt, ys, yt, w;
};
struct XiRule {
  std::vector<double> x, w3;
};
enum { CLS_DISJOINT = 0, CLS_VERTEX = 1, CLS_EDGE = 2, CLS_IDENTICAL = 3 };
SSRule ss_rule(int cls, int q);
SSRule ss_rule_identical_symmetric(int q);  // 3 of the 6 identical regions, weights doubled
XiRule xi_rule(int q);

// --------------------------------------------------------------- geometry
// Per-triangle geometry, structure of arrays: geo[f * ldg + i].
enum GeoField {
  G_V0X, G_V0Y, G_V0Z,  // first vertex
  G_E1X, G_E1Y, G_E1Z,  // v1 - v0
  G_E2X, G_E2Y, G_E2Z,  // v2 - v1
  G_SG,                 // sqrt of the Gram determinant = 2 * area
  G_NX, G_NY, G_NZ,     // outward unit normal
  G_LOX, G_LOY, G_LOZ,  // bounding box
  G_HIX, G_HIY, G_HIZ,
  GEO_NF
};

// sticky device flags
// FLAG_LIST: a sub-tile listed more pairs for the FP64 pass than its list
// holds (mirrored edge-adjacent pairs of edges shared by many triangles)
enum : unsigned { FLAG_EINVAL = 1u, FLAG_NONFINITE = 2u, FLAG_LIST = 4u };

// Device copies of the quadrature tables of one (rule, q_regular, q_singular).
struct DevRules {
  int nq = 0;         // points per triangle (regular rule)
  double *tri = nullptr;  // [3][nq]: s, t, w
  // Sauter-Schwab eta tables per class (index = class 1..3); index 0 (no
  // disjoint table is needed) holds the identical-pair table for kernels
  // symmetric in x and y (ss_rule_identical_symmetric)
  int np[4] = {0, 0, 0, 0};
  double *ss[4] = {nullptr, nullptr, nullptr, nullptr};  // [5][np]: xs, xt, ys, yt, w
  int nxi = 0;               // Sauter-Schwab order q
  double *xi = nullptr;      // [3q + 2]: xi, w xi^2, w xi, then M1 = sum w xi, M2 = sum w xi^2
};

// Device Sauter-Schwab tables as seen by the kernels.
struct SSArgs {
  const double *eta[4];  // per class [5][np]; [0]: identical pairs, symmetric kernels
  int32_t np[4];
  const double *xi;      // [4][q]
  int32_t q;
};

// Arguments of the block kernels (passed by value).
struct BlockArgs {
  const double *v;
  const int32_t *tri;
  int32_t nv, nt;
  const double *geo;
  int64_t ldg;
  int32_t nblocks;
  const int32_t *row_ptr, *row_idx, *col_ptr, *col_idx;
  int64_t row_len, col_len;
  const int64_t *out_off;
  const int64_t *mirror_off;  // coupling of a single layer: transposed copies (or null)
  void *out;
  void *out2;          // both layers in one pass: the double layer's output
  int64_t out_len;
  const double *rule;  // [3][nq]
  int32_t nq, nq_pad;
  int32_t tr, tc;      // sub-tile rows / columns
  SSArgs ss;
  double kappa;
  double near_ratio;   // mixed form: near-singular box-distance ratio
  unsigned *flags;
};

struct EntryArgs {
  const double *v;
  const int32_t *tri;
  int32_t nv, nt;
  const double *geo;
  int64_t ldg;
  int64_t n;
  const int32_t *rows, *cols;
  void *out;
  const double *rule;
  int32_t nq;
  SSArgs ss;
  double kappa;
  unsigned *flags;
};

struct GreenArgs {
  const double *geo;
  int64_t ldg;
  int32_t nt;
  int32_t ncl;
  const int32_t *row_ptr, *row_idx;
  int64_t row_len;
  int32_t m;
  const double *z, *zn, *zw, *delta;
  const int64_t *out_off;
  void *out;
  int64_t out_len;
  const double *rule;
  int32_t nq;
  double kappa;
  unsigned *flags;
};

struct ContractArgs {
  int32_t nmat;
  const int32_t *nrows, *rank, *piv_cols;
  int32_t max_rank;
  const double *pinv;
  const void *A;
  const int64_t *a_off;
  int32_t acols;
  int64_t a_len;
  void *V;
  const int64_t *v_off;
  int64_t v_len;
  unsigned *flags;
};

struct PivInvArgs {
  int32_t nmat;
  const int32_t *nrows, *rank, *piv_rows, *piv_cols;
  int32_t max_rank;
  const void *A;
  const int64_t *a_off;
  int32_t acols;
  int64_t a_len;
  double *pinv;
  unsigned *flags;
};

// Arguments of the persistent batched block kernel: one BlockArgs per batch
// entry (all with the same rule and sub-tile shape) and a queue of sub-tiles.
struct PersistentArgs {
  const BlockArgs *batches;  // device [nbatch]
  const int32_t *mode;       // device [nbatch]: bit 0 coupling block list,
                             // bits 1-2 layer (BEM_SLP, BEM_DLP, kBoth = 2)
  const int4 *tiles;         // device [ntiles]: batch, block, first row, first column
  int32_t ntiles, nbatch;
  int32_t *counter;          // device queue head, 0 at launch
  int32_t grid;              // workgroups
};

// Grouped gathered matrix-vector products of the H^2 matrix (bem_h2mv.hip).
struct GemvArgs {
  int32_t ngroups, nblocks;
  const int32_t *grp_ptr;            // [ngroups + 1] blocks of each group
  const int32_t *out_ptr, *out_idx;  // [ngroups + 1], output indices into y
  int64_t out_len;                   // length of out_idx
  const int32_t *in_ptr, *in_idx;    // [nblocks + 1], input indices into x
  int64_t in_len;                    // length of in_idx
  const int64_t *a_off;              // [nblocks] matrix offsets (entries)
  const void *A;
  int64_t a_len;
  const void *x;
  int64_t x_len;
  void *y;
  int64_t y_len;
  unsigned *flags;
};
hipError_t launch_gemv(bool cplx, bool trans, const GemvArgs &a, hipStream_t s);
size_t dot_scratch_doubles();
hipError_t launch_dot(bool cplx, bool conj, int64_t n, const double *x, const double *y,
                      double *part, double *out, hipStream_t s);
hipError_t launch_axpby(bool cplx, int64_t n, double ar, double ai, const double *x, double br,
                        double bi, double *y, hipStream_t s);
// one conjugate-gradient update with the scalars in state (bem_cg_step)
hipError_t launch_cg_step(int64_t n, double *state, double *x, double *r, double *p,
                          const double *q, double *dot_part, hipStream_t s);
hipError_t launch_mass(bool cplx, int32_t nt, const double *geo, int64_t ldg, double cr, double ci,
                       const double *x, double *y, hipStream_t s);

// Piecewise-linear bases (bem_p1.hip).
struct P1Args {
  const double *v;
  const int32_t *tri;
  int32_t nv, nt;
  const double *geo;
  int64_t ldg;
  int64_t n;
  const int32_t *rows, *cols;
  void *out;  // [n][9] entries
  const double *rule;
  int32_t nq;
  SSArgs ss;
  double kappa;
  unsigned *flags;
};
struct P1GatherArgs {
  int32_t nrv, ncv, ntr, ntc;
  const int32_t *rs_ptr, *rs_tri, *rs_loc;
  const int32_t *cs_ptr, *cs_tri, *cs_loc;
  int64_t rs_len, cs_len;
  const void *local;
  void *out;
  unsigned *flags;
};
hipError_t launch_p1_pairs(int kernel, int layer, const P1Args &a, hipStream_t s);
hipError_t launch_p1_gather(bool cplx, const P1GatherArgs &a, hipStream_t s);

// ----------------------------------------------------------- learned form
constexpr int kSelQ = 6;  // selector outputs: predicted log10 error at orders 1 .. 6

// Training samples of the order selector (inputs and targets of pairs).
struct SampleArgs {
  const int32_t *tri;
  int32_t nt;
  const double *geo;
  int64_t ldg;
  int64_t n;
  const int32_t *rows, *cols;
  float *x, *t;                   // [n][8], [n][kSelQ]
  const double *rule[kSelQ + 1];  // Duffy rules of orders 1 .. kSelQ, then the reference order
  int32_t nq[kSelQ + 1];
  double kappa;
  unsigned *flags;
};

// Order selection over the entries of near-field blocks.
struct SelectArgs {
  const int32_t *tri;
  int32_t nt;
  const double *geo;
  int64_t ldg;
  int32_t nblocks;
  const int32_t *row_ptr, *row_idx, *col_ptr, *col_idx;
  int64_t row_len, col_len;
  const int64_t *out_off;
  int8_t *orders;
  int64_t out_len;
  const void *net;                 // packed network (launch_pack_net)
  const double *tin_c, *tin_n;     // per-triangle inputs [3][ldt] (launch_tri_inputs)
  const float *tin_f;              // d, area, aspect [3][ldt]
  int64_t ldt;
  const float *range;              // device [16]: training minima, maxima of the inputs (or null)
  int32_t layer, q_plain, q_min;
  int32_t group;                   // rows of a column that share one decision (1 .. 8)
  float margin, log_tol;
  double kappa;
  unsigned *flags;
};

// Per-entry orders of the learned near-field kernel: Duffy rules of orders
// 2 .. q_max (index = order) and the order map (one byte per output entry).
struct OrderRules {
  const double *rule[BEM_MAX_ORDER + 1];
  int32_t nq[BEM_MAX_ORDER + 1];
  const int8_t *orders;
  int32_t q_max;
};

int mlp_params(int n_out);
size_t mlp_grad_scratch_floats(int n_out, int64_t n);
hipError_t launch_mlp_grad(int n_out, const float *P, int64_t n, const float *x, const float *t,
                           float *part, float *lpart, float *grad, float *loss, hipStream_t s);
hipError_t launch_mlp_adam(int64_t np, float *p, const float *g, float *m, float *v, float lr,
                           float b1, float b2, float eps, float c1, float c2, hipStream_t s);
// packed FP16 network for the matrix-core kernels (mlp_packed_bytes bytes)
size_t mlp_packed_bytes();
hipError_t launch_pack_net(int n_out, const float *P, void *packed, hipStream_t s);
hipError_t launch_tri_inputs(const double *geo, int64_t ldg, int nt, double *tc, double *tn,
                             float *tf, int64_t ldt, hipStream_t s);
hipError_t launch_mlp_forward(bool f16, int n_out, const float *P, const void *packed, int64_t n,
                              const float *x, float *y, hipStream_t s);
hipError_t launch_selector_samples(int kernel, int layer, const SampleArgs &a, hipStream_t s);
hipError_t launch_select_orders(const SelectArgs &a, int grid, hipStream_t s);
// x-points per register chunk of the learned kernel for order q
int learned_chunk(int q, int kernel);
hipError_t launch_blocks_learned(int kernel, int layer, const BlockArgs &a, const OrderRules &o,
                                 size_t lds_bytes, hipStream_t s);

// xc: x-points per register chunk (4, 5, 7, 8 or 9; nq_pad of every batch
// entry is nq rounded up to a multiple of it); the layer of each entry is in
// PersistentArgs::mode, its sub-tile shape in its BlockArgs
hipError_t launch_persistent(int kernel, bool mixed, int xc, const PersistentArgs &p,
                             size_t lds_bytes, hipStream_t s);
hipError_t launch_reset_counter(int32_t *counter, hipStream_t s);

hipError_t launch_green(int kernel, int side, const GreenArgs &a, int grid_y, hipStream_t s);
hipError_t launch_contract(bool cplx, const ContractArgs &a, int grid_y, hipStream_t s);
hipError_t launch_pivot_inverse(bool cplx, const PivInvArgs &a, hipStream_t s);

// launchers (bem_kernels.hip); return a hipError_t
// device address of the fixed geometry scratch of the allocation-free entry
// point on `device` (which must be current)
hipError_t noalloc_scratch(int device, double **ptr);
hipError_t launch_geometry(const bem_mesh &m, double *geo, int64_t ldg, unsigned *flags,
                           hipStream_t s);
hipError_t launch_blocks(int kernel, int layer, bool coupling, bool mixed, const BlockArgs &a,
                         size_t lds_bytes, hipStream_t s);
// near field of the single and the double layer in one pass (a.out: single
// layer, a.out2: double layer; plain FP64 or the mixed form)
hipError_t launch_blocks_both(int kernel, bool mixed, const BlockArgs &a, size_t lds_bytes,
                              hipStream_t s);
hipError_t launch_entries(int kernel, int layer, bool mixed, const EntryArgs &a, hipStream_t s);
// sub-tile shape (rows, columns) and LDS bytes of the block kernel for a
// padded rule size within an LDS budget; false if nothing fits
bool block_tile_shape(int nq_pad, bool mixed, size_t lds_budget, int *tr, int *tc,
                      size_t *lds_bytes, bool coupling = false, bool both = false);
size_t block_lds_bytes(int nq_pad, int tr, int tc, bool mixed, bool lists = true,
                       bool both = false);
int rule_chunk(int nq, int kernel);  // x-points per register chunk

}  // namespace bem

struct bem_ctx;

namespace bem {

struct DeviceGuard {  // make the context's device current, restore on exit
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

// shared argument checks and context helpers (bem_capi.cpp); they set the
// context's error text and return a BEM_ code
int fail(bem_ctx *ctx, int code, const std::string &msg);
int hip_fail(bem_ctx *ctx, hipError_t e, const char *where);
// hipMalloc of the library's buffers; fails when BEM_FAULT_INJECT=alloc
hipError_t dev_malloc(void **p, size_t bytes);
int check_op(bem_ctx *ctx, const bem_op *op);
int check_mesh(bem_ctx *ctx, const bem_mesh *m);
int check_blocks(bem_ctx *ctx, const bem_blocks *b, const void *out, int64_t out_len);
int get_rules(bem_ctx *ctx, const bem_op *op, const DevRules **out);
// geometry scratch of the context for nt triangles; leading dimension out
int ensure_geo(bem_ctx *ctx, int32_t nt, int64_t *ldg);
// release the device resources of the context's live plans and detach them
// (bem_plan.cpp; called by bem_destroy)
void detach_plans(bem_ctx *ctx);

}  // namespace bem

struct bem_ctx {
  int device = 0;
  size_t lds_budget = 64 * 1024;  // LDS bytes one workgroup may use
  std::string err;
  unsigned *flags = nullptr;      // device, 1 word
  double *geo = nullptr;          // device scratch
  double *noalloc_geo = nullptr;  // fixed geometry array of the allocation-free entry point
  double *dot_part = nullptr;     // device: partial sums of bem_vec_dot
  size_t geo_cap = 0;             // doubles
  float *mlp_scratch = nullptr;   // device: per-workgroup gradient partial sums
  size_t mlp_cap = 0;             // floats
  void *sel_scratch = nullptr;    // device: packed network + per-triangle selector inputs
  size_t sel_cap = 0;             // bytes
  std::map<std::tuple<int, int, int>, bem::DevRules> rules;
  std::set<bem_plan *> plans;     // live batched plans (released with the context)
};
