// Internal declarations of the MI355X BEM assembly library (not installed).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
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

// Sauter-Schwab rule of one singular class in reference coordinates
// (x^1, x^2, y^1, y^2) with weights (Gauss weight times Jacobian).
struct SSRule {
  std::vector<double> xs, xt, ys, yt, w;
};
enum { CLS_DISJOINT = 0, CLS_VERTEX = 1, CLS_EDGE = 2, CLS_IDENTICAL = 3 };
SSRule ss_rule(int cls, int q);

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
enum : unsigned { FLAG_EINVAL = 1u, FLAG_NONFINITE = 2u };

// Device copies of the quadrature tables of one (rule, q_regular, q_singular).
struct DevRules {
  int nq = 0;         // points per triangle (regular rule)
  double *tri = nullptr;  // [3][nq]: s, t, w
  int np[4] = {0, 0, 0, 0};  // Sauter-Schwab points per class (index = class)
  double *ss[4] = {nullptr, nullptr, nullptr, nullptr};  // [5][np]: xs, xt, ys, yt, w
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
  void *out;
  int64_t out_len;
  const double *rule;  // [3][nq]
  int32_t nq, nq_pad;
  int32_t tr, tc;      // sub-tile rows / columns
  const double *ss[4];
  int32_t ss_np[4];
  double kappa;
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
  const double *ss[4];
  int32_t ss_np[4];
  double kappa;
  unsigned *flags;
};

// launchers (bem_kernels.hip); return a hipError_t
hipError_t launch_geometry(const bem_mesh &m, double *geo, int64_t ldg, unsigned *flags,
                           hipStream_t s);
hipError_t launch_blocks(int kernel, int layer, bool coupling, const BlockArgs &a,
                         hipStream_t s);
hipError_t launch_entries(int kernel, int layer, const EntryArgs &a, hipStream_t s);
// choose the sub-tile shape and LDS bytes for a padded rule size
void block_tile_shape(int nq_pad, int layer, int *tr, int *tc, size_t *lds_bytes);
int rule_chunk(int nq);  // x-points per register chunk for a rule of nq points

}  // namespace bem

struct bem_ctx {
  int device = 0;
  std::string err;
  unsigned *flags = nullptr;      // device, 1 word
  double *geo = nullptr;          // device scratch
  size_t geo_cap = 0;             // doubles
  std::map<std::tuple<int, int, int>, bem::DevRules> rules;
};
