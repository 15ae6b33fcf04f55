/*
 * bem.h -- C-ABI of the MI355X Galerkin boundary-element assembly library.
 *
 * The library evaluates Galerkin matrix entries
 *
 *     G_ij = int_{tau_i} phi_i(x) int_{tau_j} k(x, y) psi_j(y) dy dx
 *
 * (Boerm & Christophersen, arXiv 1510.07244, Sec. 2.1, eq. matrix_entry) for
 * piecewise-constant bases on flat triangles (the setting of Sec. 4) and the
 * kernels of Sec. 2.1 (eq. kernels) and Sec. 4:
 *
 *     Laplace   SLP  1 / (4 pi r)          DLP  <x - y, n(y)> / (4 pi r^3)
 *     Helmholtz SLP  e^{i kappa r}/(4 pi r) DLP  e^{i kappa r}(1 - i kappa r)<x - y, n(y)>/(4 pi r^3)
 *
 * with r = |x - y| and n(y) the outward unit normal of tau_j, taken from the
 * vertex order (counter-clockwise seen from outside).  Pairs are classified by
 * their number of common vertices (Sec. 2.2): disjoint pairs use the Duffy
 * transformation and a tensor Gauss rule (or a 7-point rule per triangle);
 * identical, edge- and vertex-adjacent pairs use the Sauter-Schwab rules.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Memory.  Every array argument named "device" is device memory on the
 *   context's GPU, owned by the caller; the library never frees or retains it
 *   after the enqueued work completes.  Host structs (bem_mesh, bem_op,
 *   bem_blocks) are read during the call only.
 * Streams.  `stream` is a hipStream_t (NULL = the null stream).  Calls only
 *   enqueue work and return; completion is observed by synchronising the
 *   stream.  Calls on one context must not run concurrently from several host
 *   threads.
 * Output types.  Laplace plain: double; Helmholtz plain: double[2] (re, im)
 *   interleaved; mixed precision: float / float[2].  Sizes and offsets of
 *   outputs count entries (a complex entry is one entry).
 * Errors.  Every int-returning call returns BEM_OK or a negative code and
 *   never aborts.  Arguments the host can see are checked before anything is
 *   enqueued (BEM_EINVAL, nothing enqueued).  Device-resident indices are
 *   checked inside the kernels before use: an invalid index never causes an
 *   out-of-range access; the affected block or entry is left unwritten and a
 *   sticky device flag is raised, which bem_check() reports (BEM_EINVAL) and
 *   clears.  Non-finite results (a degenerate mesh) raise BEM_ENONFINITE the
 *   same way.  bem_last_error() gives a text for the last failure.
 */
#ifndef BEM_H
#define BEM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* return codes */
#define BEM_OK 0
#define BEM_EINVAL (-1)        /* invalid argument or index */
#define BEM_ENOMEM (-2)        /* device or host allocation failed */
#define BEM_EDEVICE (-3)       /* HIP runtime error (text in bem_last_error) */
#define BEM_EUNSUPPORTED (-4)  /* valid but not supported combination */
#define BEM_ENONFINITE (-5)    /* a computed entry is not finite */

/* bem_op.kernel */
#define BEM_LAPLACE 0
#define BEM_HELMHOLTZ 1
/* bem_op.layer */
#define BEM_SLP 0
#define BEM_DLP 1
/* bem_op.precision */
#define BEM_PLAIN_FP64 0
#define BEM_MIXED 1
/* bem_op.regular_rule */
#define BEM_RULE_DUFFY 0 /* Duffy transformation + q x q Gauss per triangle (Sec. 2.2) */
#define BEM_RULE_TRI7 1  /* seven-point degree-5 rule per triangle */

#define BEM_MAX_ORDER 12 /* largest q_regular / q_singular */

typedef struct bem_ctx bem_ctx;

/* Triangle mesh.  v: device, nv x 3 doubles row-major (x, y, z);
 * tri: device, nt x 3 int32 vertex ids, outward (counter-clockwise seen from
 * outside) and conforming (a shared vertex has one id).  Zero-area triangles
 * and ids outside [0, nv) are rejected (device flag, BEM_EINVAL). */
typedef struct {
    const double *v;
    int32_t nv;
    const int32_t *tri;
    int32_t nt;
} bem_mesh;

/* Operator and quadrature.  q_regular: Gauss points per Duffy coordinate for
 * disjoint pairs (ignored by BEM_RULE_TRI7); q_singular: Gauss points per
 * coordinate of the Sauter-Schwab rules; both in [1, BEM_MAX_ORDER].  kappa:
 * wave number (Helmholtz; kappa = 0 reproduces Laplace).
 * near_singular_ratio: mixed precision only -- a disjoint pair whose bounding
 * boxes are closer than near_singular_ratio * max(diam) is summed in FP64.
 * reserved: must be zero. */
typedef struct {
    int32_t kernel;
    int32_t layer;
    int32_t precision;
    int32_t regular_rule;
    int32_t q_regular;
    int32_t q_singular;
    double kappa;
    double near_singular_ratio;
    int32_t reserved[4];
} bem_op;

/* A list of dense blocks G[rows_b x cols_b].  Block b has the row triangles
 * row_idx[row_ptr[b] .. row_ptr[b+1]) and the column triangles
 * col_idx[col_ptr[b] .. col_ptr[b+1]) (device arrays; row_ptr / col_ptr have
 * n + 1 nondecreasing entries with row_ptr[n] <= row_len, col_ptr[n] <=
 * col_len).  Its entries go to out[out_off[b] + r + nrows_b * c] (column-major,
 * leading dimension nrows_b) with out_off[b] >= 0 and
 * out_off[b] + nrows_b * ncols_b <= out_len.  Blocks must not overlap in out. */
typedef struct {
    int32_t n;
    const int32_t *row_ptr;
    const int32_t *row_idx;
    int64_t row_len;
    const int32_t *col_ptr;
    const int32_t *col_idx;
    int64_t col_len;
    const int64_t *out_off;
} bem_blocks;

/* Create a context on HIP device `device` (tables, scratch, flags). */
int bem_create(bem_ctx **out, int device);
/* Destroy a context (waits for the device; NULL is ignored). */
void bem_destroy(bem_ctx *ctx);
/* Text of the last failure on this context ("" if none). */
const char *bem_last_error(const bem_ctx *ctx);
/* Synchronise `stream`, then report and clear the sticky device flags raised
 * by work enqueued since the last check: BEM_OK, BEM_EINVAL or
 * BEM_ENONFINITE. */
int bem_check(bem_ctx *ctx, void *stream);

/* Near-field assembly (Sec. 2.3-2.4: the inadmissible leaves G|_{t x s} of
 * the block tree, every pair class of Sec. 2.2).  Each block's disjoint pairs
 * use the regular rule, its identical / edge / vertex pairs the Sauter-Schwab
 * rules; every entry is written exactly once, so results are bitwise
 * reproducible.  `out` (device) holds out_len entries of the type given by
 * the operator. */
int bem_assemble_nearfield(bem_ctx *ctx, const bem_mesh *mesh, const bem_op *op,
                           const bem_blocks *blocks, void *out, int64_t out_len,
                           void *stream);

/* Coupling assembly (Sec. 2.3-2.4: G|_{t~ x s~} of admissible blocks on the
 * pivot sets chosen by cross approximation).  Blocks are given like
 * bem_assemble_nearfield, with the pivot triangle lists as rows and columns.
 * Only the regular rule is used: admissible blocks are separated, so every
 * pair must be disjoint; a pair that shares a vertex is left unwritten and
 * raises the device flag (BEM_EINVAL at bem_check). */
int bem_assemble_coupling(bem_ctx *ctx, const bem_mesh *mesh, const bem_op *op,
                          const bem_blocks *pivots, void *out, int64_t out_len,
                          void *stream);

/* Arbitrary entries: out[k] = G(rows[k], cols[k]) for 0 <= k < n, each pair
 * classified and integrated by its rule (Sec. 2.1 eq. matrix_entry, Sec. 2.2).
 * rows, cols: device int32[n]; out: device, n entries. */
int bem_eval_entries(bem_ctx *ctx, const bem_mesh *mesh, const bem_op *op, int64_t n,
                     const int32_t *rows, const int32_t *cols, void *out, void *stream);

/* ---------------------------------------------------------------------
 * Host-side H^2 structure (Sec. 2.3, the first and third construction steps;
 * adaptive, so plain host code).  All pointers are HOST memory, owned by the
 * caller; the calls are synchronous and touch no device.
 * --------------------------------------------------------------------- */

/* Cluster tree by geometric bisection (Sec. 2.3, cluster trees).  A cluster
 * with more than `leaf` triangles is split at the midpoint of the longest
 * side of the bounding box of its triangle centroids ((v0 + v1 + v2) / 3);
 * centroids on the midpoint go to the first son, ties between equally long
 * sides to the lowest axis, and the order inside each son is the order in
 * the father.  Clusters are numbered depth-first, the root is 0.
 * Outputs: perm[nt] (cluster c holds perm[cl_begin[c] .. cl_end[c])),
 * *ncl, cl_begin / cl_end / cl_level [ncl], cl_son [2*ncl] (-1 for leaves),
 * cl_box [6*ncl] = (lo x, y, z, hi x, y, z) of the union of the triangles'
 * vertex boxes (the bounding box B_t).  Array capacities are max_clusters
 * (2 nt - 1 always suffices).  BEM_EINVAL for bad ids, sizes or capacity. */
int bem_cluster_tree(const double *v, int32_t nv, const int32_t *tri, int32_t nt, int32_t leaf,
                     int32_t max_clusters, int32_t *perm, int32_t *ncl, int32_t *cl_begin,
                     int32_t *cl_end, int32_t *cl_son, int32_t *cl_level, double *cl_box);

/* Block tree (Sec. 2.3, block trees and admissibility).  From (root, root),
 * a block (t, s) is an admissible (far-field) leaf when
 *     max(diam B_t, diam B_s) <= eta * dist(B_t, B_s)
 * (Euclidean box diagonal and box-to-box distance), an inadmissible
 * (near-field) leaf when t or s has no sons, and otherwise has the sons
 * sons(t) x sons(s) in the order (t1,s1), (t1,s2), (t2,s1), (t2,s2).  Leaves
 * are listed depth-first as pairs (t, s) in near_ts / far_ts [2*max_blocks].
 * *nnear / *nfar receive the counts even when they exceed max_blocks (then
 * BEM_EINVAL is returned and the lists are truncated). */
int bem_block_tree(int32_t ncl, const int32_t *cl_son, const double *cl_box, double eta,
                   int32_t max_blocks, int32_t *near_ts, int32_t *nnear, int32_t *far_ts,
                   int32_t *nfar);

#ifdef __cplusplus
}
#endif

#endif /* BEM_H */
