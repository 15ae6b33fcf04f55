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
 *   threads, and work of one context enqueued on different streams must not
 *   overlap in time: calls share the context's scratch (triangle geometry,
 *   packed network, selector inputs, gradient partial sums).
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
/* Fault injection: with the environment variable BEM_FAULT_INJECT=alloc
 * (read at every call) the library's own device allocations fail as on an
 * exhausted device, and the calls that need them return BEM_ENOMEM, so that
 * callers can test their error handling. */

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
#define BEM_NOALLOC_MAX_TRI 32768 /* largest mesh of bem_assemble_nearfield_noalloc */

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
 * out_off[b] + nrows_b * ncols_b <= out_len.  Blocks must not overlap in out.
 * mirror_off (single layers and bem_assemble_nearfield_both only, else
 * NULL): the kernels g(x, y) = g(y, x) give G_ji = G_ij, so block b also
 * fills its transpose G[cols_b x rows_b] at out[mirror_off[b] + c + ncols_b * r]
 * (column-major); mirror_off[b] < 0: no mirror.  Disjoint and vertex-adjacent pairs are written once evaluated
 * (equal up to rounding); an edge-adjacent pair's mirror entry is evaluated
 * as the pair (j, i), the Sauter-Schwab rule for a shared edge not being
 * symmetric.  mirror_off[b] == out_off[b] marks a block on the diagonal of
 * the matrix (square, the same triangle list for rows and columns -- the
 * caller's promise): it is its own mirror, so only its entries with row >=
 * column are evaluated and each is also written to its transposed place.
 * Any other mirror onto the block itself, or one that does not fit in out,
 * raises the device flag and is not written; mirrors must not overlap other
 * outputs.  NULL: no mirrors. */
typedef struct {
    int32_t n;
    const int32_t *row_ptr;
    const int32_t *row_idx;
    int64_t row_len;
    const int32_t *col_ptr;
    const int32_t *col_idx;
    int64_t col_len;
    const int64_t *out_off;
    const int64_t *mirror_off;
} bem_blocks;

/* Create a context on HIP device `device` (tables, scratch, flags). */
int bem_create(bem_ctx **out, int device);
/* Destroy a context (waits for the device; NULL is ignored). */
void bem_destroy(bem_ctx *ctx);
/* Text of the last failure on this context ("" if none). */
const char *bem_last_error(const bem_ctx *ctx);
/* Synchronise `stream`, then report and clear the sticky device flags raised
 * by work enqueued since the last check: BEM_OK, BEM_EINVAL, BEM_ENONFINITE,
 * or BEM_EUNSUPPORTED when a sub-tile of a mirrored single-layer list had
 * more singular pairs than its pair list holds (each edge-adjacent pair is
 * listed twice there: only possible with edges shared by many triangles;
 * that sub-tile is left unwritten -- assemble it without mirror_off, or with
 * bem_assemble_nearfield_both, which lists each pair once). */
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

/* Near-field assembly that allocates nothing, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation).  Arguments, result (bit for bit) and
 * errors as bem_assemble_nearfield; the per-triangle geometry goes to a
 * fixed device array of the library (BEM_NOALLOC_MAX_TRI triangles, about
 * 5 MB, one per GPU, held until the process ends) instead of context
 * scratch, and no device or host memory is allocated by the call.
 * mesh->nt > BEM_NOALLOC_MAX_TRI: BEM_EINVAL.  The quadrature tables of the
 * operator's rule and orders must already exist on the context, built by an
 * earlier call of any entry point with the same regular rule, q_regular and
 * q_singular: otherwise BEM_EINVAL, nothing enqueued.  The array keeps the
 * last call's geometry; each call rewrites what it reads before reading it.
 * Every call on one GPU shares that GPU's array: calls that overlap in time
 * on one GPU (from any context or stream) race and must be serialised by
 * the caller. */
int bem_assemble_nearfield_noalloc(bem_ctx *ctx, const bem_mesh *mesh, const bem_op *op,
                                   const bem_blocks *blocks, void *out, int64_t out_len,
                                   void *stream);

/* Coupling assembly (Sec. 2.3-2.4: G|_{t~ x s~} of admissible blocks on the
 * pivot sets chosen by cross approximation).  Blocks are given like
 * bem_assemble_nearfield, with the pivot triangle lists as rows and columns.
 * Only the regular rule is used: admissible blocks are separated, so every
 * pair must be disjoint; a pair that shares a vertex is left unwritten and
 * raises the device flag (BEM_EINVAL at bem_check).  With pivots->mirror_off
 * (single layers only; BEM_EINVAL for a double layer) each block is also
 * written transposed, so that of an admissible pair (t, s), (s, t) with the
 * same bases one block is evaluated for both (likewise for near-field
 * lists: one of the blocks (t, s), (s, t), t != s). */
int bem_assemble_coupling(bem_ctx *ctx, const bem_mesh *mesh, const bem_op *op,
                          const bem_blocks *pivots, void *out, int64_t out_len,
                          void *stream);

/* Near field of the single and the double layer potential operators V and K
 * in one pass (both enter the Laplace formulation and the Brakhage-Werner
 * formulation of Sec. 4; entries as bem_assemble_nearfield's for
 * op->layer = BEM_SLP and BEM_DLP, up to rounding).  Every point pair's
 * distance, reciprocal root (and for Helmholtz its sine and cosine) serve
 * both kernels.  out_slp, out_dlp: device, out_len entries each, same layout,
 * distinct buffers; op->layer (BEM_SLP or BEM_DLP) is not used; plain FP64 or
 * BEM_MIXED (as bem_assemble_nearfield: regular pairs in FP32, singular and
 * near-singular pairs in FP64, FP32 / complex64 out).  With blocks->mirror_off, block b also
 * fills its transpose at mirror_off[b] in both outputs: the single layer as
 * for bem_assemble_nearfield, the double layer of every transposed pair
 * (j, i) evaluated from the same point pairs as (i, j) (regular pairs) or by
 * its own Sauter-Schwab rule (singular pairs) -- so one of the blocks (t, s),
 * (s, t) gives both layers of both. */
int bem_assemble_nearfield_both(bem_ctx *ctx, const bem_mesh *mesh, const bem_op *op,
                                const bem_blocks *blocks, void *out_slp, void *out_dlp,
                                int64_t out_len, void *stream);

/* Arbitrary entries: out[k] = G(rows[k], cols[k]) for 0 <= k < n, each pair
 * classified and integrated by its rule (Sec. 2.1 eq. matrix_entry, Sec. 2.2).
 * rows, cols: device int32[n]; out: device, n entries. */
int bem_eval_entries(bem_ctx *ctx, const bem_mesh *mesh, const bem_op *op, int64_t n,
                     const int32_t *rows, const int32_t *cols, void *out, void *stream);

/* ---------------------------------------------------------------------
 * Batched assembly in one persistent launch.
 *
 * Sec. 3 assembles a matrix by splitting its blocks into work lists of a
 * bounded size that worker threads dequeue and run on the GPU (Algorithms
 * add_block / assemble_gpu and schedule_tasks).  Here the lists of many
 * block lists, possibly of many meshes and of either layer, become one
 * device queue of work items (whole blocks, or sub-tiles: at most 64 x 64
 * entries, 128 x 96 in plain coupling lists), sorted by decreasing
 * estimated cost; a fixed grid of workgroups pops items from it until it is
 * empty.  The queue, per-mesh geometry and launch are built once by
 * bem_plan_batched and captured in a HIP graph (a counter-reset kernel,
 * the geometry kernels and the persistent kernel); bem_run_batched replays
 * it.  Entries are bitwise equal to those of bem_assemble_nearfield /
 * bem_assemble_coupling when the x-point chunk equals theirs (the default).
 * --------------------------------------------------------------------- */

typedef struct bem_plan bem_plan;

/* bem_batch.layers: the operator a batch entry assembles. */
#define BEM_BATCH_OP_LAYER 0 /* op->layer into out */
#define BEM_BATCH_SLP 1      /* the single layer into out */
#define BEM_BATCH_DLP 2      /* the double layer into out */
#define BEM_BATCH_BOTH 3     /* near-field lists only: both layers in one pass,
                                as bem_assemble_nearfield_both (single layer
                                into out, double layer into out2) */

/* One batch entry: a block list of one mesh and its output(s).  mirror_off
 * is allowed for the single layer and for BEM_BATCH_BOTH. */
typedef struct {
  const bem_mesh *mesh;     /* host struct; its arrays are device memory */
  const bem_blocks *blocks; /* host struct; its arrays are device memory */
  int32_t coupling;         /* 0: near-field blocks, 1: coupling blocks (no
                               common vertices allowed, as bem_assemble_coupling) */
  int32_t layers;           /* BEM_BATCH_OP_LAYER .. BEM_BATCH_BOTH */
  void *out;                /* device, out_len entries of the output type */
  int64_t out_len;
  void *out2;               /* BEM_BATCH_BOTH: device, out_len entries, not
                               out; else NULL */
} bem_batch;

/* Launch configuration of the persistent kernel.  In: a field left 0 is
 * chosen by the library (by timing candidates when autotune = 1, else its
 * default); out: the configuration used. */
typedef struct {
  int32_t grid;      /* workgroups (default 2 per compute unit) */
  int32_t tile_rows; /* sub-tile rows, 1..64, of the lists whose sub-tiles
                        carry pair lists (near-field lists; every list in the
                        mixed form); plain coupling lists take
                        bem_assemble_coupling's sub-tile (default: the
                        per-block kernel's) */
  int32_t tile_cols; /* sub-tile columns, 1..64, of the same lists */
  int32_t x_chunk;   /* regular-rule points per register chunk: 4, 5, 7, 8 or 9
                        (default: the per-block kernel's) */
  int32_t autotune;  /* 1: time the candidates of every field left 0 */
  int32_t granularity; /* work item of the queue: 1 whole blocks (each
                          popped block's sub-tiles in turn, like the
                          per-block kernel), 2 single sub-tiles; 0: the
                          library's choice (1 unless autotuned) */
  int32_t reserved[2];
  double tuned_ms;   /* out: time of one launch of the chosen configuration
                        (0 when nothing was timed) */
} bem_tune;

/* Plan the batched assembly of `nbatch` entries with one operator (kernel,
 * precision, rules; the layer per entry, see bem_batch.layers).
 * The plan keeps the device pointers of every mesh, block list and output
 * and reads their CONTENTS at every run, except the block lists' row_ptr,
 * col_ptr, out_off, row_idx and col_idx and the meshes' tri, which are read
 * once here (synchronously) to build the queue: changing those after
 * planning requires a new plan.  Meshes given by identical descriptors share
 * one geometry buffer.  The plan owns its device memory (geometry, queue,
 * counter) and a HIP graph; autotuning launches the kernel (writing the
 * outputs) on `stream`: every candidate once, then the fastest quarter (at
 * least two) three more times, the best launch of each deciding
 * (successive halving).  `cache_path` (may be NULL) names a text file of
 * tuned configurations, one JSON object per line, keyed by device and
 * workload; a hit skips the timing and a new result is appended.
 * Host-visible errors (ranges, offsets, ids) fail with BEM_EINVAL here. */
int bem_plan_batched(bem_ctx *ctx, const bem_op *op, int32_t nbatch, const bem_batch *batches,
                     bem_tune *tune, const char *cache_path, void *stream, bem_plan **plan);

/* Autotuning alone: the candidate launch configurations of the batch (the
 * fields of *tune left 0, as bem_plan_batched with tune->autotune = 1) are
 * timed by running them on `stream` (the outputs are written), the winner
 * is stored in *tune and appended to the cache file `cache_path` (a later
 * bem_plan_batched with autotune = 1 and the same cache then plans without
 * timing); no plan is kept.  A cache hit returns the cached configuration
 * without timing.  Errors as bem_plan_batched. */
int bem_autotune(bem_ctx *ctx, const bem_op *op, int32_t nbatch, const bem_batch *batches,
                 bem_tune *tune, const char *cache_path, void *stream);

/* Enqueue one replay of the plan's graph on `stream`.  Runs of one plan
 * share its queue counter and geometry: they must not overlap in time
 * (successive runs on one stream are fine).  Device flags are raised on the
 * plan's context as for the per-call entry points (see bem_check). */
int bem_run_batched(bem_plan *plan, void *stream);

/* Work items in the plan's queue (0 for a NULL plan). */
int64_t bem_plan_tiles(const bem_plan *plan);

/* Release a plan (waits for its device work).  NULL is a no-op.  Plans may
 * be destroyed before or after their context: bem_destroy releases the
 * device resources of the context's live plans, which then only accept
 * bem_plan_destroy (bem_run_batched returns BEM_EINVAL). */
void bem_plan_destroy(bem_plan *plan);

/* ---------------------------------------------------------------------
 * Learned order selection.
 *
 * The regular near-field pairs of Sec. 2.2 all take the same Duffy/Gauss
 * order, sized for the closest pairs; farther pairs reach the same accuracy
 * with fewer points (the paper's Sec. 4 varies the order by hand).  A small
 * network -- 8 inputs, three hidden layers of 64 ReLU units, n_out outputs
 * -- trained on pairs this library generates predicts, per pair, the log10
 * error of the rule at orders 1 .. 6 against order 8, and the assembly then
 * takes per entry the smallest order predicted to stay within a tolerance;
 * the plain order is the fallback.
 *
 * Parameter vector (FP32, bem_mlp_params floats): [mu(8), sigma(8),
 * W1(64 x 8), b1(64), W2(64 x 64), b2, W3(64 x 64), b3, W4(n_out x 64),
 * b4(n_out)], every W row-major; the first layer sees (x - mu) / sigma.
 * Inputs of a vertex-disjoint pair (tau_i, tau_j), with centroids c, areas
 * |tau|, longest edges d, unit normals n and D = max(d_i, d_j),
 * r = |c_i - c_j|:
 *   x0 = ln(r / D), x1 = sqrt(3)/4 d_i^2/|tau_i|, x2 = the same for tau_j,
 *   x3 = min(|tau_i|, |tau_j|) / max(..), x4 = kappa D,
 *   x5 = ln max(|n_i - n_j|^2, 1e-12), x6 = 0 (single layer) or 1 (double
 *   layer), x7 = ln max(|<c_i - c_j, n_j>| / r, 1e-8)
 * (differences in FP64, the rest in FP32).
 * Targets for q = 1 .. 6: e_q = log10(max(|G_q - G_8| / max(|G_8|,
 * 1e-3 s), 1e-16)) with s = |tau_i| |tau_j| / (4 pi r) and G_q the entry by
 * the Duffy/Gauss rule of order q.
 * --------------------------------------------------------------------- */

/* Floats in the parameter vector for n_out outputs (1 .. 16); BEM_EINVAL
 * otherwise. */
int bem_mlp_params(int32_t n_out);

/* y[n][n_out] = network(x[n][8]).  fp16 = 0: FP32 on the vector units;
 * fp16 = 1: weights, standardised inputs and activations rounded to FP16,
 * products on the matrix cores with FP32 accumulation.  All device. */
int bem_mlp_forward(bem_ctx *ctx, int32_t n_out, int32_t fp16, const float *params, int64_t n,
                    const float *x, float *y, void *stream);

/* Gradient (FP32) of the mean squared error L = mean over the n samples and
 * n_out outputs of (y - t)^2 with respect to the parameters (zero for mu and
 * sigma), by reverse-mode differentiation, summed over samples in a fixed
 * order (deterministic).  x[n][8], t[n][n_out], grad[bem_mlp_params], loss
 * (one float, may be NULL): device.  Uses context scratch (grown as
 * needed). */
int bem_mlp_grad(bem_ctx *ctx, int32_t n_out, const float *params, int64_t n, const float *x,
                 const float *t, float *grad, float *loss, void *stream);

/* One Adam step (Kingma and Ba): m = b1 m + (1 - b1) g, v = b2 v +
 * (1 - b2) g^2, p -= lr (m / (1 - b1^step)) / (sqrt(v / (1 - b2^step)) + eps).
 * params, grad, m, v: device float[np]; step counts from 1. */
int bem_mlp_adam(bem_ctx *ctx, int64_t np, float *params, const float *grad, float *m, float *v,
                 int32_t step, float lr, float beta1, float beta2, float eps, void *stream);

/* Training samples: inputs x[n][8] and targets t[n][6] of the pairs
 * (rows[k], cols[k]) for the operator's kernel and layer (plain FP64
 * rules; q_singular and the regular rule of op are not used).  Pairs with a
 * common vertex are invalid: flag raised (BEM_EINVAL at bem_check), their
 * row set to NaN. */
int bem_selector_samples(bem_ctx *ctx, const bem_mesh *mesh, const bem_op *op, int64_t n,
                         const int32_t *rows, const int32_t *cols, float *x, float *t,
                         void *stream);

/* Orders of the entries of a block list -- near-field blocks, or the
 * coupling blocks of admissible pairs (pivot lists) -- in the layout of the
 * blocks' output, one int8 per entry: 0 for pairs with a common vertex, else the smallest
 * q in [q_min, q_regular - 1] such that the FP16 network (n_out = 6,
 * params) predicts e_q' + margin <= log10(tol) at every q' in
 * [q, q_regular - 1]; q_regular when q_regular - 1 fails.  The comparison is
 * made in FP32.  range (device float[16], may be NULL): the smallest and
 * largest value of each of the 8 inputs over the training set ([min(8),
 * max(8)]); a pair with an input outside it (or not finite) gets q_regular,
 * the plain rule, whatever the network predicts.  op: Duffy rule, q_regular
 * in [2, 6].  group (1 .. 8): the rows of a block column are taken in runs
 * of `group` (the last run of a sub-tile of 64 rows may be shorter) that
 * share one network evaluation -- on the inputs of the run's pair with the
 * smallest centroid distance over the larger triangle diameter, with the
 * largest row-triangle aspect ratio of the run -- and so one order (pairs
 * with a common vertex still get 0); group = 1 decides entry by entry.  The
 * network runs once per run, so larger groups cost less to select and may
 * pick higher orders for the run's farther pairs. */
int bem_select_orders(bem_ctx *ctx, const bem_mesh *mesh, const bem_op *op,
                      const bem_blocks *blocks, const float *params, const float *range,
                      double tol, double margin, int32_t q_min, int32_t group,
                      int8_t *orders, int64_t orders_len, void *stream);

/* Near-field blocks like bem_assemble_nearfield (plain FP64, Duffy rule,
 * q_regular in [2, 6]), each regular entry with the order orders[entry]
 * (device int8, the output's layout) in [2, q_regular]; an order outside
 * raises the flag and leaves the entry unwritten.  With q_regular
 * everywhere the result equals bem_assemble_nearfield's bit for bit.  A
 * coupling list (pivot lists of admissible blocks, no common vertices) is
 * assembled the same way, entry for entry as bem_assemble_coupling with
 * q_regular; mirror_off is not used (every block is evaluated). */
int bem_assemble_nearfield_learned(bem_ctx *ctx, const bem_mesh *mesh, const bem_op *op,
                                   const bem_blocks *blocks, const int8_t *orders, void *out,
                                   int64_t out_len, void *stream);

/* Save a network and its training state to a file (host I/O, synchronous:
 * waits for `stream`): n_out, the Adam step count `step` (>= 0), the
 * parameter vector (bem_mlp_params(n_out) floats), optionally Adam's moment
 * vectors m and v (both or neither; NULL: not stored) and the training range
 * of the inputs (float[16] as bem_select_orders takes it; NULL: not
 * stored).  All arrays device memory.  Format: the 8 bytes "BEMMLP01",
 * int32 n_out, step, contents (1: moments, 2: range), 0, then the FP32
 * arrays in that order, little endian.  BEM_EINVAL if the file cannot be
 * written. */
int bem_mlp_save(bem_ctx *ctx, const char *path, int32_t n_out, const float *params,
                 const float *m, const float *v, const float *range, int32_t step, void *stream);

/* Load a file written by bem_mlp_save into device arrays (synchronous):
 * params always, m and v (both or neither) and range when not NULL, *step
 * when step is not NULL.  Training continued from the loaded state equals
 * training that was never interrupted, bit for bit.  BEM_EINVAL (nothing
 * written) for a missing or truncated file, another n_out, or contents
 * asked for that the file does not hold. */
int bem_mlp_load(bem_ctx *ctx, const char *path, int32_t n_out, float *params, float *m, float *v,
                 float *range, int32_t *step, void *stream);

/* Inputs of the rank head (the selector network with one output, predicting
 * the rank the cross approximation of Sec. 2.3 reaches for a cluster), eight
 * per cluster, computed on the host: log2 of the triangle count
 * end[c] - begin[c] (at least 1), log10 of the bounding-box diagonal D (at
 * least 1e-300), the box's middle and smallest extent over its largest,
 * height[c] (leaves 0), kappa * D, `side` (0 rows, 1 double-layer columns),
 * log10(eps) of the pivot-search tolerance.  box: host double[n][6] (lower
 * corner, upper corner); begin, end, height: host int32[n]; out: host
 * float[n][8].  BEM_EINVAL for n < 0, NULL arrays (n > 0) or eps <= 0. */
int bem_cluster_features(int32_t n, const double *box, const int32_t *begin, const int32_t *end,
                         const int32_t *height, double kappa, int32_t side, double eps,
                         float *out);

/* ---------------------------------------------------------------------
 * Cluster bases of the Green cross approximation (Sec. 2.3-2.4).
 * --------------------------------------------------------------------- */

/* Green quadrature matrices (Sec. 2.3, eq. green_matrix), one per cluster c.
 * Rows: the triangles row_idx[row_ptr[c] .. row_ptr[c+1]) (the cluster t for
 * a leaf, t^ = union of the sons' pivots for a father); columns: the m Green
 * quadrature points of the cluster, z[c][nu][3] with outward unit normals
 * zn[c][nu][3] and weights zw[c][nu], and delta[c] = diam(B_t).  Entry
 * (r, nu) and (r, m + nu) of the output (column-major, leading dimension
 * n_c, at out + out_off[c]) are
 *     side 0:  sqrt(w) int_tau g(x, z) dx,  sqrt(w) delta int_tau d/dn(z) g(x, z) dx
 *     side 1:  sqrt(w) int_tau d/dn(x) g(x, z) dx,
 *              sqrt(w) delta int_tau d/dn(x) d/dn(z) g(x, z) dx
 * (side 0: the row basis of both operators and the column basis of the
 * single layer; side 1: the column basis of the double layer, whose kernel is
 * d/dn(y) g(x, y)).  Triangle integrals use the Duffy/Gauss rule of order
 * op->q_regular; op->kernel and op->kappa select the kernel.  All arrays are
 * device memory; entry type double (Laplace) or double[2] (Helmholtz);
 * out_off[c] + 2 m n_c <= out_len.  Index errors raise the device flag.
 * max_rows (>= 0) is a hint, the largest n_c, that only sets how many
 * workgroups share one cluster; any value gives the same result. */
int bem_green_matrix(bem_ctx *ctx, const bem_mesh *mesh, const bem_op *op, int32_t side,
                     int32_t ncl, const int32_t *row_ptr, const int32_t *row_idx, int64_t row_len,
                     int32_t m, const double *z, const double *zn, const double *zw,
                     const double *delta, const int64_t *out_off, void *out, int64_t out_len,
                     int32_t max_rows, void *stream);

/* Basis contraction on the FP64 matrix cores (Sec. 2.3, algebraic
 * interpolation): for each matrix c,
 *     V_c = A_c[:, tau_c] * P_c,   P_c = A_c[t~_c, tau_c]^{-1}
 * with A_c the n_c x acols Green matrix at A + a_off[c] (column-major,
 * leading dimension n_c), tau_c = piv_cols[c * max_rank .. + rank[c]) its
 * pivot columns and P_c the rank[c] x rank[c] inverse of its pivot block at
 * pinv + c * max_rank^2 (column-major, leading dimension rank[c]; complex
 * interleaved when is_complex).  V_c (n_c x rank[c], column-major) goes to
 * V + v_off[c].  nrows, rank, piv_cols, pinv, a_off, v_off, A and V are
 * device memory; lengths a_len / v_len count entries.  For a father cluster
 * the result is the transfer matrix V^_t of the nested basis.  max_rows is
 * a launch-shape hint (the largest n_c) like in bem_green_matrix. */
int bem_basis_contract(bem_ctx *ctx, int32_t is_complex, int32_t nmat, const int32_t *nrows,
                       const int32_t *rank, int32_t max_rank, const int32_t *piv_cols,
                       const double *pinv, const void *A, const int64_t *a_off, int32_t acols,
                       int64_t a_len, void *V, const int64_t *v_off, int64_t v_len,
                       int32_t max_rows, void *stream);

/* Inverses of the pivot blocks on the device (Sec. 2.3, algebraic
 * interpolation): for each matrix c, pinv + c * max_rank^2 receives
 * P_c = A_c[t~_c, tau_c]^{-1} (rank[c] x rank[c], column-major, leading
 * dimension rank[c], complex interleaved when is_complex) -- the layout
 * bem_basis_contract reads -- with A_c the n_c x acols Green matrix at
 * A + a_off[c] (column-major, leading dimension n_c), t~_c = piv_rows[c *
 * max_rank .. + rank[c]) its pivot rows (local row numbers) and tau_c =
 * piv_cols[c * max_rank ..] its pivot columns, as bem_aca returns them.
 * Gauss-Jordan elimination in the order of the pivots, without further
 * pivoting: the cross approximation picks each pivot as the largest entry
 * of the residual, so that order is elimination with complete pivoting
 * (pivot lists from elsewhere must have the same property).  max_rank <= 512.  All arrays device memory; index
 * errors raise BEM_EINVAL, a zero or non-finite pivot BEM_ENONFINITE (device
 * flag, see bem_check). */
int bem_pivot_inverse(bem_ctx *ctx, int32_t is_complex, int32_t nmat, const int32_t *nrows,
                      const int32_t *rank, int32_t max_rank, const int32_t *piv_rows,
                      const int32_t *piv_cols, const void *A, const int64_t *a_off,
                      int32_t acols, int64_t a_len, double *pinv, void *stream);

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

/* Green boxes and quadrature points (Sec. 2.3).  For cluster c with bounding
 * box cl_box[6c .. 6c+6) = (lo, hi): delta[c] = diam(B_t) (box diagonal) and
 * omega_t = B_t grown by delta/2 on every side, so that
 * dist(B_t, boundary of omega_t) = delta/2.  Its six faces, in the order
 * (-x, +x, -y, +y, -z, +z), each carry qg x qg tensor Gauss points (first
 * tangential axis = the lower axis index, varying slowest); m = 6 qg^2 points
 * per cluster: z[c][nu][3], outward unit normals zn[c][nu][3], weights
 * zw[c][nu] (Gauss weights times the face area).  Host memory. */
int bem_green_points(int32_t ncl, const double *cl_box, int32_t qg, double *z, double *zn,
                     double *zw, double *delta);

/* Adaptive cross approximation with full pivoting (Sec. 2.3, eq. aca) of
 * nmat matrices, the adaptive part of the method (host, OpenMP over
 * matrices).  Matrix t has nrows[t] rows and ncols columns at A + a_off[t]
 * (entries; column-major, leading dimension nrows[t]; complex interleaved
 * when is_complex).  Each step takes the residual entry of largest modulus
 * (ties: smallest row, then smallest column) as pivot and subtracts its
 * cross; it stops when that modulus is at most eps times the first pivot's
 * or after max_rank steps.  Outputs: rank[t]; the pivot rows (t~, local row
 * numbers) and columns (tau) in piv_rows / piv_cols [t * max_rank ..]; and
 * the inverse of the pivot block A[t~, tau] in pinv + t * max_rank^2 (leading
 * dimension rank[t]); pinv = NULL: pivots only (bem_pivot_inverse forms the
 * inverses on the device).  BEM_ENONFINITE if a pivot block is singular. */
int bem_aca(int32_t nmat, const int64_t *a_off, const int32_t *nrows, int32_t ncols,
            int32_t is_complex, const double *A, double eps, int32_t max_rank, int32_t *rank,
            int32_t *piv_rows, int32_t *piv_cols, double *pinv);

/* ---------------------------------------------------------------------
 * Products with the H^2 matrix and the vector operations of iterative
 * solvers (Sec. 4 solves V alpha = (1/2 I + K) beta by conjugate gradients;
 * the Brakhage-Werner system of the Helmholtz experiment needs a
 * non-symmetric Krylov method).  An H^2 product y = H x (Sec. 2.3-2.4) is
 * a sequence of grouped small products: forward transformation of the
 * column basis (leaves W^_s^T x|_s, fathers W^_s^T over the sons'
 * coefficients), coupling y^_t += S_ts x^_s, backward transformation of
 * the row basis (fathers push V^_t y^_t to the sons' coefficients, leaves
 * to y|_t) and the near field y|_t += G_ts x|_s.
 * --------------------------------------------------------------------- */

/* Grouped, gathered matrix-vector products: for every group g,
 *     y[out_idx[k]] += (sum over blocks b of g of op(A_b) x_b)[k - out_ptr[g]],
 *     k in [out_ptr[g], out_ptr[g+1]),
 * the blocks of g being b in [grp_ptr[g], grp_ptr[g+1]) and
 * x_b = x[in_idx[in_ptr[b] .. in_ptr[b+1])].  op(A) = A (trans = 0; A_b is
 * m_g x n_b) or its plain transpose, not conjugated (trans = 1; A_b is
 * n_b x m_g); A_b starts at A + a_off[b] (entries), column-major with the
 * row count as leading dimension.  m_g, n_b <= 512.  Entries are double
 * (is_complex = 0) or double[2] (is_complex = 1) for A, x and y alike.
 * All arrays device memory; out_len, in_len, a_len, x_len and y_len are the
 * lengths of out_idx, in_idx, A, x and y (entries).  Sums run in a fixed
 * order (reproducible bit for bit).  Groups of one call must not share
 * output indices, and no output index of a call may be an input index of
 * the same call (x and y may be one buffer, read and written at disjoint
 * places, as the levels of a nested basis are).  Index errors raise the
 * device flag (the group or entry is skipped). */
int bem_gemv_grouped(bem_ctx *ctx, int32_t is_complex, int32_t trans, int32_t ngroups,
                     const int32_t *grp_ptr, const int32_t *out_ptr, const int32_t *out_idx,
                     int64_t out_len, int32_t nblocks, const int32_t *in_ptr,
                     const int32_t *in_idx, int64_t in_len, const int64_t *a_off, const void *A,
                     int64_t a_len, const void *x, int64_t x_len, void *y, int64_t y_len,
                     void *stream);

/* out[0] (+ i out[1]) = sum_i c(x_i) y_i with c the complex conjugate when
 * conj = 1 (is_complex = 1), else the identity; x, y device arrays of n
 * entries (double or double[2]); out: device double[2].  Fixed summation
 * order (reproducible). */
int bem_vec_dot(bem_ctx *ctx, int32_t is_complex, int32_t conj, int64_t n, const void *x,
                const void *y, double *out, void *stream);

/* y = alpha x + beta y with alpha = ar + i ai, beta = br + i bi (real
 * vectors use ar and br); x, y device arrays of n entries. */
int bem_vec_axpby(bem_ctx *ctx, int32_t is_complex, int64_t n, double ar, double ai,
                  const void *x, double br, double bi, void *y, void *stream);

/* One step of the conjugate-gradient method (Hestenes-Stiefel; Sec. 4
 * solves the single-layer system by conjugate gradients) with its scalars
 * in device memory, for real vectors of n entries:
 *     alpha = r.r / p.q,  x += alpha p,  r -= alpha q,
 *     r.r' = r.r (new),   p = r + (r.r' / r.r) p,   r.r = r.r',
 * the caller having formed q = A p and p.q (bem_vec_dot into state + 2)
 * before.  state: device double[10]:
 *   [0] r.r   [1] 0 (imaginary part of the dot product)
 *   [2] p.q   [3] 0
 *   [4] new r.r (written here)   [5] 0
 *   [6] stopping threshold on r.r (tol^2 b.b)
 *   [7] 1 while iterating, 0 once r.r <= [6], the iteration limit is
 *       reached or p.q = 0 (then the step leaves x, r and p unchanged)
 *   [8] steps taken   [9] iteration limit
 * Nothing comes back to the host: a caller may enqueue (or capture in a
 * graph) several steps and read [7] and [8] now and then.  x, r, p, q:
 * device double[n]; q is not written.  Uses the context's dot-product
 * scratch (calls on one context must not overlap in time). */
int bem_cg_step(bem_ctx *ctx, int64_t n, double *state, void *x, void *r, void *p,
                const void *q, void *stream);

/* y += c M x with c = cr + i ci and M the Galerkin mass matrix of the
 * piecewise constants, diagonal with M_ii = |tau_i| (the identity term
 * (1/2) I of Sec. 4 in Galerkin form); x, y device arrays of mesh->nt
 * entries (double, or double[2] when is_complex). */
int bem_mass_apply(bem_ctx *ctx, const bem_mesh *mesh, int32_t is_complex, double cr, double ci,
                   const void *x, void *y, void *stream);

/* ---------------------------------------------------------------------
 * Piecewise-linear (P1) bases (Sec. 2.2, eq. reference_integral: the
 * transformed basis functions are low-order polynomials).  The nodal basis
 * function of vertex v is 1 at v, 0 at the other vertices and linear on
 * every triangle; its Galerkin matrix is assembled from 3 x 3 local
 * matrices of triangle pairs.
 * --------------------------------------------------------------------- */

/* Local matrices of the triangle pairs (rows[k], cols[k]), k < n:
 *     out[9 k + 3 a + b] = int_{tau_i} int_{tau_j} lambda_a(x) k(x, y) mu_b(y) dy dx
 * with lambda_a, mu_b the barycentric coordinates of the a-th / b-th vertex
 * of tau_i / tau_j in mesh order, by the rules of the piecewise-constant
 * entries: the regular rule of op (Duffy q x q or seven points per triangle)
 * for disjoint pairs, the Sauter-Schwab rule of order q_singular for
 * identical, edge- and vertex-adjacent pairs (relabelled as for the
 * piecewise-constant entries; the shape functions follow the vertices).
 * Plain FP64 only (BEM_EUNSUPPORTED otherwise).  rows, cols: device
 * int32[n]; out: device, 9 n entries (double or double[2]). */
int bem_p1_pairs(bem_ctx *ctx, const bem_mesh *mesh, const bem_op *op, int64_t n,
                 const int32_t *rows, const int32_t *cols, void *out, void *stream);

/* Dense block of the P1 Galerkin matrix from local matrices: for row
 * vertex v < nrv and column vertex w < ncv,
 *     out[v + nrv w] = sum over p in [rs_ptr[v], rs_ptr[v+1]) and
 *                      q in [cs_ptr[w], cs_ptr[w+1]) of
 *                      local[9 (rs_tri[p] ntc + cs_tri[q]) + 3 rs_loc[p] + cs_loc[q]]
 * -- the triangles around v (indices into a row triangle set of ntr, with
 * v's position 0..2 in each) against those around w (a column set of ntc),
 * local holding the ntr x ntc pairs' matrices (bem_p1_pairs on the pairs
 * (row set [a], column set [b]) in the order a ntc + b).  Every entry is a
 * sum in list order, written once (reproducible bit for bit).  All arrays
 * device memory; rs_len, cs_len: lengths of rs_tri / rs_loc, cs_tri /
 * cs_loc; entries double or double[2] (is_complex). */
int bem_p1_gather(bem_ctx *ctx, int32_t is_complex, int32_t nrv, const int32_t *rs_ptr,
                  const int32_t *rs_tri, const int32_t *rs_loc, int64_t rs_len, int32_t ncv,
                  const int32_t *cs_ptr, const int32_t *cs_tri, const int32_t *cs_loc,
                  int64_t cs_len, int32_t ntr, int32_t ntc, const void *local, void *out,
                  void *stream);

/* ---------------------------------------------------------------------
 * Measurement.
 * --------------------------------------------------------------------- */

/* Vector-ALU peak of the context's GPU: a launch of independent fused
 * multiply-add chains (FP64 when fp64 = 1, else FP32 without packed
 * instructions, the form this library's kernels use), 16 waves per compute
 * unit, best of five timed launches after a warm-up.  *tflops receives
 * 2 x FMAs / time in TFLOP/s.  Synchronous (enqueues on `stream`, then
 * waits for it). */
int bem_valu_peak(bem_ctx *ctx, int32_t fp64, double *tflops, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* BEM_H */
