/*
 * pprviz.h - C ABI of the MI355X (gfx950) PPR -> DPPR -> PDist -> stress
 * layout library.
 *
 * Paper: "Effective and Efficient PageRank-based Positioning for Graph
 * Visualization" (arXiv 2112.14944).  Each entry point names the passage that
 * defines what it computes.
 *
 * Conventions for every call
 *  - Every array argument is a DEVICE pointer owned by the caller, unless the
 *    argument is documented as a host pointer.  The library never allocates or
 *    frees device memory: scratch space comes from a caller-provided workspace
 *    whose size is given by the matching *_workspace() query.
 *  - Matrices are dense, row-major, FP32, with the leading dimension equal to
 *    their column count unless stated otherwise.
 *  - `stream` is a hipStream_t (NULL = the default stream).  Work is enqueued
 *    asynchronously in stream order.  Argument validation happens on the host
 *    before anything is enqueued; a call that returns an error enqueues nothing.
 *  - Graphs are undirected: the CSR holds both arcs u->v and v->u of every
 *    edge, each arc carries the weight of its edge (weights must be finite and
 *    > 0), row_ptr/col_idx are int32, there are no self-loops or duplicate
 *    arcs.  A node without arcs behaves as if it had a self-loop, so each walk
 *    step stays stochastic (the paper leaves dangling nodes open; this only
 *    affects pi(v, v) of an isolated v).
 *  - The walk's restart probability alpha must lie in (0, 1).
 *  - No C++ exception crosses this boundary.  Thread safety: calls that share
 *    no output or workspace buffers may run concurrently; the library keeps no
 *    mutable global state.
 */
#ifndef PPRVIZ_H
#define PPRVIZ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PPR_OK = 0,
    PPR_EINVAL = -1,      /* bad size, NULL pointer, alpha outside (0,1), ... */
    PPR_ENOCONV = -2,     /* max_iter reached before the residual tolerance; outputs are still written */
    PPR_EWORKSPACE = -3,  /* workspace NULL or smaller than the *_workspace() query */
    PPR_EHIP = -4,        /* a HIP runtime call failed (including an earlier asynchronous error) */
    PPR_ENONFINITE = -5,  /* a checked result was NaN or Inf (e.g. from non-finite weights) */
    PPR_EUNSUPPORTED = -6 /* the size exceeds what this build handles (see each call) */
} ppr_status;

/* Undirected graph in symmetric CSR form (see conventions above). */
typedef struct {
    int32_t n;               /* node count, >= 1 */
    int64_t nnz;             /* arc count = 2 x edge count, < 2^31 */
    const int32_t* row_ptr;  /* device int32[n+1], row_ptr[0] = 0, row_ptr[n] = nnz */
    const int32_t* col_idx;  /* device int32[nnz], arcs of node v at [row_ptr[v], row_ptr[v+1]) */
    const float* weight;     /* device float[nnz] arc weights, or NULL for unit weights */
} ppr_csr;

/* Library version string (static storage). */
const char* pprviz_version(void);

/* Human-readable text for a status code (static storage). */
const char* pprviz_status_string(int status);

/*
 * Number of pushes T the power iteration performs for a given L1 residual
 * tolerance (host-only, no GPU work).
 *
 * Section 3.3 computes near-exact PPR by power iteration until the error is
 * small; the paper's push (Section 3.3, Eq. eq:fwd-invariant) moves alpha of
 * every residue into the estimate and spreads the rest over out-neighbours,
 * so with a stochastic walk the residue's L1 norm after t synchronous pushes
 * is exactly (1-alpha)^t and bounds the L1 error of each PPR row.  T is the
 * smallest t with (1-alpha)^t <= tol, capped at max_iter; tol <= 0 means
 * T = max_iter.  *converged is set to 1 when the cap was not needed.
 * Returns PPR_EINVAL for alpha outside (0,1), max_iter < 0 or NULL outputs.
 */
ppr_status pprviz_pushes_for_tolerance(float alpha, double tol, int32_t max_iter,
                                       int32_t* pushes, int32_t* converged);

/* ------------------------------------------------------------------------
 * Multi-source personalized PageRank (Section 3.1) and DPPR (Definition
 * def:pprdist), by synchronous push / power iteration (Section 3.3).
 * ---------------------------------------------------------------------- */

/* Workspace bytes needed by ppr_matrix for this graph and source count. */
size_t ppr_matrix_workspace(const ppr_csr* g, int32_t n_src, int32_t n_tgt);

/*
 * pi_hat(s, t) after T pushes from every source s in src[0..n_src), for the
 * targets t in tgt[0..n_tgt) (tgt == NULL: all nodes, n_tgt must equal n).
 *
 *  ppr_out   float[n_src * n_tgt] or NULL: ppr_out[i*n_tgt + j] = pi_hat(src[i], tgt[j])
 *  dppr_out  float[n_src * n_tgt] or NULL: d(src[i]) * pi_hat(src[i], tgt[j]),
 *            the degree-normalized PPR of Definition def:pprdist, d = weighted
 *            out-degree (sum of the node's arc weights).
 *  T is chosen by pprviz_pushes_for_tolerance(alpha, tol_l1, max_iter).
 *  resid_out HOST double[n_src] or NULL.  When non-NULL the call synchronizes
 *            `stream` and returns, per source, the FP64 L1 norm of the remaining
 *            residue, 1 - sum over ALL nodes v of pi_hat(src[i], v), computed
 *            in FP64 from the FP32 estimates; a non-finite value makes the call
 *            return PPR_ENONFINITE.  When NULL nothing is synchronized.
 *  iters_out HOST int32 or NULL: receives T.
 * Sources must be distinct valid node ids.  Precision: FP32 arithmetic,
 * FP64 for the residual check.  Returns PPR_ENOCONV (outputs still written)
 * when max_iter capped T before the tolerance was met.
 * Kernel by size: n <= 2304 keeps a tile of sources in LDS; n <= 40831 keeps
 * 4, 2 or 1 source columns of every node in LDS (these two never move the
 * iterate through HBM); larger n streams the iterate through HBM.  On the
 * first two paths a row that lists more than n arcs (repeated neighbours) can
 * exceed the workspace bound of the padded arc copy: the outputs and the
 * residual are then NaN (PPR_ENONFINITE when resid_out is asked for).
 */
ppr_status ppr_matrix(const ppr_csr* g, const int32_t* src, int32_t n_src,
                      const int32_t* tgt, int32_t n_tgt, float alpha, double tol_l1,
                      int32_t max_iter, float* ppr_out, float* dppr_out,
                      double* resid_out, int32_t* iters_out,
                      void* ws, size_t ws_bytes, void* stream);

/*
 * ppr_matrix for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same computation, kernels and results as ppr_matrix, with the workspace
 * taken from a fixed scratch array inside the library instead of a caller
 * buffer.  Inputs and outputs are still the caller's.  The call allocates
 * nothing (no hipMalloc/hipFree, no allocating library routine).
 *
 * Limit: the workspace ppr_matrix_workspace(g, n_src, n_tgt) would ask for
 * must fit ppr_matrix_noalloc_max_scratch() bytes (8 MiB), else the call
 * returns PPR_EUNSUPPORTED before any launch.  That covers, for example, the
 * LDS-resident path (n <= 2304) up to about 1 million arcs unweighted.
 *
 * The scratch is one array per GPU, held from the first call on that GPU
 * until the process ends (its device address is looked up once per device).
 * Every call on one GPU uses the same array and leaves it holding that call's
 * intermediates: calls that overlap on one GPU (on different streams, or
 * from different host threads without ordering) race and give undefined
 * results.  Calls on one stream are ordered and safe.
 */
size_t ppr_matrix_noalloc_max_scratch(void);
ppr_status ppr_matrix_noalloc(const ppr_csr* g, const int32_t* src, int32_t n_src,
                              const int32_t* tgt, int32_t n_tgt, float alpha, double tol_l1,
                              int32_t max_iter, float* ppr_out, float* dppr_out,
                              double* resid_out, int32_t* iters_out, void* stream);

/* ------------------------------------------------------------------------
 * Level-l DPPR by Group Forward-Push (Section 3.2 Definition def:spprdeg;
 * Section 4.2 Algorithm alg:fwdpushsn, Eq. eq:rmax)
 * ---------------------------------------------------------------------- */

/* Workspace bytes needed by gfp_level_dppr, gbp_level_dppr and
 * tau_push_level_dppr for k supernodes. */
size_t gfp_workspace(const ppr_csr* g, int32_t k, int32_t max_rounds);

/*
 * Approximate level-l DPPR between the k children V_0 .. V_{k-1} of a
 * supernode, from all k source supernodes at once.
 *
 * Supernode V_i is its leaf set F(V_i) = leaf_idx[leaf_ptr[i] .. leaf_ptr[i+1]):
 *  leaf_ptr  device int32[k+1], leaf_ptr[0] = 0, leaf_ptr[k] = n_leaves, each
 *            set holding 1 .. n entries;
 *  leaf_idx  device int32[n_leaves], node ids in [0, n).  The sets need not
 *            cover the graph; a node listed twice counts twice.
 * The leaf lists are checked on the device before any other work (this
 * synchronizes `stream`); invalid lists give PPR_EINVAL with no output
 * written.
 *
 * Residue r_i(v) starts at d(v) / |F(V_i)| on the leaves of V_i.  The pushes
 * of Algorithm alg:fwdpushsn run in synchronous rounds: in each round every
 * (source i, node v) pair with r_i(v) > d(v) * r_max adds alpha * r_i(v) to
 * its estimate e_i(v), sends (1 - alpha) r_i(v) w_vu / d(v) to each
 * neighbour u (received in the next round) and keeps 0.  The rounds stop
 * after the first round in which no pair pushed, or after max_rounds rounds
 * (then what the last round sent is delivered to the residues and the call
 * returns PPR_ENOCONV with every output written).  r_max = 0 pushes every
 * nonzero residue each round: max_rounds rounds are then the power series
 * truncated at max_rounds terms.  The paper's threshold is
 * r_max = eps * delta / (m * tau), tau = 1 / sqrt(k n) (Eq. eq:rmax).
 *
 *  dppr_out  float[k * k]: dppr_out[i*k + j] = sum over v in F(V_j) of
 *            e_i(v) / |F(V_j)|, the estimate of pi_d(V_i, V_j).  The FP32
 *            estimates are summed in FP64.
 *  est_out   float[k * n] or NULL: e_i(v) at [i*n + v].
 *  resid_out float[k * n] or NULL: r_i(v) at [i*n + v] when the rounds end.
 *            With est_out it satisfies Eq. eq:fwdpushsn-invariant; after a
 *            normal stop every r_i(v) <= d(v) * r_max, and then
 *            0 <= pi_d(V_i, V_j) - dppr_out[i*k+j] <= r_max * (mean degree
 *            of F(V_j)) up to FP32 rounding (Lemma lem:fpsn-correct).
 *  rounds_out HOST int32 or NULL: rounds run (including the last, empty one).
 * The call synchronizes `stream` every few rounds to read the push count.
 * Returns PPR_EINVAL for alpha outside (0,1), r_max < 0 or non-finite,
 * max_rounds < 1, k < 1 or NULL arrays; PPR_EUNSUPPORTED for n >= 2^24.
 */
ppr_status gfp_level_dppr(const ppr_csr* g, const int32_t* leaf_ptr, const int32_t* leaf_idx,
                          int32_t k, int64_t n_leaves, float alpha, double r_max,
                          int32_t max_rounds, float* dppr_out, float* est_out, float* resid_out,
                          int32_t* rounds_out, void* ws, size_t ws_bytes, void* stream);

/*
 * The backward counterpart (Algorithm alg:bwdpushsn), towards the target
 * supernodes targets[0 .. n_targets) (device int32 ids in [0, k), each a
 * column of its own), in the same synchronous rounds.  Residue r_j(v) starts
 * at 1 / |F(V_j)| on the leaves of V_j; a pair with r_j(v) > rb_max[c]
 * (device float[n_targets], the column's threshold, Eq. eq:brmax) adds
 * alpha d(v) r_j(v) to its estimate e_j(v), sends (1 - alpha) r_j(v) w_uv /
 * d(u) to each neighbour u and keeps 0.  Only the target columns of
 * dppr_out are written: dppr_out[i*k + targets[c]] = sum over v in F(V_i) of
 * e_j(v) / |F(V_i)|.  est_out / resid_out (float[n_targets * n] or NULL) give
 * e and r per column.  After a normal stop every residue is at most its
 * threshold and 0 <= pi_d(V_i, V_j) - dppr_out <= rb_max * (mean degree of
 * F(V_i)) up to FP32 rounding (Lemma lem:bpsn-correct).  Leaf lists and
 * targets are checked on the device first (PPR_EINVAL, nothing written).
 * Other conventions as gfp_level_dppr.
 */
ppr_status gbp_level_dppr(const ppr_csr* g, const int32_t* leaf_ptr, const int32_t* leaf_idx,
                          int32_t k, int64_t n_leaves, const int32_t* targets, int32_t n_targets,
                          const float* rb_max, float alpha, int32_t max_rounds, float* dppr_out,
                          float* est_out, float* resid_out, int32_t* rounds_out, void* ws,
                          size_t ws_bytes, void* stream);

/*
 * Tau-Push (Algorithm alg:taupush): tau = 1 / sqrt(k n) (or the given tau
 * when > 0), the forward threshold r_max = eps delta / (m tau) of Eq. eq:rmax
 * with m = nnz, the forward pushes from every source supernode, then for
 * every target V_j whose DNPR tau_j (Eq. eq:dnpr-dnppr; on an undirected
 * graph the mean leaf degree of V_j over m) exceeds tau, the backward pushes
 * with the threshold of Eq. eq:brmax (eps delta over the largest mean leaf
 * degree of the other supernodes) replace column j.  Every off-diagonal
 * estimate is then within eps delta below the level-l DPPR, up to FP32
 * rounding.  n_backward_out (HOST int32 or NULL): targets refined;
 * rounds_out (HOST int32[2] or NULL): forward and backward rounds.
 * Returns PPR_EINVAL for eps or delta not > 0 or not finite, a graph without
 * arcs, or the conditions of gfp_level_dppr.
 */
ppr_status tau_push_level_dppr(const ppr_csr* g, const int32_t* leaf_ptr, const int32_t* leaf_idx,
                               int32_t k, int64_t n_leaves, float alpha, double eps, double delta,
                               double tau, int32_t max_rounds, float* dppr_out,
                               int32_t* n_backward_out, int32_t* rounds_out, void* ws,
                               size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * PDist (Definition def:pprdist, Eq. eq:pprdist)
 * ---------------------------------------------------------------------- */

/*
 * delta[i*k + j] = min(max(1 - ln z, 2), 2 ln n_clamp), z = dppr[i][j] + dppr[j][i],
 * natural logarithm; z <= 0 (an unreachable pair) gives 2 ln n_clamp; the
 * diagonal is written as 0.  dppr is a k x k DPPR block whose rows (sources)
 * and columns (targets) index the same k nodes in the same order.  n_clamp is
 * the node count n of the graph the PPR ran on (the n of Eq. eq:pprdist).
 * delta may not alias dppr.
 */
ppr_status pdist(const float* dppr, int32_t k, int64_t n_clamp, float* delta, void* stream);

/*
 * Gradient of a scalar loss through pdist.  grad_delta holds dLoss/dDelta for
 * each unordered pair, stored symmetric (both [i][j] and [j][i] hold it, as
 * stress_backward writes it).  Writes grad_dppr[i][j] = grad_dppr[j][i] =
 * grad_delta[i][j] * dDelta/dz, with dDelta/dz = -1/z strictly inside the
 * clamp range of Eq. eq:pprdist and 0 on or beyond its kinks; diagonal 0.
 */
ppr_status pdist_backward(const float* dppr, const float* grad_delta, int32_t k,
                          int64_t n_clamp, float* grad_dppr, void* stream);

/* ------------------------------------------------------------------------
 * Stress layout (Section 5, Eq. eq:loss; appendix "Stress Majorization")
 * ---------------------------------------------------------------------- */

/* Workspace bytes for layout_step / stress_eval on k nodes. */
size_t layout_workspace(int32_t k);

/*
 * Stress L(X | Delta) = sum_{i<j} (1 - ||X_i - X_j|| / Delta_ij)^2 of Eq.
 * eq:loss.  delta: symmetric k x k, positive off the diagonal (diagonal
 * ignored).  x: float[k*2] (x, y per node).  stress_out: DEVICE double[1],
 * written asynchronously (FP32 pair terms, FP64 accumulation).
 */
ppr_status stress_eval(const float* delta, int32_t k, const float* x, double* stress_out,
                       void* ws, size_t ws_bytes, void* stream);

/*
 * One Jacobi sweep of the stress-majorization system L^w X = L^Y Y of the
 * appendix, from X = Y = x_in:
 *   x_out_i = sum_{j!=i} w_ij (Y_j + Delta_ij (Y_i - Y_j)/||Y_i - Y_j||) / sum_{j!=i} w_ij,
 *   w_ij = Delta_ij^-2,
 * where a coincident pair (Y_i == Y_j) contributes w_ij Y_j and no direction
 * term (L^Y is zero there).  Same fixed points as the exact update
 * X = (L^w)^-1 L^Y Y; O(k^2) per step, no linear solve.
 * x_out must not alias x_in.  stress_out: DEVICE double[1] or NULL, receives
 * L(x_in | Delta).  One launch per step: the row sweep of this entry point
 * reads Delta[i][:] for each row i, so delta need not be symmetric here.
 */
ppr_status layout_step(const float* delta, int32_t k, const float* x_in, float* x_out,
                       double* stress_out, void* ws, size_t ws_bytes, void* stream);

/* Workspace bytes needed by layout_step_exact. */
size_t layout_exact_workspace(int32_t k);

/*
 * The exact stress-majorization step (the appendix's Guttman transform,
 * eq:pprlayout-leq): x_out = (L^w)^+ L^Y(x_in) x_in, with
 *   L^w_ij = -Delta_ij^-2 and L^Y_ij = -1 / (Delta_ij ||Y_i - Y_j||) for i != j
 *   (0 for a coincident pair), each diagonal the negated row sum.
 * L^w is singular (its rows sum to zero), so the solution taken is the one
 * with zero centroid, the pseudo-inverse's.  It is reached by conjugate
 * gradients on the x and y coordinates side by side, started from the
 * centred x_in, each applying L^w by one pass over Delta (4 k^2 bytes), until
 * ||L^w x - L^Y(x_in) x_in|| <= cg_tol * ||L^Y(x_in) x_in|| for both
 * coordinates or after cg_max_iter iterations (then PPR_ENOCONV, x_out holds
 * the last iterate).  The step never increases the stress of a converged
 * solve (majorization).  Dot products are summed in FP64 in a fixed order;
 * everything else is FP32.
 *  delta     float[k*k], symmetric, positive off the diagonal (read only off it)
 *  x_in      float[k*2]; x_out float[k*2], != x_in
 *  cg_iters_out HOST int32 or NULL: iterations run.
 * The call synchronizes `stream` every few iterations to read the stop flag.
 * Returns PPR_EINVAL for NULL arrays, k < 1, x_in == x_out, cg_tol < 0 or not
 * finite, cg_max_iter < 0.
 */
ppr_status layout_step_exact(const float* delta, int32_t k, const float* x_in, float* x_out,
                             double cg_tol, int32_t cg_max_iter, int32_t* cg_iters_out,
                             void* ws, size_t ws_bytes, void* stream);

/* Workspace bytes needed by layout_metrics. */
size_t layout_metrics_workspace(int32_t k);

/*
 * Aesthetic metrics of a layout (Section 2.1):
 *  nd_out   HOST double or NULL: ND(X) = sum_{i<j} 1 / ||X_i - X_j||^2
 *           (Definition def:node-distri); +inf when two points coincide.
 *  ulcv_out HOST double or NULL: ULCV(X) = l_sigma / l_mu over the edge lengths
 *           of g (Definition def:edge-var), the population standard deviation;
 *           NaN when g has no arc or every edge has length 0.  g->n must be k.
 * x is float[k*2].  Sums are FP64 in a fixed order.  The call synchronizes
 * `stream`.  Returns PPR_EINVAL for NULL x, k < 1, both outputs NULL, or a
 * missing / mismatched g when ulcv_out is asked for.
 */
ppr_status layout_metrics(const float* x, int32_t k, const ppr_csr* g, double* nd_out,
                          double* ulcv_out, void* ws, size_t ws_bytes, void* stream);

/*
 * Gradient of grad_scale * L(X | Delta) (Eq. eq:loss):
 *   grad_x[i]  = grad_scale * sum_{j!=i} 2 w_ij (d_ij - Delta_ij)(X_i - X_j)/d_ij
 *                (= 2 (L^w X - L^X X)_i in the appendix notation; coincident
 *                pairs contribute 0),  float[k*2] or NULL;
 *   grad_delta = grad_scale * dL/dDelta_ij for each unordered pair i != j,
 *                2 (1 - d_ij/Delta_ij) d_ij / Delta_ij^2, stored symmetric,
 *                diagonal 0,  float[k*k] or NULL.
 */
ppr_status stress_backward(const float* delta, int32_t k, const float* x, float grad_scale,
                           float* grad_x, float* grad_delta, void* stream);

/* ------------------------------------------------------------------------
 * Edge-weight gradient through all-pairs PPR (chain rule through Section
 * 3.1's walk and Definition def:pprdist)
 * ---------------------------------------------------------------------- */

/* Workspace bytes for ppr_matrix_backward (recompute = ppr argument NULL). */
size_t ppr_backward_workspace(const ppr_csr* g, int recompute);

/*
 * Given grad_dppr = dLoss/dpi_d for ALL pairs (n x n, rows = sources, as
 * pdist_backward writes it), returns dLoss/dw for every arc of g:
 *   Gb = D grad_dppr                 (pi_d = D pi_hat)
 *   A  = sum_{j<T} ((1-alpha) P^T)^j Gb  (adjoint of pi = alpha (I-(1-alpha)P)^-1,
 *                                      truncated like the T-push forward)
 *   dQ[u][v] = <A[u,:], pi_hat[v,:]>
 *   grad_arc(u->v) = (1-alpha)/d_u (dQ[u][v] - sum_b P_ub dQ[u][b])
 *                    + sum_t grad_dppr[u][t] pi_hat[u][t]
 * Each edge has one weight shared by its two arcs, so grad_arc[e] receives
 * the gradient of the edge behind arc e: g(u->v) + g(v->u) (both arcs of an
 * edge hold the same value).  Requires col_idx sorted within each row.
 * ppr: the n x n all-pairs pi_hat (rows = sources) of the same T, or NULL to
 * recompute it inside the workspace.  grad_arc: float[nnz].
 * Only meaningful for graphs whose arcs each carry their own weight
 * parameter; unit-weight graphs (weight == NULL) are differentiated at w = 1.
 */
ppr_status ppr_matrix_backward(const ppr_csr* g, float alpha, int32_t T, const float* ppr,
                               const float* grad_dppr, float* grad_arc,
                               void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * Batched path: many independent subgraphs (standing in for the supernodes
 * of the multi-level hierarchy, Section 2.2), each taken through all-pairs
 * PPR -> DPPR -> PDist -> stress_iters Jacobi layout steps.
 * ---------------------------------------------------------------------- */

/* Disjoint union of n_graphs unit-weight undirected subgraphs. */
typedef struct {
    int32_t n_graphs;
    int64_t n_nodes;         /* total node count */
    int64_t nnz;             /* total arc count, < 2^31 */
    int32_t max_n;           /* largest subgraph (host-known) */
    int64_t pool_size;       /* sum of n_g^2 = mat_off[n_graphs] (host-known) */
    const int64_t* node_off; /* device int64[n_graphs+1]; graph g owns nodes [node_off[g], node_off[g+1]) */
    const int32_t* row_ptr;  /* device int32[n_nodes+1], global CSR over the union */
    const int32_t* col_idx;  /* device int32[nnz], global node ids (arcs never leave their subgraph) */
    const int64_t* mat_off;  /* device int64[n_graphs+1], prefix sums of n_g^2 (dense pool offsets) */
} ppr_batch;

/* Largest subgraph the batched path accepts (all-pairs PPR kept on chip). */
int32_t pprviz_batch_max_n(void);

/* Workspace bytes for pprviz_batch / pprviz_batch_plan_create. */
size_t pprviz_batch_workspace(const ppr_batch* b);

/*
 * For every subgraph g (n_g nodes, every node a source):
 *   dppr_pool[mat_off[g] + i*n_g + j] = d(i) pi_hat(i, j)   (T pushes, T from tol/max_iter)
 *   delta_pool[mat_off[g] + i*n_g + j] = PDist with n_clamp = n_g
 *   x_out[2*node] = layout after stress_iters Jacobi sweeps from x0
 *   stress_out[g] = L(x_out_g | Delta_g) (DEVICE double[n_graphs], or NULL)
 * dppr_pool, delta_pool: device float[pool_size].  x0, x_out: device
 * float[2*n_nodes], must not alias.  Every subgraph must have n_g in
 * [1, pprviz_batch_max_n()] (else PPR_EUNSUPPORTED).  Enqueues kernels on
 * `stream` without any host synchronization.
 */
ppr_status pprviz_batch(const ppr_batch* b, float alpha, double tol_l1, int32_t max_iter,
                        int32_t stress_iters, const float* x0, float* x_out,
                        float* dppr_pool, float* delta_pool, double* stress_out,
                        void* ws, size_t ws_bytes, void* stream);

/*
 * pprviz_batch, run once with HIP events recorded between its stages on
 * `stream`; synchronizes the stream and writes the elapsed milliseconds of
 * each stage to the HOST array stage_ms[4]: [0] degrees and planning,
 * [1] all-pairs PPR of every subgraph, [2] PDist, [3] the stress_iters
 * layout sweeps plus the final stress pass.  For measurement.
 */
ppr_status pprviz_batch_profile(const ppr_batch* b, float alpha, double tol_l1, int32_t max_iter,
                                int32_t stress_iters, const float* x0, float* x_out,
                                float* dppr_pool, float* delta_pool, double* stress_out,
                                void* ws, size_t ws_bytes, void* stream, double* stage_ms);

/*
 * The same work captured once into a HIP graph, so that it replays as one
 * launch.  The plan records the pointers it was created with; every buffer
 * must stay valid until pprviz_batch_plan_destroy.  Creation enqueues nothing
 * and does not run the work.
 */
typedef struct pprviz_batch_plan pprviz_batch_plan;

ppr_status pprviz_batch_plan_create(const ppr_batch* b, float alpha, double tol_l1,
                                    int32_t max_iter, int32_t stress_iters, const float* x0,
                                    float* x_out, float* dppr_pool, float* delta_pool,
                                    double* stress_out, void* ws, size_t ws_bytes,
                                    void* stream, pprviz_batch_plan** plan);
ppr_status pprviz_batch_plan_launch(pprviz_batch_plan* plan, void* stream);
void pprviz_batch_plan_destroy(pprviz_batch_plan* plan);

/*
 * The exact stress-majorization step of layout_step_exact (the appendix's
 * Guttman transform, eq:pprlayout-leq) for every subgraph of a batch in one
 * launch, one thread block per subgraph with its CG vectors on chip:
 *   x_out_g = (L^w_g)^+ L^Y(x_in_g) x_in_g   for Delta_g = delta_pool[mat_off[g] ..],
 * the k_g x k_g row-major PDist that pprviz_batch writes (positive off the
 * diagonal, read only off it).  Same CG, stopping rule, FP32 arithmetic and
 * fixed-order FP64 dot products as layout_step_exact; each subgraph stops on
 * its own.  No workspace, no host synchronization.
 *  x_in, x_out  device float[2*n_nodes], x_in != x_out (positions at node_off)
 *  iters_out    device int32[n_graphs] or NULL: CG iterations of each subgraph
 *               (-1 for a subgraph of size outside [1, pprviz_batch_max_n()])
 *  converged_out device int32[n_graphs] or NULL: 1 when the subgraph met
 *               cg_tol, 0 when it stopped at cg_max_iter (x_out holds the last
 *               iterate) or was skipped
 * Returns PPR_EINVAL for NULL b / arrays, x_in == x_out, cg_tol < 0 or not
 * finite, cg_max_iter < 0, b->max_n < 1; PPR_EUNSUPPORTED when b->max_n
 * exceeds pprviz_batch_max_n().
 */
ppr_status pprviz_batch_step_exact(const ppr_batch* b, const float* delta_pool, const float* x_in,
                                   float* x_out, double cg_tol, int32_t cg_max_iter, int32_t* iters_out,
                                   int32_t* converged_out, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* PPRVIZ_H */
