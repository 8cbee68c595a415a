/*
 * tvchain.h -- C ABI of the MI355X (gfx950) batched TV-chain prox and 2D TV
 * (ROF) solver.
 *
 * Method: Kolmogorov, Pock, Rolinek, "Total variation on a tree"
 * (arXiv 1502.07770).  The chain prox is the exact O(n) dynamic program of
 * Sec. 4.1 (Algorithm 2 with quadratic unaries) for eq. (1D-ROF):
 *
 *     x = argmin_x  sum_e w_e |x_{e+1} - x_e|  +  1/2 sum_i (x_i - y_i)^2 ,
 *
 * and the 2D solver is the Lagrangian decomposition of Sec. 5.1 (ROF model,
 * saddle problem eq. (rof-saddle), accelerated primal-dual iteration eq. (pd)
 * with the primal prox on row chains and the dual prox, through the Moreau
 * identity eq. (prox-tv-conj), on column chains).
 *
 * Conventions shared by every entry point:
 *  - Every data pointer is a DEVICE pointer unless marked [host].  The caller
 *    owns all memory; the library never allocates or frees device memory.
 *  - Calls are asynchronous on `stream` (0 = the default stream) unless stated
 *    otherwise, and return a tv_status.  Host-visible argument errors are
 *    reported before any HIP call is made and leave all buffers untouched.
 *  - No exception crosses the ABI.
 *  - Element types: TV_F32 (float) or TV_F64 (double) for y, w, x and all
 *    gradient buffers of one call.
 */
#ifndef TVCHAIN_H
#define TVCHAIN_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    TV_OK = 0,
    TV_ERR_INVALID_ARG = 1,   /* bad sizes, strides, null pointers, w < 0 or NaN      */
    TV_ERR_WORKSPACE = 2,     /* workspace null or smaller than the query says        */
    TV_ERR_NO_DEVICE = 3,     /* no HIP device visible                                 */
    TV_ERR_HIP = 4,           /* a HIP runtime call failed (launch, copy, sync)        */
    TV_ERR_NOT_CONVERGED = 5, /* tv2d: max_iter reached before gap_tol; stats filled   */
    TV_ERR_NONFINITE = 6,     /* tv2d: the duality gap became NaN or infinite          */
    /* range markers, not codes: they make every int a valid value of the type, so
     * an unknown code passed in from C or Python is reported, not undefined */
    TV_STATUS_MIN_ = -2147483647 - 1,
    TV_STATUS_MAX_ = 2147483647
} tv_status;

typedef enum {
    TV_F32 = 0,
    TV_F64 = 1,
    TV_DTYPE_MIN_ = -2147483647 - 1, /* range markers, as for tv_status */
    TV_DTYPE_MAX_ = 2147483647
} tv_dtype;

/* [host] A batch of chains inside one buffer.
 *  Uniform batch (offsets == NULL): chain c, node i is element
 *      c * chain_stride + i * elem_stride,  i in [0, length).
 *  Row chains of a row-major H x W image: num_chains = H, length = W,
 *  elem_stride = 1, chain_stride = W.  Column chains: num_chains = W,
 *  length = H, elem_stride = W, chain_stride = 1.
 *  Uneven batch (offsets != NULL, DEVICE array of num_chains + 1 ascending
 *  int64): chain c is elements offsets[c] .. offsets[c+1]-1 with unit stride;
 *  length is then the maximum chain length (an upper bound is fine), and
 *  elem_stride / chain_stride are ignored.  Empty chains are allowed there.
 *  Edge weights, when given per edge, use the layout of y: the weight of edge
 *  (i, i+1) sits at the slot of node i; the slot of each chain's last node is
 *  never read.  Lengths must be below 2^24 for TV_F32 (slopes are exact
 *  integers in float) and 2^31 otherwise. */
typedef struct {
    int64_t num_chains;
    int64_t length;
    int64_t elem_stride;
    int64_t chain_stride;
    const int64_t *offsets;
} tv_chain_layout;

/* Bytes of device workspace tv_chain_prox needs for this layout and dtype
 * (0 on invalid arguments).  Workspace holds the lambda^-/lambda^+ stream of
 * the forward pass (Sec. 4.1, "Backward pass": 2n numbers per chain), a
 * per-chain overflow flag and the HBM breakpoint deques of the overflow path. */
size_t tv_chain_prox_workspace(const tv_chain_layout *layout, tv_dtype dtype);

/* Batched chain prox, eq. (1D-ROF), exact (Sec. 4.1 dynamic program).
 *  y  : input signal, layout above.
 *  w  : per-edge weights in y's layout, or NULL to use w_scalar for every edge.
 *       Weights must be >= 0 (w = 0 decouples the chain at that edge); a NaN or
 *       negative w_scalar is rejected; per-edge values are not checked.
 *  x  : output in y's layout.  Its address range must not overlap y's or w's
 *       (segments of a chain run in parallel and re-read their input after
 *       neighbouring segments have written their output); an overlap that the
 *       host can see (equal pointers, or intersecting ranges of a uniform
 *       layout) is rejected with TV_ERR_INVALID_ARG.
 *  Breakpoints live in an on-chip deque; a chain whose deque outgrows it is
 *  redone exactly with its deque in the workspace, so results never depend on
 *  the data's breakpoint depth. */
tv_status tv_chain_prox(const tv_chain_layout *layout, tv_dtype dtype, const void *y,
                        const void *w, double w_scalar, void *x,
                        void *workspace, size_t workspace_bytes, hipStream_t stream);

/* The chain prox of tv_chain_prox for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): the same kernels and results (bit for bit, same launch
 * plan), with the workspace taken from a fixed device array of
 * TV_NOALLOC_SCRATCH_BYTES that the library holds on every GPU it runs on
 * until the process ends.  The call allocates and frees nothing.
 *  Arguments as tv_chain_prox, without the workspace.
 *  Returns TV_ERR_WORKSPACE, before any HIP call, if the launch needs more
 *  scratch than that (a layout whose tv_chain_prox_workspace() is at most
 *  TV_NOALLOC_SCRATCH_BYTES always fits; in FP32 the default launch plan
 *  needs about 16 bytes per node, the 8-byte lambda pair of every node plus
 *  the segments' saved deques: some 4 million nodes).
 *  Every call on one GPU uses that GPU's one scratch array: calls that overlap
 *  in time on the same GPU (other streams, other host threads) race and must
 *  be serialised by the caller (one stream is enough).  Nothing in the
 *  scratch needs to start at zero: each launch writes every value it reads.
 *  Asynchronous on `stream`. */
#define TV_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
tv_status tv_chain_prox_noalloc(const tv_chain_layout *layout, tv_dtype dtype, const void *y,
                                const void *w, double w_scalar, void *x, hipStream_t stream);

/* Several uniform batches of chains solved in ONE launch (e.g. the row and
 * the column chains of an image, or chains of different lengths), each as by
 * tv_chain_prox: batch b is layouts[b] (offsets must be NULL) over y[b] with
 * per-edge weights w[b], or with w_scalar[b] if w is NULL, into x[b].
 *  num_batches : 1 .. TV_MAX_CHAIN_BATCHES.
 *  y, w, x, w_scalar : [host] arrays of num_batches entries (y, w, x hold
 *       DEVICE pointers).  Inputs may be shared between batches; no x[b] may
 *       overlap any y, w or other x (checked as in tv_chain_prox).
 * The chains of all batches share one segmentation (the longest length sets
 * it), which gives a launch enough lanes where a single batch would not.
 * Results are bit-identical to separate tv_chain_prox calls. */
#define TV_MAX_CHAIN_BATCHES 8
size_t tv_chain_prox_multi_workspace(int num_batches, const tv_chain_layout *layouts, tv_dtype dtype);
tv_status tv_chain_prox_multi(int num_batches, const tv_chain_layout *layouts, tv_dtype dtype,
                              const void *const *y, const void *const *w, const double *w_scalar,
                              void *const *x, void *workspace, size_t workspace_bytes, hipStream_t stream);

/* [host] What the autotuner chose. */
typedef struct {
    int64_t segment_length; /* nodes per segment (lane) of a chain                 */
    int64_t halo;           /* nodes each segment's run starts before the segment  */
    int ring_slots;         /* breakpoint slots of the on-chip deque (16 .. 128)    */
    int candidates;         /* plans timed                                          */
    double ms;              /* time of one launch with the chosen plan              */
} tv_tuning_result;

/* Autotuner of the chain-prox launch (segmentation and on-chip deque size):
 * times every candidate plan that fits the workspace on this data (one untimed
 * and three timed launches each, HIP events on `stream`) and makes the fastest
 * the plan of every later tv_chain_prox / tv_chain_prox_multi launch with the
 * same total number of chains and (maximum) length, in this process.
 * Arguments as tv_chain_prox_multi; x receives the prox.  Synchronous.  Results
 * never depend on the plan (the segmented solve is exact), only speed does.
 * The workspace queries above already reserve room for every candidate. */
tv_status tv_chain_prox_autotune(int num_batches, const tv_chain_layout *layouts, tv_dtype dtype,
                                 const void *const *y, const void *const *w, const double *w_scalar,
                                 void *const *x, void *workspace, size_t workspace_bytes, hipStream_t stream,
                                 tv_tuning_result *chosen);
/* Forget every plan chosen by the autotuners (chain prox, chain DP and 2D
 * solvers). */
void tv_autotune_clear(void);

/* ---- General quadratic unaries and asymmetric weights (Sec. 4.1 in full) ----
 * The chain problem of Sec. 4.1 with strictly convex quadratic unaries and
 * piecewise-linear pairwise terms (the setting of Sec. 4, first paragraph):
 *
 *     x = argmin_x  sum_i ( a_i x_i^2 / 2 - b_i x_i )  +  sum_e f_e(x_{e+1} - x_e),
 *     f_e(z) = wm_e z  for z < 0,   f_e(z) = wp_e z  for z >= 0,
 *
 * with a_i > 0 and wm_e <= wp_e (f_e convex).  wm = -w, wp = w, a = 1, b = y is
 * eq. (1D-ROF); a_i = c_i, b_i = c_i y_i is a prox with per-node data weights.
 * The DP runs with real-valued slopes Abar_s - Abar_k (Abar = running sum of a,
 * formed once per node in FP64 by a prefix pass): slopes are no longer exact
 * integers, and each is rounded once to the working precision.
 *  layout : as for tv_chain_prox (uniform or CSR offsets); lengths below 2^24
 *           (TV_F32) or 2^31 (TV_F64).
 *  a      : per-node a_i > 0 in the layout, or NULL for a_i = 1.  Values are not
 *           checked: a_i <= 0, or a_i too small to change the FP64 running sum,
 *           gives unspecified (possibly non-finite) output, never an invalid
 *           memory access.
 *  b      : per-node b_i.
 *  wm, wp : per-edge wm_e <= wp_e in the layout (slot of node i = edge (i, i+1);
 *           each chain's last slot is never read).  wm_e > wp_e gives
 *           unspecified output.
 *  x      : output in the layout; must not overlap a, b, wm or wp (rejected with
 *           TV_ERR_INVALID_ARG where the host can see it, as in tv_chain_prox).
 * Workspace holds the FP64 prefix sums (8 bytes per node), the lambda stream and
 * the saved deques; chains whose deque outgrows the on-chip ring are redone
 * exactly with their deque in the workspace.  The segmented solve is
 * bit-identical to a sequential one, for every plan. */
size_t tv_chain_dp_workspace(const tv_chain_layout *layout, tv_dtype dtype);
tv_status tv_chain_dp(const tv_chain_layout *layout, tv_dtype dtype, const void *a, const void *b,
                      const void *wm, const void *wp, void *x,
                      void *workspace, size_t workspace_bytes, hipStream_t stream);
/* Autotuner of tv_chain_dp launches, as tv_chain_prox_autotune: times every
 * candidate plan that fits the workspace on this data, keeps the fastest for
 * later tv_chain_dp calls of the same shape in this process; x receives the
 * solution.  Synchronous. */
tv_status tv_chain_dp_autotune(const tv_chain_layout *layout, tv_dtype dtype, const void *a, const void *b,
                               const void *wm, const void *wp, void *x,
                               void *workspace, size_t workspace_bytes, hipStream_t stream,
                               tv_tuning_result *chosen);

/* ---- TV-l1 chain prox (Sec. 4.2, piecewise-quadratic unaries) ----
 *
 *     x = argmin_x  sum_e w_e |x_{e+1} - x_e| + sum_i (x_i - y_i)^2 / 2 + sum_i c_i |x_i - d_i| ,
 *
 * the chain subproblem of the TV-l1 primal prox eq. (prox-pq) with its
 * quadratic weight normalised to 1 (prox_{tau (w TV + |. - f|)}(xi) is this with
 * y = xi, d = f, c = tau, w = tau w).  Exact: the Sec. 4.2 message passing with
 * the breakpoint multiset of the message derivative (position, slope tag, jump)
 * kept sorted in on-chip memory; chains are cut into segments solved in
 * parallel from a halo, as for tv_chain_prox, and sets that outgrow the
 * on-chip ring are redone with the set in the workspace.  The sets carry
 * rounding drift (their jump remainders are re-derived at every crossing), so
 * segment boundaries accept sets that agree to 3e-5 (FP32) or 1e-12 (FP64) of
 * the data scale: results agree with a sequential solve to that level, not bit
 * for bit.  Slopes are integers, so lengths must be below 2^24 for TV_F32.
 *  y, d  : per-node inputs in the layout (uniform or CSR offsets).
 *  w     : per-edge weights in the layout (slot of node i = edge (i, i+1)), or
 *          NULL to use w_scalar (>= 0, finite, else TV_ERR_INVALID_ARG).
 *  c     : per-node data weights c_i >= 0 in the layout, or NULL to use c_scalar
 *          (>= 0, finite).  Per-node values of w and c are not checked.
 *  x     : output in the layout; must not overlap y, d, w or c (rejected where
 *          the host can see it). */
size_t tv_chain_prox_l1_workspace(const tv_chain_layout *layout, tv_dtype dtype);
tv_status tv_chain_prox_l1(const tv_chain_layout *layout, tv_dtype dtype, const void *y, const void *d,
                           const void *w, double w_scalar, const void *c, double c_scalar, void *x,
                           void *workspace, size_t workspace_bytes, hipStream_t stream);
/* Autotuner of tv_chain_prox_l1 launches, as tv_chain_prox_autotune: times
 * every candidate plan that fits the workspace on this data and keeps the
 * fastest for later calls of the same shape in this process; x receives the
 * prox.  Synchronous. */
tv_status tv_chain_prox_l1_autotune(const tv_chain_layout *layout, tv_dtype dtype, const void *y, const void *d,
                                    const void *w, double w_scalar, const void *c, double c_scalar, void *x,
                                    void *workspace, size_t workspace_bytes, hipStream_t stream,
                                    tv_tuning_result *chosen);

/* ---- Trees (Algorithm 2 on a tree, Sec. 4.2's extension to trees) ----
 *
 *     x = argmin_x  sum_i ( a_i x_i^2 / 2 - b_i x_i + c_i |x_i - d_i| )
 *                 + sum_{i not a root} f_i(x_parent(i) - x_i),
 *     f_i(z) = wm_i z (z < 0), wp_i z (z >= 0),  wm_i <= wp_i,
 *
 * on a batch of trees (a chain is the tree with parent(i) = i + 1).  The
 * message derivative of each node is the sum of its children's clipped
 * messages plus its unary; breakpoint sets are merged in order.  One tree per
 * lane, computed in FP64 whatever the dtype.
 *  offsets : DEVICE int64[num_trees + 1]: tree t is nodes offsets[t] ..
 *            offsets[t+1]-1 of every per-node array.
 *  parent  : DEVICE int64[num_nodes]: global index of each node's parent, -1 at
 *            roots.  Every tree must be numbered in depth-first post-order
 *            (each subtree a contiguous range ending at its root; a range may
 *            hold several trees); otherwise TV_ERR_INVALID_ARG is returned
 *            (detected on the device) and x is unspecified.
 *  a       : a_i > 0 per node, or NULL for 1.   b : b_i per node.
 *  c, d    : c_i >= 0 and d_i per node, or both NULL (no l1 term; d alone may be NULL).
 *  wm, wp  : slopes of the edge from each node to its parent (roots' ignored).
 *  x       : output per node; must not alias an input.
 * Synchronous (it reads the post-order check back). */
size_t tv_tree_dp_workspace(int64_t num_trees, int64_t num_nodes);
tv_status tv_tree_dp(tv_dtype dtype, int64_t num_trees, int64_t num_nodes, const int64_t *offsets,
                     const int64_t *parent, const void *a, const void *b, const void *c, const void *d,
                     const void *wm, const void *wp, void *x, void *workspace, size_t workspace_bytes,
                     hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Non-convex chains, Sec. 3: a batch of chains, each minimising
 *     sum_i f_i(x_i) + sum_e min(w_e |x_{e+1} - x_e|, C_e)
 * with f_i continuous piecewise-linear and the truncated TV of the pairwise
 * terms (Lemma 1, Lemma 2 with Algorithm 1, its reversal and the truncation,
 * and the backward pass through the mappings pi), exactly, one lane per chain.
 *  num_chains    : < 2^31.
 *  chain_offsets : DEVICE int64 [num_chains + 1], node ranges within
 *                  [0, num_nodes] (a range outside it: TV_ERR_INVALID_ARG).
 *  unary_offsets : DEVICE int64 [num_nodes + 1]; node i has t_i = unary_offsets[i+1]
 *                  - unary_offsets[i] >= 1 breakpoints ulam[unary_offsets[i] ..]
 *                  (non-decreasing) and t_i + 1 slopes uslope[unary_offsets[i] + i ..]
 *                  (slope left of the first breakpoint first; s_0 <= 0 <= s_t,
 *                  so that f_i is bounded below).
 *  w, C          : DEVICE [num_nodes], the edge from node i to node i + 1 of the
 *                  same chain (a chain's last entry is unused); w >= 0, C > 0;
 *                  C NULL or +inf: plain TV.
 *  x             : DEVICE [num_nodes] output.
 *  msg_cap       : breakpoints a message may hold (1 .. 2^24).
 *  map_cap       : intervals of the mappings pi kept per chain (1 .. 2^30).
 * FP64 inside; dtype is that of ulam, uslope, w, C and x.  Synchronous.
 * Returns TV_ERR_INVALID_ARG for an invalid unary, w < 0 or C <= 0 (found on
 * the device), TV_ERR_WORKSPACE if the workspace is too small or a message or
 * a chain's mappings outgrew msg_cap / map_cap (x is then incomplete). */
size_t tv_chain_nc_workspace(int64_t num_chains, int64_t num_nodes, int64_t msg_cap, int64_t map_cap);
tv_status tv_chain_nc(tv_dtype dtype, int64_t num_chains, int64_t num_nodes, const int64_t *chain_offsets,
                      const int64_t *unary_offsets, const void *ulam, const void *uslope, const void *w,
                      const void *C, void *x, int64_t msg_cap, int64_t map_cap, void *workspace,
                      size_t workspace_bytes, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Non-convex chains with concave pairwise terms, Sec. 3, Extensions (i): as
 * tv_chain_nc, but the term of the edge from node i to node i + 1 is
 *     f_i(z) = 0 at z = 0, else min over its pieces k on z's side of
 *              alpha_k |z| + C_k,   z = x_{i+1} - x_i,
 * i.e. any piecewise-linear f_i that is non-increasing concave for z < 0 and
 * non-decreasing concave for z > 0 (truncated TV: (w, 0) and (0, C) on both
 * sides; Potts: (0, C) on both sides).  A side without pieces makes f_i
 * infinite there (a hard order constraint).  The pieces are applied one at a
 * time (Prop. 2) by h (x) g = (h^alpha (x) g^alpha)^-alpha, exactly, FP64:
 * msg_cap <= 256 runs a wave per chain with the messages in LDS (<= 128: the
 * smaller variant), larger msg_cap one lane per chain with the messages in
 * the workspace.
 *  num_pieces    : total pieces (entries of piece_alpha, piece_C, piece_side).
 *  chain_offsets, unary_offsets, ulam, uslope : as for tv_chain_nc.
 *  piece_offsets : DEVICE int64 [num_nodes + 1]: node i's edge owns pieces
 *                  [piece_offsets[i], piece_offsets[i+1]) (within
 *                  [0, num_pieces], non-decreasing; a chain's last node's
 *                  pieces are ignored).
 *  piece_alpha, piece_C : DEVICE [num_pieces] (dtype), finite and >= 0.
 *  piece_side    : DEVICE int32 [num_pieces], +1 (z > 0) or -1 (z < 0).
 *  x             : DEVICE [num_nodes] output.
 *  msg_cap, map_cap : as for tv_chain_nc (map_cap per chain).
 * Synchronous.  Errors as tv_chain_nc (invalid pieces: TV_ERR_INVALID_ARG,
 * found on the device). */
size_t tv_chain_nc_concave_workspace(int64_t num_chains, int64_t num_nodes, int64_t num_pieces, int64_t msg_cap,
                                     int64_t map_cap);
tv_status tv_chain_nc_concave(tv_dtype dtype, int64_t num_chains, int64_t num_nodes, int64_t num_pieces,
                              const int64_t *chain_offsets, const int64_t *unary_offsets, const void *ulam,
                              const void *uslope, const int64_t *piece_offsets, const void *piece_alpha,
                              const void *piece_C, const int32_t *piece_side, void *x, int64_t msg_cap,
                              int64_t map_cap, void *workspace, size_t workspace_bytes, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Non-convex trees, Sec. 3: a batch of trees, each minimising
 *     sum_i f_i(x_i) + sum_{i not a root} min(w_i |x_parent(i) - x_i|, C_i)
 * with f_i as for tv_chain_nc; a node's message is its unary plus its
 * children's messages (Lemma 1), min-convolved with its edge (Lemma 2): a
 * wave per tree (messages in LDS) when there are fewer than 1024 trees and
 * msg_cap <= 256, else one lane per tree.
 *  tree_offsets : DEVICE int64 [num_trees + 1] node ranges within [0, num_nodes];
 *                 each tree numbered in depth-first post-order.
 *  parent       : DEVICE int64 [num_nodes], global index of the parent (in the
 *                 same tree, larger index), -1 at roots.  Other numberings
 *                 are detected on the device: TV_ERR_INVALID_ARG.
 *  unary_offsets, ulam, uslope : as for tv_chain_nc.
 *  w, C         : DEVICE [num_nodes], the edge from node i to its parent.
 *  msg_cap      : breakpoints a message may hold; map_cap: intervals of the
 *                 mappings kept per tree; stack_cap: doubles per tree for the
 *                 children's messages waiting for their parent (2t + 1 each).
 * FP64 inside.  Synchronous.  Errors as tv_chain_nc. */
size_t tv_tree_nc_workspace(int64_t num_trees, int64_t num_nodes, int64_t msg_cap, int64_t map_cap,
                            int64_t stack_cap);
tv_status tv_tree_nc(tv_dtype dtype, int64_t num_trees, int64_t num_nodes, const int64_t *tree_offsets,
                     const int64_t *parent, const int64_t *unary_offsets, const void *ulam, const void *uslope,
                     const void *w, const void *C, void *x, int64_t msg_cap, int64_t map_cap, int64_t stack_cap,
                     void *workspace, size_t workspace_bytes, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Concave pairwise terms on trees, Sec. 3 with Extensions (i): the trees of
 * tv_tree_nc with the pairwise terms of tv_chain_nc_concave, z = x_parent(i)
 * - x_i on the edge from node i to its parent (a chain numbered as a tree,
 * parent(i) = i + 1, is the chain case).  A wave per tree when there are
 * fewer than 1024 trees and msg_cap <= 256, else one lane per tree.
 *  tree_offsets, parent : as for tv_tree_nc (post-order, contiguous subtrees).
 *  unary_offsets, ulam, uslope : as for tv_chain_nc.
 *  piece_offsets, piece_alpha, piece_C, piece_side : as for
 *                 tv_chain_nc_concave, node i's pieces being those of the edge
 *                 to its parent (a root's pieces are ignored).
 *  msg_cap, map_cap, stack_cap : as for tv_tree_nc.
 * Synchronous.  Errors as tv_tree_nc. */
size_t tv_tree_nc_concave_workspace(int64_t num_trees, int64_t num_nodes, int64_t num_pieces, int64_t msg_cap,
                                    int64_t map_cap, int64_t stack_cap);
tv_status tv_tree_nc_concave(tv_dtype dtype, int64_t num_trees, int64_t num_nodes, int64_t num_pieces,
                             const int64_t *tree_offsets, const int64_t *parent, const int64_t *unary_offsets,
                             const void *ulam, const void *uslope, const int64_t *piece_offsets,
                             const void *piece_alpha, const void *piece_C, const int32_t *piece_side, void *x,
                             int64_t msg_cap, int64_t map_cap, int64_t stack_cap, void *workspace,
                             size_t workspace_bytes, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Non-convex 2D, Sec. 5.3: on an H x W grid minimise
 *     sum_horizontal min(w_h |x_i - x_j|, C) + sum_vertical min(w_v |x_i - x_j|, C)
 *       + sum_i f_i(x_i),
 * f_i piecewise-linear through cost[i][k] at the levels d0 + k dd (k < D) with
 * slopes -steep / +steep outside, by the Lagrangian splitting into row and
 * column problems and the primal-dual iteration of Sec. 5.3 (tau_k = tau0 / k,
 * sigma_k = 1 / (2 tau_k), theta = 1), each prox an exact tv_chain_nc solve of
 * the rows (columns) with the piecewise-linear interpolant of the quadratic
 * proximity term on the levels.  Starts from each pixel's minimiser of f, y = 0.
 *  cost : DEVICE [H][W][D] (dtype), D >= 2.
 *  w_h  : DEVICE [H][W-1] or NULL (w_h_scalar >= 0); w_v: [H-1][W] or NULL.
 *  C    : truncation (> 0; +inf: plain TV).  iters >= 0 iterations.
 *  x    : DEVICE [H][W] output (x_h after the last iteration).
 *  msg_cap (>= D), map_cap: as for tv_chain_nc (per row or column chain).
 * Synchronous.  Errors as tv_chain_nc; TV_ERR_INVALID_ARG for bad sizes. */
size_t tv2d_nc_workspace(int64_t H, int64_t W, int64_t D, int64_t msg_cap, int64_t map_cap);
tv_status tv2d_nc_solve(tv_dtype dtype, const void *cost, int64_t H, int64_t W, int64_t D, double d0, double dd,
                        double steep, const void *w_h, double w_h_scalar, const void *w_v, double w_v_scalar,
                        double C, double tau0, int iters, void *x, int64_t msg_cap, int64_t map_cap,
                        void *workspace, size_t workspace_bytes, hipStream_t stream);

/* Bytes of device workspace tv_chain_prox_backward needs (may be 0). */
size_t tv_chain_prox_backward_workspace(const tv_chain_layout *layout, tv_dtype dtype);

/* Adjoint of tv_chain_prox for L = <grad_x, x(y, w)>.  x is the output of the
 * forward call.  Runs are maximal blocks of exactly equal consecutive x (the
 * backward clip of Algorithm 2 produces exact copies inside a run):
 *   grad_y_i = mean of grad_x over the run containing i,
 *   dL/dw_e  = s_e (mean_left - mean_right) on a run boundary e, with
 *              s_e = sign(x_{e+1} - x_e), and 0 inside a run.
 *  grad_y : output, y's layout (may be NULL).
 *  grad_w : NULL (skip), or if w_per_edge != 0 an output in y's layout (slot of
 *           each chain's last node set to 0), else an output of num_chains
 *           values holding each chain's sum over its edges (the gradient of a
 *           scalar weight shared by that chain).
 *  At a kink (a degenerate point where a run is about to split) this is the
 *  derivative for the run structure of the given x. */
tv_status tv_chain_prox_backward(const tv_chain_layout *layout, tv_dtype dtype,
                                 const void *x, const void *grad_x, void *grad_y,
                                 void *grad_w, int w_per_edge,
                                 void *workspace, size_t workspace_bytes, hipStream_t stream);

/* [host] Options of the 2D solvers. */
typedef struct {
    int max_iter;        /* iterations to run at most (>= 0)                          */
    int gap_every;       /* evaluate the FP64 duality gap every this many iterations  */
    double gap_tol;      /* stop once (P - D) / (H W) <= gap_tol; <= 0: never stop    */
    double tau0;         /* initial primal step; sigma_0 = 1 / tau0 (tau sigma = 1)    */
    int resume;          /* nonzero: continue from the state held in the workspace    */
    double *gap_history; /* DEVICE, optional: gap after iteration k at [k-1]; entries
                            of iterations without a gap evaluation are left untouched */
    int use_graph;       /* nonzero: capture a chunk of gap_every (<= 64) iterations
                            in a HIP graph once and replay it for every full chunk
                            (same kernels and results; fewer launches from the host) */
    int lookahead;       /* 0: enqueue every iteration up to max_iter at once (the
                            call never waits on the device).  1 .. 64: the host
                            enqueues at most this many chunks of gap_every
                            iterations beyond the last one it has seen finished
                            (waiting on an event when ahead) and stops enqueuing
                            once the device has stopped, so a solve that stops early
                            costs at most this many chunks of launches that return
                            at once; the call then returns when the device is within
                            this many chunks of the end of what it enqueued.
                            Results are the same either way.  A stream being
                            captured into a graph takes 0 only (otherwise
                            TV_ERR_INVALID_ARG).  Ignored by tv2d_l1_solve,
                            which has no stopping test. */
} tv2d_options;

/* [DEVICE] Result of a 2D solve, written by the solve's last kernel on the
 * solve's stream (read it after that stream's work is done). */
typedef struct {
    int iters;        /* total iterations in the state (including resumed ones)       */
    int status;       /* TV_OK, TV_ERR_NOT_CONVERGED or TV_ERR_NONFINITE              */
    double gap_norm;  /* (P - D) / (H W) at the last evaluation                       */
    double primal;    /* P(x) = lambda (TV_h + TV_v)(x) + |x - f|^2 / 2  (FP64)        */
    double dual;      /* D(p) = |f|^2/2 - |f - D_h^T p_h - D_v^T p_v|^2 / 2  (FP64)    */
    double device_ms; /* device time from the first iteration to the stop (or to the
                         last iteration): the solve's time to its tolerance; in a
                         batched solve, to the image's own stop              */
} tv2d_stats;

/* Bytes of device workspace tv2d_solve needs for an H x W image. */
size_t tv2d_workspace(int64_t H, int64_t W, tv_dtype dtype);

/* 2D ROF, min_x lambda (TV_h + TV_v)(x) + |x - f|^2 / 2 on the 4-connected grid,
 * by the Sec. 5.1 decomposition into row chains (TV_h) and column chains
 * (TV_v), accelerated primal-dual (tau_{k+1} = theta_k tau_k,
 * sigma_{k+1} = sigma_k / theta_k, theta_k = 1/sqrt(1 + 2 tau_k), the primal
 * part being 1-strongly convex), x^0 = f, y^0 = 0 unless resuming.
 *  f      : H x W image, row-major with leading dimension ld >= W.
 *  x      : output H x W, leading dimension ld.
 *  The duality gap uses dual edge variables recovered from the two chain
 *  solves, clipped to [-lambda, lambda], so P - D >= 0 always bounds the
 *  suboptimality of x.  Reductions are FP64 whatever dtype is.
 *  ASYNCHRONOUS on `stream` with lookahead 0: every iteration up to max_iter
 *  is enqueued at once and the stopping test runs on the device: after each
 *  gap evaluation (every gap_every iterations) a device flag, once the gap is
 *  at gap_tol or not finite, makes every later kernel of the solve return at
 *  once (each such skipped iteration still costs its launches, a few
 *  microseconds each).  The schedule is generated on the device, so nothing
 *  is copied from the host and the host never waits, except once when
 *  resuming (to read which buffer holds the iterate).  With lookahead > 0 the
 *  host also mirrors the device's stop through a pinned host word (one per
 *  host thread and device, allocated on first use and kept) and stops
 *  enqueuing after it: see tv2d_options.lookahead (outside 0 .. 64:
 *  TV_ERR_INVALID_ARG).  `stats` is DEVICE memory (or NULL), written by the
 *  solve's last kernel; stats->status is TV_OK, TV_ERR_NOT_CONVERGED (gap_tol
 *  > 0 not reached) or TV_ERR_NONFINITE.
 *  Returns TV_OK once the solve is enqueued, or an argument / launch error. */
tv_status tv2d_solve(tv_dtype dtype, const void *f, int64_t H, int64_t W, int64_t ld,
                     double lambda, void *x, const tv2d_options *options, tv2d_stats *stats,
                     void *workspace, size_t workspace_bytes, hipStream_t stream);

/* Autotuner of tv2d_solve's two chain launches (the column and the row step):
 * runs 32 iterations from f in the workspace (the chains' deques deepen as the
 * dual variable builds up), then times every candidate plan of each launch on
 * the next iteration's data that fits the workspace and makes the fastest the plan
 * of every later tv2d_solve of an H x W image in this process.  Overwrites
 * the solver state held in the workspace (run a fresh solve after it, not a
 * resume).  Synchronous.  The solve's results do not depend on the plans. */
tv_status tv2d_autotune(tv_dtype dtype, const void *f, int64_t H, int64_t W, int64_t ld, double lambda,
                        double tau0, void *workspace, size_t workspace_bytes, hipStream_t stream,
                        tv_tuning_result *col, tv_tuning_result *row);

/* Bytes of device workspace tv2d_solve_batched needs. H, W: [host] arrays. */
size_t tv2d_batched_workspace(int num_images, const int64_t *H, const int64_t *W, tv_dtype dtype);

/* Autotuner of tv2d_solve_batched's two chain launches, as tv2d_autotune, for
 * this batch geometry (later batched solves with the same number of rows and
 * columns and the same largest H and W use the chosen plans).  Overwrites the
 * solver state in the workspace.  Synchronous. */
tv_status tv2d_batched_autotune(tv_dtype dtype, int num_images, const int64_t *H, const int64_t *W,
                                const int64_t *pixel_offsets, const double *lambda, const void *f, double tau0,
                                void *workspace, size_t workspace_bytes, hipStream_t stream,
                                tv_tuning_result *col, tv_tuning_result *row);

/* Many independent 2D ROF problems of different sizes in one solve: every
 * image's row chains run in one launch and its column chains in another, each
 * image with its own lambda and its own stopping test.
 *  H, W, pixel_offsets, lambda: [host] arrays of num_images entries; image j
 *  occupies f[pixel_offsets[j] .. + H[j] W[j]) row-major (ld = W[j]), and x
 *  likewise.  stats: DEVICE array of num_images results (or NULL), written by
 *  the solve's last kernel.  An image whose gap reaches gap_tol > 0, or is not
 *  finite, is frozen on the device (its chains and gap terms are skipped from
 *  then on); once every image is frozen the solve stops as tv2d_solve does.
 *  ASYNCHRONOUS on `stream` except for one wait after the chain lists are
 *  uploaded from host memory (before any iteration is enqueued), the waits of
 *  a lookahead > 0 (as for tv2d_solve; the stop comes once every image is
 *  frozen), and, with use_graph, a wait for the replays before returning.
 *  resume must be 0; lookahead outside 0 .. 64 is TV_ERR_INVALID_ARG.
 *  Returns TV_OK once the solve is enqueued, or an argument / launch error;
 *  each image's status is in its stats. */
tv_status tv2d_solve_batched(tv_dtype dtype, int num_images, const int64_t *H, const int64_t *W,
                             const int64_t *pixel_offsets, const double *lambda,
                             const void *f, void *x, const tv2d_options *options,
                             tv2d_stats *stats, void *workspace, size_t workspace_bytes,
                             hipStream_t stream);

/* ---- 2D TV-l1 (Sec. 5.2) ----
 * min_x lambda (TV_h + TV_v)(x) + sum |x - f| on the 4-connected grid, by the
 * same decomposition: the primal-dual iteration eq. (pd) with constant steps
 * tau = options->tau0, sigma = 1 / tau, theta = 1 (the data term is not
 * strongly convex).  Column step: the ROF dual step (Moreau identity,
 * eq. (prox-tv-conj)).  Row step: the primal prox eq. (prox-pq), per row the
 * TV-l1 chain prox (tv_chain_prox_l1) of xi = x - tau y' with d = f, c = tau,
 * w = tau lambda.  x^0 = xbar^0 = f, y^0 = 0.
 *  options : max_iter iterations are run; every gap_every iterations (and after
 *            the last) the FP64 energy P(x) = lambda (TV_h + TV_v)(x) + |x - f|_1
 *            is evaluated, into gap_history[k - 1] if given (DEVICE).  gap_tol
 *            must be <= 0 and resume 0 (no duality gap is formed for TV-l1);
 *            use_graph is ignored.
 *  stats   : DEVICE (or NULL): iters, status (TV_ERR_NONFINITE if the energy is
 *            not finite), primal = P(x) of the returned x, device_ms; dual and
 *            gap_norm are NaN.
 * ASYNCHRONOUS on `stream`; returns TV_OK once the solve is enqueued, or an
 * argument / launch error. */
size_t tv2d_l1_workspace(int64_t H, int64_t W, tv_dtype dtype);
tv_status tv2d_l1_solve(tv_dtype dtype, const void *f, int64_t H, int64_t W, int64_t ld, double lambda, void *x,
                        const tv2d_options *options, tv2d_stats *stats, void *workspace, size_t workspace_bytes,
                        hipStream_t stream);
/* Autotuner of the TV-l1 solver's column and row launches, as tv2d_autotune. */
tv_status tv2d_l1_autotune(tv_dtype dtype, const void *f, int64_t H, int64_t W, int64_t ld, double lambda,
                           double tau0, void *workspace, size_t workspace_bytes, hipStream_t stream,
                           tv_tuning_result *col, tv_tuning_result *row);

/* [host] Process-wide tuning of the chain-prox launches.  Each chain of length
 * n is cut into S segments of L nodes that are solved in parallel and then
 * stitched exactly (the result does not depend on the tuning):
 *   target_lanes: aim for about this many (chain, segment) lanes per launch;
 *   min_segment : never cut segments shorter than this many nodes;
 *   halo        : each segment's dynamic program starts this many nodes early
 *                 so that its breakpoint deque has usually converged to the
 *                 true one by the segment start (boundaries where it has not
 *                 are detected exactly and redone).
 * Defaults: 131072 lanes, 128 nodes, halo 128. */
typedef struct {
    int64_t target_lanes;
    int64_t min_segment;
    int64_t halo;
    int64_t ring_slots;  /* breakpoint slots of the on-chip deque: 16, 32, 64 or 128
                          * (over 32 only where entries are 8 bytes, i.e. the FP32
                          * TV-l2 chain prox and 2D steps; elsewhere it means 32) */
} tv_tuning;

/* Set the tuning (NULL restores the defaults); TV_ERR_INVALID_ARG on values < 1
 * or a ring size other than 16, 32, 64 or 128.
 * Not thread-safe with respect to concurrent prox calls: a workspace sized
 * before a change may be too small after it (TV_ERR_WORKSPACE). */
tv_status tv_set_tuning(const tv_tuning *tuning);
tv_status tv_get_tuning(tv_tuning *tuning);

/* Segment length L the current tuning gives this layout (0 on bad layouts). */
int64_t tv_chain_prox_segment_length(const tv_chain_layout *layout);

/* Static description of a status code. */
const char *tv_status_string(tv_status status);

#ifdef __cplusplus
}
#endif

#endif /* TVCHAIN_H */
