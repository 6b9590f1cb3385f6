/*
 * hh.h -- C ABI of the MI355X H-matrix mobility library.
 *
 * The library computes the per-time-step hot path of an H-matrix accelerated
 * hydrodynamic-interaction surrogate (arXiv 2505.08174, Sec. 3):
 *
 *     U = M(X) F,   U_i = alpha_1 F_i + sum_{j != i} K(x_i - x_j) F_j      (1)
 *
 * for N spheres at positions X (Eq. (2) restricted to the one-body term and
 * the two-body off-diagonal term, i.e. M^(1) F + M^(t,2) F of Eq. (6)). Every
 * matrix entry is a 3x3 block (Sec. 3, footnote). The dense two-body matrix is
 * replaced by an H-matrix: a geometric cluster tree (Definition 1, Fig. 2), a
 * block partition by the admissibility test Eq. (7) (Algorithm 1), adaptive
 * cross approximation of admissible blocks (Eqs. (8)-(10), Algorithm 2), a
 * dense on-the-fly evaluation of inadmissible leaf blocks, and the low-rank
 * product C (Q F) (Sec. 3).
 *
 * Conventions shared by every entry point
 *  - Arrays named "device" are HIP device pointers owned by the caller and
 *    borrowed for the duration of the enqueued work. Arrays named "host" are
 *    ordinary host memory; calls that read or write host arrays synchronise
 *    the context stream before returning.
 *  - Positions X are FP64, row-major [N][3], in the caller's particle order.
 *    Forces and velocities are row-major [N][3] in the caller's order, with
 *    the element type fixed by the precision (see hh_precision).
 *  - Displacements are r = x_i - x_j (target minus source).
 *  - Every call enqueues on the context's HIP stream. Calls noted "syncs"
 *    also wait for the stream (they read back list sizes to size storage).
 *  - Handles (tree, partition, low-rank factors, kernel) are owned by the
 *    library and released by the matching *_free; freeing NULL is a no-op.
 *    A handle must not outlive the context that made it.
 *  - Errors: every call returns an hh_status; hh_last_error() gives a text
 *    for the last failing call on that context. Nothing throws across the ABI.
 *    On error, output handles are set to NULL and nothing is leaked.
 *  - One context per host thread and stream; contexts are independent.
 */
#ifndef HH_H
#define HH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hh_ctx_s* hh_ctx;
typedef struct hh_tree_s* hh_tree;
typedef struct hh_part_s* hh_part;
typedef struct hh_lowrank_s* hh_lowrank;
typedef struct hh_kernel_s* hh_kernel;
typedef struct hh_batch_s* hh_batch;
typedef struct hh_short_s* hh_short;

typedef enum {
  HH_OK = 0,
  HH_ERR_INVALID_ARG = 1,      /* a size, pointer or parameter is out of range */
  HH_ERR_OUT_OF_MEMORY = 2,    /* device allocation failed */
  HH_ERR_HIP = 3,              /* a HIP runtime call failed */
  HH_ERR_DUPLICATE_POINTS = 4, /* two particles coincide: K is singular at r=0 */
  HH_ERR_CAPACITY = 5,         /* an internal list exceeded its bound */
  HH_ERR_NOT_CONVERGED = 6     /* ACA did not converge and fallback is off */
} hh_status;

/* Arithmetic of the kernel evaluation, factors and sums.
 *   HH_FP64 : F, U, factors and all sums in FP64.
 *   HH_FP32 : F, U, kernel evaluation and factors in FP32; ACA pivots and
 *             stopping norms in FP64 (as in every form).
 *   HH_BF16 : seeded-MLP layers in BF16 on MFMA with FP32 accumulation; ACA
 *             pivot selection and stopping norms in FP64; factors FP32; the
 *             final velocity sum in FP64. F is FP32 and U is FP64. The ACA
 *             samples carry the activations as BF16 hi + lo; the near field
 *             rounds them to BF16 once (about 1e-4 relative per entry).
 *   HH_BF16_SPLIT : as HH_BF16, with hi + lo activations in the near field
 *             too (about 1e-6 per entry, about 1.5x the near-field work). */
typedef enum { HH_FP64 = 0, HH_FP32 = 1, HH_BF16 = 2, HH_BF16_SPLIT = 3 } hh_precision;

/* Input of the seeded MLP kernel: the unit direction r/|r| (default; gives
 * an asymptotically smooth kernel, the premise of the low-rank step at the
 * end of Sec. 3.1) or the raw displacement r. */
typedef enum { HH_MLP_INPUT_DIRECTION = 0, HH_MLP_INPUT_DISPLACEMENT = 1 } hh_mlp_input;

/* Size of the packed MLP parameter vector: W1[64][3] b1[64] W2[64][64] b2[64]
 * W3[64][64] b3[64] W4[9][64] b4[9], each row-major [out][in]. */
#define HH_MLP_NPARAM 9161

/* ---------------------------------------------------------------- context */

/* Create a context on HIP device `device` that enqueues on `stream`
 * (a hipStream_t; NULL = the null stream). The context also owns a second
 * stream (default priority, non-blocking) and two events: the ACA runs its
 * workgroup-team kernel there, forked from `stream` and joined back before
 * any later work on `stream`, so callers only ever order against `stream`.
 * Released by hh_ctx_destroy. */
hh_status hh_ctx_create(int device, void* stream, hh_ctx* out);
void hh_ctx_destroy(hh_ctx ctx);
const char* hh_last_error(hh_ctx ctx);
/* Replace the stream used by later calls. */
hh_status hh_ctx_set_stream(hh_ctx ctx, void* stream);
/* Device memory (bytes) that ACA factors may occupy. When the factors of all
 * admissible blocks would not fit in half of it, hh_aca_build only plans
 * and hh_matvec builds and applies them in batches of blocks whose factors
 * fit (a fixed buffer filled, applied and reused, Sec. 3.3.2). The default is
 * 40% of the free device memory at context creation. */
hh_status hh_ctx_set_budget(hh_ctx ctx, size_t bytes);
/* Work split of hh_aca_build / hh_matvec: admissible blocks with
 * c + q >= team_min (rounded up to a power of two) are approximated by a
 * whole workgroup of 8 waves, smaller ones by a single wave each (results
 * agree to rounding). Default 4096; team_min in [64, 2^30]. */
hh_status hh_ctx_set_team_min(hh_ctx ctx, int32_t team_min);
/* Wait for all work enqueued by this context. */
hh_status hh_synchronize(hh_ctx ctx);

/* ---------------------------------------------------------------- kernels */

/* Rotne-Prager-Yamakawa tensor for spheres of radius a in a fluid of
 * viscosity mu (the dilute two-body mobility the paper cites, Sec. 1); self
 * mobility alpha_1 = 1/(6 pi mu a) I (Eq. (2)). Requires a > 0, mu > 0. */
hh_status hh_kernel_create_rpy(hh_ctx ctx, double a, double mu, hh_kernel* out);

/* Seeded MLP stand-in for the learned two-body term h/|r| of Eq. (4):
 * o = W4 tanh(W3 tanh(W2 tanh(W1 v + b1) + b2) + b3) + b4, O = o as 3x3
 * row-major, K(r) = (O + O^T)/2 / (8 pi |r|), v per `input_mode`.
 * params: host, HH_MLP_NPARAM doubles (layout above); copied. The self
 * mobility is 1/(6 pi mu a). */
hh_status hh_kernel_create_mlp(hh_ctx ctx, const double* params, int input_mode, double a,
                               double mu, hh_kernel* out);
/* The 6N mobility with rotations, [U; w] = M [F; T] of Eq. (1), with the
 * Rotne-Prager blocks for spheres of radius a in a fluid of viscosity mu
 * (r = x_i - x_j, d = |r|, [r]_x u = r x u):
 *   U from F: the RPY tensor of hh_kernel_create_rpy, self 1/(6 pi mu a) I;
 *   w from F and U from T: -[r]_x / (8 pi mu d^3) (the same function of r in
 *                          both places), self 0;
 *   w from T: -(I - 3 r r^T / d^2) / (16 pi mu d^3), self 1/(8 pi mu a^3) I.
 * The rotational blocks are the non-overlapping forms (d >= 2a); the
 * translational block is the full RPY tensor. The paper limits itself to
 * translation and names this extension (end of Sec. 2.2). The kernel works
 * on the 2n rows of a tree from hh_build_tree6 (and only there): each 3x3
 * entry of the 6N matrix is one ACA entry (Algorithm 2 as for 3N), with the
 * |det| pivot magnitude in every precision (the translation-rotation entries
 * are singular). HH_FP64 and HH_FP32 only; no backward. Requires a, mu > 0. */
hh_status hh_kernel_create_rpy6(hh_ctx ctx, double a, double mu, hh_kernel* out);
void hh_kernel_free(hh_kernel k);

/* ----------------------------------------------------------- the hot path */

/* Cluster tree (Definition 1; bisection of boxes along x, y, z, Fig. 2).
 * X: device FP64 [n][3]. c_leaf >= 2: a cluster with fewer than c_leaf
 * particles is a leaf. The root box is the power-of-two cube anchored at the
 * per-axis minimum of X; particles are ordered by 63-bit Morton key of their
 * 21-bit quantised coordinates, ties by input index; nodes are numbered in
 * pre-order. Errors: n < 1, c_leaf < 2, n >= 2^31 or non-finite X ->
 * HH_ERR_INVALID_ARG; two identical positions -> HH_ERR_DUPLICATE_POINTS.
 * Syncs. */
hh_status hh_build_tree(hh_ctx ctx, const double* X, int64_t n, int32_t c_leaf, hh_tree* out);

/* Tree of the 6N mobility: the cluster tree of hh_build_tree on the n
 * particles X (c_leaf counts particles), with every particle's two rows
 * (2i: translation and force, 2i + 1: rotation and torque) next to each other,
 * so the tree has 2n rows, every cluster twice its particles' rows and the
 * same boxes and nodes. hh_partition, hh_aca_build and hh_matvec then work on
 * it with hh_kernel_create_rpy6; hh_matvec takes F as [n][6] = (F_i, T_i)
 * and returns U as [n][6] = (U_i, w_i). hh_tree_info reports 2n rows and
 * hh_tree_export their permutation (row 2p + r of the sorted order is input
 * row 2 perm[p] + r); hh_tree_refit takes the n particle positions. Not for
 * hh_short_create or batched trees. Errors as hh_build_tree with n < 2^30 - 1.
 * Syncs. */
hh_status hh_build_tree6(hh_ctx ctx, const double* X, int64_t n, int32_t c_leaf, hh_tree* out);

/* Many independent systems in one tree (the batched form): X is the
 * concatenation of n_sys systems, offsets (host, n_sys + 1 values, offsets[0]
 * = 0, strictly increasing) delimit them. Each system gets its own root box
 * and its own subtree, identical to hh_build_tree on that system alone (node
 * ids and particle positions shifted by the systems before it); hh_partition
 * then starts Algorithm 1 at (root_s, root_s) for every system, so no block
 * couples two systems, and hh_aca_build / hh_matvec / hh_matvec_backward
 * process all systems' blocks in the same launches. Errors as hh_build_tree,
 * plus an empty system -> HH_ERR_INVALID_ARG. Syncs. */
hh_status hh_build_tree_batch(hh_ctx ctx, const double* X, const int64_t* offsets,
                              int32_t n_sys, int32_t c_leaf, hh_tree* out);
/* As hh_build_tree_batch with a leaf size per system: c_leafs is a host
 * array of n_sys values, each >= 2 (system s is the tree hh_build_tree would
 * build on it with c_leafs[s]). NULL c_leafs -> HH_ERR_INVALID_ARG. Syncs. */
hh_status hh_build_tree_batch_leaf(hh_ctx ctx, const double* X, const int64_t* offsets,
                                   int32_t n_sys, const int32_t* c_leafs, hh_tree* out);

/* New positions for an existing tree, keeping its particle order, nodes and
 * leaves (Definition 1's clusters as index sets) and recomputing the sorted
 * positions and the tight boxes of every node. X: device FP64 [n][3] in the
 * caller's order (for a tree of hh_build_tree6: the n particles, not its 2n
 * rows). The Morton keys are not recomputed, and a partition built
 * on the tree keeps its blocks (Eq. (7) is not re-tested). Used to evaluate
 * the frozen-structure product at perturbed positions (finite differences
 * of hh_matvec_backward) and for time steps that keep the structure.
 * Non-finite X -> HH_ERR_INVALID_ARG. Syncs. */
hh_status hh_tree_refit(hh_ctx ctx, hh_tree tree, const double* X);

/* Block partition (Algorithm 1) with the admissibility test Eq. (7) on tight
 * bounding boxes of the member centres: admissible iff dist^2 > 0 and
 * max(diam_tau^2, diam_sigma^2) <= eta^2 dist^2. eta > 0. dense_mode != 0
 * admits nothing (every leaf pair is dense), which reproduces the dense
 * product. Output lists are sorted by (tau, sigma) node id. Syncs. */
hh_status hh_partition(hh_ctx ctx, hh_tree tree, double eta, int dense_mode, hh_part* out);

/* Adaptive cross approximation (Algorithm 2, Eqs. (8)-(10)) of every
 * admissible block, with 3x3 entries: first column j_1 = floor(q/2), row and
 * column pivots by the largest magnitude of the residual entry (squared
 * Frobenius norm in HH_FP64, |det| in the single-precision forms; ties to
 * the lowest index), c_k normalised by the inverse of its pivot entry, stop
 * when nu^2 <= eps^2 lambda^2 (exact block norms through 3x3 Gram matrices)
 * or when min(c, q) terms interpolate the block. A block that reaches l_max
 * terms without converging is evaluated densely (counted in
 * hh_lowrank_info). eps >= 0, 1 <= l_max <= 64. Syncs.
 * When the factors would not fit half the context budget the handle is in
 * streamed mode: this call only plans, and hh_matvec runs the ACA with the
 * product fused in and keeps no factors (Sec. 3.3.2).
 * freeze_pivots_from (nullable): a stored-mode handle built on the same
 * partition. The recursion of Algorithm 2 is then replayed with its pivots
 * (i_k, j_k), ranks and dense fallbacks instead of searching and testing
 * (eps and l_max are ignored); kern may differ from the one it was built
 * with. Together with hh_tree_refit this evaluates the frozen-structure
 * product at new positions or kernel parameters, the function whose
 * derivatives hh_matvec_backward returns. A pivot entry that is singular at
 * the new positions turns its block into a dense fallback. HH_FP64 and
 * HH_FP32 only; a streamed source -> HH_ERR_INVALID_ARG. */
hh_status hh_aca_build(hh_ctx ctx, hh_tree tree, hh_part part, hh_kernel kern,
                       hh_precision prec, double eps, int32_t l_max,
                       hh_lowrank freeze_pivots_from, hh_lowrank* out);

/* As hh_aca_build with freeze_pivots_from, with the pivots given in host
 * arrays in the layout of hh_lowrank_export: rank[nG], fallback[nG] (0 or 1;
 * a block with 1 is evaluated densely), piv_i[nG][64] and piv_j[nG][64]
 * (local row and column indices, entries past the rank ignored). Blocks are
 * in the partition's order. Ranks must lie in [0, min(c, q, 64)] and pivots
 * inside the block, else HH_ERR_INVALID_ARG. HH_FP64 and HH_FP32 only. Syncs. */
hh_status hh_aca_build_pivots(hh_ctx ctx, hh_tree tree, hh_part part, hh_kernel kern,
                              hh_precision prec, const int32_t* rank, const int32_t* fallback,
                              const int32_t* piv_i, const int32_t* piv_j, hh_lowrank* out);

/* U = alpha_1 F + sum_{P^H} H F + sum_{P^G} C (Q F)  (Eq. (6), first two
 * terms). F: device [n][3] (FP64 for HH_FP64, FP32 otherwise). U: device
 * [n][3] (FP32 for HH_FP32, FP64 otherwise), fully overwritten, input order.
 * lr must come from hh_aca_build with the same tree, partition, kernel and
 * precision. Does not sync. Workspaces live in lr: the first call sizes
 * them; later calls allocate nothing and record no memset, so they can be
 * captured in a HIP graph (with profiling off). Products on one lr must not
 * overlap in time. In streamed mode, where huge blocks hold 5% or more of a
 * launch's rows, the ACA's workgroup-team kernel runs on the context's second
 * stream, forked from and joined back to the context stream inside this call
 * (a capture includes it). */
hh_status hh_matvec(hh_ctx ctx, hh_tree tree, hh_part part, hh_lowrank lr, hh_kernel kern,
                    hh_precision prec, const void* F, void* U);

/* Bytes of the static device scratch of hh_matvec_noalloc (one copy per
 * device, held until the process ends). */
#define HH_NOALLOC_SCRATCH_BYTES (64ull << 20)

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * product of hh_matvec (same kernels, same result bit for bit) with its
 * workspaces -- the sorted forces and the near-field rows, 3 n values each --
 * in a file-scope device array of HH_NOALLOC_SCRATCH_BYTES instead of device
 * memory kept in lr; it calls no allocating routine and records no phase
 * events. Stored factors only (a streamed-mode lr -> HH_ERR_INVALID_ARG). A
 * product that needs more scratch than HH_NOALLOC_SCRATCH_BYTES (about 1.4M
 * particles in HH_FP64, 1.8M in HH_BF16, 2.8M in HH_FP32) -> HH_ERR_CAPACITY,
 * checked before anything else. Every call on a device shares that device's
 * scratch: calls that overlap in time on one device (any streams, any
 * contexts) race and must be ordered by the caller. Does not sync. */
hh_status hh_matvec_noalloc(hh_ctx ctx, hh_tree tree, hh_part part, hh_lowrank lr,
                            hh_kernel kern, hh_precision prec, const void* F, void* U);

/* Gradients of L = sum_i dU_i . U_i for the product hh_matvec computes, with
 * the tree, the partition and the ACA pivots frozen.
 *   dF (device, same type as F, nullable): the transposed product M_H^T dU.
 *   dX (device FP64 [n][3], nullable): d L / d x through the kernel (near
 *       blocks re-evaluate each pair; admissible blocks use the frozen
 *       cross approximation as the function of X it is).
 *   dparams (device FP64 [HH_MLP_NPARAM], nullable, MLP kernel only):
 *       d L / d theta, accumulated into (not overwritten).
 * F and dU as in hh_matvec. Precision HH_FP64 or HH_FP32; stored factors
 * only. The cotangents of the sampled kernel entries are kept for chunks of
 * consecutive blocks of at most 2^28 values (1 GiB in FP32) at a time. Syncs
 * (reads back the ranks to plan those chunks). */
hh_status hh_matvec_backward(hh_ctx ctx, hh_tree tree, hh_part part, hh_lowrank lr,
                             hh_kernel kern, hh_precision prec, const void* F, const void* dU,
                             void* dF, double* dX, double* dparams);

void hh_tree_free(hh_tree t);
void hh_part_free(hh_part p);
void hh_lowrank_free(hh_lowrank l);

/* ------------------------------------------------------- the batched form */

/* Parameters of a batch of independent systems (suspensions) concatenated in
 * one position array. */
typedef struct {
  int32_t n_sys;           /* number of systems, >= 1 */
  const int64_t* offsets;  /* host, n_sys + 1 particle offsets (0, ..., n), increasing */
  const int32_t* c_leafs;  /* host, leaf size per system (each >= 2), or NULL ... */
  int32_t c_leaf;          /* ... for this leaf size in every system */
  double eta;              /* admissibility parameter of Eq. (7), > 0 */
  double eps;              /* ACA tolerance (Eq. (10)), >= 0 */
  int32_t l_max;           /* ACA rank cap, 1..64 */
  hh_precision prec;
} hh_batch_params;

/* Builds the H-matrix of every system of a batch in one handle: the batched
 * tree (hh_build_tree_batch_leaf), the partition (Algorithm 1 from every
 * system's root, so no block couples two systems) and the ACA plan or
 * factors (hh_aca_build), with all systems' blocks in the same launches.
 * X: device FP64 [n][3]. kern must outlive the batch. Errors as the calls
 * it makes. Syncs. */
hh_status hh_batch_create(hh_ctx ctx, const double* X, const hh_batch_params* params,
                          hh_kernel kern, hh_batch* out);

/* U = M F for every system of the batch (as hh_matvec; F and U device
 * arrays of the batch's n particles, types per precision). The first call
 * with a given (F, U) computes U eagerly, which sizes every workspace, and
 * records the whole product (every launch of hh_matvec, in streamed mode the
 * ACA with its fused apply and the team kernel on the context's second
 * stream) in a HIP graph on a private stream; it syncs. Every later call
 * with the same pointers is one graph launch on the context stream that
 * recomputes U from the current contents of F (no sync, no allocation, no
 * host work per system). A call with other pointers records a new graph.
 * Calls on one batch must not overlap in time. */
hh_status hh_batch_matvec(hh_ctx ctx, hh_batch b, const void* F, void* U);

/* Sizes and parts of a batch (each output nullable): particles, systems,
 * nodes of the recorded graph (0 before the first product), graph launches
 * so far, and the tree, partition and low-rank handles it owns (valid until
 * hh_batch_free; do not free them). */
hh_status hh_batch_info(hh_batch b, int64_t* n, int32_t* n_sys, int64_t* graph_nodes,
                        int64_t* graph_launches, hh_tree* tree, hh_part* part, hh_lowrank* lr);
void hh_batch_free(hh_batch b);

/* ------------------------------------------ short-range many-body terms */

/* Size of the packed parameter vector of the three-body network g:
 * W1[64][6] b1[64] W2[64][64] b2[64] W3[64][64] b3[64] W4[18][64] b4[18]. */
#define HH_G3_NPARAM 9938

/* The remaining terms of Eq. (6), M^(s,2) F + M^(t,3) F + M^(s,3) F (Eq. (2)
 * normalised as in Eq. (4)), over the neighbours N(i) within the cut-off
 * r_cut (Sec. 2.2; 5 in Sec. 2.4) and the 3-cliques (j, k, i) with k in N(i),
 * j in N(k), j != i (Sec. 2.3). With d_j = x_j - x_i, d_k = x_k - x_i:
 *   alpha_2^(s) = sym(h_s(d_j / |d_j|)) / (8 pi |d_j|)         (times F_i)
 *   alpha_3^(s), alpha_3^(t) = sym(g_s), sym(g_t) / (8 pi |x_j - x_k| |x_k - x_i|)
 *                                                    (times F_i and F_j)
 * where h_s is a 3-64-64-64-9 tanh MLP (s2_params: HH_MLP_NPARAM doubles, the
 * layout of hh_kernel_create_mlp), g a 6-64-64-64-18 tanh MLP on
 * (d_j, d_k) / r_cut whose outputs 0..8 and 9..17 are the row-major 3x3
 * blocks g_s and g_t (g3_params: HH_G3_NPARAM doubles), sym(O) = (O + O^T)/2:
 * seeded stand-ins for the trained networks.
 * hh_short_create builds the neighbour lists of the tree's current positions
 * (a uniform grid of cells of edge r_cut over the root box; a single-system
 * tree only, else HH_ERR_INVALID_ARG; parameters are copied). The tree must
 * outlive the handle. Syncs. */
hh_status hh_short_create(hh_ctx ctx, hh_tree tree, const double* s2_params,
                          const double* g3_params, double r_cut, hh_short* out);
/* U += M^(s,2) F + M^(t,3) F + M^(s,3) F for the positions of the tree the
 * handle was built on. F, U: device arrays in the caller's order with the
 * types of hh_matvec for prec (the networks run on the VALU in FP64 for
 * HH_FP64, FP32 otherwise, sums in FP64). Does not sync. */
hh_status hh_short_matvec(hh_ctx ctx, hh_short s, hh_precision prec, const void* F, void* U);
/* Neighbour pairs (sum of |N(i)|) and 3-cliques of the handle. */
hh_status hh_short_info(hh_short s, int64_t* n_pairs, int64_t* n_cliques);
void hh_short_free(hh_short s);

/* --------------------------------------------------------- time stepping */

/* Forces of a time step (Sec. 4.3): the uniform external force gravity
 * (host, 3 values; (0, 0, -1) in Sec. 4.3.1) on every particle, plus the
 * internal forces of n_fil filaments, each a chain of n_beads consecutive
 * particles (chain c holds particles [c n_beads, (c + 1) n_beads) of X; the
 * remaining particles are free), Sec. 4.3.2:
 *   tension on every bond r = x_{i+1} - x_i: f = k_t (|r| - l0) r / |r|,
 *     added to bead i and subtracted from bead i+1;
 *   COS bending on every interior bead i: t_1, t_2 the unit bond vectors into
 *     and out of i, T = -k_b (t_1 x t_2) |t_1 x t_2|, forces T x t_1 on i-1,
 *     -T x t_2 on i+1 and minus their sum on i.
 * X: device FP64 [n][3]; F: device [n][3], FP64 for HH_FP64, FP32 otherwise
 * (the force type of hh_matvec), fully overwritten. n_fil * n_beads <= n,
 * n_beads >= 2 when n_fil > 0, else HH_ERR_INVALID_ARG. Does not sync. */
hh_status hh_filament_forces(hh_ctx ctx, const double* X, int64_t n, int64_t n_fil,
                             int32_t n_beads, double k_t, double l0, double k_b,
                             const double* gravity, hh_precision prec, void* F);
/* Explicit Euler step of dX/dt = U (Sec. 4.3): X += dt U. X: device FP64
 * [n][3], updated in place; U: device [n][3] of the type hh_matvec returns
 * for prec (FP32 for HH_FP32, FP64 otherwise). Does not sync. */
hh_status hh_euler_step(hh_ctx ctx, double* X, const void* U, int64_t n, double dt,
                        hh_precision prec);

/* ------------------------------------------------------- export and stats */

/* Sizes of a tree: particles, nodes, leaves. Host outputs (nullable). */
hh_status hh_tree_info(hh_tree t, int64_t* n, int64_t* n_nodes, int64_t* n_leaves);
/* Copy a tree to host arrays (each nullable):
 * perm[n] int64 -- input index at sorted position s; keys[n] uint64 -- Morton
 * key at sorted position s; nodes[n_nodes][4] int32 -- (begin, end, left,
 * right), -1 children for leaves; bbox[n_nodes][6] FP64 -- (lo xyz, hi xyz).
 * Syncs. */
hh_status hh_tree_export(hh_tree t, int64_t* perm, uint64_t* keys, int32_t* nodes, double* bbox);

/* Sizes of a partition: admissible (nG) and inadmissible (nH) blocks. */
hh_status hh_part_info(hh_part p, int64_t* nG, int64_t* nH);
/* Work measures of a partition: near_pairs = sum over P^H of |tau||sigma|
 * (the dense kernel evaluations of the near field, self pairs included) and
 * far_entries = sum over P^G of |tau||sigma|. Host outputs (nullable). */
hh_status hh_part_stats(hh_part p, int64_t* near_pairs, int64_t* far_entries);
/* Copy the block lists to host arrays [nG][2], [nH][2] of (tau, sigma) node
 * ids, sorted. Each nullable. Syncs. */
hh_status hh_part_export(hh_part p, int32_t* G, int32_t* H);

/* Factor summary: number of admissible blocks, sum of ranks, number of
 * dense fallbacks, total kernel samples taken (sum over blocks of
 * rank*(c+q)), factor bytes. Host outputs (nullable). */
hh_status hh_lowrank_info(hh_lowrank l, int64_t* n_blocks, int64_t* rank_sum,
                          int64_t* n_fallback, int64_t* samples, int64_t* bytes);
/* Per admissible block (in partition order): rank[nG] int32, fallback flag
 * [nG] int32, and the pivots piv_i[nG][64], piv_j[nG][64] int32 (local
 * indices, -1 past the rank). Each nullable. Syncs. */
hh_status hh_lowrank_export(hh_lowrank l, int32_t* rank, int32_t* fallback, int32_t* piv_i,
                            int32_t* piv_j);
/* Copy factor k of admissible block b to host: c_k as [c][3][3] and q_k as
 * [q][3][3], in FP64 regardless of storage type. Syncs. */
hh_status hh_lowrank_factor(hh_lowrank l, int64_t b, int32_t k, double* ck, double* qk);

/* ------------------------------------------------------------ profiling */

/* Phases timed with HIP events recorded on the context stream around each
 * phase's kernel launches, while profiling is on (off by default). */
#define HH_PHASE_TREE 0      /* hh_build_tree (whole call, incl. its readbacks) */
#define HH_PHASE_PARTITION 1 /* hh_partition (whole call, incl. its readbacks) */
#define HH_PHASE_ACA 2       /* the ACA kernel launch(es) of hh_aca_build */
#define HH_PHASE_NEAR 3      /* the near-field kernel launch of hh_matvec */
#define HH_PHASE_FAR 4       /* the t_k = Q_k F launch of hh_matvec */
#define HH_PHASE_COMBINE 5   /* the combine/unpermute launch of hh_matvec */
#define HH_PHASE_BACKWARD 6  /* the launches of hh_matvec_backward */
#define HH_PHASE_SHORT 7     /* hh_short_create (whole call) and the hh_short_matvec launches */
#define HH_NPHASE 8
hh_status hh_ctx_set_profiling(hh_ctx ctx, int on);
/* Accumulated milliseconds and event pairs per phase since the last reset
 * (host arrays of HH_NPHASE, nullable). Syncs. reset != 0 clears them after
 * reading. */
hh_status hh_ctx_phase_times(hh_ctx ctx, double* ms, int64_t* count, int reset);

/* Build-time constants of the library (for tests): returns 1 if compiled for
 * gfx950. */
int hh_device_arch_ok(void);

#ifdef __cplusplus
}
#endif
#endif /* HH_H */
