/*
 * hps_leaf.h - batched leaf-level static condensation for the Hierarchical
 * Poincare-Steklov (HPS) discretisation on AMD Instinct MI355X (gfx950).
 *
 * Reference: A. Yesypenko, P.-G. Martinsson, "GPU Optimizations for the
 * Hierarchical Poincare-Steklov Scheme", arxiv 2211.14969.
 *
 * The problem (Sec. 1, eqs. (bvp), (var_helm)): A u = f in a domain, u = g on
 * its boundary, with A a second-order elliptic operator.  In the reference
 * coordinates of a leaf box this library collocates
 *
 *     A u = -(a11 u_11 + 2 a12 u_12 + a22 u_22 + c1 u_1 + c2 u_2) - k2b u
 *
 * (the variable-coefficient Helmholtz operator has a11 = a22 = 1,
 * a12 = c1 = c2 = 0, k2b = kappa^2 b; a mapped domain such as the curved one
 * of Sec. 3.2, eq. (chain_rule), brings the mixed term).  With a12 the
 * interior rows reach the leaf corners, which carry no unknown: each corner
 * value is taken as the mean of the degree-(p-3) polynomials through its two
 * edges' nodes, evaluated at the corner, which folds the corner columns into
 * A_ib.  Operators with a12 are condensed in FP64 only.
 *
 * Discretisation (Sec. 2): each leaf carries a p x p tensor grid of Chebyshev
 * extreme points; the PDE is collocated at the (p-2)^2 interior nodes by
 * spectral differentiation, and the outward normal derivative (the flux that
 * must be continuous between neighbouring leaves) is taken at the 4(p-2)
 * edge nodes.  Corners are not used.  Static condensation (Sec. 2, before
 * eq. (hps_reduced)) eliminates the interior nodes:
 *
 *     X = A_ii^{-1} A_ib,  h = A_ii^{-1} f_i,  S = A_bb - A_bi X,  w = A_bi h,
 *
 * and after the reduced system is solved the interior values are recovered
 * as u_i = h - X u_b (Sec. 3, text after eq. (constant_coeff_helm)).
 *
 * Layouts (all arrays row-major, leaves concatenated in group order):
 *   node (i, j) of a leaf, i along x1, j along x2, has flat index i + p*j;
 *   interior order: (i, j), 1 <= i, j <= p-2, i fastest       -> ni = (p-2)^2
 *   boundary order: W (i=0, j up), E (i=p-1, j up),
 *                   S (j=0, i up), N (j=p-1, i up)            -> nb = 4(p-2)
 *   flux sign: outward (W: -d/dx1, E: +d/dx1, S: -d/dx2, N: +d/dx2).
 *
 * Memory: every array argument is caller-owned DEVICE memory unless stated
 * otherwise, and must stay valid until the context stream has executed the
 * call.  Calls are asynchronous on the context stream; argument errors are
 * detected on the host, returned synchronously, and nothing is enqueued.
 * No C++ exception crosses this interface.  Device-side failures are written
 * per leaf into `info` and are folded into the return code only with
 * HPS_SYNC.
 */
#ifndef HPS_LEAF_H
#define HPS_LEAF_H

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  HPS_OK = 0,
  HPS_ERR_INVALID = -1,       /* bad argument; nothing was enqueued            */
  HPS_ERR_OOM = -2,           /* device allocation failed                      */
  HPS_ERR_HIP = -3,           /* a HIP runtime call failed                     */
  HPS_ERR_SINGULAR = -4,      /* (HPS_SYNC) some leaf had an exactly zero pivot */
  HPS_ERR_NOT_CONVERGED = -5, /* reserved (refinement failures fall back to FP64) */
  HPS_ERR_NONFINITE = -6      /* (HPS_SYNC) a leaf produced Inf or NaN         */
} hps_status;

typedef enum {
  HPS_FP64 = 0,        /* LU, triangular solves and Schur complement in FP64   */
  HPS_FP32_REFINE = 1  /* LU and solves on FP32-stored work matrices (tile
                          products on the FP64 MFMA from FP32 operands), FP64
                          iterative refinement of X with an FP64 residual
                          A_ib - A_ii X; S in FP64 */
} hps_precision;

/* flags */
#define HPS_SYNC 1                /* synchronise and fold `info` into the result */
#define HPS_RECOVER_REFACTOR 2    /* recover: re-form and re-factor the leaves
                                     instead of using the stored X, h (the
                                     paper's storage-free mode, Sec. 2 remark) */

/* Limits of this build. */
#define HPS_P_MIN 4
#define HPS_P_MAX 32
/* Size of the device array that holds the pass scratch of
 * hps_leaf_condense_noalloc (one copy per GPU, kept for the process). */
#define HPS_NOALLOC_SCRATCH_BYTES (512ull << 20)

/* One group of leaves sharing the order p (a whole problem, or one order
 * class of a multi-problem batch).
 *   box : device [nleaf][4] = x0, x1, y0, y1 of each leaf (reference coords)
 *   a11, a12, a22, c1, c2, k2b : device [nleaf][p*p] samples at every node
 *         (flat index i + p*j), or NULL for the default (a11 = a22 = 1,
 *         others 0).  Sample them at the coordinates returned by
 *         hps_leaf_nodes.  A group with a12 must be condensed with HPS_FP64
 *         (HPS_FP32_REFINE returns HPS_ERR_INVALID).                      */
typedef struct {
  int p;
  int nleaf;
  const double *box;
  const double *a11, *a12, *a22, *c1, *c2, *k2b;
} hps_leaf_desc;

typedef struct hps_ctx hps_ctx;
typedef struct hps_batch hps_batch;

/* Create a context bound to `stream` (a hipStream_t; NULL = default stream)
 * on the current device.  *out receives the handle. */
hps_status hps_ctx_create(void *stream, hps_ctx **out);
/* Release a context (NULL is a no-op).  Batches built on it must be
 * destroyed first.  Everything is released even if a HIP call fails; the
 * first failure is returned as HPS_ERR_HIP. */
hps_status hps_ctx_destroy(hps_ctx *ctx);

/* Set up a batch of leaf groups: validates the descriptors, builds the
 * Chebyshev tables for each order (Sec. 2: p x p Chebyshev grid and spectral
 * differentiation) and allocates every device buffer the batch will use: the
 * FP64 X and h kept for recovery, per-leaf flags, and the pass scratch (LU
 * work matrices, pivots, refinement bookkeeping) of the leaves in flight,
 * sized once for the largest mode (FP64 with a body-load column) within the
 * workspace cap (environment HPS_WORKSPACE_MB, default 32 GiB, shared between
 * the lanes in proportion to their work; larger groups are condensed in
 * several passes).  After this call no entry point of the
 * batch allocates or frees device memory, so condense and recover calls may
 * be captured in a HIP graph.  Groups are dealt to up to four lanes (largest
 * work first; environment HPS_LANES lowers the cap, 1 = a single stream),
 * each with its own stream and scratch, so that groups of different orders
 * run concurrently.  The descriptor arrays are only read
 * when the batch is used, so they must stay valid for the batch's lifetime.
 * Synchronous. */
hps_status hps_leaf_build(hps_ctx *ctx, const hps_leaf_desc *groups, int ngroups,
                          hps_batch **out);

/* Total number of leaves, and ni / nb of group g. */
int hps_batch_nleaf(const hps_batch *b);
hps_status hps_batch_group_dims(const hps_batch *b, int g, int *p, int *nleaf,
                                int *ni, int *nb);

/* Write the physical coordinates of every node of group g:
 * xy device [nleaf][p*p][2].  Async. */
hps_status hps_leaf_nodes(hps_batch *b, int g, double *xy);

/* Write the dense leaf blocks of group g (Sec. 2: the p^2 x p^2 leaf matrix,
 * partitioned into interior / boundary):  Aii [nleaf][ni][ni],
 * Aib [nleaf][ni][nb], Abi [nleaf][nb][ni], Abb [nleaf][nb][nb];
 * any pointer may be NULL.  For checking the operator; the condensation
 * itself never materialises A_bi or A_bb.  Async. */
hps_status hps_leaf_operator(hps_batch *b, int g, double *Aii, double *Aib,
                             double *Abi, double *Abb);

/* Static condensation of every leaf (Sec. 2; cost O(p^4 N), Sec. 2 batching
 * paragraph): forms the leaf operator on the device, factors A_ii with
 * partial pivoting, computes X (and h when f != NULL), refines X in FP64
 * when prec == HPS_FP32_REFINE, and forms S and w in FP64.
 *   prec       : HPS_FP64 or HPS_FP32_REFINE
 *   tol        : refinement target (HPS_FP32_REFINE; ignored for HPS_FP64):
 *                a leaf stops refining when the estimated relative forward
 *                error of X, 16 rho / (1 - rho) ||dX_k|| / ||X_k||, is at
 *                most tol, with dX_k the last correction and rho < 1 the
 *                contraction per step, estimated as the larger of
 *                ||r_k|| / ||r_{k-1}|| and ||dX_1|| / ||X_1||
 *                (r = A_ib - A_ii X evaluated in FP64; the factor 16
 *                covers how far both estimates of rho can fall short).
 *                <= 0 selects 1e-10; >= 1 applies exactly max_refine
 *                corrections and accepts the result without a test (no
 *                FP64 redo).
 *   max_refine : FP32 correction steps at most, 0..16.  The residual is
 *                evaluated before each correction and once more after the
 *                last.  Leaves that never pass (A_ii too ill-conditioned for
 *                an FP32 factorisation, e.g. near a leaf resonance) are
 *                condensed again in FP64, so every leaf ends accurate.
 *   f          : device [total leaves][ni] interior body load, or NULL (f = 0)
 *   S          : device [total leaves][nb][nb]   (output)
 *   w          : device [total leaves][nb] or NULL (output; 0 when f == NULL)
 *   info       : device [total leaves] or NULL (output):
 *                0 ok; k > 0 exact zero pivot in column k (1-based, LAPACK
 *                getrf convention); -2 non-finite value in X or S.
 *   flags      : HPS_SYNC or 0
 * The stored X and h are kept in the batch for hps_leaf_recover.  Async
 * unless HPS_SYNC. */
hps_status hps_leaf_condense(hps_batch *b, hps_precision prec, double tol,
                             int max_refine, const double *f, double *S,
                             double *w, int *info, int flags);

/* The same computation as hps_leaf_condense (same arguments, results equal
 * up to rounding), for callers that cannot allocate device memory at call
 * time (code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation): its pass scratch (LU work matrices, pivots, retire
 * steps and refinement bookkeeping) lives in a device array of
 * HPS_NOALLOC_SCRATCH_BYTES inside the library, one per GPU, instead of in
 * the batch; it calls no allocating routine.  Each order group is processed
 * in passes of as many leaves as that array holds (at p = 32 in FP64, 67
 * leaves per pass), all on the context stream.  Returns HPS_ERR_INVALID,
 * with nothing enqueued, if a single leaf of some group does not fit the
 * array.  Every call on one GPU shares that GPU's array and overwrites it:
 * calls that overlap on one GPU (two streams, or two threads) race and must
 * be serialised by the caller.  The batch's stored X, h, flags and per-leaf
 * status are updated as by hps_leaf_condense.  Async unless HPS_SYNC. */
hps_status hps_leaf_condense_noalloc(hps_batch *b, hps_precision prec, double tol,
                                     int max_refine, const double *f, double *S,
                                     double *w, int *info, int flags);

/* Interior recovery (Sec. 3, after eq. (constant_coeff_helm)):
 *   ub : device [total leaves][nb]  boundary values
 *   f  : device [total leaves][ni] or NULL; used only with
 *        HPS_RECOVER_REFACTOR (the stored h already holds the f given to
 *        hps_leaf_condense)
 *   ui : device [total leaves][ni]  (output)
 * Default: u_i = h - X u_b from the stored FP64 X and h (requires a prior
 * hps_leaf_condense).  With HPS_RECOVER_REFACTOR: re-forms and re-factors
 * every leaf in FP64 and solves A_ii u_i = f_i - A_ib u_b (the paper's mode:
 * factorisations are not kept).  Async unless HPS_SYNC. */
hps_status hps_leaf_recover(hps_batch *b, const double *ub, const double *f,
                            double *ui, int flags);

/* Tuning of group g's factorisation (for an autotuner; the defaults are
 * chosen automatically):
 *   factor_variant : 0 automatic, 4 left-looking: each 32-column block
 *                    column held in registers, formed from the operator,
 *                    updated by the earlier panels (multipliers read, never
 *                    rewritten) with rows kept in pivot order, then its own
 *                    panels factored (chunk_cols ignored),
 *                    1 one 16-column panel per trailing pass,
 *                    2 panels in pairs (one trailing pass per 32 columns;
 *                    both panels in LDS when (p-2)^2 <= 256 (FP64: < 256),
 *                    else the first panel's multipliers re-read from the
 *                    work matrix), 3 the whole work matrix held in registers
 *                    (HPS_FP32_REFINE and p <= 16 only; elsewhere the
 *                    automatic choice).  Automatic is 4 for HPS_FP64 above
 *                    400 rows (p >= 23), else 2, except 1 for
 *                    HPS_FP32_REFINE when 256 < (p-2)^2 < 400.
 *   chunk_cols     : 0 automatic, else the column width (multiple of 16, at
 *                    most 1024) of the U12 / trailing passes; ignored when
 *                    its LDS footprint does not fit.
 * Results do not depend on the tuning beyond rounding.  Takes effect on the
 * next hps_leaf_condense / hps_leaf_recover. */
hps_status hps_batch_set_tuning(hps_batch *b, int g, int factor_variant, int chunk_cols);

/* Copy the stored FP64 solution operator out of the batch:
 *   Xt : device [total leaves][nb][ni]  (X transposed: Xt[l][b][i] = X_l[i][b])
 *   h  : device [total leaves][ni]
 * Either may be NULL.  Async. */
hps_status hps_batch_export(hps_batch *b, double *Xt, double *h);

/* Per-leaf record of the last condense: flags device [total leaves] gets 1
 * for every leaf the FP32 + refinement path handed to the FP64 redo (its
 * refinement could not meet tol within max_refine corrections), else 0.
 * Async. */
hps_status hps_batch_redo_flags(hps_batch *b, int *flags);

/* Number of lanes (concurrent streams) the batch's groups were dealt to. */
int hps_batch_lanes(const hps_batch *b);

/* Statistics of the last hps_leaf_condense (host pointers, either may be
 * NULL): the refinement step limit it ran with, and the number of leaves the
 * FP32 + refinement path handed to the FP64 fallback.  Reading fp64_redo
 * synchronises the context stream. */
hps_status hps_batch_stats(const hps_batch *b, int *refine_steps, int *fp64_redo);

/* Per-phase timing with HIP events on the context stream (tracing aid).
 * While enabled, every kernel launch of hps_leaf_condense / hps_leaf_recover
 * is bracketed by events and the elapsed time is accumulated per phase:
 *   0 (unused)   1 operator build and LU factorisation (with forward
 *   elimination of the right-hand sides)   2 back substitution
 *   3 refinement correction solves and stop tests   4 Schur complement
 *   5 recovery   6 refinement FP64 residuals   7 FP64 redo of leaves the
 *   refinement could not serve.
 * hps_ctx_phase_times synchronises the stream, writes the accumulated
 * milliseconds and launch counts of the HPS_NPHASE phases (host arrays,
 * either may be NULL) and resets them. */
#define HPS_NPHASE 8
hps_status hps_ctx_set_timing(hps_ctx *ctx, int enable);
hps_status hps_ctx_phase_times(hps_ctx *ctx, double *ms, int *launches);

/* Free a batch and its device buffers (NULL is a no-op).  hipFree
 * synchronises the device, so work still queued on the batch completes
 * first.  Every buffer is released even if one free fails (HPS_ERR_HIP). */
hps_status hps_batch_destroy(hps_batch *b);

/* Static text naming a status code. */
const char *hps_status_string(hps_status s);

#ifdef __cplusplus
}
#endif
#endif /* HPS_LEAF_H */
