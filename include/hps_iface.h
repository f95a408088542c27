/*
 * hps_iface.h - FP64 direct solve of the reduced (interface) system of the
 * HPS discretisation on AMD Instinct MI355X (gfx950).
 *
 * Reference: A. Yesypenko, P.-G. Martinsson, "GPU Optimizations for the
 * Hierarchical Poincare-Steklov Scheme", arxiv 2211.14969.
 *
 * After static condensation every leaf t has its Dirichlet-to-Neumann map
 * S_t (nb x nb) and particular flux w_t (hps_leaf.h).  Continuity of the
 * flux across every shared leaf edge (Sec. 2) gives the reduced system of
 * eq. (hps_reduced) on the edge nodes:
 *
 *     sum over the leaves t at node e of (S_t u_b + w_t)[e] = 0,
 *
 * with u_b = g on edges that lie on the outer boundary.  Sec. 2 solves it
 * with a sparse direct solver in nested-dissection order (O(N^{3/2}) to
 * factor, O(N log N) to apply).  This library does exactly that on the GPU:
 * the leaf grid is bisected recursively (longer side first); each bisection
 * has a separator (the leaf edges on the cut) whose unknowns are eliminated
 * from a dense frontal matrix assembled from the two halves' Schur
 * complements.  Fronts of one tree level are independent and run as one
 * batch: assembly, LU with partial pivoting of the separator block, the
 * multi-column triangular solve and the Schur-complement update (FP64 MFMA).
 * Pivoting is within each separator block (no exchanges between fronts).
 *
 * Grid and layouts: one problem on an nx x ny grid of equal leaves, leaf
 * t = ix + nx*iy (ix along x1), all of order p (hps_iface_create) or each
 * of its own order (hps_iface_create_orders); each leaf's S is [nb][nb]
 * and w, g and u_b are [nb] in the boundary order of hps_leaf.h (W, E, S,
 * N, each p-2 nodes in increasing coordinate), leaves concatenated in leaf
 * order unless offsets are given.
 * All arrays are caller-owned DEVICE memory and must stay valid until the
 * context stream has executed the call; calls are asynchronous on the
 * context stream.  Argument errors are returned synchronously and nothing
 * is enqueued.
 */
#ifndef HPS_IFACE_H
#define HPS_IFACE_H

#include "hps_leaf.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Largest separator (nodes on one cut) this build factors. */
#define HPS_IFACE_MAX_SEPARATOR 1024

typedef struct hps_iface hps_iface;

/* Host-only planning (no device call): the nested-dissection tree of an
 * nx x ny grid of order-p leaves.  Outputs (each may be NULL): number of
 * fronts (nx*ny - 1), tree levels, largest separator, FLOP of one
 * factorisation, device bytes the factorisation keeps.
 * HPS_ERR_INVALID: p outside [HPS_P_MIN, HPS_P_MAX], nx or ny < 1, or a
 * separator above HPS_IFACE_MAX_SEPARATOR. */
hps_status hps_iface_plan(int p, int nx, int ny, int *nfront, int *levels, int *max_sep,
                          double *factor_flop, size_t *bytes);

/* Host-only planning of a grid whose leaves differ in order (Sec. 2: p
 * chosen per leaf from a fixed set).  orders: host [nx*ny], the p of leaf
 * t = ix + nx*iy.  A shared edge carries the nodes of the lower of its two
 * leaves' orders; the other leaf's trace is the polynomial through them,
 * evaluated at its own edge nodes, and its flux is carried back to the
 * edge's nodes by the polynomial through its nodal fluxes (the fluxes
 * balance there).  Outputs and errors as hps_iface_plan. */
hps_status hps_iface_plan_orders(int nx, int ny, const int *orders, int *nfront, int *levels,
                                 int *max_sep, double *factor_flop, size_t *bytes);

/* Host-only: per-front sizes of that plan, in the order the fronts are
 * factored (by tree level, leaves' parents first): separator nodes nS,
 * exterior nodes nE and tree level of each front; arrays of nfront entries
 * (from hps_iface_plan), any may be NULL. */
hps_status hps_iface_plan_fronts(int p, int nx, int ny, int *nS, int *nE, int *level);

/* Plans the tree and allocates its device storage (the fronts' factors and
 * Schur complements, sized by hps_iface_plan's `bytes`).  Errors as
 * hps_iface_plan, plus HPS_ERR_OOM / HPS_ERR_HIP. */
hps_status hps_iface_create(hps_ctx *ctx, int p, int nx, int ny, hps_iface **out);

/* As hps_iface_create for leaves of different orders (orders: host
 * [nx*ny], as in hps_iface_plan_orders).  s_off / b_off: host [nx*ny], the
 * offset (in doubles) of leaf t's S [nb_t][nb_t] in the S array, and of its
 * nb_t boundary slots in the w, g and ub arrays, nb_t = 4(p_t - 2) (the
 * layout of a leaf batch with one group per order: groups concatenated);
 * NULL for leaf-major order.  Leaves on an edge of lower order on their
 * other side have their S taken to the edge basis at factorisation time. */
hps_status hps_iface_create_orders(hps_ctx *ctx, int nx, int ny, const int *orders,
                                   const long long *s_off, const long long *b_off,
                                   hps_iface **out);

/* Factorisation (the build of Sec. 2's direct solver) from the leaves' maps
 * S [nx*ny][nb][nb].  Per front it keeps the LU factors of the separator
 * block, X = F_ss^{-1} F_se and F_es, and passes the Schur complement
 * F_ee - F_es X up the tree.  `info` (device [nfront] or NULL): 0, or k > 0
 * when the separator block of that front had a zero (or NaN) pivot at
 * column k (LAPACK getrf convention; the factorisation goes on).  The
 * handle enqueues on the stream of `ctx`, which must outlive it.
 * With HPS_SYNC: synchronises and returns HPS_ERR_SINGULAR if any front
 * had a zero pivot. */
hps_status hps_iface_factor(hps_iface *it, const double *S, int *info, int flags);

/* Solve (the apply of the direct solver) after hps_iface_factor with the
 * same S.  w [nx*ny][nb] (NULL: w = 0, i.e. f = 0) and g [nx*ny][nb] (only
 * the slots on the outer boundary are read: the Dirichlet data) give the
 * right-hand side; the result ub [nx*ny][nb] holds every leaf's edge
 * values (solved interface values, g on the outer boundary), ready for
 * hps_leaf_recover.  Upward pass: reduced right-hand sides; downward pass:
 * u_sep = F_ss^{-1} r_s - X u_ext from the root.  HPS_SYNC: synchronise. */
hps_status hps_iface_solve(hps_iface *it, const double *S, const double *w, const double *g,
                           double *ub, int flags);

hps_status hps_iface_destroy(hps_iface *it);

#ifdef __cplusplus
}
#endif

#endif /* HPS_IFACE_H */
