/*
 * imq.h -- C interface of the MI355X (gfx950) fast product with the
 * inverse-multiquadric (IMQ) interpolation matrix, and of the solver built
 * on it.
 *
 * The operator (Sec. 2, eqs. IMQ_def and interp_system):
 *     A_ij = 1 / sqrt(|x_i - x_j|^2 + c^2),   x_i in R^2 distinct data sites,
 * and the product b = A u that the translation technique of Sec. 2.2
 * (Algorithm 1) computes.  Each point is lifted to the plane z = -c/2 as a
 * source and z = +c/2 as a target (eq. G_eq_phi), so A_ij is the 3-D Laplace
 * Green's function (eq. G_def) between the lifted points; its spectral
 * expansion (eq. GreenDecompositionG, truncated at order p as in
 * eq. serieTroncata, error bound of Theorem 2.1) is applied through a
 * quadtree of the plane: per-leaf expansions (P2M), upward shifts (M2M),
 * expansion-to-local translations between well-separated boxes (M2L),
 * downward shifts (L2L), local evaluation (L2P), and the direct near field
 * (P2P) of the last loop of Algorithm 1.
 *
 * Conventions for every entry point below:
 *  - Array arguments are DEVICE pointers on the current HIP device, owned by
 *    the caller, unless the comment says "host".
 *  - All work is enqueued on `stream` (0 = the default stream) and is
 *    stream-ordered; only the calls that say so synchronise.
 *  - Errors are returned as a status, never thrown; imq_last_error() gives a
 *    thread-local detail string for the last failing call.
 *  - A tree handle may be used by one stream at a time.  A call on a handle
 *    that imq_tree_free has freed returns IMQ_EINVAL.
 *  - Calls on a tree run on the device the tree was built on; the caller's
 *    current device is the same after the call as before it.
 */
#ifndef IMQ_H
#define IMQ_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct imq_tree_s *imq_tree;     /* opaque, owned by the library */

typedef enum {
    IMQ_OK = 0,
    IMQ_ENOTCONVERGED = 1,  /* warning: outputs are valid, tolerance not met */
    IMQ_EINVAL = -1,        /* bad argument (size, pointer, c <= 0, NaN ...)  */
    IMQ_EDUPLICATE = -2,    /* two data sites coincide: A would be singular   */
    IMQ_ENOMEM = -3,        /* device or host allocation failed               */
    IMQ_EHIP = -4,          /* a HIP runtime call failed                      */
    IMQ_EUNSUPPORTED = -5   /* valid request the library does not support     */
} imq_status;

/* Element type of the vectors handed across the boundary. */
typedef enum { IMQ_F64 = 0, IMQ_F32 = 1 } imq_dtype;

/* Arithmetic of the expansions, translations and near field inside the
 * product.  IMQ_PREC_FP32 keeps FP64 only for the final accumulation of b
 * and for the operator tables' generation. */
typedef enum { IMQ_PREC_FP64 = 0, IMQ_PREC_FP32 = 1 } imq_prec;

#define IMQ_MAX_LEVELS 31

/* Tree and expansion parameters.
 *  leaf_max   : a box is split while it holds more than leaf_max points
 *               (the finest partition of Sec. 2.2 is reached adaptively).
 *  order_p    : truncation index M of eq. serieTroncata (1 <= p <= 16).
 *  max_level  : deepest level of the quadtree (<= 30; 0 = 30).
 *  level_order: optional per-level truncation of the M2L translation
 *               (0 = use order_p); entry l applies to boxes at level l.
 *               Multipoles are always kept to order_p.                     */
typedef struct {
    int leaf_max;
    int order_p;
    int max_level;
    int level_order[IMQ_MAX_LEVELS + 1];
    int direct_max;      /* adaptive W/X interactions whose finer box holds at
                            most this many points are summed directly instead
                            of through an expansion (0 = 2*leaf_max, < 0 = never) */
    int autotune;        /* imq_build_tree(_alloc) only: nonzero = after the
                            build, tune the per-level translation orders (from
                            order_p down), the internal precision and the
                            translation and near-field kernels for the fastest
                            product whose relative 2-norm error over 1000
                            sampled rows (a fixed pseudo-random weight vector,
                            against exact FP64 sums) is at most 0.8 x
                            autotune_tol; the tree is left configured and
                            imq_get_tree_info reports the choice (tuned_prec,
                            tuned_err, tuned_ms).  Runs products on `stream`
                            and synchronises it.  IMQ_EINVAL if neither
                            precision reaches the target at order_p.  Ignored
                            by imq_build_eval_tree. */
    double autotune_tol; /* target relative error (0 = 1e-6) */
} imq_tree_params;

/* Build the quadtree forest of `nsets` independent point sets.
 *  set_offsets : host, nsets+1 entries; set s owns points
 *                [set_offsets[s], set_offsets[s+1]) of the concatenation.
 *  xy          : device FP64, structure of arrays: x[0..Ntot), y[0..Ntot)
 *                with Ntot = set_offsets[nsets].
 *  c           : host, nsets shape parameters (c > 0, finite).
 * Copies the points to the host, builds the trees, interaction lists and
 * translation tables, and uploads them; synchronises `stream` once.
 * Returns IMQ_EDUPLICATE if two points of a set coincide exactly. */
imq_status imq_build_tree(int nsets, const int64_t *set_offsets, const double *xy,
                          const double *c, const imq_tree_params *params,
                          hipStream_t stream, imq_tree *out);

/* Device memory of a tree (its lists, tables and workspaces) from the
 * caller's allocator instead of hipMalloc/hipFree, e.g. a framework's caching
 * allocator.  alloc returns at least `bytes` of device memory on the current
 * device, 256-byte aligned, or NULL on failure (the call then returns
 * IMQ_ENOMEM); free releases a pointer alloc returned.  Both are called on
 * the host, from the thread of the imq_ call that needs them (every call on
 * the tree may allocate; imq_tree_free frees), with `ctx` passed through;
 * the allocator and ctx must stay valid until imq_tree_free returns. */
typedef struct {
    void *(*alloc)(size_t bytes, void *ctx);
    void (*free)(void *ptr, void *ctx);
    void *ctx;
} imq_allocator;

/* imq_build_tree with the tree's device memory from `alloc` (NULL: hipMalloc). */
imq_status imq_build_tree_alloc(int nsets, const int64_t *set_offsets, const double *xy,
                                const double *c, const imq_tree_params *params,
                                const imq_allocator *alloc, hipStream_t stream, imq_tree *out);

/* b = A u for every set and right-hand side, in the caller's point order.
 *  u : nrhs columns of length Ntot, column r at u + r*ldu (ldu >= Ntot),
 *      element type `dtype`.
 *  b : same layout with ldb, element type `dtype`.
 * Uses the tree's expansions at the given internal precision. */
imq_status imq_matvec(imq_tree tree, int nrhs, imq_dtype dtype, const void *u,
                      int64_t ldu, void *b, int64_t ldb, imq_prec prec,
                      hipStream_t stream);

/* imq_matvec for callers that cannot allocate device memory: code under HIP
 * graph capture, serving loops, harnesses that forbid hipMalloc.  Same
 * arguments, kernels and result as imq_matvec (up to the order of the
 * floating-point sums: the stages run one after another on `stream`, none
 * beside another), but the product's workspace (gathered weights,
 * expansions, partial sums, the FP64 accumulator) is a fixed device array of
 * imq_matvec_noalloc_max_bytes() bytes (128 MiB) that the library holds on
 * every device it runs on until the process ends, instead of buffers the
 * tree allocates on first use; the call allocates nothing.  A product that
 * needs more workspace returns IMQ_EINVAL (about 80 bytes per point and
 * right-hand side at p = 12 in FP64: some 1.6 million points at one
 * right-hand side).  Every call on one device shares that array: calls that
 * overlap in time on one device (other streams, other threads, other trees)
 * race and must be serialised by the caller. */
imq_status imq_matvec_noalloc(imq_tree tree, int nrhs, imq_dtype dtype, const void *u,
                              int64_t ldu, void *b, int64_t ldb, imq_prec prec,
                              hipStream_t stream);
size_t imq_matvec_noalloc_max_bytes(void);

/* Exact product restricted to some rows: b[r*ldb + k] = sum_j A_{rows[k], j} u_j
 * for k < nrows (device int64 row indices, caller order).  Direct sums over
 * all points of the row's set in FP64; used to measure the error of the fast
 * product on sampled rows. */
imq_status imq_rows_exact(imq_tree tree, int nrhs, const double *u, int64_t ldu,
                          int64_t nrows, const int64_t *rows, double *b,
                          int64_t ldb, hipStream_t stream);

/* Evaluation of the interpolant (Sec. 2, eq. interp_eq)
 *     P(y) = sum_j lambda_j / sqrt(|y - x_j|^2 + c^2)
 * at points y that need not be data sites, for one set of n data sites x_j.
 * imq_build_eval_tree builds a tree over the data sites and the m evaluation
 * points together; the evaluation points are targets only (weight zero in
 * every product of this tree).  An evaluation point that coincides with a
 * data site or with an earlier evaluation point is not inserted and takes
 * the value of that point.
 *  xy_src : device FP64 SoA x[0..n), y[0..n): the data sites (IMQ_EDUPLICATE
 *           if two coincide)
 *  xy_tgt : device FP64 SoA x[0..m), y[0..m): the evaluation points (m >= 0)
 *  c      : shape parameter (> 0)
 * The tree answers imq_matvec and imq_rows_exact over its own points (the
 * data sites first, then the inserted evaluation points, Ntot in all) and
 * imq_evaluate.  Synchronises `stream`. */
imq_status imq_build_eval_tree(const double *xy_src, int64_t n, const double *xy_tgt, int64_t m, double c,
                               const imq_tree_params *params, hipStream_t stream, imq_tree *out);

/* s[r*lds + k] = P_r(y_k), k < m, for the coefficients lambda (nrhs columns
 * of length n, leading dimension ldl >= n, element type `dtype`; s the same
 * with lds >= m) on a tree from imq_build_eval_tree (else IMQ_EINVAL): one
 * fast product over the tree's points with the evaluation points' weights
 * zero, read at the evaluation points.  Keeps a workspace of 2 * nrhs * Ntot
 * elements in the tree (allocated on first use, grown when nrhs grows). */
imq_status imq_evaluate(imq_tree tree, int nrhs, imq_dtype dtype, const void *lambda, int64_t ldl, void *s,
                        int64_t lds, imq_prec prec, hipStream_t stream);

typedef struct {
    double tol;        /* stop when ||f - A~ a|| <= tol ||f||, A~ the FP64
                          fast product (below)                              */
    int restart;       /* GMRES restart length m (1 .. 4096)                */
    int max_iters;     /* cap on inner iterations summed over everything     */
    int mixed_ir;      /* 1: FP32 inner GMRES inside FP64 refinement         */
    int max_outer;     /* cap on refinement steps (mixed_ir only; 0 = 10)    */
    double *history;   /* host, optional (NULL: none): nrhs x max_iters
                          entries; entry r*max_iters + k is column r's GMRES
                          residual estimate |g_(k+1)| / ||f|| after its
                          inner iteration k, f the system of that iteration
                          (the refinement's correction systems in mixed_ir);
                          entries from stats[r].iters on are zero          */
    int precond;       /* 0: none; 1: leaf block-Jacobi on the right,
                          A M^-1 y = f, a = M^-1 y, M = blockdiag(A_bb)
                          over runs of at most 64 points of each leaf (the
                          structure-based preconditioning the paper leaves
                          for future work, Sec. 4).  Built on the first
                          preconditioned solve and kept in the tree: FP64
                          inverses, sum of n_b^2 doubles.                   */
} imq_solve_opts;

typedef struct {        /* host */
    int iters;          /* inner GMRES iterations (matrix products)          */
    int outer_iters;    /* refinement steps (1 without mixed_ir)             */
    int converged;      /* 1 if relres_fast64 <= tol                         */
    double relres_fast64; /* final explicit ||f - A~ a|| / ||f||: the residual
                           of the system the solver solves, whose operator A~
                           is the FP64 fast product of the tree as configured
                           (order, per-level orders).  It is not the residual
                           with the exact A: that differs by (A - A~) a,
                           which grows with ||a|| and can be far above tol on
                           ill-conditioned systems; imq_rows_exact gives
                           exact rows to measure it.                        */
} imq_solve_stats;

/* Solve A a = f (eq. interp_system) by restarted GMRES on the fast product,
 * all nrhs columns in one Krylov cycle: every Arnoldi step applies the
 * product to the nrhs basis vectors at once; each column has its own basis,
 * Hessenberg matrix and Givens rotations (on the device) and stops at its
 * own tolerance.
 *  f, a : FP64, nrhs columns with leading dimensions ldf, lda; `a` holds the
 *         initial guess on entry (zeros for none) and the solution on exit.
 *  stats: host array of nrhs entries, filled on return.
 * Synchronises `stream` once per restart and reads one 4-byte count per
 * Arnoldi step (one step behind the device).  Returns IMQ_ENOTCONVERGED if
 * some column stopped above tol. */
imq_status imq_solve(imq_tree tree, int nrhs, const double *f, int64_t ldf,
                     double *a, int64_t lda, const imq_solve_opts *opts,
                     imq_solve_stats *stats, hipStream_t stream);

/* Adjoint of B = A(c, X) V (nrhs columns b_r = A v_r) for a scalar loss L
 * with upstream gradients g_r = dL/db_r.  Derivatives of the entries of
 * eq. IMQ_def:
 *   dv_r  = A g_r                                (A is symmetric)
 *   dc[s] = sum_r sum_ij g_ri v_rj dA_ij/dc,  dA_ij/dc = -c (r_ij^2 + c^2)^(-3/2)
 *   dxy   = sum_r d/dx_k of sum_ij g_ri A_ij v_rj
 *         = -sum_r sum_j (g_rk v_rj + v_rk g_rj)(x_k - x_j)(r_kj^2 + c^2)^(-3/2)
 * for every set s.
 *  v, g : nrhs columns of length Ntot (leading dimensions ldv, ldg >= Ntot),
 *         FP64 or FP32 per `dtype`
 *  dv   : same layout with lddv, same dtype (written)
 *  dc   : device FP64, nsets entries (written, summed over the columns)
 *  dxy  : device FP64 SoA 2 x Ntot: d/dx then d/dy (written, summed over the
 *         columns)
 * The interaction lists are those of `tree`, adaptive W/X lists included
 * (an X-list leaf enters the odd local coefficients from its points, a
 * W-list box's multipole is evaluated with its derivatives at the leaf's
 * points).  The vertical derivative uses translation tables to the n+m-odd
 * local coefficients, generated on the first call.  IMQ_EINVAL for nrhs < 1,
 * a null pointer or a leading dimension below Ntot. */
imq_status imq_matvec_backward(imq_tree tree, int nrhs, imq_dtype dtype, const void *v, int64_t ldv,
                               const void *g, int64_t ldg, void *dv, int64_t lddv, double *dc,
                               double *dxy, imq_prec prec, hipStream_t stream);

/* Launch shape of the batched translations, chosen by the autotuner or by
 * hand; 0 = default.
 *  m2l_kc     : coefficients staged per M2L pipeline step (16, 32 or 64 in
 *               FP32; 16 or 32 in FP64)
 *  m2l_split  : the output rows of one M2L tile are spread over this many
 *               workgroups (1 .. 10)
 *  shift_cols : columns (box, rhs) per workgroup of the level-by-level
 *               shifts, 16 or 32 (32 only in FP32; 0 picks by level size)
 *  m2l_mode   : M2L kernel per level: 0 = operands streamed through
 *               registers where a box has at most 80 coefficients, the
 *               staged GEMM above; 1 = staged GEMM everywhere; 2 = as 0,
 *               with the FP32 products of the streamed levels taken on the
 *               BF16 matrix cores: each operand split into three BF16 parts
 *               (24 significant bits in all), six part products summed in
 *               FP32 (the FP64 product runs as 0); 3 = operands streamed
 *               through registers at every level up to 160 coefficients (p
 *               <= 16; one output row block per workgroup above 80), which
 *               the wide expansions of high orders favour on some trees and
 *               not on others (the autotuner times it).
 *               m2l_kc and m2l_split apply to the staged GEMM only.
 *  p2p_wg     : workgroups of the near-field kernel while it runs alongside
 *               the tree passes (each takes every p2p_wg-th leaf); 0 = 3072
 *  p2p_mode   : near field with one right-hand side (FP32 or FP64): 0 =
 *               vector form everywhere; 1 = matrix-core form (squared
 *               distances as a rank-4 product on the FP32 or FP64 matrix
 *               cores) for the leaves whose neighbourhood is small against
 *               c, vector form for the rest
 *  far_field  : 0 = the tree passes above (multipole shifts, translations to
 *               local expansions, local evaluation); 1 = the paper's
 *               Algorithm 1 (Sec. 2.2): the multipole of every box from its
 *               own points, evaluated directly at the points of every box of
 *               its same-level interaction (V) list, at every level, plus
 *               the direct near field.  Uniform order p on every level.  The
 *               adaptive W/X interactions must be summed directly (a tree
 *               built with a large direct_max; a uniform tree has none), else
 *               the product returns IMQ_EUNSUPPORTED. */
typedef struct {
    int m2l_kc, m2l_split;
    int shift_cols;
    int m2l_mode;
    int p2p_wg;
    int p2p_mode;
    int far_field;
} imq_kernel_config;

imq_status imq_set_kernel_config(imq_tree tree, const imq_kernel_config *cfg);

/* Change the per-level truncation of the M2L translations (and of the local
 * shifts that follow them) on an existing tree: orders[l] for l < nlevels
 * (levels beyond are left as they are), each in [1, order_p] or 0 for
 * order_p.  The truncated translation is the leading block of the full
 * table, so nothing is regenerated; the batches' sizes are re-uploaded with a
 * synchronous copy.  Multipoles stay at order_p. */
imq_status imq_set_level_orders(imq_tree tree, int nlevels, const int *orders);

typedef struct {          /* host */
    int64_t npoints, nboxes, nleaves;
    int depth;            /* deepest level present                           */
    int order_p, K;       /* truncation index and real coefficients per box  */
    int64_t p2p_pairs;    /* near-field (target, source) pairs per product   */
    int64_t m2l_pairs;    /* (target box, source box) translations           */
    int64_t m2p_evals;    /* (target point, source box) multipole evaluations */
    int64_t p2l_evals;    /* (source point, target box) local accumulations  */
    int64_t m2m_pairs, l2l_pairs;
    int nlevels;                            /* levels 0 .. nlevels-1       */
    int64_t level_boxes[IMQ_MAX_LEVELS + 1];
    int64_t level_m2l_pairs[IMQ_MAX_LEVELS + 1];
    int level_K[IMQ_MAX_LEVELS + 1];        /* translation size per level  */
    int tuned_prec;       /* build-time autotuner's precision (imq_prec), -1 if not tuned */
    double tuned_err;     /* its sampled-row relative error                  */
    double tuned_ms;      /* its measured time per product (ms)              */
} imq_tree_info;

imq_status imq_get_tree_info(imq_tree tree, imq_tree_info *info);

/* Per-stage device times of the products run on this tree since stage
 * timing was (re)started with imq_set_stage_timing(tree, 1): event pairs are
 * recorded on the product's stream around every stage (no synchronisation
 * inside the product), and imq_get_stage_times synchronises on them and
 * returns the mean per stage in ms (host array of IMQ_NSTAGES entries, stage
 * order as in imq_stage_name).  At most 256 products are recorded.  While
 * timing is on, the near field runs on the product's stream between the
 * translations and L2P instead of concurrently with the tree passes, so the
 * stage times add up to a longer product than an untimed one. */
#define IMQ_NSTAGES 10
imq_status imq_set_stage_timing(imq_tree tree, int on);
imq_status imq_get_stage_times(imq_tree tree, double *ms);
const char *imq_stage_name(int stage);

void imq_tree_free(imq_tree tree);
const char *imq_status_string(imq_status s);
const char *imq_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* IMQ_H */
