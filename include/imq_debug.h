/*
 * imq_debug.h -- host-only inspection hooks of the IMQ library.
 *
 * These make no HIP call, so a test-suite can check the host logic (the
 * quadtree, its interaction lists and the FP64 translation tables) on a
 * machine without a GPU.  They are not part of the product path.
 */
#ifndef IMQ_DEBUG_H
#define IMQ_DEBUG_H

#include <stdint.h>
#include "imq.h"

#ifdef __cplusplus
extern "C" {
#endif

/* One translation table as a row-major K x K real matrix, K = (p+1)(p+2)/2,
 * in the stored n+m-even coefficient layout (host buffer `out`).
 *  kind 0: child -> parent multipole shift for child position `pos`
 *  kind 1: parent -> child local shift for child position `pos`
 *  kind 2: multipole -> local translation at `level` between boxes (dx, dy)
 *          edges apart, lifted planes c' = cnorm apart (units of the root)
 *  kind 3: the K per-coefficient constants of the point evaluations
 *  kind 4: as kind 2, to the p(p+1)/2 n+m-odd local coefficients that give
 *          the vertical derivative at the target plane (first rows of K x K)
 *  kind 5: parent -> child shift of those odd coefficients (leading block)
 * Returns 0, or -1 for a bad argument. */
int imq_debug_table(int kind, int p, int pos, int level, int dx, int dy, double cnorm, double *out);

/* Build the host part of a tree from HOST coordinates (x[N], y[N]); returns
 * an opaque handle or NULL (then *status holds the reason). */
void *imq_debug_host_tree(int nsets, const int64_t *set_offsets, const double *x, const double *y,
                          const double *c, const imq_tree_params *prm, int *status);

/* Number of elements of a named array of the host tree, or -1: "perm",
 * "xl", "yl", "level", "set", "ix", "iy", "parent", "child0", "nchild",
 * "pos", "begin", "end", "isleaf", "cx", "cy", "level_begin", "leaves",
 * "u_off", "u_idx", "v_off", "v_idx", "v_cls", "w_off", "w_idx", "x_off",
 * "x_idx", "Klev", "side", "cn", "sh_par", "sh_kids", "sh_level_begin",
 * "near_expand", "pt_scale", "pt_leaf", "lox", "loy". */
int64_t imq_debug_host_tree_size(void *h, const char *what);

/* Copy a named array into `out` (host, large enough); returns 0 or -1. */
int imq_debug_host_tree_get(void *h, const char *what, void *out);

void imq_debug_host_tree_free(void *h);

/* The M2L table (set, level, displacement class) of a tree as the
 * translation kernels read it: layout 0 = FP64 row-major KP x KP, 1 = FP64
 * in the streaming kernel's lane order, 2 and 3 the same in FP32; copied
 * into `out` (host, KP*KP elements).  Returns KP, or -1. */
int imq_debug_tree_table(imq_tree t, int set, int level, int cls, int layout, void *out);

/* The same tree built by the device construction (needs a GPU) from HOST
 * coordinates copied to the device: a handle for the getters above (free it
 * with imq_debug_host_tree_free), or NULL with *status set. */
void *imq_debug_device_tree(int nsets, const int64_t *set_offsets, const double *x, const double *y,
                            const double *c, const imq_tree_params *prm, int *status);

/* The point list of an evaluation tree (host arrays): data sites xs, ys (n)
 * and evaluation points xt, yt (m); writes map[k] for k < m (the index, in
 * the tree's point list, of the point evaluation point k takes its value
 * from) and returns the number of points in the tree, or a negative
 * imq_status (IMQ_EINVAL, IMQ_EDUPLICATE). */
int64_t imq_debug_eval_points(int64_t n, const double *xs, const double *ys, int64_t m, const double *xt,
                              const double *yt, int64_t *map);

#ifdef __cplusplus
}
#endif
#endif /* IMQ_DEBUG_H */
