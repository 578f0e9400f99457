// Internal declarations of the IMQ fast-product library (not installed).
//
// Geometry.  Every point set is mapped to the unit square by
// x' = (x - lo) / side with `side` the edge of its bounding square, so box
// sizes are exact powers of two and box centres exact dyadic numbers.  In
// these units the kernel is phi'(r') = 1/sqrt(r'^2 + c'^2), c' = c/side, and
// A = A' / side.  Points are stored in Morton order, with coordinates
// relative to the centre of their own leaf, so that differences between
// nearby points keep full relative precision in FP32.
//
// Expansions (Sec. 2.1-2.2).  Sources sit in the plane z = -c/2 and targets
// in z = +c/2 (eq. G_eq_phi).  Relative to a centre in its own plane every
// point has cos(theta) = 0, where the associated Legendre function
// P_n^m(0) vanishes unless n + m is even; multipole and local expansions
// therefore only carry the n+m-even terms, exactly K = (p+1)(p+2)/2 real
// numbers per box.  Real layout, degree by degree (n = 0..p), m ascending
// over the values with n+m even, real part then imaginary part (m > 0):
//     idx(n, m) = n(n+1)/2 + max(m-1, 0)      (prefix of length K(p') for p' < p)
// Stored quantities (w = (x - z)/s in complex form, s = box edge):
//     multipole  Mt[n,m] = sum_j u_j |w_j|^(n-m) conj(w_j)^m
//     local      Lt[n,m]  with  potential(x) = sum Re(Lt[n,m] |w|^(n-m) w^m)
// All normalisation constants of the spectral series live in the FP64
// translation tables.
#pragma once

#include "../../include/imq.h"

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

namespace imq {

constexpr int PMAX = 16;
constexpr int KMAX = (PMAX + 1) * (PMAX + 2) / 2;
constexpr int NCLASS = 49;            // displacement (dx, dy) in [-3, 3]^2
constexpr int MORTON_BITS = 30;       // bits per coordinate -> depth <= 30

inline int Kof(int p) { return (p + 1) * (p + 2) / 2; }
inline int class_of(int dx, int dy) { return (dx + 3) * 7 + (dy + 3); }

void set_error(const std::string &msg);

// ------------------------------------------------------------------ tables
// Real K x K matrices (row-major, row = output coefficient) in FP64.
// m2m/l2l: one per child position (bit 0: x half, bit 1: y half), level
// independent in box-size units.  m2l: translation from a source box to a
// target box of the same level at in-plane offset (dx, dy) boxes, with the
// lifted vertical offset c' (normalised), already including the 1/s factor
// of the level.  wx: per-coefficient constants eps_m * P_n^m(0)/(n+m)! used by
// the multipole-to-point and point-to-local evaluations.
void make_m2m_table(int p, int pos, double *T);
void make_l2l_table(int p, int pos, double *T);
void make_m2l_table(int p, int level, int dx, int dy, double cnorm, double *T);
void make_wx_consts(int p, double *w);
// n+m-odd local coefficients (vertical derivative at the target plane):
// translation with the same inputs as make_m2l_table (already including the
// 1/s^2 of the level), and the parent -> child shift of odd coefficients.
void make_m2l_odd_table(int p, int level, int dx, int dy, double cnorm, double *T);
void make_l2l_odd_table(int p, int pos, double *T);
inline int Kodd(int p) { return p * (p + 1) / 2; }
double legendre_at_zero(int n, int m);     // P_n^m(0), Condon-Shortley sign
double legendre_coef(int n, int m);        // P_n^m(0) / (n+m)!

// ------------------------------------------------------------------ tree

// A batch of the dense translations y[:, t] (+)= sum_s T_s x[:, src(t, s)]
// for up to GEMM_TILE target boxes t that share every slot's table T_s
// (same set, level and child position).  Columns are (box, right-hand side)
// pairs; one task is one workgroup's tile.
constexpr int GEMM_TILE = 64;
constexpr int GEMM_MAXSLOT = 27;  // V-list classes per child position
struct GemmTask {
    int32_t box0;     // first target in GemmList::tbox
    int32_t nbox;     // targets in this task (<= GEMM_TILE)
    int32_t nslot;    // source slots per target
    int32_t kin;      // coefficients read from each source
    int32_t kout;     // coefficients written to each target
    int32_t tab0;     // first table index in GemmList::tab (nslot entries)
    int32_t src0;     // first source in GemmList::src (nbox * nslot entries, -1 = none)
    int32_t level;    // level of the targets
};

struct GemmList {
    std::vector<GemmTask> tasks;
    std::vector<int32_t> tbox, tab, src;
    std::vector<int32_t> level_task_begin;   // tasks of level l: [begin[l], begin[l+1])
};

// Stride of one expansion in the M and L arrays: K rounded up to 4, so that
// every expansion starts on a 16-byte (FP32) or 32-byte (FP64) boundary.
inline int coef_stride(int K) { return (K + 3) & ~3; }

struct HostTree;
void build_gemm_lists(HostTree &t);

struct HostTree {
    int nsets = 0;
    int64_t N = 0;
    int p = 0, K = 0;
    int nlev = 0;                            // levels 0..nlev-1 present
    std::vector<int64_t> set_off;
    std::vector<double> c, side, lox, loy, cn;
    std::vector<int> Klev;                   // M2L order per level (K units)

    std::vector<int32_t> perm;               // sorted index -> caller index
    std::vector<double> xl, yl;              // leaf-local coordinates
    std::vector<double> pt_scale;            // 1/side of the point's set
    std::vector<int32_t> pt_leaf;            // leaf box of each sorted point

    // boxes in (level, set, Morton) order
    std::vector<int32_t> level, set, ix, iy, parent, child0, nchild, pos, begin, end, isleaf;
    std::vector<double> cx, cy;
    std::vector<int32_t> level_begin;        // nlev + 1
    std::vector<int32_t> leaves;

    // interaction lists, CSR over boxes
    std::vector<int32_t> u_off, u_idx;       // near field (leaves)
    std::vector<int32_t> v_off, v_idx, v_cls; // same-level translations
    std::vector<int32_t> w_off, w_idx;       // multipole -> target points (leaves)
    std::vector<int32_t> x_off, x_idx;       // source points -> local
    // per leaf (leaf-list order): 1 if its near field may form the squared
    // distances from the expansion about the leaf's centre (see tree.cpp)
    std::vector<int32_t> near_expand;

    // expansion-to-local batches (targets = boxes with a V list); tables are
    // indexed (set*nlev + level)*NCLASS + class
    GemmList m2l;

    // level-by-level shifts: every box with children, level by level, and its
    // child at each of the four positions (-1 if that quadrant is empty)
    std::vector<int32_t> sh_par, sh_kids;    // kids: 4 per parent
    std::vector<int32_t> sh_level_begin;     // nlev + 1, into sh_par
    // shallowest level whose multipoles are read (V, W lists) and whose local
    // expansions are written (V, X lists); shifts above them move nothing used
    int need_m = 0, need_l = 0;

    int64_t p2p_pairs = 0, m2l_pairs = 0, m2p_evals = 0, p2l_evals = 0;
    int64_t m2m_pairs = 0, l2l_pairs = 0;
};

// Points of an evaluation tree: the n data sites (xs, ys), then each of the m
// evaluation points (xt, yt) that coincides with no earlier point, data site
// or evaluation point (-0 and +0 coincide); map[k] is the index, in that
// list, of the point whose value evaluation point k takes.  Returns IMQ_OK,
// IMQ_EINVAL (a coordinate not finite) or IMQ_EDUPLICATE (two data sites
// coincide).
imq_status eval_points(int64_t n, const double *xs, const double *ys, int64_t m, const double *xt,
                       const double *yt, std::vector<double> &x, std::vector<double> &y,
                       std::vector<int64_t> &map);

// Argument checks shared by the host and device builds.
imq_status check_tree_params(int nsets, const int64_t *set_offsets, const double *c, const imq_tree_params &prm);
// Translation batches, shift lists, near-field flags and work counts of a
// tree whose boxes, points and lists are built.  leaf_r2: per leaf (in the
// order of t.leaves) the largest squared distance of its points from the
// leaf's centre; null: computed from t.xl and t.yl.
imq_status finish_host_tree(HostTree &t, const std::vector<double> *leaf_r2 = nullptr);

// Returns IMQ_OK, IMQ_EINVAL or IMQ_EDUPLICATE.
imq_status build_host_tree(int nsets, const int64_t *set_offsets, const double *x,
                           const double *y, const double *c, const imq_tree_params &prm,
                           HostTree &t);

}  // namespace imq
