// Device-side state of a tree handle and the views handed to kernels.
#pragma once

#include "imq_internal.h"

#include <hip/hip_runtime.h>

#include <cstddef>
#include <string>
#include <vector>

namespace imq {

struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    const imq_allocator *al = nullptr;   // the allocator p came from (null: hipMalloc)
    template <typename T> T *as() const { return static_cast<T *>(p); }
};

// Allocations use the allocator of the tree whose imq_ call is running on this
// thread (set on entry by every such call; null: hipMalloc).
extern thread_local const imq_allocator *g_alloc;
hipError_t dev_alloc(DevBuf &b, size_t bytes);
void dev_free(DevBuf &b);

// One leaf: its box, first and past-the-end point, level (one 16-byte load).
struct alignas(16) LeafRec {
    int box, begin, end, level;
};

// One run of the leaf block-Jacobi preconditioner: points [begin, begin + n)
// of the tree's order (within one leaf), the set, and the offset of its
// n x n inverse.
struct alignas(8) BJRun {
    int begin, n, set, pad;
    int64_t off;
};

// A box whose multipole is formed from its own points (Algorithm 1 mode):
// the leaves under it are entries [leaf0, leaf1) of the point-ordered leaf
// index list (one 16-byte load).
struct alignas(16) BoxRec {
    int box, leaf0, leaf1, level;
};

// One U-list entry of a target leaf, as the near field reads it (one 16- or
// 32-byte load): the source leaf's points [beg, beg + cnt) in sorted order and
// its centre minus the target leaf's centre, rounded to T.
template <typename T>
struct alignas(16) URec {
    int beg, cnt;
    T ox, oy;
};

// One leaf as the near field reads it (one 32-byte load): its points
// [begin, end), its U-list entries [u0, u1), c^2 of its set in the scaled
// coordinates, and whether its squared distances may be taken from the
// expansion about the leaf's centre (expand = 1).
struct alignas(16) NearLeaf {
    int begin, end, u0, u1;
    double c2;
    int expand, pad;
};

// Coefficient count of the translations at every level, by value.
struct LevelK {
    int K[32];
};

// Read-only view of the forest for kernels, in arithmetic type T.
template <typename T>
struct DTree {
    int nbox, nsets, nlev, K, P;
    int KS;                    // stride of one expansion in M and L (K rounded up to 4)
    int64_t N;
    const int32_t *level, *set, *parent, *child0, *nchild, *pos, *begin, *end;
    const double *cx, *cy;
    const int32_t *u_off, *u_idx, *v_off, *v_idx, *v_cls, *w_off, *w_idx, *x_off, *x_idx;
    const int32_t *Klev;
    const LeafRec *leafrec;    // per leaf, in the order of the leaf list
    const NearLeaf *nleaf;     // per leaf, costliest first (not the leaf-list order)
    const double *cn;          // per set: c / side
    const T *xl, *yl;          // leaf-local coordinates, sorted order
    const URec<T> *urec;       // per U-list entry (aligned with u_idx)
};

struct PrecData {              // everything that exists once per arithmetic type
    DevBuf xl, yl, wx;
    DevBuf urec;               // URec<T> per U-list entry
    DevBuf m2m, l2l;           // shift tables, 4 quadrants, packed for k_shift
    DevBuf m2l;                // translation tables, zero-padded to KP x KP each
    DevBuf m2l_pk;             // the same, packed for k_m2l_stream
    DevBuf m2l_bf3;            // FP32 only: the packed tables as three BF16 parts per entry
    DevBuf us, M, L;           // workspace
    size_t ws_nrhs = 0;
    DevBuf Lx;                 // per-pair local expansions of the X lists
    size_t lx_nrhs = 0;
    DevBuf m2l_odd, l2l_odd;   // adjoint: tables to the n+m-odd local coefficients
                               // (l2l_odd packed like l2l)
    DevBuf m2l_odd_pk;         // adjoint: m2l_odd in the streamed kernel's lane order
    DevBuf Lodd;               // adjoint: odd local coefficients
    DevBuf wxo;                // adjoint: eps_k c_{j-1,k} per odd coefficient
};

// Per row block of a packed shift table: the 16-coefficient input chunks
// [lo, hi) that hold nonzero entries (the shifts are triangular in the degree).
constexpr int SHIFT_MAXRB = 10;
struct ShiftCuts {
    int lo[SHIFT_MAXRB], hi[SHIFT_MAXRB];
};

// tabs: ntab tables of KP x KP (row-major, zero-padded); packed: same size in
// the matrix-core lane order of k_shift.
void pack_shift_tables(const std::vector<double> &tabs, int KP, std::vector<double> &packed, ShiftCuts &cuts);

// One level of shifts.  up: out[par] = sum_q T_q in[kids_q]; else
// out[kids_q] += T_q in[par].  par/kids: npar parents and their 4 children
// (-1 = none); columns are (box, rhs) with box-major layout and leading
// dimensions ldin/ldout; cols = 0 (automatic), 16 or 32 (tile width).
template <typename T>
void launch_shift(hipStream_t s, bool up, int cols, int npar, int nrhs, const int32_t *par,
                  const int32_t *kids, const T *Apk, int KP, int kin, int kout, const ShiftCuts &cuts,
                  const T *in, int ldin, T *out, int ldout);

// Near field of every leaf (grid-stride over the nleaves leaves with `grid`
// workgroups): bs[r N + i] = sum over the U list of the kernel times us, in
// sorted order, for nrhs right-hand sides.  SIDE tells apart in profiles the
// launch beside the tree passes (true) from the one on the caller's stream.
// mf: FP32 leaves flagged in v.nleaf take the matrix-core form (one
// right-hand side only).
template <typename T, bool SIDE>
void launch_p2p(hipStream_t s, unsigned grid, const DTree<T> &v, int nleaves, const T *us, int nrhs, double *bs,
                bool mf);


// Expansion-to-local translations of tasks [task0, task0 + ntask), operands
// streamed through registers class by class (acc: added to out, else stored);
// for coefficient counts up to kmax <= 80, else launches nothing and returns
// false.
// Leaf block-Jacobi preconditioner: its runs and inverses (once per tree),
// and out = M^-1 in for nrhs columns of length N in the tree's point order.
imq_status precond_setup(imq_tree_s *t, hipStream_t s);
template <typename V>
imq_status precond_apply(imq_tree_s *t, int nrhs, const V *in, V *out, hipStream_t s);

// Abf (FP32 only, else null): the tables as three BF16 parts per entry, read
// by the BF16 matrix-core form instead of Apk.  kout_ovr > 0: output rows per
// box (tables with another output layout), else the tasks' own.
template <typename T>
bool launch_m2l_stream(hipStream_t s, int acc, int kmax, int ntask, int task0, int nrhs, const GemmTask *tasks,
                       const int32_t *tbox, const int32_t *tab, const int32_t *src, const T *Apk,
                       const uint16_t *Abf, int KP, int KS, const T *in, T *out, int kout_ovr = 0);
// Batched translation GEMM (fmm.hip); kc = staged coefficients per step.
template <typename T>
void launch_gemm(hipStream_t s, int kc, int split, int ntask, int nrhs, const GemmTask *tasks, int t0,
                 const int32_t *tbox, const int32_t *tab, const int32_t *src, const T *tables, int KP, int KS,
                 const T *in, T *out, int acc, int kin_ovr, int kout_ovr);

// Caller-order vectors for the kernels that read the weights or write the
// result directly (the overlapped product skips the separate gather into
// Morton order on its critical path, and the scatter): element (r, i) of the
// sorted order is v[r * ld + perm[i]], FP32 or FP64.
struct UserVec {
    const void *in = nullptr;    // weights u (null: read the gathered copy)
    void *out = nullptr;         // result b (null: leave it in bs)
    int64_t ldu = 0, ldb = 0;
    int f32 = 0;
    const int32_t *perm = nullptr;
    const double *scale = nullptr;   // 1/side per sorted point
    __device__ __forceinline__ double get(int r, int i) const
    {
        const int64_t j = r * ldu + perm[i];
        return f32 ? double(static_cast<const float *>(in)[j]) : static_cast<const double *>(in)[j];
    }
    __device__ __forceinline__ void put(int r, int i, double v) const
    {
        const int64_t j = r * ldb + perm[i];
        v *= scale[i];
        if (f32) static_cast<float *>(out)[j] = float(v);
        else static_cast<double *>(out)[j] = v;
    }
};

// The tree passes (gather, P2M, the shifts, the translations, L2P, M2P,
// scatter) form a chain of dependent launches; the near field runs beside
// them as independent bulk work.  Their waves take a higher issue priority
// than the near field's on a shared SIMD, so the chain advances as soon as
// its waves are ready (the wave's own priority, not the queue's).
__device__ __forceinline__ void tree_pass_priority() { __builtin_amdgcn_s_setprio(2); }

// Workgroups of the near field while it runs beside the tree passes (each
// walks every P2P_WG_DEFAULT-th leaf); twelve per CU measured best on the
// clustered 1M-point product, the autotuner searches around it.
constexpr int P2P_WG_DEFAULT = 3072;

struct DevGemm {               // device copy of a GemmList
    DevBuf tasks, tbox, tab, src;
    std::vector<int32_t> level_task_begin;
    int ntasks = 0;
};

}  // namespace imq

struct imq_tree_s {
    imq::HostTree h;
    int device = 0;
    // topology (shared by both precisions)
    imq::DevBuf perm, pt_scale, level, set, parent, child0, nchild, pos, begin, end, cx, cy;
    imq::DevBuf u_off, u_idx, v_off, v_idx, v_cls, w_off, w_idx, x_off, x_idx, Klev, cn, leaves;
    imq::DevBuf xy_user, set_off;          // caller-order FP64 copy, for exact rows
    imq::DevBuf leafrec;                   // LeafRec per leaf
    int max_leaf = 0;                      // most points in one leaf
    int nnear = 0;                         // near-field leaf records (empty ones included)
    imq::DevBuf boxrec;                    // BoxRec per box at levels >= need_m (Algorithm 1 mode)
    imq::DevBuf boxleaf;                   // leaf-list indices in point order (BoxRec ranges)
    int nboxrec = 0;
    imq::DevBuf nleaf;                     // NearLeaf per leaf, costliest first
    imq::PrecData f64, f32;
    imq::DevGemm g_m2l;
    imq::DevBuf sh_par, sh_kids;           // shift lists (HostTree::sh_*)
    imq::ShiftCuts cut_m2m = {}, cut_l2l = {}, cut_l2l_odd = {};
    imq_kernel_config kcfg = {};
    imq_allocator alloc = {};              // the caller's allocator, if alloc.alloc is set
    const imq_allocator *allocator() const { return alloc.alloc ? &alloc : nullptr; }
    int KP = 0;                            // K rounded up to the MFMA tile (16)
    imq::DevBuf bs;                        // FP64 result accumulator, sorted order
    size_t bs_nrhs = 0;
    // W and X lists as pairs: target of every pair, per-pair scratch offsets,
    // and the boxes that own at least one pair
    imq::DevBuf w_tgt, w_scr, w_leaves, x_tgt, x_boxes, Pw;
    int nwpairs = 0, nwleaves = 0, nwscr = 0, nxpairs = 0, nxboxes = 0;
    // extra streams: side[0] runs the near field alongside the tree passes,
    // side[1..] run translation levels concurrently (with the caller's stream
    // that makes 4 streams, the hardware queues a process gets by default)
    static constexpr int NSIDE = 3;
    hipStream_t side[NSIDE] = {};
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;          // near field
    hipEvent_t ev_tfork = nullptr, ev_tjoin[NSIDE] = {};      // translations
    hipEvent_t ev_start = nullptr, ev_prep = nullptr;         // gathered weights; L cleared + X lists added
    static constexpr int NGROUP_EV = 32;                      // M2L level groups done (the L2L chain waits)
    hipEvent_t ev_grp[NGROUP_EV] = {};
    imq_status ensure_side();
    // result of the build-time autotuner (tuned_prec < 0: not tuned)
    int tuned_prec = -1;
    double tuned_err = 0.0, tuned_ms = 0.0;
    // evaluation tree (imq_build_eval_tree): data sites, evaluation points,
    // per evaluation point the tree point it reads, and the product's workspace
    int64_t eval_n = -1, eval_m = 0;
    imq::DevBuf eval_map, eval_u, eval_b;
    // solver workspace
    imq::DevBuf sol;
    size_t sol_bytes = 0;
    // leaf block-Jacobi preconditioner (built on the first preconditioned solve)
    imq::DevBuf bj_runs, bj_inv;
    int nbj = 0;
    // adjoint: per-point fields and partial sums; odd tables generated on first use
    imq::DevBuf adj;
    bool odd_ready = false;
    // stage timing: one set of IMQ_NSTAGES+1 events per recorded product,
    // read back (and summed) only when the caller asks for the times
    static constexpr int TIMING_RING = 256;
    bool timing = false;
    std::vector<hipEvent_t> ev;          // TIMING_RING * (IMQ_NSTAGES + 1)
    int ev_used = 0;                     // products recorded since the last reset
    hipEvent_t *stage_events();          // events of the product being launched, or null
};

namespace imq {
template <typename T> DTree<T> make_view(const imq_tree_s *t);
template <typename T> PrecData &prec_data(imq_tree_s *t);

// FP64 or FP32 fast product on sorted, already-gathered vectors:
// us (T, nrhs x N) -> bs (FP64, nrhs x N) in normalised units.
template <typename T>
imq_status fmm_sorted(imq_tree_s *t, int nrhs, hipStream_t s, const UserVec *io = nullptr);

template <typename T>
imq_status ensure_workspace(imq_tree_s *t, int nrhs);

// Every M2L table of a built tree (four layouts, both precisions) generated
// on the device; KP = the padded table edge.
imq_status make_m2l_tables_device(imq_tree_s *t, int KP);
// The build-time autotuner (tune.hip): orders, precision and kernels of a
// built, registered tree for a sampled-row relative error <= tol.
imq_status autotune_tree(imq_tree_s *t, double tol, hipStream_t s);

// Device buffers that receive a build's per-point arrays in tree order:
// the permutation (int32), the leaf-local coordinates and the scale 1/side
// (double); and the near field's U-list records (URec<double>, URec<float>).
struct DeviceKeep {
    DevBuf *perm, *xl, *yl, *scale, *urec64, *urec32;
};
// The host build's tree (build_host_tree) computed on the device from device
// coordinates; synchronises `s`.  With keep the per-point arrays stay on the
// device (and are not copied into t).
imq_status build_device_tree(int nsets, const int64_t *off, const double *xy, const double *c,
                             const imq_tree_params &prm, hipStream_t s, HostTree &t,
                             const DeviceKeep *keep = nullptr);
}  // namespace imq

#define IMQ_HIP(call)                                                                 \
    do {                                                                              \
        hipError_t e_ = (call);                                                       \
        if (e_ != hipSuccess) {                                                       \
            imq::set_error(std::string(#call) + ": " + hipGetErrorString(e_));        \
            return e_ == hipErrorOutOfMemory ? IMQ_ENOMEM : IMQ_EHIP;                 \
        }                                                                             \
    } while (0)
