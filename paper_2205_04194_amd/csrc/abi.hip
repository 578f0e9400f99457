// C entry points: argument checks, tree upload, dispatch by precision.
#include "device.h"
#include "../../include/imq_debug.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <future>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_set>
#include <vector>

namespace imq {

static thread_local std::string g_last_error;
void set_error(const std::string &msg) { g_last_error = msg; }

template <typename T, typename Tio>
imq_status matvec_typed(imq_tree_s *t, int nrhs, const Tio *u, int64_t ldu, Tio *b, int64_t ldb,
                        hipStream_t s);
imq_status rows_exact(imq_tree_s *t, int nrhs, const double *u, int64_t ldu, int64_t nrows,
                      const int64_t *rows, double *b, int64_t ldb, hipStream_t s);
imq_status solve_batched(imq_tree_s *t, int nrhs, const double *f_user, int64_t ldf, double *a_user, int64_t lda,
                         const imq_solve_opts &o, imq_solve_stats *stats, hipStream_t s);
imq_status matvec_noalloc(imq_tree_s *t, int nrhs, imq_dtype dtype, const void *u, int64_t ldu, void *b,
                          int64_t ldb, imq_prec prec, hipStream_t s);
size_t noalloc_scratch_bytes();
template <typename T, typename Tio>
imq_status backward_typed(imq_tree_s *t, const Tio *v, const Tio *g, Tio *dv, double *dc, double *dxy,
                          int accumulate, hipStream_t s);

template <typename V>
static imq_status upload(DevBuf &d, const std::vector<V> &h)
{
    IMQ_HIP(dev_alloc(d, sizeof(V) * h.size()));
    if (!h.empty()) IMQ_HIP(hipMemcpy(d.p, h.data(), sizeof(V) * h.size(), hipMemcpyHostToDevice));
    return IMQ_OK;
}

template <typename V>
static std::vector<float> to_f32(const std::vector<V> &v)
{
    std::vector<float> o(v.size());
    for (size_t i = 0; i < v.size(); ++i) o[i] = float(v[i]);
    return o;
}

// All translation tables of a tree, generated in FP64 on the host.
static void make_tables(const HostTree &h, std::vector<double> &m2m, std::vector<double> &l2l,
                        std::vector<double> &wx)
{
    const int K = h.K, p = h.p;
    const size_t KK = size_t(K) * K;
    m2m.assign(4 * KK, 0.0);
    l2l.assign(4 * KK, 0.0);
    for (int pos = 0; pos < 4; ++pos) {
        make_m2m_table(p, pos, m2m.data() + pos * KK);
        make_l2l_table(p, pos, l2l.data() + pos * KK);
    }
    wx.assign(K, 0.0);
    make_wx_consts(p, wx.data());
}

// The near field's per-leaf records (the expansion flag comes from the host
// tree), arranged for the eight XCDs.  The workgroups of a launch are dealt
// to the XCDs in turn, so with a grid that is a multiple of 8 the records at
// slots r, r + 8, r + 16, ... are all summed on XCD r.  The leaves in point
// (Morton) order are cut into 8 runs of about equal cost (targets x U-list
// sources); run r takes the slots of XCD r, largest leaf first (the tail is
// made of cheap leaves), and empty records pad the shorter runs.  An XCD's
// sources then come from one region of the plane and stay in its L2, instead
// of every XCD reading the whole point set.
static std::vector<NearLeaf> near_leaves(const HostTree &h)
{
    const size_t n = h.leaves.size();
    std::vector<NearLeaf> nl(n);
    std::vector<int64_t> cost(n);
    int64_t total = 0;
    for (size_t l = 0; l < n; ++l) {
        const int b = h.leaves[l];
        const double cn = h.cn[h.set[b]];
        nl[l] = NearLeaf{h.begin[b], h.end[b], h.u_off[b], h.u_off[b + 1], cn * cn, h.near_expand[l], 0};
        int64_t src = 0;
        for (int u = nl[l].u0; u < nl[l].u1; ++u) src += h.end[h.u_idx[u]] - h.begin[h.u_idx[u]];
        cost[l] = src * (nl[l].end - nl[l].begin);
        total += cost[l];
    }
    std::vector<size_t> ord(n);
    for (size_t l = 0; l < n; ++l) ord[l] = l;
    std::stable_sort(ord.begin(), ord.end(), [&](size_t a, size_t b) { return nl[a].begin < nl[b].begin; });
    constexpr int NX = 8;
    std::vector<size_t> run[NX];
    int64_t acc = 0;
    for (size_t k : ord) {
        // the run that holds the middle of this leaf's share of the cost
        const double mid = total > 0 ? (double(acc) + 0.5 * double(cost[k])) / double(total) : 0.0;
        run[std::min(NX - 1, int(mid * NX))].push_back(k);
        acc += cost[k];
    }
    size_t most = 0;
    for (auto &r : run) {
        std::stable_sort(r.begin(), r.end(), [&](size_t a, size_t b) { return cost[a] > cost[b]; });
        most = std::max(most, r.size());
    }
    std::vector<NearLeaf> out(NX * most, NearLeaf{0, 0, 0, 0, 1.0, 0, 0});
    for (int r = 0; r < NX; ++r)
        for (size_t j = 0; j < run[r].size(); ++j) out[NX * j + r] = nl[run[r][j]];
    return out;
}

__global__ void k_to_f32(int64_t n, const double *__restrict__ a, float *__restrict__ o)
{
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) o[i] = float(a[i]);
}

// The tree's device arrays from its host build; the per-point arrays (perm,
// scale, FP64 leaf-local coordinates) are already on the device.
static imq_status upload_tree(imq_tree_s *t, const double *xy_dev)
{
    const HostTree &h = t->h;
    imq_status st;
    // the near field's leaf order (costs and a sort) on a second thread (on
    // this one, when it is needed, where no thread can be started)
    std::future<std::vector<NearLeaf>> nleaf;
    try {
        nleaf = std::async(std::launch::async, [&h] { return near_leaves(h); });
    } catch (const std::exception &) {
        nleaf = std::async(std::launch::deferred, [&h] { return near_leaves(h); });
    }
#define UP(field) if ((st = upload(t->field, h.field)) != IMQ_OK) return st
    UP(level); UP(set); UP(parent); UP(child0); UP(nchild); UP(pos);
    UP(begin); UP(end); UP(cx); UP(cy); UP(u_off); UP(u_idx); UP(v_off); UP(v_idx); UP(v_cls);
    UP(w_off); UP(w_idx); UP(x_off); UP(x_idx); UP(Klev); UP(leaves);
#undef UP
    {   // leaf records
        std::vector<LeafRec> lr(h.leaves.size());
        for (size_t i = 0; i < lr.size(); ++i) {
            const int b = h.leaves[i];
            lr[i] = LeafRec{b, h.begin[b], h.end[b], h.level[b]};
            t->max_leaf = std::max(t->max_leaf, h.end[b] - h.begin[b]);
        }
        if ((st = upload(t->leafrec, lr)) != IMQ_OK) return st;
        // every box that can be a V-list source, with the leaves under it: a
        // contiguous range of the leaves in point order
        std::vector<int32_t> lord(lr.size()), lbeg(lr.size());
        for (size_t i = 0; i < lr.size(); ++i) lord[i] = int32_t(i);
        std::sort(lord.begin(), lord.end(), [&](int32_t a, int32_t b) { return lr[a].begin < lr[b].begin; });
        for (size_t i = 0; i < lr.size(); ++i) lbeg[i] = lr[lord[i]].begin;
        if ((st = upload(t->boxleaf, lord)) != IMQ_OK) return st;
        // first leaf at or after a point: a forward scan while the queries
        // ascend (boxes of a level come in point order), else a binary search
        size_t at = 0;
        auto first_leaf = [&](int32_t v) -> int {
            if (at > 0 && lbeg[at - 1] >= v) at = size_t(std::lower_bound(lbeg.begin(), lbeg.end(), v) - lbeg.begin());
            while (at < lbeg.size() && lbeg[at] < v) ++at;
            return int(at);
        };
        std::vector<BoxRec> br;
        br.reserve(h.level.size());
        for (int b = 0; b < int(h.level.size()); ++b) {
            if (h.level[b] < h.need_m) continue;
            const int l0 = first_leaf(h.begin[b]);
            const int l1 = first_leaf(h.end[b]);
            br.push_back(BoxRec{b, l0, l1, h.level[b]});
        }
        if ((st = upload(t->boxrec, br)) != IMQ_OK) return st;
        t->nboxrec = int(br.size());
        const std::vector<NearLeaf> recs = nleaf.get();
        t->nnear = int(recs.size());
        if ((st = upload(t->nleaf, recs)) != IMQ_OK) return st;
    }
    {   // W and X lists as flat pairs
        std::vector<int32_t> w_tgt, w_scr, w_leaves, x_tgt, x_boxes;
        int32_t scr = 0;
        const int nbox = int(h.level.size());
        for (int b = 0; b < nbox; ++b) {
            if (h.w_off[b + 1] > h.w_off[b]) w_leaves.push_back(b);
            for (int k = h.w_off[b]; k < h.w_off[b + 1]; ++k) {
                w_tgt.push_back(b);
                w_scr.push_back(scr);
                scr += h.end[b] - h.begin[b];
            }
            if (h.x_off[b + 1] > h.x_off[b]) x_boxes.push_back(b);
            for (int k = h.x_off[b]; k < h.x_off[b + 1]; ++k) x_tgt.push_back(b);
        }
        t->nwpairs = int(w_tgt.size());
        t->nwleaves = int(w_leaves.size());
        t->nwscr = scr;
        t->nxpairs = int(x_tgt.size());
        t->nxboxes = int(x_boxes.size());
        if ((st = upload(t->w_tgt, w_tgt)) != IMQ_OK) return st;
        if ((st = upload(t->w_scr, w_scr)) != IMQ_OK) return st;
        if ((st = upload(t->w_leaves, w_leaves)) != IMQ_OK) return st;
        if ((st = upload(t->x_tgt, x_tgt)) != IMQ_OK) return st;
        if ((st = upload(t->x_boxes, x_boxes)) != IMQ_OK) return st;
    }
    std::vector<double> cc(h.cn);
    cc.insert(cc.end(), h.c.begin(), h.c.end());      // [c/side per set, c per set]
    if ((st = upload(t->cn, cc)) != IMQ_OK) return st;
    if ((st = upload(t->set_off, h.set_off)) != IMQ_OK) return st;
    IMQ_HIP(dev_alloc(t->xy_user, sizeof(double) * 2 * size_t(h.N)));
    IMQ_HIP(hipMemcpy(t->xy_user.p, xy_dev, sizeof(double) * 2 * size_t(h.N), hipMemcpyDeviceToDevice));

    IMQ_HIP(dev_alloc(t->f32.xl, sizeof(float) * size_t(h.N)));
    IMQ_HIP(dev_alloc(t->f32.yl, sizeof(float) * size_t(h.N)));
    const unsigned nb = unsigned((h.N + 255) / 256);
    hipLaunchKernelGGL(k_to_f32, dim3(nb), dim3(256), 0, nullptr, h.N, t->f64.xl.as<const double>(),
                       t->f32.xl.as<float>());
    hipLaunchKernelGGL(k_to_f32, dim3(nb), dim3(256), 0, nullptr, h.N, t->f64.yl.as<const double>(),
                       t->f32.yl.as<float>());
    IMQ_HIP(hipGetLastError());
    IMQ_HIP(hipStreamSynchronize(nullptr));

    std::vector<double> m2m, l2l, wx;
    make_tables(h, m2m, l2l, wx);
    // zero-pad every K x K table to KP x KP for the MFMA tiles
    const int K = h.K, KP = (K + 15) & ~15;
    t->KP = KP;
    auto pad = [&](std::vector<double> &v) {
        const size_t n = v.size() / (size_t(K) * K);
        std::vector<double> o(n * size_t(KP) * KP, 0.0);
        for (size_t tb = 0; tb < n; ++tb)
            for (int r = 0; r < K; ++r)
                std::copy(v.begin() + (tb * K + r) * K, v.begin() + (tb * K + r + 1) * K,
                          o.begin() + (tb * KP + r) * KP);
        v.swap(o);
    };
    pad(m2m);
    pad(l2l);
    {
        std::vector<double> pk;
        pack_shift_tables(m2m, KP, pk, t->cut_m2m);
        m2m.swap(pk);
        pack_shift_tables(l2l, KP, pk, t->cut_l2l);
        l2l.swap(pk);
    }
    if ((st = make_m2l_tables_device(t, KP)) != IMQ_OK) return st;
    {
        const GemmList &g = h.m2l;
        DevGemm &d = t->g_m2l;
        if ((st = upload(d.tasks, g.tasks)) != IMQ_OK) return st;
        if ((st = upload(d.tbox, g.tbox)) != IMQ_OK) return st;
        if ((st = upload(d.tab, g.tab)) != IMQ_OK) return st;
        if ((st = upload(d.src, g.src)) != IMQ_OK) return st;
        d.level_task_begin = g.level_task_begin;
        d.ntasks = int(g.tasks.size());
    }
    if ((st = upload(t->sh_par, h.sh_par)) != IMQ_OK) return st;
    if ((st = upload(t->sh_kids, h.sh_kids)) != IMQ_OK) return st;
    if ((st = upload(t->f64.m2m, m2m)) != IMQ_OK) return st;
    if ((st = upload(t->f64.l2l, l2l)) != IMQ_OK) return st;
    if ((st = upload(t->f64.wx, wx)) != IMQ_OK) return st;
    if ((st = upload(t->f32.m2m, to_f32(m2m))) != IMQ_OK) return st;
    if ((st = upload(t->f32.l2l, to_f32(l2l))) != IMQ_OK) return st;
    if ((st = upload(t->f32.wx, to_f32(wx))) != IMQ_OK) return st;
    return IMQ_OK;
}

static void free_tree(imq_tree_s *t)
{
    if (g_alloc == &t->alloc) g_alloc = nullptr;   // never left pointing into a freed tree
    DevBuf *bufs[] = {&t->perm, &t->pt_scale, &t->level, &t->set, &t->parent, &t->child0, &t->nchild,
                      &t->pos, &t->begin, &t->end, &t->cx, &t->cy, &t->u_off, &t->u_idx, &t->v_off,
                      &t->v_idx, &t->v_cls, &t->w_off, &t->w_idx, &t->x_off, &t->x_idx, &t->Klev,
                      &t->cn, &t->leaves, &t->leafrec, &t->boxrec, &t->boxleaf, &t->nleaf, &t->xy_user, &t->set_off, &t->bs, &t->sol, &t->bj_runs, &t->bj_inv,
                      &t->w_tgt, &t->w_scr, &t->w_leaves, &t->x_tgt, &t->x_boxes, &t->Pw, &t->adj,
                      &t->sh_par, &t->sh_kids, &t->eval_map, &t->eval_u, &t->eval_b};
    for (DevBuf *b : bufs) dev_free(*b);
    for (DevGemm *g : {&t->g_m2l}) {
        dev_free(g->tasks); dev_free(g->tbox); dev_free(g->tab); dev_free(g->src);
    }
    for (PrecData *pd : {&t->f64, &t->f32}) {
        DevBuf *pb[] = {&pd->xl, &pd->yl, &pd->urec, &pd->m2m, &pd->l2l, &pd->m2l, &pd->m2l_pk, &pd->m2l_bf3, &pd->wx, &pd->us, &pd->M, &pd->L,
                        &pd->Lx, &pd->m2l_odd, &pd->l2l_odd, &pd->m2l_odd_pk, &pd->Lodd, &pd->wxo};
        for (DevBuf *b : pb) dev_free(*b);
    }
    for (auto &e : t->ev)
        if (e) (void)hipEventDestroy(e);
    for (hipStream_t &x : t->side)
        if (x) {
            (void)hipStreamSynchronize(x);
            (void)hipStreamDestroy(x);
        }
    for (hipEvent_t e : {t->ev_fork, t->ev_join, t->ev_tfork, t->ev_start, t->ev_prep})
        if (e) (void)hipEventDestroy(e);
    for (hipEvent_t e : t->ev_tjoin)
        if (e) (void)hipEventDestroy(e);
    for (hipEvent_t e : t->ev_grp)
        if (e) (void)hipEventDestroy(e);
    delete t;
}

// Handles of the trees that exist: a call on a freed handle is rejected with
// IMQ_EINVAL instead of reading freed memory (an address reused by a later
// tree is that tree's handle).
static std::mutex g_live_mu;
static std::unordered_set<const imq_tree_s *> g_live;

static void live_add(const imq_tree_s *t)
{
    std::lock_guard<std::mutex> lk(g_live_mu);
    g_live.insert(t);
}

static bool live_remove(const imq_tree_s *t)
{
    std::lock_guard<std::mutex> lk(g_live_mu);
    return g_live.erase(t) > 0;
}

static bool live_has(const imq_tree_s *t)
{
    std::lock_guard<std::mutex> lk(g_live_mu);
    return g_live.count(t) > 0;
}

// Entry of every call on a tree: checks the handle, makes the tree's device
// current and selects the tree's allocator; the caller's device is current
// again when the call returns.
struct TreeCall {
    imq_status st = IMQ_OK;
    int prev = -1;
    explicit TreeCall(imq_tree t)
    {
        if (!t) { set_error("null tree handle"); st = IMQ_EINVAL; return; }
        if (!live_has(t)) { set_error("tree handle was freed or never built"); st = IMQ_EINVAL; return; }
        g_alloc = t->allocator();                 // the tree's buffers come from its allocator
        int dev = -1;
        hipError_t e = hipGetDevice(&dev);
        if (e == hipSuccess && dev != t->device) {
            e = hipSetDevice(t->device);
            if (e == hipSuccess) prev = dev;
        }
        if (e != hipSuccess) {
            set_error(std::string("selecting the tree's device: ") + hipGetErrorString(e));
            st = IMQ_EHIP;
        }
    }
    ~TreeCall()
    {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
    TreeCall(const TreeCall &) = delete;
    TreeCall &operator=(const TreeCall &) = delete;
};

namespace {
// the product's input: the coefficients at the data sites, zero at the
// evaluation points
template <typename V>
__global__ void k_eval_in(int64_t n, int64_t N, const V *__restrict__ lam, int64_t ldl, V *__restrict__ u)
{
    const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    const int r = blockIdx.y;
    if (i < N) u[r * N + i] = i < n ? lam[r * ldl + i] : V(0);
}

template <typename V>
__global__ void k_eval_out(int64_t m, int64_t N, const int64_t *__restrict__ map, const V *__restrict__ b,
                           V *__restrict__ s, int64_t lds)
{
    const int64_t k = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    const int r = blockIdx.y;
    if (k < m) s[r * lds + k] = b[r * N + map[k]];
}

template <typename V>
imq_status evaluate_typed(imq_tree_s *t, int nrhs, const V *lam, int64_t ldl, V *s, int64_t lds, imq_prec prec,
                          hipStream_t stream)
{
    const int64_t N = t->h.N, n = t->eval_n, m = t->eval_m;
    const size_t bytes = sizeof(V) * size_t(nrhs) * size_t(N);
    if (t->eval_u.bytes < bytes) {
        dev_free(t->eval_u);
        dev_free(t->eval_b);
        IMQ_HIP(dev_alloc(t->eval_u, bytes));
        IMQ_HIP(dev_alloc(t->eval_b, bytes));
    }
    V *u = t->eval_u.as<V>(), *b = t->eval_b.as<V>();
    hipLaunchKernelGGL(k_eval_in<V>, dim3(unsigned((N + 255) / 256), nrhs), dim3(256), 0, stream, n, N, lam, ldl, u);
    IMQ_HIP(hipGetLastError());
    const imq_status st = imq_matvec(t, nrhs, sizeof(V) == 8 ? IMQ_F64 : IMQ_F32, u, N, b, N, prec, stream);
    if (st != IMQ_OK) return st;
    hipLaunchKernelGGL(k_eval_out<V>, dim3(unsigned((m + 255) / 256), nrhs), dim3(256), 0, stream, m, N,
                       t->eval_map.as<int64_t>(), b, s, lds);
    IMQ_HIP(hipGetLastError());
    return IMQ_OK;
}
}  // namespace

}  // namespace imq

using namespace imq;

hipEvent_t *imq_tree_s::stage_events()
{
    if (!timing || ev_used >= TIMING_RING || ev.empty()) return nullptr;
    return ev.data() + size_t(ev_used++) * (IMQ_NSTAGES + 1);
}

extern "C" {

const char *imq_last_error(void) { return g_last_error.c_str(); }

const char *imq_status_string(imq_status s)
{
    switch (s) {
    case IMQ_OK: return "ok";
    case IMQ_ENOTCONVERGED: return "tolerance not reached";
    case IMQ_EINVAL: return "invalid argument";
    case IMQ_EDUPLICATE: return "duplicate data sites";
    case IMQ_ENOMEM: return "out of memory";
    case IMQ_EHIP: return "HIP runtime error";
    case IMQ_EUNSUPPORTED: return "unsupported";
    }
    return "unknown status";
}

const char *imq_stage_name(int k)
{
    static const char *names[IMQ_NSTAGES] = {"gather", "p2m", "m2m", "p2l", "m2l",
                                             "l2l", "p2p", "l2p", "m2p", "scatter"};
    return (k >= 0 && k < IMQ_NSTAGES) ? names[k] : "?";
}

imq_status imq_build_tree(int nsets, const int64_t *set_offsets, const double *xy, const double *c,
                          const imq_tree_params *params, hipStream_t stream, imq_tree *out)
{
    return imq_build_tree_alloc(nsets, set_offsets, xy, c, params, nullptr, stream, out);
}

imq_status imq_build_tree_alloc(int nsets, const int64_t *set_offsets, const double *xy, const double *c,
                                const imq_tree_params *params, const imq_allocator *alloc, hipStream_t stream,
                                imq_tree *out)
{
    if (alloc && (!alloc->alloc || !alloc->free)) { set_error("allocator without alloc or free"); return IMQ_EINVAL; }
    if (!out) { set_error("out is null"); return IMQ_EINVAL; }
    *out = nullptr;
    if (nsets < 1 || !set_offsets || !xy || !c || !params) { set_error("null argument or nsets < 1"); return IMQ_EINVAL; }
    const int64_t N = set_offsets[nsets];
    if (N < 1) { set_error("no points"); return IMQ_EINVAL; }
    auto *t = new imq_tree_s();
    const hipError_t e = hipGetDevice(&t->device);
    if (e != hipSuccess) {
        delete t;
        set_error(std::string("hipGetDevice: ") + hipGetErrorString(e));
        return IMQ_EHIP;
    }
    if (alloc) t->alloc = *alloc;
    g_alloc = t->allocator();
    const DeviceKeep keep{&t->perm, &t->f64.xl, &t->f64.yl, &t->pt_scale, &t->f64.urec, &t->f32.urec};
    imq_status st = build_device_tree(nsets, set_offsets, xy, c, *params, stream, t->h, &keep);
    if (st != IMQ_OK) { free_tree(t); return st; }
    st = upload_tree(t, xy);
    if (st != IMQ_OK) { free_tree(t); return st; }
    live_add(t);
    if (params->autotune) {
        if (!(params->autotune_tol >= 0.0) || !std::isfinite(params->autotune_tol)) {
            imq_tree_free(t);
            set_error("autotune_tol must be finite and >= 0");
            return IMQ_EINVAL;
        }
        st = autotune_tree(t, params->autotune_tol > 0.0 ? params->autotune_tol : 1e-6, stream);
        if (st != IMQ_OK) {
            const std::string why = imq_last_error();
            imq_tree_free(t);
            set_error(why);
            return st;
        }
    }
    *out = t;
    return IMQ_OK;
}

imq_status imq_build_eval_tree(const double *xy_src, int64_t n, const double *xy_tgt, int64_t m, double c,
                               const imq_tree_params *params, hipStream_t stream, imq_tree *out)
{
    if (!out) { set_error("out is null"); return IMQ_EINVAL; }
    *out = nullptr;
    if (!xy_src || n < 1 || m < 0 || (m > 0 && !xy_tgt) || !params) {
        set_error("null argument, n < 1 or m < 0");
        return IMQ_EINVAL;
    }
    if (n + m > 0x7fffffff) { set_error("too many points"); return IMQ_EINVAL; }
    std::vector<double> hs(2 * size_t(n)), ht(2 * size_t(m));
    IMQ_HIP(hipMemcpyAsync(hs.data(), xy_src, sizeof(double) * hs.size(), hipMemcpyDeviceToHost, stream));
    if (m > 0) IMQ_HIP(hipMemcpyAsync(ht.data(), xy_tgt, sizeof(double) * ht.size(), hipMemcpyDeviceToHost, stream));
    IMQ_HIP(hipStreamSynchronize(stream));
    std::vector<double> x, y;
    std::vector<int64_t> map;
    imq_status st = eval_points(n, hs.data(), hs.data() + n, m, ht.data(), ht.data() + m, x, y, map);
    if (st != IMQ_OK) return st;
    const int64_t N = int64_t(x.size());
    std::vector<double> soa(x);
    soa.insert(soa.end(), y.begin(), y.end());
    DevBuf dxy;
    g_alloc = nullptr;                                    // a temporary of this call: hipMalloc
    if ((st = upload(dxy, soa)) != IMQ_OK) return st;   // the tree copies what it keeps
    const int64_t offs[2] = {0, N};
    st = imq_build_tree(1, offs, dxy.as<double>(), &c, params, stream, out);
    dev_free(dxy);
    if (st != IMQ_OK) return st;
    imq_tree t = *out;
    t->eval_n = n;
    t->eval_m = m;
    if ((st = upload(t->eval_map, map)) != IMQ_OK) {
        imq_tree_free(t);
        *out = nullptr;
        return st;
    }
    return IMQ_OK;
}


imq_status imq_evaluate(imq_tree t, int nrhs, imq_dtype dtype, const void *lambda, int64_t ldl, void *s,
                        int64_t lds, imq_prec prec, hipStream_t stream)
{
    TreeCall call(t);
    if (call.st != IMQ_OK) return call.st;
    imq_status st = IMQ_OK;
    if (t->eval_n < 0) { set_error("not an evaluation tree (imq_build_eval_tree)"); return IMQ_EINVAL; }
    if (nrhs < 1 || nrhs > 65535 || !lambda || ldl < t->eval_n || (t->eval_m > 0 && (!s || lds < t->eval_m))) {
        set_error("bad nrhs, pointer or leading dimension");
        return IMQ_EINVAL;
    }
    if (dtype != IMQ_F64 && dtype != IMQ_F32) { set_error("unknown dtype"); return IMQ_EINVAL; }
    if (prec != IMQ_PREC_FP64 && prec != IMQ_PREC_FP32) { set_error("unknown precision"); return IMQ_EINVAL; }
    if (t->eval_m == 0) return IMQ_OK;
    if (dtype == IMQ_F64)
        return evaluate_typed<double>(t, nrhs, (const double *)lambda, ldl, (double *)s, lds, prec, stream);
    return evaluate_typed<float>(t, nrhs, (const float *)lambda, ldl, (float *)s, lds, prec, stream);
}

imq_status imq_matvec(imq_tree t, int nrhs, imq_dtype dtype, const void *u, int64_t ldu, void *b,
                      int64_t ldb, imq_prec prec, hipStream_t stream)
{
    TreeCall call(t);
    if (call.st != IMQ_OK) return call.st;
    imq_status st = IMQ_OK;
    if (nrhs < 1 || !u || !b || ldu < t->h.N || ldb < t->h.N) { set_error("bad nrhs, pointer or leading dimension"); return IMQ_EINVAL; }
    if (dtype == IMQ_F64 && prec == IMQ_PREC_FP64)
        return matvec_typed<double, double>(t, nrhs, (const double *)u, ldu, (double *)b, ldb, stream);
    if (dtype == IMQ_F32 && prec == IMQ_PREC_FP64)
        return matvec_typed<double, float>(t, nrhs, (const float *)u, ldu, (float *)b, ldb, stream);
    if (dtype == IMQ_F64 && prec == IMQ_PREC_FP32)
        return matvec_typed<float, double>(t, nrhs, (const double *)u, ldu, (double *)b, ldb, stream);
    if (dtype == IMQ_F32 && prec == IMQ_PREC_FP32)
        return matvec_typed<float, float>(t, nrhs, (const float *)u, ldu, (float *)b, ldb, stream);
    set_error("unknown dtype or precision");
    return IMQ_EINVAL;
}

imq_status imq_matvec_noalloc(imq_tree t, int nrhs, imq_dtype dtype, const void *u, int64_t ldu, void *b,
                              int64_t ldb, imq_prec prec, hipStream_t stream)
{
    TreeCall call(t);
    if (call.st != IMQ_OK) return call.st;
    if (nrhs < 1 || !u || !b || ldu < t->h.N || ldb < t->h.N) {
        set_error("bad nrhs, pointer or leading dimension");
        return IMQ_EINVAL;
    }
    return matvec_noalloc(t, nrhs, dtype, u, ldu, b, ldb, prec, stream);
}

size_t imq_matvec_noalloc_max_bytes(void) { return noalloc_scratch_bytes(); }

imq_status imq_rows_exact(imq_tree t, int nrhs, const double *u, int64_t ldu, int64_t nrows,
                          const int64_t *rows, double *b, int64_t ldb, hipStream_t stream)
{
    TreeCall call(t);
    if (call.st != IMQ_OK) return call.st;
    imq_status st = IMQ_OK;
    if (nrhs < 1 || nrows < 0 || (nrows > 0 && (!u || !rows || !b)) || ldu < t->h.N || ldb < nrows) {
        set_error("bad argument to imq_rows_exact");
        return IMQ_EINVAL;
    }
    if (nrows > 0x7fffffff) { set_error("too many rows"); return IMQ_EINVAL; }
    std::vector<int64_t> hr(nrows);
    IMQ_HIP(hipMemcpyAsync(hr.data(), rows, sizeof(int64_t) * nrows, hipMemcpyDeviceToHost, stream));
    IMQ_HIP(hipStreamSynchronize(stream));
    for (int64_t r : hr)
        if (r < 0 || r >= t->h.N) { set_error("row index out of range"); return IMQ_EINVAL; }
    return rows_exact(t, nrhs, u, ldu, nrows, rows, b, ldb, stream);
}

imq_status imq_get_tree_info(imq_tree t, imq_tree_info *info)
{
    if (!info) { set_error("null argument"); return IMQ_EINVAL; }
    TreeCall call(t);
    if (call.st != IMQ_OK) return call.st;
    const HostTree &h = t->h;
    info->npoints = h.N;
    info->nboxes = int64_t(h.level.size());
    info->nleaves = int64_t(h.leaves.size());
    info->depth = h.nlev - 1;
    info->order_p = h.p;
    info->K = h.K;
    info->p2p_pairs = h.p2p_pairs;
    info->m2l_pairs = h.m2l_pairs;
    info->m2p_evals = h.m2p_evals;
    info->p2l_evals = h.p2l_evals;
    info->m2m_pairs = h.m2m_pairs;
    info->l2l_pairs = h.l2l_pairs;
    info->nlevels = h.nlev;
    for (int l = 0; l <= IMQ_MAX_LEVELS; ++l) {
        info->level_boxes[l] = 0;
        info->level_m2l_pairs[l] = 0;
        info->level_K[l] = 0;
    }
    for (int l = 0; l < h.nlev && l <= IMQ_MAX_LEVELS; ++l) {
        info->level_K[l] = h.Klev[l];
        info->level_boxes[l] = h.level_begin[l + 1] - h.level_begin[l];
        info->level_m2l_pairs[l] = h.v_off[h.level_begin[l + 1]] - h.v_off[h.level_begin[l]];
    }
    info->tuned_prec = t->tuned_prec;
    info->tuned_err = t->tuned_err;
    info->tuned_ms = t->tuned_ms;
    return IMQ_OK;
}

imq_status imq_set_kernel_config(imq_tree t, const imq_kernel_config *cfg)
{
    if (!cfg) { set_error("null argument"); return IMQ_EINVAL; }
    TreeCall call(t);
    if (call.st != IMQ_OK) return call.st;
    auto ok_kc = [](int v) { return v == 0 || v == 16 || v == 32 || v == 64; };
    if (!ok_kc(cfg->m2l_kc) || cfg->m2l_split < 0 || cfg->m2l_split > 10 ||
        (cfg->shift_cols != 0 && cfg->shift_cols != 16 && cfg->shift_cols != 32) ||
        cfg->m2l_mode < 0 || cfg->m2l_mode > 3 || cfg->p2p_wg < 0 || cfg->p2p_mode < 0 || cfg->p2p_mode > 1 ||
        cfg->far_field < 0 || cfg->far_field > 1) {
        set_error("kernel config out of range");
        return IMQ_EINVAL;
    }
    t->kcfg = *cfg;
    return IMQ_OK;
}

imq_status imq_set_level_orders(imq_tree t, int nlevels, const int *orders)
{
    TreeCall call(t);
    if (call.st != IMQ_OK) return call.st;
    imq_status st = IMQ_OK;
    if (nlevels < 0 || (nlevels > 0 && !orders)) { set_error("bad level orders"); return IMQ_EINVAL; }
    HostTree &h = t->h;
    for (int l = 0; l < nlevels && l < h.nlev; ++l)
        if (orders[l] < 0 || orders[l] > h.p) { set_error("level order out of [0, order_p]"); return IMQ_EINVAL; }
    for (int l = 0; l < nlevels && l < h.nlev; ++l) h.Klev[l] = Kof(orders[l] > 0 ? orders[l] : h.p);
    for (GemmTask &k : h.m2l.tasks) k.kin = k.kout = h.Klev[k.level];
    IMQ_HIP(hipDeviceSynchronize());
    if ((st = upload(t->Klev, h.Klev)) != IMQ_OK) return st;
    if ((st = upload(t->g_m2l.tasks, h.m2l.tasks)) != IMQ_OK) return st;
    return IMQ_OK;
}

imq_status imq_set_stage_timing(imq_tree t, int on)
{
    TreeCall call(t);
    if (call.st != IMQ_OK) return call.st;
    imq_status st = IMQ_OK;
    if (on && t->ev.empty()) {
        t->ev.assign(size_t(imq_tree_s::TIMING_RING) * (IMQ_NSTAGES + 1), nullptr);
        for (auto &e : t->ev) IMQ_HIP(hipEventCreate(&e));
    }
    t->timing = on != 0;
    t->ev_used = 0;
    return IMQ_OK;
}

imq_status imq_get_stage_times(imq_tree t, double *ms)
{
    TreeCall call(t);
    if (call.st != IMQ_OK) return call.st;
    imq_status st = IMQ_OK;
    if (!ms) { set_error("null argument"); return IMQ_EINVAL; }
    for (int k = 0; k < IMQ_NSTAGES; ++k) ms[k] = 0.0;
    const int n = t->ev_used;
    for (int r = 0; r < n; ++r) {
        hipEvent_t *e = t->ev.data() + size_t(r) * (IMQ_NSTAGES + 1);
        IMQ_HIP(hipEventSynchronize(e[IMQ_NSTAGES]));
        for (int k = 0; k < IMQ_NSTAGES; ++k) {
            float v = 0;
            IMQ_HIP(hipEventElapsedTime(&v, e[k], e[k + 1]));
            ms[k] += v / n;
        }
    }
    return IMQ_OK;
}

void imq_tree_free(imq_tree t)
{
    if (t && live_remove(t)) {
        int dev = -1;
        const bool other = hipGetDevice(&dev) == hipSuccess && dev != t->device &&
                           hipSetDevice(t->device) == hipSuccess;
        free_tree(t);
        if (other) (void)hipSetDevice(dev);
    }
}

// ------------------------------------------------------------------ host-only hooks

int imq_debug_table(int kind, int p, int pos, int level, int dx, int dy, double cnorm, double *out)
{
    if (p < 1 || p > PMAX || !out) return -1;
    switch (kind) {
    case 0: make_m2m_table(p, pos & 3, out); return 0;
    case 1: make_l2l_table(p, pos & 3, out); return 0;
    case 2: make_m2l_table(p, level, dx, dy, cnorm, out); return 0;
    case 3: make_wx_consts(p, out); return 0;
    case 4: make_m2l_odd_table(p, level, dx, dy, cnorm, out); return 0;
    case 5: make_l2l_odd_table(p, pos & 3, out); return 0;
    }
    return -1;
}

void *imq_debug_host_tree(int nsets, const int64_t *set_offsets, const double *x, const double *y,
                          const double *c, const imq_tree_params *prm, int *status)
{
    auto *h = new HostTree();
    imq_status st = build_host_tree(nsets, set_offsets, x, y, c, *prm, *h);
    if (status) *status = st;
    if (st != IMQ_OK) { delete h; return nullptr; }
    return h;
}

static const void *field(const HostTree &h, const char *w, int64_t &n, int &elem)
{
#define F(name) if (!std::strcmp(w, #name)) { n = int64_t(h.name.size()); elem = int(sizeof(h.name[0])); return h.name.data(); }
    F(perm) F(xl) F(yl) F(level) F(set) F(ix) F(iy) F(parent) F(child0) F(nchild) F(pos) F(begin)
    F(end) F(isleaf) F(cx) F(cy) F(level_begin) F(leaves) F(u_off) F(u_idx) F(v_off) F(v_idx)
    F(v_cls) F(w_off) F(w_idx) F(x_off) F(x_idx) F(Klev) F(side) F(cn) F(sh_par) F(sh_kids)
    F(sh_level_begin) F(near_expand) F(pt_scale) F(pt_leaf) F(lox) F(loy)
#undef F
    n = -1;
    elem = 0;
    return nullptr;
}

int64_t imq_debug_host_tree_size(void *hp, const char *what)
{
    int64_t n; int e;
    field(*static_cast<HostTree *>(hp), what, n, e);
    return n;
}

int imq_debug_host_tree_get(void *hp, const char *what, void *out)
{
    int64_t n; int e;
    const void *src = field(*static_cast<HostTree *>(hp), what, n, e);
    if (n < 0) return -1;
    if (n > 0) std::memcpy(out, src, size_t(n) * e);
    return 0;
}

void imq_debug_host_tree_free(void *hp) { delete static_cast<HostTree *>(hp); }

int imq_debug_tree_table(imq_tree t, int set, int level, int cls, int layout, void *out)
{
    TreeCall call(t);
    if (call.st != IMQ_OK) return -1;
    const HostTree &h = t->h;
    if (set < 0 || set >= h.nsets || level < 0 || level >= h.nlev || cls < 0 || cls >= NCLASS || !out) return -1;
    const size_t PP = size_t(t->KP) * t->KP, id = (size_t(set) * h.nlev + level) * NCLASS + cls;
    const DevBuf *src[4] = {&t->f64.m2l, &t->f64.m2l_pk, &t->f32.m2l, &t->f32.m2l_pk};
    if (layout < 0 || layout > 3) return -1;
    const size_t es = layout < 2 ? sizeof(double) : sizeof(float);
    if (hipMemcpy(out, static_cast<const char *>(src[layout]->p) + id * PP * es, PP * es, hipMemcpyDeviceToHost) !=
        hipSuccess)
        return -1;
    return t->KP;
}

void *imq_debug_device_tree(int nsets, const int64_t *set_offsets, const double *x, const double *y,
                            const double *c, const imq_tree_params *prm, int *status)
{
    const int64_t N = set_offsets[nsets];
    double *dxy = nullptr;
    auto fail = [&](imq_status st) -> void * {
        if (status) *status = st;
        if (dxy) (void)hipFree(dxy);
        return nullptr;
    };
    if (hipMalloc(reinterpret_cast<void **>(&dxy), sizeof(double) * 2 * size_t(std::max<int64_t>(N, 1))) != hipSuccess)
        return fail(IMQ_ENOMEM);
    if (N > 0 && (hipMemcpy(dxy, x, sizeof(double) * N, hipMemcpyHostToDevice) != hipSuccess ||
                  hipMemcpy(dxy + N, y, sizeof(double) * N, hipMemcpyHostToDevice) != hipSuccess))
        return fail(IMQ_EHIP);
    g_alloc = nullptr;
    auto *h = new HostTree();
    const imq_status st = build_device_tree(nsets, set_offsets, dxy, c, *prm, 0, *h);
    (void)hipFree(dxy);
    dxy = nullptr;
    if (status) *status = st;
    if (st != IMQ_OK) { delete h; return nullptr; }
    return h;
}

int64_t imq_debug_eval_points(int64_t n, const double *xs, const double *ys, int64_t m, const double *xt,
                              const double *yt, int64_t *map)
{
    if (n < 1 || m < 0 || !xs || !ys || (m > 0 && (!xt || !yt || !map))) return IMQ_EINVAL;
    std::vector<double> x, y;
    std::vector<int64_t> mp;
    const imq_status st = eval_points(n, xs, ys, m, xt, yt, x, y, mp);
    if (st != IMQ_OK) return st;
    std::copy(mp.begin(), mp.end(), map);
    return int64_t(x.size());
}

imq_status imq_solve(imq_tree t, int nrhs, const double *f, int64_t ldf, double *a, int64_t lda,
                     const imq_solve_opts *opts, imq_solve_stats *stats, hipStream_t stream)
{
    TreeCall call(t);
    if (call.st != IMQ_OK) return call.st;
    imq_status st = IMQ_OK;
    if (nrhs < 1 || !f || !a || !opts || !stats || ldf < t->h.N || lda < t->h.N) {
        set_error("bad argument to imq_solve");
        return IMQ_EINVAL;
    }
    if (!(opts->tol > 0.0) || opts->restart < 1 || opts->restart > 4096 || opts->max_iters < 1 ||
        opts->max_outer < 0 || opts->precond < 0 || opts->precond > 1) {
        set_error("solve options out of range (tol > 0, 1 <= restart <= 4096, max_iters >= 1, precond 0 or 1)");
        return IMQ_EINVAL;
    }
    if ((st = solve_batched(t, nrhs, f, ldf, a, lda, *opts, stats, stream)) != IMQ_OK) return st;
    bool all = true;
    for (int r = 0; r < nrhs; ++r) all = all && stats[r].converged;
    return all ? IMQ_OK : IMQ_ENOTCONVERGED;
}

imq_status imq_matvec_backward(imq_tree t, int nrhs, imq_dtype dtype, const void *v, int64_t ldv,
                               const void *g, int64_t ldg, void *dv, int64_t lddv, double *dc, double *dxy,
                               imq_prec prec, hipStream_t stream)
{
    TreeCall call(t);
    if (call.st != IMQ_OK) return call.st;
    const int64_t N = t->h.N;
    if (nrhs < 1 || !v || !g || !dv || !dc || !dxy || ldv < N || ldg < N || lddv < N) {
        set_error("bad nrhs, pointer or leading dimension in imq_matvec_backward");
        return IMQ_EINVAL;
    }
    if ((dtype != IMQ_F64 && dtype != IMQ_F32) || (prec != IMQ_PREC_FP64 && prec != IMQ_PREC_FP32)) {
        set_error("unknown dtype or precision");
        return IMQ_EINVAL;
    }
    const size_t es = dtype == IMQ_F64 ? sizeof(double) : sizeof(float);
    for (int r = 0; r < nrhs; ++r) {
        const char *vr = static_cast<const char *>(v) + size_t(r) * ldv * es;
        const char *gr = static_cast<const char *>(g) + size_t(r) * ldg * es;
        char *dvr = static_cast<char *>(dv) + size_t(r) * lddv * es;
        imq_status st;
        if (dtype == IMQ_F64 && prec == IMQ_PREC_FP64)
            st = backward_typed<double, double>(t, (const double *)vr, (const double *)gr, (double *)dvr, dc, dxy,
                                                r > 0, stream);
        else if (dtype == IMQ_F32 && prec == IMQ_PREC_FP64)
            st = backward_typed<double, float>(t, (const float *)vr, (const float *)gr, (float *)dvr, dc, dxy,
                                               r > 0, stream);
        else if (dtype == IMQ_F64)
            st = backward_typed<float, double>(t, (const double *)vr, (const double *)gr, (double *)dvr, dc, dxy,
                                               r > 0, stream);
        else
            st = backward_typed<float, float>(t, (const float *)vr, (const float *)gr, (float *)dvr, dc, dxy,
                                              r > 0, stream);
        if (st != IMQ_OK) return st;
    }
    return IMQ_OK;
}

}  // extern "C"
