// Host construction of the quadtree forest and its interaction lists.
//
// Sec. 2.2 partitions a square D containing the data into 4^l blocks at
// level l and, per block, separates the blocks whose points are far enough
// for the expansion (well separated) from the near ones, whose contribution
// is summed directly at the finest level.  The paper analyses uniform
// levels only; here the partition is refined adaptively (a box is split
// while it holds more than leaf_max points), and the well-separated /
// near classification becomes the usual adaptive lists:
//   U(b)  leaves adjacent to leaf b (edge or corner, b included): direct sum
//   V(b)  children of the neighbours of b's parent that are not adjacent
//         to b (same level as b): expansion-to-local translation
//   W(b)  for a leaf b, the largest descendants of b's neighbours that are
//         not adjacent to b although their parent is: multipole evaluated
//         at b's points
//   X(b)  the dual of W: b in W(a) <=> a in X(b): a's points summed into
//         b's local expansion
// Every ordered pair of points of a set is covered exactly once by these
// lists (checked by the test-suite).
#include "imq_internal.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <stdexcept>
#include <thread>

namespace imq {

static inline uint64_t spread(uint32_t v)
{
    uint64_t x = v & 0x3fffffffu;
    x = (x | (x << 16)) & 0x0000FFFF0000FFFFull;
    x = (x | (x << 8)) & 0x00FF00FF00FF00FFull;
    x = (x | (x << 4)) & 0x0F0F0F0F0F0F0F0Full;
    x = (x | (x << 2)) & 0x3333333333333333ull;
    x = (x | (x << 1)) & 0x5555555555555555ull;
    return x;
}

static inline uint64_t morton(uint32_t ix, uint32_t iy) { return spread(ix) | (spread(iy) << 1); }

namespace {
struct Builder {
    HostTree &t;
    std::vector<std::vector<int32_t>> lvl_set_begin;   // [level][set] -> first box

    explicit Builder(HostTree &tt) : t(tt) {}

    int find(int s, int l, int64_t ix, int64_t iy) const
    {
        const int64_t n = int64_t(1) << l;
        if (ix < 0 || iy < 0 || ix >= n || iy >= n) return -1;
        int lo = lvl_set_begin[l][s], hi = lvl_set_begin[l][s + 1];
        const uint64_t key = morton(uint32_t(ix), uint32_t(iy));
        while (lo < hi) {
            int mid = (lo + hi) / 2;
            uint64_t km = morton(uint32_t(t.ix[mid]), uint32_t(t.iy[mid]));
            if (km < key) lo = mid + 1; else hi = mid;
        }
        if (lo < lvl_set_begin[l][s + 1] && t.ix[lo] == ix && t.iy[lo] == iy) return lo;
        return -1;
    }

    void colleagues(int b, std::vector<int> &out) const
    {
        out.clear();
        for (int dx = -1; dx <= 1; ++dx)
            for (int dy = -1; dy <= 1; ++dy) {
                int c = find(t.set[b], t.level[b], int64_t(t.ix[b]) + dx, int64_t(t.iy[b]) + dy);
                if (c >= 0) out.push_back(c);
            }
    }

    bool adjacent(int a, int b) const
    {
        const int L = std::max(t.level[a], t.level[b]);
        const int sa = L - t.level[a], sb = L - t.level[b];
        const int64_t ax0 = int64_t(t.ix[a]) << sa, ax1 = int64_t(t.ix[a] + 1) << sa;
        const int64_t ay0 = int64_t(t.iy[a]) << sa, ay1 = int64_t(t.iy[a] + 1) << sa;
        const int64_t bx0 = int64_t(t.ix[b]) << sb, bx1 = int64_t(t.ix[b] + 1) << sb;
        const int64_t by0 = int64_t(t.iy[b]) << sb, by1 = int64_t(t.iy[b] + 1) << sb;
        return ax0 <= bx1 && bx0 <= ax1 && ay0 <= by1 && by0 <= ay1;
    }
};
}  // namespace

// Per leaf, whether its near field may take the squared distances from the
// expansion |x_i - x_j|^2 = |x_i|^2 + |x_j|^2 - 2 x_i . x_j about the leaf's
// centre (one operation fewer per pair than the differences, and a rank-4
// product for the matrix cores).  In |x_i - x_j|^2 + c^2 the expansion
// carries about (1 + (|x_i|^2 + |x_j|^2) / c^2) units of rounding against
// about 2 for the differences.  A leaf qualifies when that ratio, bounded with
// the largest point radius r of each leaf of its U list
// (r_b^2 + max_a (|c_a - c_b| + r_a)^2 <= NEAR_EXPAND_RATIO c^2), is at most
// NEAR_EXPAND_RATIO, so at most about 3 units.
static constexpr double NEAR_EXPAND_RATIO = 2.0;

static void near_expansion_flags(HostTree &h, const std::vector<double> *leaf_r2)
{
    const int nbox = int(h.level.size());
    std::vector<double> rad(nbox, 0.0);
    for (size_t l = 0; l < h.leaves.size(); ++l) {
        const int b = h.leaves[l];
        double r2 = 0.0;
        if (leaf_r2) {
            r2 = (*leaf_r2)[l];
        } else {
            for (int i = h.begin[b]; i < h.end[b]; ++i) {
                const double xx = h.xl[i] * h.xl[i];
                const double yy = h.yl[i] * h.yl[i];
                r2 = std::max(r2, xx + yy);
            }
        }
        rad[b] = std::sqrt(r2);                   // the largest distance: sqrt is monotone
    }
    h.near_expand.assign(h.leaves.size(), 0);
    for (size_t l = 0; l < h.leaves.size(); ++l) {
        const int b = h.leaves[l];
        double far = 0.0;
        for (int k = h.u_off[b]; k < h.u_off[b + 1]; ++k) {
            const int a = h.u_idx[k];
            far = std::max(far, std::hypot(h.cx[a] - h.cx[b], h.cy[a] - h.cy[b]) + rad[a]);
        }
        const double cn = h.cn[h.set[b]];
        h.near_expand[l] = (rad[b] * rad[b] + far * far) <= NEAR_EXPAND_RATIO * cn * cn ? 1 : 0;
    }
}

imq_status check_tree_params(int nsets, const int64_t *off, const double *c, const imq_tree_params &prm)
{
    if (nsets < 1) { set_error("nsets must be >= 1"); return IMQ_EINVAL; }
    if (off[0] != 0) { set_error("set_offsets[0] must be 0"); return IMQ_EINVAL; }
    for (int s = 0; s < nsets; ++s) {
        if (off[s + 1] <= off[s]) { set_error("every set needs at least one point"); return IMQ_EINVAL; }
        if (!(c[s] > 0.0) || !std::isfinite(c[s])) { set_error("shape parameter c must be finite and > 0"); return IMQ_EINVAL; }
    }
    if (off[nsets] > INT32_MAX) { set_error("more than 2^31-1 points"); return IMQ_EINVAL; }
    if (prm.order_p < 1 || prm.order_p > PMAX) { set_error("order_p must be in [1, 16]"); return IMQ_EINVAL; }
    if (prm.leaf_max < 1) { set_error("leaf_max must be >= 1"); return IMQ_EINVAL; }
    const int max_level = prm.max_level == 0 ? MORTON_BITS : prm.max_level;
    if (max_level < 0 || max_level > MORTON_BITS) { set_error("max_level must be in [0, 30]"); return IMQ_EINVAL; }
    return IMQ_OK;
}

// What follows the lists: the translation batches and shift lists, the
// near-field expansion flags, the work counts.
imq_status finish_host_tree(HostTree &t, const std::vector<double> *leaf_r2)
{
    // the flags and the batches write disjoint fields: built side by side
    // (one after the other where no thread can be started)
    std::thread flags;
    try {
        flags = std::thread([&] { near_expansion_flags(t, leaf_r2); });
    } catch (const std::exception &) {
        near_expansion_flags(t, leaf_r2);
    }
    build_gemm_lists(t);
    if (flags.joinable()) flags.join();
    const int nbox = int(t.level.size());
    auto npts = [&](int b) { return int64_t(t.end[b] - t.begin[b]); };
    for (int b = 0; b < nbox; ++b) {
        for (int k = t.u_off[b]; k < t.u_off[b + 1]; ++k) t.p2p_pairs += npts(b) * npts(t.u_idx[k]);
        t.m2l_pairs += t.v_off[b + 1] - t.v_off[b];
        t.m2p_evals += int64_t(t.w_off[b + 1] - t.w_off[b]) * npts(b);
        for (int k = t.x_off[b]; k < t.x_off[b + 1]; ++k) t.p2l_evals += npts(t.x_idx[k]);
        if (t.parent[b] >= 0) { t.m2m_pairs++; t.l2l_pairs++; }
    }
    return IMQ_OK;
}

imq_status build_host_tree(int nsets, const int64_t *off, const double *x, const double *y,
                           const double *c, const imq_tree_params &prm, HostTree &t)
{
    imq_status st0 = check_tree_params(nsets, off, c, prm);
    if (st0 != IMQ_OK) return st0;
    const int64_t N = off[nsets];
    const int max_level = prm.max_level == 0 ? MORTON_BITS : prm.max_level;
    for (int64_t i = 0; i < N; ++i)
        if (!std::isfinite(x[i]) || !std::isfinite(y[i])) { set_error("non-finite coordinate"); return IMQ_EINVAL; }

    t = HostTree();
    t.nsets = nsets;
    t.N = N;
    t.p = prm.order_p;
    t.K = Kof(t.p);
    t.set_off.assign(off, off + nsets + 1);
    t.c.assign(c, c + nsets);
    t.side.resize(nsets); t.lox.resize(nsets); t.loy.resize(nsets); t.cn.resize(nsets);

    // ---- normalise, Morton keys, sort per set
    std::vector<uint64_t> key(N);
    std::vector<double> xn(N), yn(N);
    t.perm.resize(N);
    for (int s = 0; s < nsets; ++s) {
        double x0 = x[off[s]], x1 = x0, y0 = y[off[s]], y1 = y0;
        for (int64_t i = off[s]; i < off[s + 1]; ++i) {
            x0 = std::min(x0, x[i]); x1 = std::max(x1, x[i]);
            y0 = std::min(y0, y[i]); y1 = std::max(y1, y[i]);
        }
        double ext = std::max(x1 - x0, y1 - y0);
        double side = ext > 0 ? ext * (1.0 + std::ldexp(1.0, -20)) : 1.0;
        t.side[s] = side; t.lox[s] = x0; t.loy[s] = y0; t.cn[s] = c[s] / side;
        const double q = std::ldexp(1.0, MORTON_BITS);
        std::vector<std::pair<uint64_t, int32_t>> kv;
        kv.reserve(off[s + 1] - off[s]);
        for (int64_t i = off[s]; i < off[s + 1]; ++i) {
            double a = (x[i] - x0) / side, b = (y[i] - y0) / side;
            int64_t qa = std::min<int64_t>(int64_t(a * q), (int64_t(1) << MORTON_BITS) - 1);
            int64_t qb = std::min<int64_t>(int64_t(b * q), (int64_t(1) << MORTON_BITS) - 1);
            qa = std::max<int64_t>(qa, 0); qb = std::max<int64_t>(qb, 0);
            kv.emplace_back(morton(uint32_t(qa), uint32_t(qb)), int32_t(i));
        }
        std::sort(kv.begin(), kv.end());
        for (size_t k = 0; k < kv.size(); ++k) {
            int64_t i = off[s] + int64_t(k);
            key[i] = kv[k].first;
            t.perm[i] = kv[k].second;
            xn[i] = (x[kv[k].second] - x0) / side;
            yn[i] = (y[kv[k].second] - y0) / side;
        }
        // exact duplicates can only share a Morton key
        for (int64_t i = off[s]; i < off[s + 1];) {
            int64_t j = i + 1;
            while (j < off[s + 1] && key[j] == key[i]) ++j;
            for (int64_t a = i; a < j; ++a)
                for (int64_t b = a + 1; b < j; ++b)
                    if (x[t.perm[a]] == x[t.perm[b]] && y[t.perm[a]] == y[t.perm[b]]) {
                        set_error("duplicate data sites: points " + std::to_string(t.perm[a]) +
                                  " and " + std::to_string(t.perm[b]));
                        return IMQ_EDUPLICATE;
                    }
            i = j;
        }
    }

    // ---- breadth-first adaptive split: boxes come out in (level, set, Morton) order
    auto push_box = [&](int l, int s, int64_t bx, int64_t by, int64_t b, int64_t e, int par) {
        t.level.push_back(l); t.set.push_back(s);
        t.ix.push_back(int32_t(bx)); t.iy.push_back(int32_t(by));
        t.parent.push_back(par); t.child0.push_back(-1); t.nchild.push_back(0);
        t.pos.push_back(int32_t((bx & 1) | ((by & 1) << 1)));
        t.begin.push_back(int32_t(b)); t.end.push_back(int32_t(e));
        t.isleaf.push_back(1);
        const double sz = std::ldexp(1.0, -l);
        t.cx.push_back((double(bx) + 0.5) * sz); t.cy.push_back((double(by) + 0.5) * sz);
    };
    t.level_begin.push_back(0);
    for (int s = 0; s < nsets; ++s) push_box(0, s, 0, 0, off[s], off[s + 1], -1);
    int lvl_lo = 0, lvl_hi = nsets;
    for (int l = 0;; ++l) {
        t.level_begin.push_back(lvl_hi);
        if (l >= max_level) break;
        const int shift = 2 * (MORTON_BITS - l - 1);
        for (int b = lvl_lo; b < lvl_hi; ++b) {
            if (t.end[b] - t.begin[b] <= prm.leaf_max) continue;
            int64_t lo = t.begin[b];
            const int64_t hi = t.end[b];
            const int first = int(t.level.size());
            int cnt = 0;
            for (int ch = 0; ch < 4; ++ch) {
                int64_t e = std::partition_point(key.begin() + lo, key.begin() + hi,
                                                 [&](uint64_t k) { return int((k >> shift) & 3) <= ch; }) -
                            key.begin();
                if (e > lo) {
                    push_box(l + 1, t.set[b], 2 * int64_t(t.ix[b]) + (ch & 1),
                             2 * int64_t(t.iy[b]) + (ch >> 1), lo, e, b);
                    ++cnt;
                }
                lo = e;
            }
            t.child0[b] = first; t.nchild[b] = cnt; t.isleaf[b] = 0;
        }
        lvl_lo = lvl_hi;
        lvl_hi = int(t.level.size());
        if (lvl_hi == lvl_lo) break;
    }
    const int nbox = int(t.level.size());
    t.nlev = int(t.level_begin.size()) - 1;
    t.Klev.resize(t.nlev);
    for (int l = 0; l < t.nlev; ++l) {
        int pl = (l <= IMQ_MAX_LEVELS && prm.level_order[l] > 0) ? prm.level_order[l] : t.p;
        pl = std::min(pl, t.p);
        t.Klev[l] = Kof(pl);
    }

    // ---- points: leaf-local coordinates
    t.xl.resize(N); t.yl.resize(N); t.pt_scale.resize(N); t.pt_leaf.resize(N);
    for (int b = 0; b < nbox; ++b) {
        if (!t.isleaf[b]) continue;
        t.leaves.push_back(b);
        for (int i = t.begin[b]; i < t.end[b]; ++i) {
            t.xl[i] = xn[i] - t.cx[b];
            t.yl[i] = yn[i] - t.cy[b];
            t.pt_scale[i] = 1.0 / t.side[t.set[b]];
            t.pt_leaf[i] = b;
        }
    }

    // ---- lookup structure
    Builder B(t);
    B.lvl_set_begin.assign(t.nlev, std::vector<int32_t>(nsets + 1, 0));
    for (int l = 0; l < t.nlev; ++l) {
        int b = t.level_begin[l];
        for (int s = 0; s <= nsets; ++s) {
            while (b < t.level_begin[l + 1] && t.set[b] < s) ++b;
            B.lvl_set_begin[l][s] = b;
        }
        B.lvl_set_begin[l][nsets] = t.level_begin[l + 1];
    }

    // ---- lists
    std::vector<std::vector<int32_t>> U(nbox), V(nbox), Vc(nbox), W(nbox), X(nbox);
    std::vector<int> col, pcol, stack;
    for (int b = 0; b < nbox; ++b) {
        if (t.parent[b] >= 0) {
            B.colleagues(t.parent[b], pcol);
            for (int pc : pcol)
                for (int ch = t.child0[pc]; ch >= 0 && ch < t.child0[pc] + t.nchild[pc]; ++ch) {
                    int dx = t.ix[b] - t.ix[ch], dy = t.iy[b] - t.iy[ch];
                    if (std::abs(dx) > 1 || std::abs(dy) > 1) {
                        V[b].push_back(ch);
                        Vc[b].push_back(class_of(dx, dy));
                    }
                }
        }
        if (!t.isleaf[b]) continue;
        B.colleagues(b, col);
        stack.assign(col.begin(), col.end());
        while (!stack.empty()) {
            int cb = stack.back();
            stack.pop_back();
            if (t.isleaf[cb]) { U[b].push_back(cb); continue; }
            for (int ch = t.child0[cb]; ch < t.child0[cb] + t.nchild[cb]; ++ch) {
                if (B.adjacent(b, ch)) stack.push_back(ch);
                else W[b].push_back(ch);
            }
        }
        for (int a = t.parent[b]; a >= 0; a = t.parent[a]) {
            B.colleagues(a, pcol);
            for (int cb : pcol)
                if (cb != a && t.isleaf[cb] && B.adjacent(b, cb)) U[b].push_back(cb);
        }
        std::sort(U[b].begin(), U[b].end());
        std::sort(W[b].begin(), W[b].end());
    }
    for (int b = 0; b < nbox; ++b)
        for (int w : W[b]) X[w].push_back(b);

    // W/X interactions whose finer box is small are cheaper as direct sums:
    // move them to the near list of every leaf under the target box.
    const int dmax = prm.direct_max == 0 ? 2 * prm.leaf_max : prm.direct_max;
    if (dmax > 0) {
        std::vector<int> under;
        auto leaves_under = [&](int box) {
            under.clear();
            stack.assign(1, box);
            while (!stack.empty()) {
                int q = stack.back();
                stack.pop_back();
                if (t.isleaf[q]) under.push_back(q);
                else for (int ch = t.child0[q]; ch < t.child0[q] + t.nchild[q]; ++ch) stack.push_back(ch);
            }
        };
        std::vector<std::vector<int32_t>> Wk(nbox), Xk(nbox);
        for (int b = 0; b < nbox; ++b) {
            for (int w : W[b]) {               // targets b (leaf), sources w
                if (t.end[w] - t.begin[w] <= dmax) {
                    leaves_under(w);
                    U[b].insert(U[b].end(), under.begin(), under.end());
                } else {
                    Wk[b].push_back(w);
                }
            }
            for (int a : X[b]) {               // targets b, sources a (leaf)
                if (t.end[b] - t.begin[b] <= dmax) {
                    leaves_under(b);
                    for (int l : under) U[l].push_back(a);
                } else {
                    Xk[b].push_back(a);
                }
            }
        }
        W.swap(Wk);
        X.swap(Xk);
        for (int b = 0; b < nbox; ++b) std::sort(U[b].begin(), U[b].end());
    }

    auto flatten = [&](const std::vector<std::vector<int32_t>> &L, std::vector<int32_t> &offv,
                       std::vector<int32_t> &idx) {
        offv.assign(nbox + 1, 0);
        for (int b = 0; b < nbox; ++b) offv[b + 1] = offv[b] + int32_t(L[b].size());
        idx.resize(offv[nbox]);
        for (int b = 0; b < nbox; ++b) std::copy(L[b].begin(), L[b].end(), idx.begin() + offv[b]);
    };
    flatten(U, t.u_off, t.u_idx);
    flatten(V, t.v_off, t.v_idx);
    {
        std::vector<int32_t> dummy;
        flatten(Vc, dummy, t.v_cls);
    }
    flatten(W, t.w_off, t.w_idx);
    flatten(X, t.x_off, t.x_idx);

    return finish_host_tree(t);
}

// ---- translation batches
//
// For a box at child position (px, py) of its parent, the sources of its V
// list lie at offsets (dx, dy) with dx in [px-3, px+2], dy in [py-3, py+2]
// and max(|dx|, |dy|) >= 2: 27 classes, fixed per position.  Grouping the
// targets of a (set, level, position) makes every slot's table uniform
// across a task.
static void v_classes(int pos, std::vector<int> &cls)
{
    cls.clear();
    const int px = pos & 1, py = (pos >> 1) & 1;
    for (int dx = px - 3; dx <= px + 2; ++dx)
        for (int dy = py - 3; dy <= py + 2; ++dy)
            if (std::max(std::abs(dx), std::abs(dy)) >= 2) cls.push_back(class_of(dx, dy));
}

// Tasks of up to GEMM_TILE consecutive targets; src holds nslot sources per
// target, in the order of boxes.
static void add_tasks(GemmList &g, const std::vector<int32_t> &boxes, const std::vector<int32_t> &src, int nslot,
                      int kin, int kout, int level, const std::vector<int32_t> &tabs)
{
    for (size_t b0 = 0; b0 < boxes.size(); b0 += GEMM_TILE) {
        GemmTask k;
        k.box0 = int32_t(g.tbox.size());
        k.nbox = int32_t(std::min<size_t>(GEMM_TILE, boxes.size() - b0));
        k.nslot = nslot;
        k.kin = kin;
        k.kout = kout;
        k.tab0 = int32_t(g.tab.size());
        k.src0 = int32_t(g.src.size());
        k.level = level;
        g.tab.insert(g.tab.end(), tabs.begin(), tabs.end());
        g.tbox.insert(g.tbox.end(), boxes.begin() + b0, boxes.begin() + b0 + k.nbox);
        g.src.insert(g.src.end(), src.begin() + b0 * nslot, src.begin() + (b0 + k.nbox) * nslot);
        g.tasks.push_back(k);
    }
}

void build_gemm_lists(HostTree &t)
{
    const int nbox = int(t.level.size());
    const int L = t.nlev;
    t.m2l = GemmList();
    // Multipoles are read by V lists (as sources) and W lists; locals are
    // written by V and X lists.  Shifts above the first level that needs them
    // would only move zeros or unused coefficients, so they are skipped.
    t.need_m = L;
    t.need_l = L;
    for (int b = 0; b < nbox; ++b) {
        if (t.v_off[b + 1] > t.v_off[b] || t.x_off[b + 1] > t.x_off[b]) t.need_l = std::min(t.need_l, t.level[b]);
        for (int v = t.v_off[b]; v < t.v_off[b + 1]; ++v) t.need_m = std::min(t.need_m, t.level[t.v_idx[v]]);
        for (int w = t.w_off[b]; w < t.w_off[b + 1]; ++w) t.need_m = std::min(t.need_m, t.level[t.w_idx[w]]);
    }
    // parents level by level with their children by quadrant
    t.sh_par.clear();
    t.sh_kids.clear();
    t.sh_level_begin.assign(L + 1, 0);
    for (int l = 0; l < L; ++l) {
        t.sh_level_begin[l] = int32_t(t.sh_par.size());
        for (int b = t.level_begin[l]; b < t.level_begin[l + 1]; ++b) {
            if (t.nchild[b] == 0) continue;
            t.sh_par.push_back(b);
            int32_t k4[4] = {-1, -1, -1, -1};
            for (int c = t.child0[b]; c < t.child0[b] + t.nchild[b]; ++c) k4[t.pos[c]] = c;
            t.sh_kids.insert(t.sh_kids.end(), k4, k4 + 4);
        }
    }
    t.sh_level_begin[L] = int32_t(t.sh_par.size());
    // expansion-to-local: (set, level, position) groups, 27 slots; slot of
    // every displacement class at each child position (-1: not a V class)
    std::vector<int> cls[4];
    int slot_of[4][NCLASS];
    for (int pos = 0; pos < 4; ++pos) {
        v_classes(pos, cls[pos]);
        std::fill(slot_of[pos], slot_of[pos] + NCLASS, -1);
        for (int i = 0; i < int(cls[pos].size()); ++i) slot_of[pos][cls[pos][i]] = i;
    }
    t.m2l.level_task_begin.assign(L + 1, 0);
    {
        size_t ntgt = 0;
        for (int b = 0; b < nbox; ++b) ntgt += t.v_off[b + 1] > t.v_off[b] ? 1 : 0;
        t.m2l.tbox.reserve(ntgt);
        t.m2l.src.reserve(ntgt * 27);
    }
    std::vector<int32_t> tgt, grp, src, tabs, cnt;
    for (int l = 0; l < L; ++l) {
        t.m2l.level_task_begin[l] = int32_t(t.m2l.tasks.size());
        // the level's targets in (set, position, box) order: a counting sort
        // on set * 4 + position
        cnt.assign(size_t(t.nsets) * 4 + 1, 0);
        int ntgt = 0;
        for (int b = t.level_begin[l]; b < t.level_begin[l + 1]; ++b)
            if (t.v_off[b + 1] > t.v_off[b]) {
                ++cnt[size_t(t.set[b]) * 4 + t.pos[b] + 1];
                ++ntgt;
            }
        for (size_t k = 1; k < cnt.size(); ++k) cnt[k] += cnt[k - 1];
        tgt.resize(ntgt);
        for (int b = t.level_begin[l]; b < t.level_begin[l + 1]; ++b)
            if (t.v_off[b + 1] > t.v_off[b]) tgt[cnt[size_t(t.set[b]) * 4 + t.pos[b]]++] = b;
        for (size_t g0 = 0; g0 < tgt.size();) {
            const int s = t.set[tgt[g0]], pos = t.pos[tgt[g0]];
            size_t g1 = g0;
            while (g1 < tgt.size() && t.set[tgt[g1]] == s && t.pos[tgt[g1]] == pos) ++g1;
            const int nslot = int(cls[pos].size());
            grp.assign(tgt.begin() + g0, tgt.begin() + g1);
            src.assign(grp.size() * nslot, -1);
            for (size_t i = 0; i < grp.size(); ++i) {
                const int32_t b = grp[i];
                int32_t *row = src.data() + i * nslot;
                for (int v = t.v_off[b]; v < t.v_off[b + 1]; ++v) {
                    const int sl = slot_of[pos][t.v_cls[v]];
                    if (sl >= 0 && row[sl] < 0) row[sl] = t.v_idx[v];
                }
            }
            tabs.clear();
            for (int c : cls[pos]) tabs.push_back((s * L + l) * NCLASS + c);
            add_tasks(t.m2l, grp, src, nslot, t.Klev[l], t.Klev[l], l, tabs);
            g0 = g1;
        }
    }
    t.m2l.level_task_begin[L] = int32_t(t.m2l.tasks.size());
}

imq_status eval_points(int64_t n, const double *xs, const double *ys, int64_t m, const double *xt,
                       const double *yt, std::vector<double> &x, std::vector<double> &y,
                       std::vector<int64_t> &map)
{
    // Open-addressing hash of the kept points by their coordinates' bit
    // patterns (-0 read as +0: the same point); a slot holds a point index.
    auto bits = [](double a) {
        a += 0.0;                                // -0 -> +0
        uint64_t k;
        std::memcpy(&k, &a, 8);
        return k;
    };
    auto hash = [](uint64_t kx, uint64_t ky) {
        uint64_t h = kx * 0x9E3779B97F4A7C15ull ^ (ky + 0x632BE59BD9B4E019ull + (kx << 6));
        h ^= h >> 29;
        h *= 0xBF58476D1CE4E5B9ull;
        return h ^ (h >> 32);
    };
    size_t cap = 16;
    while (cap < 2 * size_t(n + m)) cap <<= 1;
    std::vector<int64_t> slot(cap, -1);
    x.assign(xs, xs + n);
    y.assign(ys, ys + n);
    x.reserve(size_t(n + m));
    y.reserve(size_t(n + m));
    map.assign(size_t(m), -1);
    // index of the kept point at (a, b), or -1 with `at` the empty slot for it
    auto find = [&](double a, double b, size_t &at) -> int64_t {
        const uint64_t ka = bits(a), kb = bits(b);
        for (size_t h = hash(ka, kb) & (cap - 1);; h = (h + 1) & (cap - 1)) {
            const int64_t i = slot[h];
            if (i < 0) { at = h; return -1; }
            if (bits(x[size_t(i)]) == ka && bits(y[size_t(i)]) == kb) return i;
        }
    };
    for (int64_t i = 0; i < n; ++i) {
        if (!std::isfinite(xs[i]) || !std::isfinite(ys[i])) { set_error("non-finite data site"); return IMQ_EINVAL; }
        size_t at = 0;
        const int64_t j = find(xs[i], ys[i], at);
        if (j >= 0) {
            set_error("duplicate data sites: points " + std::to_string(j) + " and " + std::to_string(i));
            return IMQ_EDUPLICATE;
        }
        slot[at] = i;
    }
    for (int64_t k = 0; k < m; ++k) {
        if (!std::isfinite(xt[k]) || !std::isfinite(yt[k])) { set_error("non-finite evaluation point"); return IMQ_EINVAL; }
        size_t at = 0;
        int64_t j = find(xt[k], yt[k], at);
        if (j < 0) {
            j = int64_t(x.size());
            x.push_back(xt[k]);
            y.push_back(yt[k]);
            slot[at] = j;
        }
        map[size_t(k)] = j;
    }
    return IMQ_OK;
}

}  // namespace imq
