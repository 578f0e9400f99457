// Construction of the quadtree forest on the device: the same partition,
// point order and interaction lists as the host construction in tree.cpp
// (Sec. 2.2: the hierarchical partition of a square containing the data and
// the well-separated / near classification, refined adaptively), array for
// array, computed in parallel:
//   1. per-set bounding squares (block reductions) and the finiteness check;
//   2. 30-bit Morton keys of the normalised points and a stable radix sort
//      of (key, index) per set: the order of std::sort on the pairs;
//   3. exact-duplicate detection among points that share a key;
//   4. the adaptive split, level by level: a box with more than leaf_max
//      points is cut at the partition points of its keys' two bits at that
//      level (binary searches), its children numbered by a prefix sum, so
//      boxes come out in (level, set, Morton) order;
//   5. leaf-local coordinates;
//   6. the U, V, W, X lists, one thread per box: colleagues by binary search
//      in the (level, set) range, V from the parent's colleagues' children,
//      U and W by the walk down the colleagues, coarser adjacent leaves; the
//      small W/X interactions moved to the U lists of the leaves under the
//      small box (counts by atomics, positions by prefix sums), every list
//      then sorted where the host sorts it.
// The floating-point steps (normalisation, quantisation, box centres,
// leaf-local coordinates) are the host's operations in the same order, and
// this file is compiled without contraction of multiplies and adds, so the
// results are equal bit for bit.
#include "device.h"

#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

namespace imq {

namespace {

constexpr int TB = 256;
inline unsigned nblk(int64_t n) { return unsigned((n + TB - 1) / TB); }

__device__ __forceinline__ uint64_t spread_d(uint32_t v)
{
    uint64_t x = v & 0x3fffffffu;
    x = (x | (x << 16)) & 0x0000FFFF0000FFFFull;
    x = (x | (x << 8)) & 0x00FF00FF00FF00FFull;
    x = (x | (x << 4)) & 0x0F0F0F0F0F0F0F0Full;
    x = (x | (x << 2)) & 0x3333333333333333ull;
    x = (x | (x << 1)) & 0x5555555555555555ull;
    return x;
}

__device__ __forceinline__ uint64_t morton_d(uint32_t ix, uint32_t iy) { return spread_d(ix) | (spread_d(iy) << 1); }

// set of sorted (or input) position i: off has nsets + 1 entries
__device__ __forceinline__ int set_of(const int64_t *off, int nsets, int64_t i)
{
    int lo = 0, hi = nsets;                          // off[lo] <= i < off[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (off[mid] <= i) lo = mid; else hi = mid;
    }
    return lo;
}

// per set: min and max of x and y (exact whatever the order), and a flag
// for a coordinate that is not finite; gridDim.x blocks per set (blockIdx.y)
// each write their partial bounds, k_bounds_final combines them
__global__ __launch_bounds__(TB) void k_bounds(const int64_t *__restrict__ off, const double *__restrict__ x,
                                               const double *__restrict__ y, double *__restrict__ part,
                                               int *__restrict__ bad)
{
    __shared__ double r[4][TB];
    const int s = blockIdx.y;
    double x0 = INFINITY, x1 = -INFINITY, y0 = INFINITY, y1 = -INFINITY;
    for (int64_t i = off[s] + int64_t(blockIdx.x) * TB + threadIdx.x; i < off[s + 1];
         i += int64_t(gridDim.x) * TB) {
        const double a = x[i], b = y[i];
        if (!isfinite(a) || !isfinite(b)) atomicOr(bad, 1);
        x0 = fmin(x0, a); x1 = fmax(x1, a);
        y0 = fmin(y0, b); y1 = fmax(y1, b);
    }
    r[0][threadIdx.x] = x0; r[1][threadIdx.x] = x1; r[2][threadIdx.x] = y0; r[3][threadIdx.x] = y1;
    __syncthreads();
    for (int w = TB / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            r[0][threadIdx.x] = fmin(r[0][threadIdx.x], r[0][threadIdx.x + w]);
            r[1][threadIdx.x] = fmax(r[1][threadIdx.x], r[1][threadIdx.x + w]);
            r[2][threadIdx.x] = fmin(r[2][threadIdx.x], r[2][threadIdx.x + w]);
            r[3][threadIdx.x] = fmax(r[3][threadIdx.x], r[3][threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x < 4) part[(size_t(s) * gridDim.x + blockIdx.x) * 4 + threadIdx.x] = r[threadIdx.x][0];
}

__global__ void k_bounds_final(int nsets, int nblk_set, const double *__restrict__ part, double *__restrict__ bnd)
{
    const int s = blockIdx.x * TB + threadIdx.x;
    if (s >= nsets) return;
    const double *q = part + size_t(s) * nblk_set * 4;
    double x0 = q[0], x1 = q[1], y0 = q[2], y1 = q[3];
    for (int g = 1; g < nblk_set; ++g) {
        x0 = fmin(x0, q[4 * g]); x1 = fmax(x1, q[4 * g + 1]);
        y0 = fmin(y0, q[4 * g + 2]); y1 = fmax(y1, q[4 * g + 3]);
    }
    bnd[4 * s] = x0; bnd[4 * s + 1] = x1; bnd[4 * s + 2] = y0; bnd[4 * s + 3] = y1;
}

// Morton key of the point quantised in its set's square (the host's
// expressions: (x - x0) / side, times 2^30, truncated, clamped)
__global__ void k_keys(int64_t N, int nsets, const int64_t *__restrict__ off, const double *__restrict__ x,
                       const double *__restrict__ y, const double *__restrict__ geo, uint64_t *__restrict__ key,
                       int32_t *__restrict__ idx)
{
    const int64_t i = blockIdx.x * int64_t(TB) + threadIdx.x;
    if (i >= N) return;
    const int s = set_of(off, nsets, i);
    const double x0 = geo[3 * s], y0 = geo[3 * s + 1], side = geo[3 * s + 2];
    const double q = 1073741824.0;                   // 2^30
    const double a = (x[i] - x0) / side, b = (y[i] - y0) / side;
    const int64_t top = (int64_t(1) << MORTON_BITS) - 1;
    int64_t qa = min(int64_t(a * q), top), qb = min(int64_t(b * q), top);
    qa = max(qa, int64_t(0));
    qb = max(qb, int64_t(0));
    key[i] = morton_d(uint32_t(qa), uint32_t(qb));
    idx[i] = int32_t(i);
}

// Exact duplicates can only share a key: the first pair (sorted positions
// packed high/low) of equal points in a run of equal keys of one set.
__global__ void k_dups(int64_t N, int nsets, const int64_t *__restrict__ off, const uint64_t *__restrict__ key,
                       const int32_t *__restrict__ perm, const double *__restrict__ x, const double *__restrict__ y,
                       unsigned long long *__restrict__ first)
{
    const int64_t i = blockIdx.x * int64_t(TB) + threadIdx.x;
    if (i >= N) return;
    const int s = set_of(off, nsets, i);
    const int64_t hi = off[s + 1];
    const double xa = x[perm[i]], ya = y[perm[i]];
    for (int64_t j = i + 1; j < hi && key[j] == key[i]; ++j)
        if (x[perm[j]] == xa && y[perm[j]] == ya) {
            atomicMin(first, (static_cast<unsigned long long>(i) << 32) | static_cast<unsigned long long>(j));
            return;
        }
}

// normalised coordinates in sorted order
__global__ void k_normal(int64_t N, int nsets, const int64_t *__restrict__ off, const int32_t *__restrict__ perm,
                         const double *__restrict__ x, const double *__restrict__ y, const double *__restrict__ geo,
                         double *__restrict__ xn, double *__restrict__ yn)
{
    const int64_t i = blockIdx.x * int64_t(TB) + threadIdx.x;
    if (i >= N) return;
    const int s = set_of(off, nsets, i);
    const int32_t k = perm[i];
    xn[i] = (x[k] - geo[3 * s]) / geo[3 * s + 2];
    yn[i] = (y[k] - geo[3 * s + 1]) / geo[3 * s + 2];
}

// One level of boxes (structure of arrays; box i of the level is box
// base + i of the forest).
struct LevelBoxes {
    int32_t *set = nullptr, *ix = nullptr, *iy = nullptr, *beg = nullptr, *end = nullptr, *parent = nullptr,
            *pos = nullptr;
    int32_t *child0 = nullptr, *nchild = nullptr, *cnt = nullptr, *first = nullptr,
            *cut = nullptr;                       // split results (cut: 5 per box)
    int n = 0;
};

// the children of a box with more than leaf_max points: the partition
// points of its sorted keys by the two bits of level l + 1
__global__ void k_split_count(int n, int l, int leaf_max, const int32_t *__restrict__ beg,
                              const int32_t *__restrict__ end, const uint64_t *__restrict__ key,
                              int32_t *__restrict__ cnt, int32_t *__restrict__ cut)
{
    const int b = blockIdx.x * TB + threadIdx.x;
    if (b >= n) return;
    const int32_t lo0 = beg[b], hi = end[b];
    if (hi - lo0 <= leaf_max) {
        cnt[b] = 0;
        return;
    }
    const int shift = 2 * (MORTON_BITS - l - 1);
    int32_t lo = lo0;
    int c = 0;
    cut[5 * b] = lo0;
    for (int ch = 0; ch < 4; ++ch) {
        int32_t a = lo, z = hi;                      // first position whose quadrant exceeds ch
        while (a < z) {
            const int32_t mid = a + ((z - a) >> 1);
            if (int((key[mid] >> shift) & 3) <= ch) a = mid + 1; else z = mid;
        }
        cut[5 * b + ch + 1] = a;
        if (a > lo) ++c;
        lo = a;
    }
    cnt[b] = c;
}

__global__ void k_split_fill(int n, int base_next, const int32_t *__restrict__ set, const int32_t *__restrict__ ix,
                             const int32_t *__restrict__ iy, int base, const int32_t *__restrict__ cnt,
                             const int32_t *__restrict__ first, const int32_t *__restrict__ cut,
                             int32_t *__restrict__ child0, int32_t *__restrict__ nchild, int32_t *__restrict__ nset,
                             int32_t *__restrict__ nix, int32_t *__restrict__ niy, int32_t *__restrict__ nbeg,
                             int32_t *__restrict__ nend, int32_t *__restrict__ npar, int32_t *__restrict__ npos)
{
    const int b = blockIdx.x * TB + threadIdx.x;
    if (b >= n) return;
    const int c = cnt[b];
    nchild[b] = c;
    if (c == 0) {
        child0[b] = -1;
        return;
    }
    int o = first[b];
    child0[b] = base_next + o;
    for (int ch = 0; ch < 4; ++ch) {
        const int32_t lo = cut[5 * b + ch], hi = cut[5 * b + ch + 1];
        if (hi <= lo) continue;
        const int32_t bx = 2 * ix[b] + (ch & 1), by = 2 * iy[b] + (ch >> 1);
        nset[o] = set[b];
        nix[o] = bx;
        niy[o] = by;
        nbeg[o] = lo;
        nend[o] = hi;
        npar[o] = base + b;
        npos[o] = (bx & 1) | ((by & 1) << 1);
        ++o;
    }
}

// leaf-local coordinates of every point of a leaf (one block per leaf)
__global__ void k_points(const int32_t *__restrict__ leaves, const int32_t *__restrict__ level,
                         const int32_t *__restrict__ set, const int32_t *__restrict__ ix, const int32_t *__restrict__ iy,
                         const int32_t *__restrict__ beg, const int32_t *__restrict__ end,
                         const double *__restrict__ geo, const double *__restrict__ xn, const double *__restrict__ yn,
                         double *__restrict__ xl, double *__restrict__ yl, double *__restrict__ scale,
                         int32_t *__restrict__ pt_leaf, double *__restrict__ leaf_r2)
{
    const int b = leaves[blockIdx.x];
    const double sz = ldexp(1.0, -level[b]);
    const double cx = (double(ix[b]) + 0.5) * sz, cy = (double(iy[b]) + 0.5) * sz;
    const double sc = 1.0 / geo[3 * set[b] + 2];
    double r2 = 0.0;
    for (int i = beg[b] + threadIdx.x; i < end[b]; i += blockDim.x) {
        const double x = xn[i] - cx, y = yn[i] - cy;
        xl[i] = x;
        yl[i] = y;
        scale[i] = sc;
        pt_leaf[i] = b;
        const double xx = x * x, yy = y * y;
        r2 = fmax(r2, xx + yy);
    }
    // the leaf's largest squared distance from its centre (one wave per leaf)
    for (int o = 32; o > 0; o >>= 1) r2 = fmax(r2, __shfl_xor(r2, o));
    if (threadIdx.x == 0) leaf_r2[blockIdx.x] = r2;
}

// the near field's record of every U-list entry, in both precisions: the
// source leaf's points and its centre minus the target's (the host's
// expressions for the centres)
__global__ void k_urec(int nbox, const int32_t *__restrict__ level, const int32_t *__restrict__ ix,
                       const int32_t *__restrict__ iy, const int32_t *__restrict__ beg,
                       const int32_t *__restrict__ end, const int32_t *__restrict__ u_off,
                       const int32_t *__restrict__ u_idx, URec<double> *__restrict__ r64,
                       URec<float> *__restrict__ r32)
{
    const int b = blockIdx.x * TB + threadIdx.x;
    if (b >= nbox) return;
    const double sb = ldexp(1.0, -level[b]);
    const double cxb = (double(ix[b]) + 0.5) * sb, cyb = (double(iy[b]) + 0.5) * sb;
    for (int k = u_off[b]; k < u_off[b + 1]; ++k) {
        const int a = u_idx[k];
        const double sa = ldexp(1.0, -level[a]);
        const double cxa = (double(ix[a]) + 0.5) * sa, cya = (double(iy[a]) + 0.5) * sa;
        const double ox = cxa - cxb, oy = cya - cyb;
        r64[k] = URec<double>{beg[a], end[a] - beg[a], ox, oy};
        r32[k] = URec<float>{beg[a], end[a] - beg[a], float(ox), float(oy)};
    }
}

// ---- interaction lists

struct DBoxes {
    const int32_t *level, *set, *ix, *iy, *parent, *child0, *nchild, *beg, *end, *isleaf;
    const int32_t *lsb;          // [level][set] -> first box, nsets + 1 per level
    const int32_t *lbeg;         // leaves in point order: their first point
    int nsets, nleaves;

    __device__ int find(int s, int l, int64_t x, int64_t y) const
    {
        const int64_t n = int64_t(1) << l;
        if (x < 0 || y < 0 || x >= n || y >= n) return -1;
        int lo = lsb[l * (nsets + 1) + s], hi = lsb[l * (nsets + 1) + s + 1];
        const int top = hi;
        const uint64_t k = morton_d(uint32_t(x), uint32_t(y));
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (morton_d(uint32_t(ix[mid]), uint32_t(iy[mid])) < k) lo = mid + 1; else hi = mid;
        }
        return (lo < top && ix[lo] == x && iy[lo] == y) ? lo : -1;
    }
    // up to 9 boxes of b's level and set touching b (b included), in the
    // host's order
    __device__ int colleagues(int b, int *out) const
    {
        int n = 0;
        for (int dx = -1; dx <= 1; ++dx)
            for (int dy = -1; dy <= 1; ++dy) {
                const int c = find(set[b], level[b], int64_t(ix[b]) + dx, int64_t(iy[b]) + dy);
                if (c >= 0) out[n++] = c;
            }
        return n;
    }
    __device__ bool adjacent(int a, int b) const
    {
        const int L = max(level[a], level[b]);
        const int sa = L - level[a], sb = L - level[b];
        const int64_t ax0 = int64_t(ix[a]) << sa, ax1 = int64_t(ix[a] + 1) << sa;
        const int64_t ay0 = int64_t(iy[a]) << sa, ay1 = int64_t(iy[a] + 1) << sa;
        const int64_t bx0 = int64_t(ix[b]) << sb, bx1 = int64_t(ix[b] + 1) << sb;
        const int64_t by0 = int64_t(iy[b]) << sb, by1 = int64_t(iy[b] + 1) << sb;
        return ax0 <= bx1 && bx0 <= ax1 && ay0 <= by1 && by0 <= ay1;
    }
    // the leaves under box w: entries [l0, l1) of the point-ordered leaf list
    __device__ void leaves_under(int w, int &l0, int &l1) const
    {
        auto lb = [&](int32_t v) {
            int lo = 0, hi = nleaves;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (lbeg[mid] < v) lo = mid + 1; else hi = mid;
            }
            return lo;
        };
        l0 = lb(beg[w]);
        l1 = lb(end[w]);
    }
};

constexpr int DFS_STACK = 192;

// V lists (every box) and, for leaves, the U entries of the walk and of the
// coarser adjacent leaves, and the W lists before any move.  Counts when
// the output pointers are null, else writes at the given offsets.
__global__ void k_lists(int nbox, DBoxes t, int32_t *__restrict__ vcnt, int32_t *__restrict__ ucnt,
                        int32_t *__restrict__ wcnt, const int32_t *__restrict__ v_off, int32_t *__restrict__ v_idx,
                        int32_t *__restrict__ v_cls, const int32_t *__restrict__ u_off, int32_t *__restrict__ u_idx,
                        const int32_t *__restrict__ w_off, int32_t *__restrict__ w_idx, int *__restrict__ overflow)
{
    const int b = blockIdx.x * TB + threadIdx.x;
    if (b >= nbox) return;
    const bool fill = v_idx != nullptr;
    int col[9], pcol[9];
    int nv = 0;
    if (t.parent[b] >= 0) {
        const int np = t.colleagues(t.parent[b], pcol);
        for (int k = 0; k < np; ++k) {
            const int pc = pcol[k];
            if (t.child0[pc] < 0) continue;
            for (int ch = t.child0[pc]; ch < t.child0[pc] + t.nchild[pc]; ++ch) {
                const int dx = t.ix[b] - t.ix[ch], dy = t.iy[b] - t.iy[ch];
                if (abs(dx) > 1 || abs(dy) > 1) {
                    if (fill) {
                        v_idx[v_off[b] + nv] = ch;
                        v_cls[v_off[b] + nv] = (dx + 3) * 7 + (dy + 3);
                    }
                    ++nv;
                }
            }
        }
    }
    int nu = 0, nw = 0;
    if (t.isleaf[b]) {
        int stack[DFS_STACK];
        int sp = 0;
        const int nc = t.colleagues(b, col);
        for (int k = 0; k < nc; ++k) stack[sp++] = col[k];
        while (sp > 0) {
            const int cb = stack[--sp];
            if (t.isleaf[cb]) {
                if (fill) u_idx[u_off[b] + nu] = cb;
                ++nu;
                continue;
            }
            for (int ch = t.child0[cb]; ch < t.child0[cb] + t.nchild[cb]; ++ch) {
                if (t.adjacent(b, ch)) {
                    if (sp < DFS_STACK) stack[sp++] = ch;
                    else atomicOr(overflow, 1);
                } else {
                    if (fill) w_idx[w_off[b] + nw] = ch;
                    ++nw;
                }
            }
        }
        for (int a = t.parent[b]; a >= 0; a = t.parent[a]) {
            const int na = t.colleagues(a, pcol);
            for (int k = 0; k < na; ++k) {
                const int cb = pcol[k];
                if (cb != a && t.isleaf[cb] && t.adjacent(b, cb)) {
                    if (fill) u_idx[u_off[b] + nu] = cb;
                    ++nu;
                }
            }
        }
    }
    if (!fill) {
        vcnt[b] = nv;
        ucnt[b] = nu;
        wcnt[b] = nw;
    }
}

// ascending order of each list (insertion sort per box; lists are short)
__global__ void k_sort_lists(int nbox, const int32_t *__restrict__ off, int32_t *__restrict__ idx)
{
    const int b = blockIdx.x * TB + threadIdx.x;
    if (b >= nbox) return;
    for (int i = off[b] + 1; i < off[b + 1]; ++i) {
        const int32_t v = idx[i];
        int j = i - 1;
        while (j >= off[b] && idx[j] > v) {
            idx[j + 1] = idx[j];
            --j;
        }
        idx[j + 1] = v;
    }
}

// The moves of the small W/X interactions to the near field: a W entry w of
// leaf a is small when dmax > 0 and w holds at most dmax points.  Then a's
// U list gains the leaves under w and every leaf under w gains a; W keeps
// the other entries, and X (the transpose of W) only those.  Counting pass
// (one thread per box a): own moves, kept W entries, X entries per box,
// incoming moves per leaf.
__global__ void k_moves_count(int nbox, DBoxes t, int dmax, const int32_t *__restrict__ w_off,
                              const int32_t *__restrict__ w_idx, const int32_t *__restrict__ lord,
                              int32_t *__restrict__ uown, int32_t *__restrict__ wkeep, int32_t *__restrict__ xcnt,
                              int32_t *__restrict__ uin)
{
    const int a = blockIdx.x * TB + threadIdx.x;
    if (a >= nbox) return;
    int own = 0, keep = 0;
    for (int k = w_off[a]; k < w_off[a + 1]; ++k) {
        const int w = w_idx[k];
        if (dmax > 0 && t.end[w] - t.beg[w] <= dmax) {
            int l0, l1;
            t.leaves_under(w, l0, l1);
            own += l1 - l0;
            for (int l = l0; l < l1; ++l) atomicAdd(&uin[lord[l]], 1);
        } else {
            ++keep;
            atomicAdd(&xcnt[w], 1);
        }
    }
    uown[a] = own;
    wkeep[a] = keep;
}

// Filling pass: the U list of box a is its walk entries, then the leaves
// under its small W entries, then (by atomic cursors, in any order: the
// list is sorted afterwards) the incoming moves; the kept W entries in
// order; the kept X entries by atomic cursors (sorted afterwards).
__global__ void k_moves_fill(int nbox, DBoxes t, int dmax, const int32_t *__restrict__ w0_off,
                             const int32_t *__restrict__ w0_idx, const int32_t *__restrict__ u0_off,
                             const int32_t *__restrict__ u0_idx, const int32_t *__restrict__ lord,
                             const int32_t *__restrict__ u_off, int32_t *__restrict__ u_idx, int32_t *__restrict__ ucur,
                             const int32_t *__restrict__ w_off, int32_t *__restrict__ w_idx,
                             int32_t *__restrict__ xcur, int32_t *__restrict__ x_idx)
{
    const int a = blockIdx.x * TB + threadIdx.x;
    if (a >= nbox) return;
    int o = u_off[a];
    for (int k = u0_off[a]; k < u0_off[a + 1]; ++k) u_idx[o++] = u0_idx[k];
    int ow = w_off[a];
    for (int k = w0_off[a]; k < w0_off[a + 1]; ++k) {
        const int w = w0_idx[k];
        if (dmax > 0 && t.end[w] - t.beg[w] <= dmax) {
            int l0, l1;
            t.leaves_under(w, l0, l1);
            for (int l = l0; l < l1; ++l) {
                u_idx[o++] = lord[l];
                u_idx[atomicAdd(&ucur[lord[l]], 1)] = a;
            }
        } else {
            w_idx[ow++] = w;
            x_idx[atomicAdd(&xcur[w], 1)] = a;
        }
    }
}

__global__ void k_iota_add(int n, const int32_t *__restrict__ base, const int32_t *__restrict__ a,
                           const int32_t *__restrict__ b, int32_t *__restrict__ out)
{
    const int i = blockIdx.x * TB + threadIdx.x;
    if (i < n) out[i] = base[i] + a[i] + b[i];
}

__global__ void k_sum3(int n, const int32_t *__restrict__ a, const int32_t *__restrict__ b,
                       const int32_t *__restrict__ c, int32_t *__restrict__ out)
{
    const int i = blockIdx.x * TB + threadIdx.x;
    if (i < n) out[i] = a[i] + b[i] + c[i];
}

// Temporaries of one build, freed on every path: carved from a few large
// chunks (256-byte aligned pieces), so a build makes a handful of device
// allocations instead of one per array.
struct Scratch {
    static constexpr size_t CHUNK = size_t(32) << 20;
    std::vector<DevBuf> chunks;
    size_t used = 0;                              // bytes taken from chunks.back()
    ~Scratch()
    {
        for (DevBuf &b : chunks) dev_free(b);
    }
    template <typename V>
    V *get(size_t n, imq_status &st)
    {
        const size_t bytes = (sizeof(V) * std::max<size_t>(n, 1) + 255) & ~size_t(255);
        if (chunks.empty() || used + bytes > chunks.back().bytes) {
            chunks.emplace_back();
            const hipError_t e = dev_alloc(chunks.back(), std::max(bytes, CHUNK));
            if (e != hipSuccess) {
                chunks.pop_back();
                set_error(std::string("device tree build: ") + hipGetErrorString(e));
                st = e == hipErrorOutOfMemory ? IMQ_ENOMEM : IMQ_EHIP;
                return nullptr;
            }
            used = 0;
        }
        V *p = reinterpret_cast<V *>(static_cast<char *>(chunks.back().p) + used);
        used += bytes;
        return p;
    }
};

template <typename V>
imq_status to_host(std::vector<V> &h, const V *d, size_t n, hipStream_t s)
{
    h.resize(n);
    if (n) IMQ_HIP(hipMemcpyAsync(h.data(), d, sizeof(V) * n, hipMemcpyDeviceToHost, s));
    return IMQ_OK;
}

template <typename V>
imq_status to_dev(V *d, const std::vector<V> &h, hipStream_t s)
{
    if (!h.empty()) IMQ_HIP(hipMemcpyAsync(d, h.data(), sizeof(V) * h.size(), hipMemcpyHostToDevice, s));
    return IMQ_OK;
}

// exclusive prefix sums of n counts into n + 1 offsets (counts[n] must be 0)
imq_status scan(Scratch &S, const int32_t *cnt, int32_t *off, int n, hipStream_t s)
{
    size_t bytes = 0;
    IMQ_HIP(hipcub::DeviceScan::ExclusiveSum(nullptr, bytes, cnt, off, n + 1, s));
    imq_status st = IMQ_OK;
    void *tmp = S.get<unsigned char>(bytes, st);
    if (!tmp) return st;
    IMQ_HIP(hipcub::DeviceScan::ExclusiveSum(tmp, bytes, cnt, off, n + 1, s));
    return IMQ_OK;
}

}  // namespace

// The forest of tree.cpp's build_host_tree, computed on the device from the
// device coordinates xy (x then y, N each); on return t holds the same
// partition, point order, coordinates and interaction lists as the host
// build (its remaining fields are filled by finish_host_tree).  With keep,
// the per-point arrays (perm, leaf-local x and y, scale) stay on the device
// in keep's buffers, allocated here, and t's copies of them (and of
// pt_leaf) are left empty; the near field's U-list records are made there
// too.
imq_status build_device_tree(int nsets, const int64_t *off, const double *xy, const double *c,
                             const imq_tree_params &prm, hipStream_t s, HostTree &t, const DeviceKeep *keep)
{
    imq_status st = check_tree_params(nsets, off, c, prm);
    if (st != IMQ_OK) return st;
    const int64_t N = off[nsets];
    const int max_level = prm.max_level == 0 ? MORTON_BITS : prm.max_level;
    t = HostTree();
    t.nsets = nsets;
    t.N = N;
    t.p = prm.order_p;
    t.K = Kof(t.p);
    t.set_off.assign(off, off + nsets + 1);
    t.c.assign(c, c + nsets);
    t.side.resize(nsets); t.lox.resize(nsets); t.loy.resize(nsets); t.cn.resize(nsets);
    const double *x = xy, *y = xy + N;

    Scratch S;
#define TMP(var, V, n)                          \
    V *var = S.get<V>(size_t(n), st);           \
    if (!var) return st
    TMP(d_off, int64_t, nsets + 1);
    IMQ_HIP(hipMemcpyAsync(d_off, off, sizeof(int64_t) * (nsets + 1), hipMemcpyHostToDevice, s));
    // ---- bounding squares
    int64_t max_set = 0;
    for (int k = 0; k < nsets; ++k) max_set = std::max(max_set, off[k + 1] - off[k]);
    const int nbs = int(std::min<int64_t>(256, std::max<int64_t>(1, (max_set + 16 * TB - 1) / (16 * TB))));
    TMP(d_part, double, 4 * size_t(nsets) * nbs);
    TMP(d_bnd, double, 4 * nsets);
    TMP(d_bad, int, 1);
    IMQ_HIP(hipMemsetAsync(d_bad, 0, sizeof(int), s));
    hipLaunchKernelGGL(k_bounds, dim3(nbs, nsets), dim3(TB), 0, s, d_off, x, y, d_part, d_bad);
    hipLaunchKernelGGL(k_bounds_final, dim3(nblk(nsets)), dim3(TB), 0, s, nsets, nbs, d_part, d_bnd);
    std::vector<double> bnd(4 * size_t(nsets));
    int bad = 0;
    IMQ_HIP(hipMemcpyAsync(bnd.data(), d_bnd, sizeof(double) * bnd.size(), hipMemcpyDeviceToHost, s));
    IMQ_HIP(hipMemcpyAsync(&bad, d_bad, sizeof(int), hipMemcpyDeviceToHost, s));
    IMQ_HIP(hipStreamSynchronize(s));
    if (bad) { set_error("non-finite coordinate"); return IMQ_EINVAL; }
    std::vector<double> geo(3 * size_t(nsets));
    for (int k = 0; k < nsets; ++k) {
        const double x0 = bnd[4 * k], x1 = bnd[4 * k + 1], y0 = bnd[4 * k + 2], y1 = bnd[4 * k + 3];
        const double ext = std::max(x1 - x0, y1 - y0);
        const double side = ext > 0 ? ext * (1.0 + std::ldexp(1.0, -20)) : 1.0;
        t.side[k] = side; t.lox[k] = x0; t.loy[k] = y0; t.cn[k] = c[k] / side;
        geo[3 * k] = x0; geo[3 * k + 1] = y0; geo[3 * k + 2] = side;
    }
    TMP(d_geo, double, 3 * nsets);
    if ((st = to_dev(d_geo, geo, s)) != IMQ_OK) return st;
    // ---- keys and the stable sort per set
    TMP(key0, uint64_t, N);
    TMP(idx0, int32_t, N);
    TMP(key, uint64_t, N);
    int32_t *perm = nullptr;
    if (keep) {
        IMQ_HIP(dev_alloc(*keep->perm, sizeof(int32_t) * N));
        perm = keep->perm->as<int32_t>();
    } else {
        TMP(perm_tmp, int32_t, N);
        perm = perm_tmp;
    }
    hipLaunchKernelGGL(k_keys, dim3(nblk(N)), dim3(TB), 0, s, N, nsets, d_off, x, y, d_geo, key0, idx0);
    {
        size_t bytes = 0;
        if (nsets == 1) {
            IMQ_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, bytes, key0, key, idx0, perm, int(N), 0,
                                                       2 * MORTON_BITS, s));
            TMP(tmp, unsigned char, bytes);
            IMQ_HIP(hipcub::DeviceRadixSort::SortPairs(tmp, bytes, key0, key, idx0, perm, int(N), 0,
                                                       2 * MORTON_BITS, s));
        } else {
            std::vector<int32_t> off32(off, off + nsets + 1);
            TMP(d_off32, int32_t, nsets + 1);
            if ((st = to_dev(d_off32, off32, s)) != IMQ_OK) return st;
            IMQ_HIP(hipcub::DeviceSegmentedRadixSort::SortPairs(nullptr, bytes, key0, key, idx0, perm, int(N), nsets,
                                                                d_off32, d_off32 + 1, 0, 2 * MORTON_BITS, s));
            TMP(tmp, unsigned char, bytes);
            IMQ_HIP(hipcub::DeviceSegmentedRadixSort::SortPairs(tmp, bytes, key0, key, idx0, perm, int(N), nsets,
                                                                d_off32, d_off32 + 1, 0, 2 * MORTON_BITS, s));
            IMQ_HIP(hipStreamSynchronize(s));          // off32 goes out of scope
        }
    }
    {
        TMP(d_first, unsigned long long, 1);
        IMQ_HIP(hipMemsetAsync(d_first, 0xff, sizeof(unsigned long long), s));
        hipLaunchKernelGGL(k_dups, dim3(nblk(N)), dim3(TB), 0, s, N, nsets, d_off, key, perm, x, y, d_first);
        unsigned long long first = 0;
        IMQ_HIP(hipMemcpyAsync(&first, d_first, sizeof(first), hipMemcpyDeviceToHost, s));
        IMQ_HIP(hipStreamSynchronize(s));
        if (first != ~0ull) {
            int32_t pa = 0, pb = 0;
            IMQ_HIP(hipMemcpy(&pa, perm + (first >> 32), sizeof(int32_t), hipMemcpyDeviceToHost));
            IMQ_HIP(hipMemcpy(&pb, perm + (first & 0xffffffffull), sizeof(int32_t), hipMemcpyDeviceToHost));
            set_error("duplicate data sites: points " + std::to_string(pa) + " and " + std::to_string(pb));
            return IMQ_EDUPLICATE;
        }
    }
    TMP(xn, double, N);
    TMP(yn, double, N);
    hipLaunchKernelGGL(k_normal, dim3(nblk(N)), dim3(TB), 0, s, N, nsets, d_off, perm, x, y, d_geo, xn, yn);
    IMQ_HIP(hipGetLastError());

    // ---- adaptive split, level by level
    std::vector<LevelBoxes> lv(1);
    {
        LevelBoxes &L0 = lv[0];
        L0.n = nsets;
        std::vector<int32_t> sset(nsets), zero(nsets, 0), beg(nsets), en(nsets), par(nsets, -1);
        for (int k = 0; k < nsets; ++k) {
            sset[k] = k;
            beg[k] = int32_t(off[k]);
            en[k] = int32_t(off[k + 1]);
        }
        for (int32_t **b : {&L0.set, &L0.ix, &L0.iy, &L0.beg, &L0.end, &L0.parent, &L0.pos})
            if (!(*b = S.get<int32_t>(nsets, st))) return st;
        if ((st = to_dev(L0.set, sset, s)) != IMQ_OK) return st;
        if ((st = to_dev(L0.ix, zero, s)) != IMQ_OK) return st;
        if ((st = to_dev(L0.iy, zero, s)) != IMQ_OK) return st;
        if ((st = to_dev(L0.beg, beg, s)) != IMQ_OK) return st;
        if ((st = to_dev(L0.end, en, s)) != IMQ_OK) return st;
        if ((st = to_dev(L0.parent, par, s)) != IMQ_OK) return st;
        if ((st = to_dev(L0.pos, zero, s)) != IMQ_OK) return st;
        IMQ_HIP(hipStreamSynchronize(s));             // the host vectors go out of scope
    }
    t.level_begin.push_back(0);
    int base = 0;
    for (int l = 0;; ++l) {
        LevelBoxes &L = lv[l];
        const int n = L.n;
        t.level_begin.push_back(base + n);
        for (int32_t **b : {&L.child0, &L.nchild})
            if (!(*b = S.get<int32_t>(n, st))) return st;
        if (l >= max_level) {
            std::vector<int32_t> m1(n, -1), z(n, 0);
            if ((st = to_dev(L.child0, m1, s)) != IMQ_OK) return st;
            if ((st = to_dev(L.nchild, z, s)) != IMQ_OK) return st;
            IMQ_HIP(hipStreamSynchronize(s));
            break;
        }
        if (!(L.cnt = S.get<int32_t>(size_t(n) + 1, st))) return st;
        if (!(L.first = S.get<int32_t>(size_t(n) + 1, st))) return st;
        if (!(L.cut = S.get<int32_t>(5 * size_t(n), st))) return st;
        IMQ_HIP(hipMemsetAsync(L.cnt, 0, sizeof(int32_t) * (n + 1), s));
        hipLaunchKernelGGL(k_split_count, dim3(nblk(n)), dim3(TB), 0, s, n, l, prm.leaf_max, L.beg, L.end, key,
                           L.cnt, L.cut);
        if ((st = scan(S, L.cnt, L.first, n, s)) != IMQ_OK) return st;
        int32_t total = 0;
        IMQ_HIP(hipMemcpyAsync(&total, L.first + n, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        IMQ_HIP(hipStreamSynchronize(s));
        LevelBoxes nx;
        nx.n = total;
        if (total > 0)
            for (int32_t **b : {&nx.set, &nx.ix, &nx.iy, &nx.beg, &nx.end, &nx.parent, &nx.pos})
                if (!(*b = S.get<int32_t>(total, st))) return st;
        hipLaunchKernelGGL(k_split_fill, dim3(nblk(n)), dim3(TB), 0, s, n, base + n, L.set, L.ix, L.iy, base, L.cnt,
                           L.first, L.cut, L.child0, L.nchild, nx.set, nx.ix, nx.iy, nx.beg, nx.end, nx.parent,
                           nx.pos);
        IMQ_HIP(hipGetLastError());
        base += n;
        if (total == 0) break;
        lv.push_back(nx);
    }
    const int nbox = t.level_begin.back();
    t.nlev = int(t.level_begin.size()) - 1;

    // ---- box arrays: one device array each (levels concatenated), copied to the host
    TMP(d_level, int32_t, nbox + 1);
    TMP(d_set, int32_t, nbox + 1);
    TMP(d_ix, int32_t, nbox + 1);
    TMP(d_iy, int32_t, nbox + 1);
    TMP(d_par, int32_t, nbox + 1);
    TMP(d_c0, int32_t, nbox + 1);
    TMP(d_nc, int32_t, nbox + 1);
    TMP(d_pos, int32_t, nbox + 1);
    TMP(d_beg, int32_t, nbox + 1);
    TMP(d_end, int32_t, nbox + 1);
    TMP(d_leaf, int32_t, nbox + 1);
    {
        std::vector<int32_t> lvl(nbox);
        for (int l = 0; l < t.nlev; ++l)
            std::fill(lvl.begin() + t.level_begin[l], lvl.begin() + t.level_begin[l + 1], l);
        if ((st = to_dev(d_level, lvl, s)) != IMQ_OK) return st;
        int o = 0;
        for (int l = 0; l < t.nlev; ++l) {
            const LevelBoxes &L = lv[l];
            const size_t bytes = sizeof(int32_t) * L.n;
            const std::pair<int32_t *, const int32_t *> cp[] = {{d_set, L.set}, {d_ix, L.ix}, {d_iy, L.iy},
                                                               {d_par, L.parent}, {d_c0, L.child0},
                                                               {d_nc, L.nchild}, {d_pos, L.pos}, {d_beg, L.beg},
                                                               {d_end, L.end}};
            for (const auto &e : cp)
                IMQ_HIP(hipMemcpyAsync(e.first + o, e.second, bytes, hipMemcpyDeviceToDevice, s));
            o += L.n;
        }
        t.level = lvl;
        IMQ_HIP(hipStreamSynchronize(s));
    }
    if ((st = to_host(t.set, d_set, nbox, s)) != IMQ_OK) return st;
    if ((st = to_host(t.ix, d_ix, nbox, s)) != IMQ_OK) return st;
    if ((st = to_host(t.iy, d_iy, nbox, s)) != IMQ_OK) return st;
    if ((st = to_host(t.parent, d_par, nbox, s)) != IMQ_OK) return st;
    if ((st = to_host(t.child0, d_c0, nbox, s)) != IMQ_OK) return st;
    if ((st = to_host(t.nchild, d_nc, nbox, s)) != IMQ_OK) return st;
    if ((st = to_host(t.pos, d_pos, nbox, s)) != IMQ_OK) return st;
    if ((st = to_host(t.begin, d_beg, nbox, s)) != IMQ_OK) return st;
    if ((st = to_host(t.end, d_end, nbox, s)) != IMQ_OK) return st;
    IMQ_HIP(hipStreamSynchronize(s));
    t.isleaf.resize(nbox);
    t.cx.resize(nbox);
    t.cy.resize(nbox);
    for (int b = 0; b < nbox; ++b) {
        t.isleaf[b] = t.nchild[b] == 0 ? 1 : 0;
        const double sz = std::ldexp(1.0, -t.level[b]);
        t.cx[b] = (double(t.ix[b]) + 0.5) * sz;
        t.cy[b] = (double(t.iy[b]) + 0.5) * sz;
        if (t.isleaf[b]) t.leaves.push_back(b);
    }
    t.Klev.resize(t.nlev);
    for (int l = 0; l < t.nlev; ++l) {
        int pl = (l <= IMQ_MAX_LEVELS && prm.level_order[l] > 0) ? prm.level_order[l] : t.p;
        t.Klev[l] = Kof(std::min(pl, t.p));
    }
    const int nleaves = int(t.leaves.size());
    // leaves in point order (box indices) and their first points
    std::vector<int32_t> lord(t.leaves), lbeg(nleaves);
    std::sort(lord.begin(), lord.end(), [&](int32_t a, int32_t b) { return t.begin[a] < t.begin[b]; });
    for (int i = 0; i < nleaves; ++i) lbeg[i] = t.begin[lord[i]];
    // first box of every (level, set)
    std::vector<int32_t> lsb(size_t(t.nlev) * (nsets + 1));
    for (int l = 0; l < t.nlev; ++l) {
        int b = t.level_begin[l];
        for (int k = 0; k <= nsets; ++k) {
            while (b < t.level_begin[l + 1] && t.set[b] < k) ++b;
            lsb[size_t(l) * (nsets + 1) + k] = b;
        }
        lsb[size_t(l) * (nsets + 1) + nsets] = t.level_begin[l + 1];
    }
    TMP(d_leaves, int32_t, nleaves);
    TMP(d_lord, int32_t, nleaves);
    TMP(d_lbeg, int32_t, nleaves);
    TMP(d_lsb, int32_t, lsb.size());
    if ((st = to_dev(d_leaves, t.leaves, s)) != IMQ_OK) return st;
    if ((st = to_dev(d_lord, lord, s)) != IMQ_OK) return st;
    if ((st = to_dev(d_lbeg, lbeg, s)) != IMQ_OK) return st;
    if ((st = to_dev(d_lsb, lsb, s)) != IMQ_OK) return st;
    {
        std::vector<int32_t> isl(t.isleaf);
        if ((st = to_dev(d_leaf, isl, s)) != IMQ_OK) return st;
        IMQ_HIP(hipStreamSynchronize(s));
    }

    // ---- points
    double *d_xl = nullptr, *d_yl = nullptr, *d_sc = nullptr;
    if (keep) {
        for (DevBuf *b : {keep->xl, keep->yl, keep->scale}) IMQ_HIP(dev_alloc(*b, sizeof(double) * N));
        d_xl = keep->xl->as<double>();
        d_yl = keep->yl->as<double>();
        d_sc = keep->scale->as<double>();
    } else {
        TMP(xl_tmp, double, N);
        TMP(yl_tmp, double, N);
        TMP(sc_tmp, double, N);
        d_xl = xl_tmp;
        d_yl = yl_tmp;
        d_sc = sc_tmp;
    }
    TMP(d_pl, int32_t, N);
    TMP(d_r2, double, nleaves);
    hipLaunchKernelGGL(k_points, dim3(nleaves), dim3(64), 0, s, d_leaves, d_level, d_set, d_ix, d_iy, d_beg, d_end,
                       d_geo, xn, yn, d_xl, d_yl, d_sc, d_pl, d_r2);
    IMQ_HIP(hipGetLastError());

    // ---- lists
    DBoxes db{d_level, d_set, d_ix, d_iy, d_par, d_c0, d_nc, d_beg, d_end, d_leaf, d_lsb, d_lbeg, nsets, nleaves};
    TMP(vcnt, int32_t, nbox + 1);
    TMP(u0cnt, int32_t, nbox + 1);
    TMP(w0cnt, int32_t, nbox + 1);
    TMP(d_ovf, int, 1);
    for (int32_t *p : {vcnt, u0cnt, w0cnt}) IMQ_HIP(hipMemsetAsync(p, 0, sizeof(int32_t) * (nbox + 1), s));
    IMQ_HIP(hipMemsetAsync(d_ovf, 0, sizeof(int), s));
    hipLaunchKernelGGL(k_lists, dim3(nblk(nbox)), dim3(TB), 0, s, nbox, db, vcnt, u0cnt, w0cnt, nullptr, nullptr,
                       nullptr, nullptr, nullptr, nullptr, nullptr, d_ovf);
    TMP(v_off, int32_t, nbox + 1);
    TMP(u0_off, int32_t, nbox + 1);
    TMP(w0_off, int32_t, nbox + 1);
    if ((st = scan(S, vcnt, v_off, nbox, s)) != IMQ_OK) return st;
    if ((st = scan(S, u0cnt, u0_off, nbox, s)) != IMQ_OK) return st;
    if ((st = scan(S, w0cnt, w0_off, nbox, s)) != IMQ_OK) return st;
    int32_t tot[3] = {0, 0, 0};
    IMQ_HIP(hipMemcpyAsync(&tot[0], v_off + nbox, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    IMQ_HIP(hipMemcpyAsync(&tot[1], u0_off + nbox, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    IMQ_HIP(hipMemcpyAsync(&tot[2], w0_off + nbox, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    IMQ_HIP(hipStreamSynchronize(s));
    TMP(v_idx, int32_t, tot[0]);
    TMP(v_cls, int32_t, tot[0]);
    TMP(u0_idx, int32_t, tot[1]);
    TMP(w0_idx, int32_t, tot[2]);
    hipLaunchKernelGGL(k_lists, dim3(nblk(nbox)), dim3(TB), 0, s, nbox, db, nullptr, nullptr, nullptr, v_off, v_idx,
                       v_cls, u0_off, u0_idx, w0_off, w0_idx, d_ovf);
    hipLaunchKernelGGL(k_sort_lists, dim3(nblk(nbox)), dim3(TB), 0, s, nbox, w0_off, w0_idx);
    IMQ_HIP(hipGetLastError());
    // moves of the small W/X interactions (none when dmax <= 0)
    const int dmax = prm.direct_max == 0 ? 2 * prm.leaf_max : prm.direct_max;
    TMP(uown, int32_t, nbox + 1);
    TMP(uin, int32_t, nbox + 1);
    TMP(wkeep, int32_t, nbox + 1);
    TMP(xcnt, int32_t, nbox + 1);
    TMP(ucnt, int32_t, nbox + 1);
    for (int32_t *p : {uown, uin, wkeep, xcnt, ucnt}) IMQ_HIP(hipMemsetAsync(p, 0, sizeof(int32_t) * (nbox + 1), s));
    hipLaunchKernelGGL(k_moves_count, dim3(nblk(nbox)), dim3(TB), 0, s, nbox, db, dmax, w0_off, w0_idx, d_lord, uown,
                       wkeep, xcnt, uin);
    hipLaunchKernelGGL(k_sum3, dim3(nblk(nbox)), dim3(TB), 0, s, nbox, u0cnt, uown, uin, ucnt);
    TMP(u_off, int32_t, nbox + 1);
    TMP(w_off, int32_t, nbox + 1);
    TMP(x_off, int32_t, nbox + 1);
    if ((st = scan(S, ucnt, u_off, nbox, s)) != IMQ_OK) return st;
    if ((st = scan(S, wkeep, w_off, nbox, s)) != IMQ_OK) return st;
    if ((st = scan(S, xcnt, x_off, nbox, s)) != IMQ_OK) return st;
    int32_t tot2[3] = {0, 0, 0}, ovf = 0;
    IMQ_HIP(hipMemcpyAsync(&tot2[0], u_off + nbox, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    IMQ_HIP(hipMemcpyAsync(&tot2[1], w_off + nbox, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    IMQ_HIP(hipMemcpyAsync(&tot2[2], x_off + nbox, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    IMQ_HIP(hipMemcpyAsync(&ovf, d_ovf, sizeof(int), hipMemcpyDeviceToHost, s));
    IMQ_HIP(hipStreamSynchronize(s));
    if (ovf) {
        set_error("device tree build: list walk deeper than its stack");
        return IMQ_EUNSUPPORTED;
    }
    TMP(u_idx, int32_t, tot2[0]);
    TMP(w_idx, int32_t, tot2[1]);
    TMP(x_idx, int32_t, tot2[2]);
    TMP(ucur, int32_t, nbox + 1);
    TMP(xcur, int32_t, nbox + 1);
    // incoming U entries go after each box's own entries; X entries from the start
    hipLaunchKernelGGL(k_iota_add, dim3(nblk(nbox)), dim3(TB), 0, s, nbox, u_off, u0cnt, uown, ucur);
    IMQ_HIP(hipMemcpyAsync(xcur, x_off, sizeof(int32_t) * (nbox + 1), hipMemcpyDeviceToDevice, s));
    hipLaunchKernelGGL(k_moves_fill, dim3(nblk(nbox)), dim3(TB), 0, s, nbox, db, dmax, w0_off, w0_idx, u0_off, u0_idx,
                       d_lord, u_off, u_idx, ucur, w_off, w_idx, xcur, x_idx);
    hipLaunchKernelGGL(k_sort_lists, dim3(nblk(nbox)), dim3(TB), 0, s, nbox, u_off, u_idx);
    hipLaunchKernelGGL(k_sort_lists, dim3(nblk(nbox)), dim3(TB), 0, s, nbox, x_off, x_idx);
    IMQ_HIP(hipGetLastError());
    if (keep) {
        IMQ_HIP(dev_alloc(*keep->urec64, sizeof(URec<double>) * std::max(tot2[0], 1)));
        IMQ_HIP(dev_alloc(*keep->urec32, sizeof(URec<float>) * std::max(tot2[0], 1)));
        hipLaunchKernelGGL(k_urec, dim3(nblk(nbox)), dim3(TB), 0, s, nbox, d_level, d_ix, d_iy, d_beg, d_end, u_off,
                           u_idx, keep->urec64->as<URec<double>>(), keep->urec32->as<URec<float>>());
        IMQ_HIP(hipGetLastError());
    }

    // ---- back to the host tree
    if (!keep) {
        if ((st = to_host(t.xl, d_xl, N, s)) != IMQ_OK) return st;
        if ((st = to_host(t.yl, d_yl, N, s)) != IMQ_OK) return st;
        if ((st = to_host(t.pt_scale, d_sc, N, s)) != IMQ_OK) return st;
        if ((st = to_host(t.pt_leaf, d_pl, N, s)) != IMQ_OK) return st;
        if ((st = to_host(t.perm, perm, N, s)) != IMQ_OK) return st;
    }
    std::vector<double> leaf_r2;
    if ((st = to_host(leaf_r2, d_r2, nleaves, s)) != IMQ_OK) return st;
    if ((st = to_host(t.u_off, u_off, nbox + 1, s)) != IMQ_OK) return st;
    if ((st = to_host(t.u_idx, u_idx, tot2[0], s)) != IMQ_OK) return st;
    if ((st = to_host(t.v_off, v_off, nbox + 1, s)) != IMQ_OK) return st;
    if ((st = to_host(t.v_idx, v_idx, tot[0], s)) != IMQ_OK) return st;
    if ((st = to_host(t.v_cls, v_cls, tot[0], s)) != IMQ_OK) return st;
    if ((st = to_host(t.w_off, w_off, nbox + 1, s)) != IMQ_OK) return st;
    if ((st = to_host(t.w_idx, w_idx, tot2[1], s)) != IMQ_OK) return st;
    if ((st = to_host(t.x_off, x_off, nbox + 1, s)) != IMQ_OK) return st;
    if ((st = to_host(t.x_idx, x_idx, tot2[2], s)) != IMQ_OK) return st;
    IMQ_HIP(hipStreamSynchronize(s));
#undef TMP
    return finish_host_tree(t, &leaf_r2);
}

}  // namespace imq
