// HIP kernels of the fast product b = A u and their schedule.
//
// Stage order (one product):
//   gather   u -> Morton order, arithmetic type T
//   P2M      leaf expansions from points (the v_k, w_k sums of Algorithm 1)
//   M2M      children -> parent, level by level upward
//   M2L      source box -> target box of the same level (V list)
//   P2L      points of a coarser leaf -> local expansion (X list)
//   L2L      parent -> children, level by level downward
//   L2P      local expansion evaluated at the leaf's points
//   P2P      direct near field (last loop of Algorithm 1, U list)
//   M2P      multipole of a finer box evaluated at points (W list)
//   scatter  FP64 result -> caller order and type, times 1/side
#include "device.h"
#include "mfma.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

namespace imq {

// ------------------------------------------------------------------ helpers

__device__ __forceinline__ int cidx(int n, int m) { return n * (n + 1) / 2 + (m > 0 ? m - 1 : 0); }

__device__ __forceinline__ float rsqrt_t(float x) { return __frsqrt_rn(x); }
__device__ __forceinline__ double rsqrt_t(double x) { return 1.0 / sqrt(x); }

template <typename T> __device__ __forceinline__ T pow2i(int l) { return T(ldexp(1.0, l)); }

// Irregular solid harmonics I_n^m(v), 0 <= m <= n <= P, generated column by
// column in m with the three-term recurrence in n; calls f(n, m, re, im)
// for every n+m-even pair.
template <typename T, typename F>
__device__ __forceinline__ void irregular_even(int P, T vx, T vy, T vz, F &&f)
{
    const T r2 = vx * vx + vy * vy + vz * vz;
    const T inv_r2 = T(1) / r2;
    T mr = rsqrt_t(r2), mi = T(0);                 // I_m^m
    for (int m = 0; m <= P; ++m) {
        if (m > 0) {
            const T a = -T(2 * m - 1) * inv_r2;
            const T nr = a * (vx * mr - vy * mi);
            const T ni = a * (vx * mi + vy * mr);
            mr = nr;
            mi = ni;
        }
        T p2r = 0, p2i = 0, p1r = mr, p1i = mi;   // I_{n-2}^m, I_{n-1}^m
        f(m, m, mr, mi);
        for (int n = m + 1; n <= P; ++n) {
            const T a = T(2 * n - 1) * vz;
            const T b = T((n + m - 1) * (n - m - 1));
            const T cr = (a * p1r - b * p2r) * inv_r2;
            const T ci = (a * p1i - b * p2i) * inv_r2;
            if (((n + m) & 1) == 0) f(n, m, cr, ci);
            p2r = p1r; p2i = p1i; p1r = cr; p1i = ci;
        }
    }
}

// ------------------------------------------------------------------ kernels


template <typename Tin, typename T>
__global__ void k_gather(int64_t N, const int32_t *__restrict__ perm, const Tin *__restrict__ u,
                         int64_t ldu, T *__restrict__ us)
{
    tree_pass_priority();
    const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    const int r = blockIdx.y;
    if (i < N) us[r * N + i] = T(u[r * ldu + perm[i]]);
}

template <typename Tout>
__global__ void k_scatter(int64_t N, const int32_t *__restrict__ perm, const double *__restrict__ scale,
                          const double *__restrict__ bs, Tout *__restrict__ b, int64_t ldb)
{
    tree_pass_priority();
    const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    const int r = blockIdx.y;
    if (i < N) b[r * ldb + perm[i]] = Tout(bs[r * N + i] * scale[i]);
}

// Monomials of one point for every stored coefficient: f(k, value, imag)
// with value the real (imag = false) or imaginary part of |w|^(n-m) w^m (the
// caller passes conj(w) for multipoles).  P is a compile-time order, so every
// coefficient index is a constant.
template <int P, typename T, typename F>
__device__ __forceinline__ void monomials(T wx, T wy, F &&f)
{
    const T r2 = wx * wx + wy * wy;
    T pr = T(1), pi = T(0);
#pragma unroll
    for (int m = 0; m <= P; ++m) {
        T tr = pr, ti = pi;
#pragma unroll
        for (int n = m; n <= P; n += 2) {
            const int k = n * (n + 1) / 2 + (m > 0 ? m - 1 : 0);
            f(k, tr, false);
            if (m > 0) f(k + 1, ti, true);
            tr *= r2;
            ti *= r2;
        }
        const T nr = pr * wx - pi * wy;
        pi = pr * wy + pi * wx;
        pr = nr;
    }
}

// Launch kern<T, P>(args...) for the runtime order p in [1, 16].
#define IMQ_DISPATCH_P(p, LAUNCH)                                                        \
    switch (p) {                                                                         \
    case 1: LAUNCH(1); break;   case 2: LAUNCH(2); break;   case 3: LAUNCH(3); break;   \
    case 4: LAUNCH(4); break;   case 5: LAUNCH(5); break;   case 6: LAUNCH(6); break;   \
    case 7: LAUNCH(7); break;   case 8: LAUNCH(8); break;   case 9: LAUNCH(9); break;   \
    case 10: LAUNCH(10); break; case 11: LAUNCH(11); break; case 12: LAUNCH(12); break; \
    case 13: LAUNCH(13); break; case 14: LAUNCH(14); break; case 15: LAUNCH(15); break; \
    default: LAUNCH(16); break;                                                          \
    }

// Column sums of an LDS matrix: sum_{j < n} a[j*ld + k] * w[j], unrolled so
// that several reads are in flight.
template <typename T>
__device__ __forceinline__ T lds_dot(const T *a, int ld, int k, const T *w, int n)
{
    T s0 = T(0), s1 = T(0), s2 = T(0), s3 = T(0);
    int j = 0;
    for (; j + 4 <= n; j += 4) {
        s0 += a[j * ld + k] * w[j];
        s1 += a[(j + 1) * ld + k] * w[j + 1];
        s2 += a[(j + 2) * ld + k] * w[j + 2];
        s3 += a[(j + 3) * ld + k] * w[j + 3];
    }
    for (; j < n; ++j) s0 += a[j * ld + k] * w[j];
    return (s0 + s1) + (s2 + s3);
}

// P2M: Mt[n,m] = sum_j u_j |w_j|^(n-m) conj(w_j)^m over a leaf's points.
// With n = m + 2e the coefficient is sum_j (u_j |w_j|^(2e)) conj(w_j)^m:
// each lane (a point of the chunk) writes its powers conj(w)^m, m <= P, and
// u |w|^(2e), e <= P/2, as one row of an LDS matrix (odd row stride, 3P/2 + 3
// values where the monomials would be (P+1)(P+2)/2), and each lane then
// forms its coefficients as sums over the rows of the product of two entries
// (the same entry for every lane of one m or one e: mostly broadcast reads).
// With caller-order weights the kernels also store them in point order (us),
// for the stages that read them there.
constexpr int P2M_CHUNK = 64;      // points staged per round
constexpr int P2M_PIPE_CH = 32;    // the same in the one-column kernel (occupancy)
constexpr int P2M_PIPE_WG = 8192;  // its workgroups
constexpr int LEAF_WG_MAX = 4096;  // workgroups of the leaf-by-leaf kernels (P2M, L2P)
template <int P> constexpr int p2m_ld() { return (2 * (P + 1) + P / 2 + 1) | 1; }

// The chunk's rows and the coefficient sums, shared by both P2M kernels.
// A point's row holds the monomials conj(w)^m (re, im) for m <= P and the
// weighted radial powers u |w|^(2e), e <= P/2; coefficient (n, m) of the
// leaf is the sum over points of  conj(w)^m  times  u |w|^(n-m).  Over a
// chunk this is one small matrix product on the matrix cores,
//     C[w][e] = sum_j  row_j[w] row_j[EOFF + e]     (2(P+1) x points) x (points x (P/2+1)),
// four points per 16x16x4 step, and coefficient (n, m) is C[2m (+1)][(n-m)/2].
template <typename T, int P>
struct P2MRows {
    static constexpr int K = (P + 1) * (P + 2) / 2;
    static constexpr int LD = p2m_ld<P>();
    static constexpr int NW = 2 * (P + 1);        // monomial entries of a row
    static constexpr int EOFF = NW;               // then u |w|^(2e)
    static constexpr int NE = P / 2 + 1;
    static constexpr int NT = (NW + 15) / 16;     // 16-row tiles of C
    static_assert(NE <= 16, "radial powers per column tile");
    using acc_t = typename Mfma<T>::acc_t;
    // row of one point: w = (x, -y) / s, weight u
    __device__ __forceinline__ static void write(T *row, T wx, T wy, T u)
    {
        const T rr = wx * wx + wy * wy;
        T pr = T(1), pi = T(0);
#pragma unroll
        for (int m = 0; m <= P; ++m) {
            row[2 * m] = pr;
            row[2 * m + 1] = pi;
            const T t_ = pr * wx - pi * wy;
            pi = pr * wy + pi * wx;
            pr = t_;
        }
        T q = u;
#pragma unroll
        for (int e = 0; e < NE; ++e) {
            row[EOFF + e] = q;
            q *= rr;
        }
    }
    __device__ __forceinline__ static void clear(acc_t (&acc)[NT])
    {
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[t][v] = T(0);
    }
    // acc += C over the rows j < n of S (n a multiple of 4 at most the rows
    // S holds, or less than that): lane l feeds row l%16 of
    // each tile and radial power l%16 of point 4 s + l/16 in step s; rows
    // past n and entries past the row's count enter as zeros
    __device__ __forceinline__ static void sums(const T *S, int n, int lane, acc_t (&acc)[NT])
    {
        const int r16 = lane & 15, q = lane >> 4;
        for (int j0 = 0; j0 < n; j0 += 4) {
            const int j = j0 + q;                     // a row of S: j0 < n, j0 % 4 == 0
            const T *row = S + j * LD;
            const bool ok = j < n;
            const T bv = row[EOFF + (r16 < NE ? r16 : 0)];
            const T b = (ok && r16 < NE) ? bv : T(0);
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                const int w = 16 * t + r16;
                const T av = row[w < NW ? w : 0];
                acc[t] = Mfma<T>::mac((ok && w < NW) ? av : T(0), b, acc[t]);
            }
        }
    }
    // M[k] for the coefficients this lane holds: C[w][e] with w = 2m + part,
    // n = m + 2e, stored at n(n+1)/2 + max(m-1, 0) + part
    __device__ __forceinline__ static void store(const acc_t (&acc)[NT], int lane, T *__restrict__ Mb)
    {
        const int e = lane & 15, q = lane >> 4;
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int w = 16 * t + Mfma<T>::row(q, v);
                const int m = w >> 1, part = w & 1, n = m + 2 * e;
                if (w < NW && e < NE && n <= P && (m > 0 || part == 0))
                    Mb[n * (n + 1) / 2 + (m > 0 ? m - 1 : 0) + part] = acc[t][v];
            }
    }
};

// IN: where the weights are read: 0 = us (point order), 1 = the caller's FP64
// vector, 2 = the caller's FP32 vector (caller order, through io.perm).
template <typename T, int IN>
__device__ __forceinline__ T p2m_weight(const UserVec &io, const T *us, int64_t N, int j, int r)
{
    if constexpr (IN == 0) return us[r * N + j];
    else if constexpr (IN == 1) return T(static_cast<const double *>(io.in)[r * io.ldu + j]);
    else return T(static_cast<const float *>(io.in)[r * io.ldu + j]);
}

// One right-hand side, leaves of at most 64 points (a lane per point; the
// rows go through LDS P2M_PIPE_CH at a time, which keeps the LDS of a
// workgroup small enough for many leaves in flight per CU).  recs: the
// leaves; workgroup g takes leaves g, g + G, ... (G workgroups).  The point
// and weight of the next leaf are requested before the current leaf is
// worked on, and the point and caller-order index of the leaf after it one
// leaf earlier still, so neither the loads nor the gather of caller-order
// weights (two dependent loads) stall the wave; no other load is issued in
// the loop.
template <typename T, int P, int IN>
__global__ __launch_bounds__(64) void k_p2m_pipe(DTree<T> t, const LeafRec *__restrict__ recs, int nrec,
                                                 T *__restrict__ us, T *__restrict__ M, UserVec io)
{
    tree_pass_priority();
    using R = P2MRows<T, P>;
    __shared__ T S[P2M_PIPE_CH * R::LD];
    const int lane = threadIdx.x;
    const int G = gridDim.x;
    int li = blockIdx.x;
    if (li >= nrec) return;
    struct Pa {                                      // point, caller-order index of its weight
        T x, y;
        int j;
    };
    struct Pb {                                      // point, weight
        T x, y, u;
    };
    // lanes past the leaf read its first point, an empty leaf point 0
    auto stage_a = [&](const LeafRec &r) -> Pa {
        const int ip = r.end > r.begin ? r.begin + (lane < r.end - r.begin ? lane : 0) : 0;
        if constexpr (IN == 0) return Pa{t.xl[ip], t.yl[ip], ip};
        else return Pa{t.xl[ip], t.yl[ip], io.perm[ip]};
    };
    auto stage_b = [&](const Pa &a) -> Pb { return Pb{a.x, a.y, p2m_weight<T, IN>(io, us, t.N, a.j, 0)}; };
    // records of the current leaf and the two after it (the current one
    // stands in past the end: loaded again, not used)
    LeafRec lr = recs[li];
    LeafRec r1 = li + G < nrec ? recs[li + G] : lr;
    LeafRec r2 = li + 2 * G < nrec ? recs[li + 2 * G] : lr;
    Pb cur = stage_b(stage_a(lr));
    Pa nxa = stage_a(r1);
    for (;;) {
        const bool more = li + G < nrec;
        const Pb nxb = stage_b(nxa);
        const Pa nna = stage_a(r2);
        const int n = lr.end - lr.begin;
        if (IN != 0 && lane < n) us[lr.begin + lane] = cur.u;
        typename R::acc_t acc[R::NT];
        R::clear(acc);
        for (int c = 0; c < n; c += P2M_PIPE_CH) {
            __syncthreads();                         // the previous rows are no longer read
            if (lane >= c && lane < c + P2M_PIPE_CH && lane < n) {
                const T inv_s = pow2i<T>(lr.level);
                R::write(S + (lane - c) * R::LD, cur.x * inv_s, -cur.y * inv_s, cur.u);
            }
            __syncthreads();
            R::sums(S, min(P2M_PIPE_CH, n - c), lane, acc);
        }
        R::store(acc, lane, M + int64_t(lr.box) * t.KS);
        if (!more) break;
        li += G;
        lr = r1;
        r1 = r2;
        r2 = li + 2 * G < nrec ? recs[li + 2 * G] : lr;
        cur = nxb;
        nxa = nna;
    }
}

// Any number of right-hand sides (below the matrix-core form's) and leaf
// size: one leaf per workgroup, chunk by chunk.
template <typename T, int P, int IN>
__global__ __launch_bounds__(64) void k_p2m(DTree<T> t, const LeafRec *__restrict__ recs, T *__restrict__ us,
                                            int nrhs, T *__restrict__ M, UserVec io)
{
    tree_pass_priority();
    using R = P2MRows<T, P>;
    __shared__ T S[P2M_CHUNK * R::LD];
    const int lane = threadIdx.x;
    const LeafRec lr = recs[blockIdx.x];
    const T inv_s = pow2i<T>(lr.level);
    for (int r = 0; r < nrhs; ++r) {
        typename R::acc_t acc[R::NT];
        R::clear(acc);
        for (int c0 = lr.begin; c0 < lr.end; c0 += P2M_CHUNK) {
            const int n = min(P2M_CHUNK, lr.end - c0);
            const int ip = c0 + (lane < n ? lane : 0);
            const T x = t.xl[ip], y = t.yl[ip];
            const T u = p2m_weight<T, IN>(io, us, t.N, IN == 0 ? ip : io.perm[ip], r);
            if (IN != 0 && lane < n) us[r * t.N + ip] = u;
            __syncthreads();
            if (lane < n) R::write(S + lane * R::LD, x * inv_s, -y * inv_s, u);
            __syncthreads();
            R::sums(S, n, lane, acc);
        }
        R::store(acc, lane, M + (int64_t(lr.box) * nrhs + r) * t.KS);
    }
}

template <typename T, int P, int IN>
void launch_p2m_in(hipStream_t s, int nleaves, int max_leaf, const DTree<T> &v, const LeafRec *recs, T *us,
                   int nrhs, T *M, const UserVec &uv)
{
    if (nrhs == 1 && max_leaf <= P2M_CHUNK)
        hipLaunchKernelGGL((k_p2m_pipe<T, P, IN>), dim3(unsigned(std::min(nleaves, P2M_PIPE_WG))), dim3(64), 0, s,
                           v, recs, nleaves, us, M, uv);
    else
        hipLaunchKernelGGL((k_p2m<T, P, IN>), dim3(unsigned(nleaves)), dim3(64), 0, s, v, recs, us, nrhs, M, uv);
}

template <typename T, int P>
void launch_p2m(hipStream_t s, int nleaves, int max_leaf, const DTree<T> &v, const LeafRec *recs, T *us, int nrhs,
                T *M, const UserVec &uv)
{
    if (nleaves <= 0) return;
    if (!uv.in) launch_p2m_in<T, P, 0>(s, nleaves, max_leaf, v, recs, us, nrhs, M, uv);
    else if (!uv.f32) launch_p2m_in<T, P, 1>(s, nleaves, max_leaf, v, recs, us, nrhs, M, uv);
    else launch_p2m_in<T, P, 2>(s, nleaves, max_leaf, v, recs, us, nrhs, M, uv);
}

// P2M of any box from its own points (Algorithm 1 mode): the leaves under
// the box (lord: leaf-list indices in point order), chunk by chunk, with each leaf's points moved from its centre to
// the box's; the column sums are kept in registers and stored once.  For a
// leaf this is k_p2m's arithmetic.
template <typename T, int P>
__global__ __launch_bounds__(64) void k_p2m_box(DTree<T> t, const BoxRec *__restrict__ recs,
                                                const int32_t *__restrict__ lord, const T *__restrict__ us,
                                                int nrhs, T *__restrict__ M, int ld)
{
    tree_pass_priority();
    extern __shared__ unsigned char smem_raw[];
    T *mono = reinterpret_cast<T *>(smem_raw);   // [P2M_CHUNK][ld]
    T *su = mono + P2M_CHUNK * ld;               // [P2M_CHUNK]
    constexpr int K = (P + 1) * (P + 2) / 2, KPL = (K + 63) / 64;
    const BoxRec rc = recs[blockIdx.x];
    const int b = rc.box, lane = threadIdx.x;
    const double inv_sd = ldexp(1.0, rc.level);
    const T inv_s = T(inv_sd);
    for (int r = 0; r < nrhs; ++r) {
        T acc[KPL];
#pragma unroll
        for (int j = 0; j < KPL; ++j) acc[j] = T(0);
        for (int li = rc.leaf0; li < rc.leaf1; ++li) {
            const LeafRec lr = t.leafrec[lord[li]];
            const T ox = T((t.cx[lr.box] - t.cx[b]) * inv_sd), oy = T((t.cy[lr.box] - t.cy[b]) * inv_sd);
            for (int c0 = lr.begin; c0 < lr.end; c0 += P2M_CHUNK) {
                const int n = min(P2M_CHUNK, lr.end - c0);
                T x = T(0), y = T(0), u = T(0);
                if (lane < n) {
                    x = t.xl[c0 + lane] * inv_s + ox;
                    y = t.yl[c0 + lane] * inv_s + oy;
                    u = us[r * t.N + c0 + lane];
                }
                __syncthreads();                 // the previous chunk is no longer read
                if (lane < n) {
                    T *row = mono + lane * ld;
                    monomials<P>(x, -y, [&](int k, T v, bool) { row[k] = v; });
                    su[lane] = u;
                }
                __syncthreads();
#pragma unroll
                for (int j = 0; j < KPL; ++j) {
                    const int k = lane + 64 * j;
                    if (k < K) acc[j] += lds_dot(mono, ld, k, su, n);
                }
            }
        }
#pragma unroll
        for (int j = 0; j < KPL; ++j) {
            const int k = lane + 64 * j;
            if (k < K) M[(size_t(b) * nrhs + r) * t.KS + k] = acc[j];
        }
    }
}

// P2L, one workgroup per (target box b, X-list leaf a) pair k: the local
// expansion of a's points about b's centre,
//     Lx[k] = (1/s) sum_j u_j eps_k c_{jk} conj(I_j^k((y_j - z_b)/s)),
// written to scratch and summed per box afterwards in list order.
template <typename T>
__global__ __launch_bounds__(64) void k_p2l_pairs(DTree<T> t, const int32_t *__restrict__ x_tgt,
                                                  const T *__restrict__ us, int nrhs,
                                                  const T *__restrict__ wx, T *__restrict__ Lx, int ld,
                                                  int npairs)
{
    tree_pass_priority();
    extern __shared__ unsigned char smem_raw[];
    T *mono = reinterpret_cast<T *>(smem_raw);   // [64][ld]
    T *su = mono + 64 * ld;
    const int kp = blockIdx.x;
    const int b = x_tgt[kp], a = t.x_idx[kp];
    const int P = t.P, K = t.K, lane = threadIdx.x;
    const double inv_sd = ldexp(1.0, t.level[b]);
    const T inv_s = T(inv_sd);
    const T vz = T(-t.cn[t.set[b]] * inv_sd);
    const T ox = T((t.cx[a] - t.cx[b]) * inv_sd), oy = T((t.cy[a] - t.cy[b]) * inv_sd);
    for (int c0 = t.begin[a]; c0 < t.end[a]; c0 += 64) {
        const int n = min(64, t.end[a] - c0);
        __syncthreads();
        if (lane < n) {
            T *row = mono + lane * ld;
            irregular_even<T>(P, t.xl[c0 + lane] * inv_s + ox, t.yl[c0 + lane] * inv_s + oy, vz,
                              [&](int nn, int m, T re, T im) {
                                  const int k = cidx(nn, m);
                                  row[k] = re;
                                  if (m > 0) row[k + 1] = -im;
                              });
        }
        for (int r = 0; r < nrhs; ++r) {
            __syncthreads();
            if (lane < n) su[lane] = us[r * t.N + c0 + lane];
            __syncthreads();
            for (int k = lane; k < K; k += 64) {
                const T v = lds_dot(mono, ld, k, su, n) * wx[k] * inv_s;
                T &dst = Lx[(size_t(r) * npairs + kp) * K + k];
                dst = (c0 == t.begin[a]) ? v : dst + v;
            }
        }
    }
}

// L[b] += sum of the pair expansions of b's X list, in list order.
template <typename T>
__global__ void k_p2l_reduce(DTree<T> t, const int32_t *__restrict__ xboxes, int nrhs,
                             const T *__restrict__ Lx, int npairs, T *__restrict__ L)
{
    tree_pass_priority();
    const int b = xboxes[blockIdx.x];
    const int K = t.K;
    for (int r = 0; r < nrhs; ++r)
        for (int k = threadIdx.x; k < K; k += blockDim.x) {
            T s = T(0);
            for (int kp = t.x_off[b]; kp < t.x_off[b + 1]; ++kp) s += Lx[(size_t(r) * npairs + kp) * K + k];
            L[(size_t(b) * nrhs + r) * t.KS + k] += s;
        }
}

// ------------------------------------------------------------------ MFMA translations

constexpr int GEMM_MAXRB = 10;        // row blocks of 16: KP <= 160 (p <= 16)

// One task = one workgroup of 4 waves: out[:, col] (+)= sum_s T_s in[:, src(col, s)]
// for the 64 columns (target box, rhs) of blockIdx.y and the row blocks of
// split blockIdx.z.  Wave w owns columns [16w, 16w+16).  The contraction runs
// over a sequence of (slot, k-chunk) steps; each step's table chunk
// (rows x KC) and source chunk (KC x 64 columns) are staged in LDS, and the
// next step's are loaded into registers while the matrix cores work on the
// current one.
template <typename T, int KC_, int MAXRB_>
struct GemmStage {
    static constexpr int KC = KC_;                                  // k per step
    static constexpr int LD = KC + (sizeof(T) == 4 ? 1 : 2);       // LDS row stride
    static constexpr int NA = MAXRB_ * 16 * KC / 256;              // table elems / thread
    static constexpr int NB = GEMM_TILE * KC / 256;                // source elems / thread
};

template <typename T, int KC_, int MAXRB>
__global__ __launch_bounds__(256) void k_gemm_tasks(const GemmTask *__restrict__ tasks, int task0,
                                                    const int32_t *__restrict__ tbox,
                                                    const int32_t *__restrict__ tab,
                                                    const int32_t *__restrict__ src,
                                                    const T *__restrict__ tables, int KP, int KS, int nrhs,
                                                    const T *__restrict__ in, T *__restrict__ out,
                                                    int accumulate, int kin_ovr, int kout_ovr)
{
    tree_pass_priority();
    using S = GemmStage<T, KC_, MAXRB>;
    constexpr int KC = S::KC, LD = S::LD;
    __shared__ T As[MAXRB * 16 * LD];
    __shared__ T Bs[GEMM_TILE * LD];
    __shared__ int s_col[GEMM_MAXSLOT][GEMM_TILE];
    __shared__ int s_tab[GEMM_MAXSLOT];
    __shared__ int s_has[GEMM_MAXSLOT];
    __shared__ int s_step[GEMM_MAXSLOT];
    __shared__ int s_nstep;
    using acc_t = typename Mfma<T>::acc_t;
    GemmTask tk = tasks[task0 + blockIdx.x];
    if (kin_ovr > 0) tk.kin = kin_ovr;
    if (kout_ovr > 0) tk.kout = kout_ovr;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int r16 = lane & 15, q = lane >> 4;
    const int ncols = tk.nbox * nrhs;
    const int col0 = blockIdx.y * GEMM_TILE;
    if (col0 >= ncols) return;
    const int nrb_all = (tk.kout + 15) >> 4;
    const int per = (nrb_all + gridDim.z - 1) / gridDim.z;
    const int rb0 = blockIdx.z * per;
    const int nrb = min(nrb_all - rb0, per);          // row blocks of this split
    if (nrb <= 0) return;
    const int kin4 = (tk.kin + 3) & ~3;
    const int nkc = (kin4 + KC - 1) / KC;
    const int arows = nrb * 16;
    const int row0 = rb0 * 16;

    if (tid < tk.nslot) {
        s_tab[tid] = tab[tk.tab0 + tid];
        s_has[tid] = 0;
    }
    __syncthreads();
    for (int e = tid; e < tk.nslot * GEMM_TILE; e += 256) {
        const int sl = e / GEMM_TILE, c = e - sl * GEMM_TILE;
        const int gc = col0 + c;
        int ci = -1;
        if (gc < ncols) {
            const int bl = gc / nrhs, r = gc - bl * nrhs;
            const int sb = src[tk.src0 + bl * tk.nslot + sl];
            if (sb >= 0) ci = sb * nrhs + r;
        }
        s_col[sl][c] = ci;
        if (ci >= 0) s_has[sl] = 1;
    }
    __syncthreads();
    if (tid == 0) {
        int n = 0;
        for (int sl = 0; sl < tk.nslot; ++sl)
            if (s_has[sl]) s_step[n++] = sl;
        s_nstep = n;
    }
    __syncthreads();
    const int nstep = s_nstep * nkc;

    T ra[S::NA], rb_[S::NB];
    auto fetch = [&](int step) {
        const int sl = s_step[step / nkc];
        const int kc0 = (step % nkc) * KC;
        const T *A = tables + size_t(s_tab[sl]) * KP * KP + size_t(row0) * KP;
#pragma unroll
        for (int i = 0; i < S::NA; ++i) {
            const int e = tid + i * 256;
            const int r = e / KC, k = e % KC;
            ra[i] = (r < arows && kc0 + k < kin4) ? A[size_t(r) * KP + kc0 + k] : T(0);
        }
#pragma unroll
        for (int i = 0; i < S::NB; ++i) {
            const int e = tid + i * 256;
            const int c = e / KC, k = e % KC;
            const int ci = s_col[sl][c];
            const int kk = kc0 + k;
            rb_[i] = (ci >= 0 && kk < tk.kin) ? in[size_t(ci) * KS + kk] : T(0);
        }
    };

    acc_t acc[MAXRB];
#pragma unroll
    for (int i = 0; i < MAXRB; ++i)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[i][v] = T(0);

    if (nstep > 0) fetch(0);
    for (int step = 0; step < nstep; ++step) {
        __syncthreads();
#pragma unroll
        for (int i = 0; i < S::NA; ++i) {
            const int e = tid + i * 256;
            const int r = e / KC, k = e % KC;
            if (r < arows) As[r * LD + k] = ra[i];
        }
#pragma unroll
        for (int i = 0; i < S::NB; ++i) {
            const int e = tid + i * 256;
            const int c = e / KC, k = e % KC;
            Bs[c * LD + k] = rb_[i];
        }
        __syncthreads();
        if (step + 1 < nstep) fetch(step + 1);
        const T *Bw = Bs + (wave * 16 + r16) * LD + q;
        const T *Aw = As + r16 * LD + q;
#pragma unroll
        for (int k0 = 0; k0 < KC; k0 += 4) {
            const T b = Bw[k0];
#pragma unroll
            for (int rb = 0; rb < MAXRB; ++rb)
                if (rb < nrb) acc[rb] = Mfma<T>::mac(Aw[rb * 16 * LD + k0], b, acc[rb]);
        }
    }

    const int gc = col0 + wave * 16 + r16;
    if (gc < ncols) {
        const int bl = gc / nrhs, r = gc - bl * nrhs;
        T *o = out + (size_t(tbox[tk.box0 + bl]) * nrhs + r) * KS;
#pragma unroll
        for (int rb = 0; rb < MAXRB; ++rb)
            if (rb < nrb)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int row = row0 + rb * 16 + Mfma<T>::row(q, v);
                    if (row < tk.kout) {
                        if (accumulate) o[row] += acc[rb][v];
                        else o[row] = acc[rb][v];
                    }
                }
    }
}

// Launch one batch of translation tasks: kc coefficients per pipeline step
// (0 = 32) and the rows of a tile spread over `split` workgroups.
template <typename T>
void launch_gemm(hipStream_t s, int kc, int split, int ntask, int nrhs, const GemmTask *tasks,
                 int t0, const int32_t *tbox, const int32_t *tab, const int32_t *src,
                 const T *tables, int KP, int KS, const T *in, T *out, int acc, int kin_ovr, int kout_ovr)
{
#define IMQ_GEMM(KCV, RB)                                                                            \
    hipLaunchKernelGGL((k_gemm_tasks<T, KCV, RB>), grid, dim3(256), 0, s, tasks, t0, tbox, tab, src,  \
                       tables, KP, KS, nrhs, in, out, acc, kin_ovr, kout_ovr)
    if (kc == 0) kc = 32;
    const dim3 grid(ntask, nrhs, split > 0 ? split : 1);
    if constexpr (sizeof(T) == 4) {
        if (kc >= 64) IMQ_GEMM(64, GEMM_MAXRB);
        else if (kc >= 32) IMQ_GEMM(32, GEMM_MAXRB);
        else IMQ_GEMM(16, GEMM_MAXRB);
    } else {
        if (kc >= 32) IMQ_GEMM(32, GEMM_MAXRB);
        else IMQ_GEMM(16, GEMM_MAXRB);
    }
#undef IMQ_GEMM
}

template <typename T>
__global__ void k_fill(size_t n, T *__restrict__ p, T v)
{
    tree_pass_priority();
    const size_t i = blockIdx.x * size_t(blockDim.x) + threadIdx.x;
    if (i < n) p[i] = v;
}

// The per-pair W-list (M2P) evaluations that L2P adds for its leaf's points
// (Pw null: none; they are then added by k_m2p_reduce).
struct M2PParts {
    const int32_t *w_scr = nullptr;
    const double *Pw = nullptr;
    int nscr = 0;
};

// L2P: potential = sum Re(Lt[n,m] |w|^(n-m) w^m) at each point of a leaf.
// The leaf's local expansion carries only the coefficients of its level's
// translation order Q <= P (the rest are zero), so the evaluation runs at Q:
// the kernel is instantiated for the tree's order P and switches, per leaf,
// to the fully unrolled evaluation of order Q.  The expansion is staged in LDS.
template <typename T, int Q>
__device__ __forceinline__ T l2p_eval(T x, T y, const T *Ls)
{
    T acc = T(0);
    // real part of Lt * monomial: Re*Re - Im*Im
    monomials<Q>(x, y, [&](int k, T v, bool im) { acc += im ? -Ls[k] * v : Ls[k] * v; });
    return acc;
}

// the order q with (q+1)(q+2)/2 = Kl
__device__ __forceinline__ int order_of(int Kl)
{
    int q = 0;
    while ((q + 2) * (q + 3) / 2 <= Kl) ++q;
    return q;
}

template <typename T, int P>
__device__ __forceinline__ T l2p_value(int q, T x, T y, const T *Ls)
{
#define IMQ_L2P_Q(Q) \
    case Q: if constexpr (Q <= P) return l2p_eval<T, Q>(x, y, Ls); else break;
    switch (q) {
        IMQ_L2P_Q(1) IMQ_L2P_Q(2) IMQ_L2P_Q(3) IMQ_L2P_Q(4) IMQ_L2P_Q(5) IMQ_L2P_Q(6) IMQ_L2P_Q(7)
        IMQ_L2P_Q(8) IMQ_L2P_Q(9) IMQ_L2P_Q(10) IMQ_L2P_Q(11) IMQ_L2P_Q(12) IMQ_L2P_Q(13) IMQ_L2P_Q(14)
        IMQ_L2P_Q(15) IMQ_L2P_Q(16)
        default: break;
    }
#undef IMQ_L2P_Q
    return l2p_eval<T, P>(x, y, Ls);
}

// Adds the leaf's W-list evaluations (in list order) and stores the result.
template <typename T>
__device__ __forceinline__ void l2p_store(const DTree<T> &t, const LeafRec &lr, int r, int i, double val,
                                          double *__restrict__ bs, const UserVec &io, const M2PParts &wp)
{
    if (wp.Pw)
        for (int kp = t.w_off[lr.box]; kp < t.w_off[lr.box + 1]; ++kp)
            val += wp.Pw[size_t(r) * wp.nscr + wp.w_scr[kp] + (i - lr.begin)];
    if (io.out) io.put(r, i, val);
    else bs[r * t.N + i] = val;
}

// Any number of right-hand sides (below the matrix-core form's) and leaf
// size: one leaf per workgroup.
template <typename T, int P>
__global__ __launch_bounds__(64) void k_l2p(DTree<T> t, LevelK lk, const T *__restrict__ L, int nrhs,
                                            double *__restrict__ bs, int add, UserVec io, M2PParts wp)
{
    tree_pass_priority();
    constexpr int KP = (P + 1) * (P + 2) / 2;
    __shared__ T Ls[KP];
    const LeafRec lr = t.leafrec[blockIdx.x];
    const int Kl = lk.K[lr.level];
    const int q = order_of(Kl);
    const T inv_s = pow2i<T>(lr.level);
    for (int i0 = lr.begin; i0 < lr.end; i0 += 64) {
        const int i = i0 + threadIdx.x;
        const bool ok = i < lr.end;
        for (int r = 0; r < nrhs; ++r) {
            __syncthreads();                     // the previous expansion is no longer read
            // the point, the partial result and the expansion are requested together
            const T x = ok ? t.xl[i] * inv_s : T(0), y = ok ? t.yl[i] * inv_s : T(0);
            const double prev = (ok && add) ? bs[r * t.N + i] : 0.0;
            for (int k = threadIdx.x; k < KP; k += 64) Ls[k] = k < Kl ? L[(size_t(lr.box) * nrhs + r) * t.KS + k] : T(0);
            __syncthreads();
            if (ok) l2p_store(t, lr, r, i, prev + double(l2p_value<T, P>(q, x, y, Ls)), bs, io, wp);
        }
    }
}

// One right-hand side, leaves of at most 64 points.  Workgroup g takes leaves
// g, g + G, ... (G workgroups) and requests the next leaf's points, partial
// results, expansion and caller-order output slots before it evaluates the
// current one.
template <typename T, int P>
__global__ __launch_bounds__(64) void k_l2p_pipe(DTree<T> t, const LeafRec *__restrict__ recs, LevelK lk,
                                                 const T *__restrict__ L, double *__restrict__ bs, int add, UserVec io,
                                                 M2PParts wp, const int32_t *__restrict__ w_off, int nrec)
{
    tree_pass_priority();
    constexpr int KP = (P + 1) * (P + 2) / 2;
    constexpr int NL = (KP + 63) / 64;
    __shared__ T Ls[KP];
    const int lane = threadIdx.x;
    const int G = gridDim.x;
    int li = blockIdx.x;
    if (li >= nrec) return;
    struct Pass {
        T x, y;
        double prev;
        int dst;                                  // caller-order slot and scale (io.out)
        double sc;
        T l[NL];
    };
    // every lane loads: lanes past the leaf read point 0, coefficients past
    // the level's count read coefficient 0 and are zeroed
    auto load = [&](const LeafRec &lr, Pass &o) {
        const int i = lr.begin + lane;
        const int ii = i < lr.end ? i : 0;
        o.x = t.xl[ii];
        o.y = t.yl[ii];
        o.prev = add ? bs[ii] : 0.0;
        o.dst = io.out ? io.perm[ii] : ii;
        o.sc = io.out ? io.scale[ii] : 1.0;
        const int Kl = lk.K[lr.level];
#pragma unroll
        for (int j = 0; j < NL; ++j) {
            const int k = lane + 64 * j;
            const T v = L[size_t(lr.box) * t.KS + (k < Kl ? k : 0)];
            o.l[j] = k < Kl ? v : T(0);
        }
    };
    LeafRec lr = recs[li];
    LeafRec nr = li + G < nrec ? recs[li + G] : lr;
    Pass cur;
    load(lr, cur);
    for (;;) {
        const bool more = li + G < nrec;
        Pass nx;
        load(nr, nx);                              // the next leaf (the current one again at the end)
        __syncthreads();                           // the previous expansion is no longer read
#pragma unroll
        for (int j = 0; j < NL; ++j)
            if (lane + 64 * j < KP) Ls[lane + 64 * j] = cur.l[j];
        __syncthreads();
        const int i = lr.begin + lane;
        if (i < lr.end) {
            const T inv_s = pow2i<T>(lr.level);
            double val = cur.prev + double(l2p_value<T, P>(order_of(lk.K[lr.level]), cur.x * inv_s,
                                                           cur.y * inv_s, Ls));
            if (wp.Pw)
                for (int kp = w_off[lr.box]; kp < w_off[lr.box + 1]; ++kp)
                    val += wp.Pw[wp.w_scr[kp] + (i - lr.begin)];
            if (io.out) {
                val *= cur.sc;
                if (io.f32) static_cast<float *>(io.out)[cur.dst] = float(val);
                else static_cast<double *>(io.out)[cur.dst] = val;
            } else {
                bs[i] = val;
            }
        }
        if (!more) break;
        li += G;
        lr = nr;
        nr = li + G < nrec ? recs[li + G] : lr;
        cur = nx;
    }
}

template <typename T, int P>
void launch_l2p(hipStream_t s, int nleaves, int max_leaf, const DTree<T> &v, const LevelK &lk, const T *L, int nrhs,
                double *bs, const UserVec &uv, const M2PParts &wp)
{
    if (nleaves <= 0) return;
    if (nrhs == 1 && max_leaf <= 64)
        hipLaunchKernelGGL((k_l2p_pipe<T, P>), dim3(unsigned(std::min(nleaves, LEAF_WG_MAX))), dim3(64), 0, s, v,
                           v.leafrec, lk, L, bs, 1, uv, wp, v.w_off, nleaves);
    else
        hipLaunchKernelGGL((k_l2p<T, P>), dim3(unsigned(nleaves)), dim3(64), 0, s, v, lk, L, nrhs, bs, 1, uv, wp);
}

// Many right-hand sides: the leaf expansions and their evaluation as
// matrix-core products over a leaf,
//   P2M  M[k][r]  = sum_j mono_k(conj w_j) u_r[j]       (K x points) x (points x rhs)
//   L2P  b_r[j]  += sum_k s_k mono_k(w_j) L[k][r]       (points x K) x (K x rhs)
// with s_k = -1 on imaginary parts (the real part of Lt * monomial).  One wave
// per (leaf, block of RB right-hand sides); the monomials of up to 64 points
// are the rows of an LDS matrix (row stride = 17 mod 32 words: conflict-free
// row writes, nearly conflict-free reads) and the right-hand-side block is
// staged rhs-major (stride = 2 mod 32).
constexpr int BATCH_RHS_MIN = 8;   // from this many right-hand sides on

template <int K> constexpr int mono_ld() { return ((K + 15) / 16) * 16 + (((K + 15) / 16) & 1 ? 1 : 17); }

template <typename T, int P, int RB>
__global__ __launch_bounds__(64) void k_p2m_mfma(DTree<T> t, const int32_t *__restrict__ leaves,
                                                 const T *__restrict__ us, int nrhs, T *__restrict__ M)
{
    tree_pass_priority();
    constexpr int K = (P + 1) * (P + 2) / 2, NRB = (K + 15) / 16, LDM = mono_ld<K>();
    constexpr int NCB = RB / 16, LDU = 64 + 2;
    using acc_t = typename Mfma<T>::acc_t;
    __shared__ T mono[64 * LDM];
    __shared__ T su[RB * LDU];
    const int b = leaves[blockIdx.x];
    const int r0 = blockIdx.y * RB;
    const int lane = threadIdx.x, i16 = lane & 15, q = lane >> 4;
    const int beg = t.begin[b], end = t.end[b];
    const T inv_s = pow2i<T>(t.level[b]);
    const int64_t N = t.N;
    acc_t acc[NRB][NCB];
#pragma unroll
    for (int rb = 0; rb < NRB; ++rb)
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[rb][cb][v] = T(0);
    for (int c0 = beg; c0 < end; c0 += 64) {
        const int n = min(64, end - c0);
        __syncthreads();
        {
            T *row = mono + lane * LDM;
            if (lane < n)
                monomials<P>(t.xl[c0 + lane] * inv_s, -t.yl[c0 + lane] * inv_s,
                             [&](int k, T v, bool) { row[k] = v; });
            else
#pragma unroll
                for (int k = 0; k < K; ++k) row[k] = T(0);
#pragma unroll
            for (int k = K; k < NRB * 16; ++k) row[k] = T(0);
        }
#pragma unroll
        for (int rr = 0; rr < RB; rr += 16) {            // 16 loads in flight per lane
            T v[16];
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                const bool ok = lane < n && r0 + rr + j < nrhs;
                v[j] = ok ? us[(r0 + rr + j) * N + c0 + lane] : T(0);
            }
#pragma unroll
            for (int j = 0; j < 16; ++j) su[(rr + j) * LDU + lane] = v[j];
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < 16; ++ks) {
            T bv[NCB];
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) bv[cb] = su[(cb * 16 + i16) * LDU + 4 * ks + q];
#pragma unroll
            for (int rb = 0; rb < NRB; ++rb) {
                const T av = mono[(4 * ks + q) * LDM + rb * 16 + i16];
#pragma unroll
                for (int cb = 0; cb < NCB; ++cb) acc[rb][cb] = Mfma<T>::mac(av, bv[cb], acc[rb][cb]);
            }
        }
    }
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) {
        const int r = r0 + cb * 16 + i16;
        if (r >= nrhs) continue;
        T *o = M + (size_t(b) * nrhs + r) * t.KS;
#pragma unroll
        for (int rb = 0; rb < NRB; ++rb)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int k = rb * 16 + Mfma<T>::row(q, v);
                if (k < K) o[k] = acc[rb][cb][v];
            }
    }
}

template <typename T, int P, int RB>
__global__ __launch_bounds__(64) void k_l2p_mfma(DTree<T> t, const int32_t *__restrict__ leaves,
                                                 const T *__restrict__ L, int nrhs, double *__restrict__ bs)
{
    tree_pass_priority();
    constexpr int K = (P + 1) * (P + 2) / 2, NRB = (K + 15) / 16, LDM = mono_ld<K>();
    constexpr int NCB = RB / 16, LDL = NRB * 16 + 2;
    using acc_t = typename Mfma<T>::acc_t;
    __shared__ T mono[64 * LDM];
    __shared__ T sl[RB * LDL];
    const int b = leaves[blockIdx.x];
    const int r0 = blockIdx.y * RB;
    const int lane = threadIdx.x, i16 = lane & 15, q = lane >> 4;
    const int beg = t.begin[b], end = t.end[b];
    const T inv_s = pow2i<T>(t.level[b]);
    const int64_t N = t.N;
    constexpr int NSL = RB * NRB * 16 / 64;            // staged values per lane
#pragma unroll
    for (int e0 = 0; e0 < NSL; e0 += 16) {               // 16 loads in flight per lane
        T v[16];
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const int e = lane + 64 * (e0 + j);
            const int r = e / (NRB * 16), k = e - r * (NRB * 16);
            v[j] = (e0 + j < NSL && r0 + r < nrhs && k < K) ? L[(size_t(b) * nrhs + r0 + r) * t.KS + k] : T(0);
        }
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const int e = lane + 64 * (e0 + j);
            const int r = e / (NRB * 16), k = e - r * (NRB * 16);
            if (e0 + j < NSL) sl[r * LDL + k] = v[j];
        }
    }
    for (int c0 = beg; c0 < end; c0 += 64) {
        const int n = min(64, end - c0);
        __syncthreads();
        {
            T *row = mono + lane * LDM;
            if (lane < n)
                monomials<P>(t.xl[c0 + lane] * inv_s, t.yl[c0 + lane] * inv_s,
                             [&](int k, T v, bool im) { row[k] = im ? -v : v; });
            else
#pragma unroll
                for (int k = 0; k < K; ++k) row[k] = T(0);
#pragma unroll
            for (int k = K; k < NRB * 16; ++k) row[k] = T(0);
        }
        __syncthreads();
        // transposed product (rhs x points) = L^T (rhs x K) . mono^T (K x points):
        // a lane's outputs are one point of four right-hand sides, so each store
        // instruction writes 16 consecutive points of a right-hand side
        acc_t acc[NCB][4];
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
            for (int pb = 0; pb < 4; ++pb)
#pragma unroll
                for (int v = 0; v < 4; ++v) acc[cb][pb][v] = T(0);
#pragma unroll
        for (int ks = 0; ks < NRB * 4; ++ks) {
            T bv[4];
#pragma unroll
            for (int pb = 0; pb < 4; ++pb) bv[pb] = mono[(pb * 16 + i16) * LDM + 4 * ks + q];
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) {
                const T av = sl[(cb * 16 + i16) * LDL + 4 * ks + q];
#pragma unroll
                for (int pb = 0; pb < 4; ++pb) acc[cb][pb] = Mfma<T>::mac(av, bv[pb], acc[cb][pb]);
            }
        }
#pragma unroll
        for (int pb = 0; pb < 4; ++pb) {
            const int j = pb * 16 + i16;
            if (j >= n) continue;
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int r = r0 + cb * 16 + Mfma<T>::row(q, v);
                    if (r < nrhs) bs[r * N + c0 + j] += double(acc[cb][pb][v]);
                }
        }
    }
}

// M2P, one wave per (target leaf b, W-list box a) pair k: the multipole of
// a evaluated at b's points,
//     potential = (1/s_a) sum Re(Mt[n,m] eps_m c_{nm} I_n^m((x - z_a)/s_a)),
// written to scratch (offset w_scr[k]) and summed per point afterwards in
// list order.  The multipole, premultiplied by the constants, is staged in LDS.
template <typename T>
__global__ __launch_bounds__(64) void k_m2p_pairs(DTree<T> t, const int32_t *__restrict__ w_tgt,
                                                  const int32_t *__restrict__ w_scr,
                                                  const T *__restrict__ M, const T *__restrict__ wx,
                                                  int nrhs, double *__restrict__ Pw, int nscr)
{
    tree_pass_priority();
    __shared__ T mw[KMAX + 1];
    const int kp = blockIdx.x;
    const int b = w_tgt[kp], a = t.w_idx[kp];
    const int P = t.P, K = t.K, lane = threadIdx.x;
    const double cnd = t.cn[t.set[b]];
    const double inv_sd = ldexp(1.0, t.level[a]);
    const T inv_s = T(inv_sd);
    const T ox = T((t.cx[b] - t.cx[a]) * inv_sd), oy = T((t.cy[b] - t.cy[a]) * inv_sd);
    const T vz = T(cnd * inv_sd);
    for (int r = 0; r < nrhs; ++r) {
        __syncthreads();
        for (int k = lane; k < K; k += 64) mw[k] = M[(size_t(a) * nrhs + r) * t.KS + k] * wx[k];
        __syncthreads();
        for (int i = t.begin[b] + lane; i < t.end[b]; i += 64) {
            T s = T(0);
            irregular_even<T>(P, t.xl[i] * inv_s + ox, t.yl[i] * inv_s + oy, vz,
                              [&](int n, int m, T re, T im) {
                                  const int k = cidx(n, m);
                                  s += mw[k] * re;
                                  if (m > 0) s -= mw[k + 1] * im;
                              });
            Pw[size_t(r) * nscr + w_scr[kp] + (i - t.begin[b])] = double(s * inv_s);
        }
    }
}

// b_i += sum over the W-list pairs of i's leaf, in list order.
template <typename T>
__global__ __launch_bounds__(64) void k_m2p_reduce(DTree<T> t, const int32_t *__restrict__ wleaves,
                                                   const int32_t *__restrict__ w_scr, int nrhs,
                                                   const double *__restrict__ Pw, int nscr,
                                                   double *__restrict__ bs)
{
    tree_pass_priority();
    const int b = wleaves[blockIdx.x];
    for (int r = 0; r < nrhs; ++r)
        for (int i = t.begin[b] + threadIdx.x; i < t.end[b]; i += blockDim.x) {
            double s = 0.0;
            for (int kp = t.w_off[b]; kp < t.w_off[b + 1]; ++kp)
                s += Pw[size_t(r) * nscr + w_scr[kp] + (i - t.begin[b])];
            bs[r * t.N + i] += s;
        }
}

// The far field of the paper's Algorithm 1 (Sec. 2.2, eq. MatxVec): every
// box's multipole is formed from its own points, and evaluated directly at
// the points of each box of its V list (the well-separated boxes of the same
// partition not already treated at a coarser one).  One workgroup per leaf:
// for the leaf and each of its ancestors b, for each box a in b's V list, the
// multipole of a at the leaf's points (the V-list relation is symmetric, so
// this visits every pair of Algorithm 1 once), summed per point in FP64 and
// added to bs.  The multipole, premultiplied by the constants, is staged in LDS.
template <typename T>
__global__ __launch_bounds__(64) void k_alg1_far(DTree<T> t, const T *__restrict__ M, const T *__restrict__ wx,
                                                 int nrhs, double *__restrict__ bs)
{
    tree_pass_priority();
    __shared__ T mw[KMAX + 1];
    const LeafRec lr = t.leafrec[blockIdx.x];
    const int P = t.P, K = t.K, lane = threadIdx.x;
    const double cnd = t.cn[t.set[lr.box]];
    for (int r = 0; r < nrhs; ++r)
        for (int i0 = lr.begin; i0 < lr.end; i0 += 64) {
            const int i = i0 + lane;
            const bool ok = i < lr.end;
            const T xi = ok ? t.xl[i] : T(0), yi = ok ? t.yl[i] : T(0);
            double acc = 0.0;
            for (int b = lr.box; b >= 0; b = t.parent[b])
                for (int v = t.v_off[b]; v < t.v_off[b + 1]; ++v) {
                    const int a = t.v_idx[v];
                    const double inv_sd = ldexp(1.0, t.level[a]);
                    const T inv_s = T(inv_sd);
                    const T ox = T((t.cx[lr.box] - t.cx[a]) * inv_sd), oy = T((t.cy[lr.box] - t.cy[a]) * inv_sd);
                    const T vz = T(cnd * inv_sd);
                    __syncthreads();                 // the previous multipole is no longer read
                    for (int k = lane; k < K; k += 64) mw[k] = M[(size_t(a) * nrhs + r) * t.KS + k] * wx[k];
                    __syncthreads();
                    if (ok) {
                        T sv = T(0);
                        irregular_even<T>(P, xi * inv_s + ox, yi * inv_s + oy, vz, [&](int n, int m, T re, T im) {
                            const int k = cidx(n, m);
                            sv += mw[k] * re;
                            if (m > 0) sv -= mw[k + 1] * im;
                        });
                        acc += double(sv * inv_s);
                    }
                }
            if (ok) bs[r * t.N + i] += acc;
        }
}

// Exact rows: b[r*ldb + k] = sum_j A_{rows[k], j} u_j in FP64 over the row's set.
__global__ __launch_bounds__(256) void k_rows_exact(int nsets, const int64_t *__restrict__ set_off,
                                                    const double *__restrict__ c, const double *__restrict__ xy,
                                                    int64_t N, const double *__restrict__ u, int64_t ldu,
                                                    const int64_t *__restrict__ rows, double *__restrict__ b,
                                                    int64_t ldb)
{
    __shared__ double red[256];
    const int64_t row = rows[blockIdx.x];
    const int r = blockIdx.y;
    int s = 0;
    while (s + 1 < nsets && set_off[s + 1] <= row) ++s;
    const double xi = xy[row], yi = xy[N + row], cc = c[s] * c[s];
    double acc = 0.0, comp = 0.0;
    for (int64_t j = set_off[s] + threadIdx.x; j < set_off[s + 1]; j += blockDim.x) {
        const double dx = xi - xy[j], dy = yi - xy[N + j];
        const double term = u[r * ldu + j] / sqrt(dx * dx + dy * dy + cc);
        const double y = term - comp;
        const double tt = acc + y;
        comp = (tt - acc) - y;
        acc = tt;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) b[r * ldb + blockIdx.x] = red[0];
}

// ------------------------------------------------------------------ host side

// The allocator of the tree an entry point is working on (null: hipMalloc).
// Every entry point that allocates sets it first: the tree builders to the
// new tree's, the calls on a tree through their argument check; a freed
// tree's is cleared.  Each buffer remembers the allocator that made it.
thread_local const imq_allocator *g_alloc = nullptr;

hipError_t dev_alloc(DevBuf &b, size_t bytes)
{
    dev_free(b);
    if (bytes == 0) bytes = 8;
    hipError_t e;
    if (g_alloc) {
        b.p = g_alloc->alloc(bytes, g_alloc->ctx);
        e = b.p ? hipSuccess : hipErrorOutOfMemory;
    } else {
        e = hipMalloc(&b.p, bytes);
    }
    if (e == hipSuccess) {
        b.bytes = bytes;
        b.al = g_alloc;
    } else {
        b.p = nullptr;
    }
    return e;
}

void dev_free(DevBuf &b)
{
    if (b.p) {
        if (b.al) b.al->free(b.p, b.al->ctx);
        else (void)hipFree(b.p);
    }
    b.p = nullptr;
    b.bytes = 0;
    b.al = nullptr;
}

template <typename T> PrecData &prec_data(imq_tree_s *t);
template <> PrecData &prec_data<double>(imq_tree_s *t) { return t->f64; }
template <> PrecData &prec_data<float>(imq_tree_s *t) { return t->f32; }

template <typename T>
DTree<T> make_view(const imq_tree_s *t)
{
    DTree<T> v;
    const HostTree &h = t->h;
    v.nbox = int(h.level.size());
    v.nsets = h.nsets;
    v.nlev = h.nlev;
    v.K = h.K;
    v.KS = coef_stride(h.K);
    v.P = h.p;
    v.N = h.N;
    v.level = t->level.as<int32_t>(); v.set = t->set.as<int32_t>(); v.parent = t->parent.as<int32_t>();
    v.child0 = t->child0.as<int32_t>(); v.nchild = t->nchild.as<int32_t>(); v.pos = t->pos.as<int32_t>();
    v.begin = t->begin.as<int32_t>(); v.end = t->end.as<int32_t>();
    v.cx = t->cx.as<double>(); v.cy = t->cy.as<double>();
    v.u_off = t->u_off.as<int32_t>(); v.u_idx = t->u_idx.as<int32_t>();
    v.v_off = t->v_off.as<int32_t>(); v.v_idx = t->v_idx.as<int32_t>(); v.v_cls = t->v_cls.as<int32_t>();
    v.w_off = t->w_off.as<int32_t>(); v.w_idx = t->w_idx.as<int32_t>();
    v.x_off = t->x_off.as<int32_t>(); v.x_idx = t->x_idx.as<int32_t>();
    v.Klev = t->Klev.as<int32_t>();
    v.leafrec = t->leafrec.as<LeafRec>();
    v.nleaf = t->nleaf.as<NearLeaf>();
    v.cn = t->cn.as<double>();
    const PrecData &pd = prec_data<T>(const_cast<imq_tree_s *>(t));
    v.xl = pd.xl.as<T>();
    v.yl = pd.yl.as<T>();
    v.urec = pd.urec.as<URec<T>>();
    return v;
}

template <typename T>
imq_status ensure_workspace(imq_tree_s *t, int nrhs)
{
    PrecData &pd = prec_data<T>(t);
    const size_t nbox = t->h.level.size();
    if (pd.ws_nrhs < size_t(nrhs)) {
        IMQ_HIP(dev_alloc(pd.us, sizeof(T) * size_t(t->h.N) * nrhs));
        IMQ_HIP(dev_alloc(pd.M, sizeof(T) * nbox * nrhs * coef_stride(t->h.K)));
        IMQ_HIP(dev_alloc(pd.L, sizeof(T) * nbox * nrhs * coef_stride(t->h.K)));
        pd.ws_nrhs = nrhs;
    }
    if (pd.lx_nrhs < size_t(nrhs)) {
        IMQ_HIP(dev_alloc(pd.Lx, sizeof(T) * size_t(t->nxpairs) * nrhs * t->h.K));
        pd.lx_nrhs = nrhs;
    }
    if (t->bs_nrhs < size_t(nrhs)) {
        IMQ_HIP(dev_alloc(t->bs, sizeof(double) * size_t(t->h.N) * nrhs));
        IMQ_HIP(dev_alloc(t->Pw, sizeof(double) * size_t(t->nwscr) * nrhs));
        t->bs_nrhs = nrhs;
    }
    return IMQ_OK;
}

static thread_local hipEvent_t *g_cur_events = nullptr;
// Every stage in order on the caller's stream (no side streams, no events):
// the product of the entry point that allocates nothing.
static thread_local bool g_serial = false;
void set_serial_product(bool on) { g_serial = on; }

static inline void mark(imq_tree_s *, int stage, hipStream_t s)
{
    if (g_cur_events) (void)hipEventRecord(g_cur_events[stage], s);
}

// Upward pass: leaf expansions and multipole shifts (stages P2M, M2M).
}  // namespace imq

imq_status imq_tree_s::ensure_side()
{
    if (side[0]) return IMQ_OK;
    for (hipStream_t &x : side) IMQ_HIP(hipStreamCreateWithFlags(&x, hipStreamNonBlocking));
    for (hipEvent_t *e : {&ev_fork, &ev_join, &ev_tfork, &ev_start, &ev_prep})
        IMQ_HIP(hipEventCreateWithFlags(e, hipEventDisableTiming));
    for (hipEvent_t &e : ev_tjoin) IMQ_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    for (hipEvent_t &e : ev_grp) IMQ_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    return IMQ_OK;
}

namespace imq {

template <typename T>
imq_status prep_locals(imq_tree_s *t, int nrhs, hipStream_t s);

// Launch the near field on the tree's second stream once everything queued
// on s so far (the gathered charges, P2M and the first shift levels) is done;
// ev_join marks its completion.
template <typename T>
imq_status fork_p2p(imq_tree_s *t, int nrhs, hipStream_t s)
{
    imq_status st = t->ensure_side();
    if (st != IMQ_OK) return st;
    PrecData &pd = prec_data<T>(t);
    IMQ_HIP(hipEventRecord(t->ev_fork, s));
    IMQ_HIP(hipStreamWaitEvent(t->side[0], t->ev_fork, 0));
    const int nrec = t->nnear;
    const int wg = t->kcfg.p2p_wg > 0 ? t->kcfg.p2p_wg : P2P_WG_DEFAULT;
    launch_p2p<T, true>(t->side[0], unsigned(std::min(nrec, wg)), make_view<T>(t), nrec, pd.us.as<T>(),
                        nrhs, t->bs.as<double>(), t->kcfg.p2p_mode == 1);
    IMQ_HIP(hipGetLastError());
    IMQ_HIP(hipEventRecord(t->ev_join, t->side[0]));
    return IMQ_OK;
}

template <typename T>
imq_status fmm_upward(imq_tree_s *t, int nrhs, hipStream_t s, bool fork, const UserVec *io)
{
    const HostTree &h = t->h;
    PrecData &pd = prec_data<T>(t);
    DTree<T> v = make_view<T>(t);
    const int nleaves = int(h.leaves.size());
    const int K = h.K, KS = coef_stride(K);
    T *M = pd.M.as<T>();
    mark(t, 1, s);
    const UserVec uv = io ? *io : UserVec();
    if (fork) {
        imq_status st = t->ensure_side();
        if (st != IMQ_OK) return st;
        IMQ_HIP(hipEventRecord(t->ev_start, s));
        // P2M reads the caller's weights; the point-order copy is for P2P and
        // P2L.  With few right-hand sides P2M stores that copy itself (ev_start
        // is then recorded after it), else a gather on side[0] makes it.
        if (uv.in && nrhs >= BATCH_RHS_MIN) {
            IMQ_HIP(hipStreamWaitEvent(t->side[0], t->ev_start, 0));
            const int64_t N = h.N;
            const dim3 gg(unsigned((N + 255) / 256), nrhs);
            if (uv.f32)
                hipLaunchKernelGGL((k_gather<float, T>), gg, dim3(256), 0, t->side[0], N, t->perm.as<int32_t>(),
                                   static_cast<const float *>(uv.in), uv.ldu, pd.us.template as<T>());
            else
                hipLaunchKernelGGL((k_gather<double, T>), gg, dim3(256), 0, t->side[0], N, t->perm.as<int32_t>(),
                                   static_cast<const double *>(uv.in), uv.ldu, pd.us.template as<T>());
            IMQ_HIP(hipGetLastError());
            IMQ_HIP(hipEventRecord(t->ev_start, t->side[0]));   // now: the copy is ready
        }
    }
    constexpr int RB = sizeof(T) == 4 ? 64 : 32;
    const dim3 gb(unsigned(nleaves), unsigned((nrhs + RB - 1) / RB));
#define IMQ_P2M(PP)                                                                                    \
    if (nrhs >= BATCH_RHS_MIN)                                                                         \
        hipLaunchKernelGGL((k_p2m_mfma<T, PP, RB>), gb, dim3(64), 0, s, v, t->leaves.as<int32_t>(),     \
                           pd.us.as<T>(), nrhs, M);                                                    \
    else                                                                                               \
        launch_p2m<T, PP>(s, nleaves, t->max_leaf, v, t->leafrec.as<LeafRec>(), pd.us.as<T>(), nrhs, M, uv)
    IMQ_DISPATCH_P(h.p, IMQ_P2M)
#undef IMQ_P2M
    IMQ_HIP(hipGetLastError());
    if (fork && uv.in && nrhs < BATCH_RHS_MIN) IMQ_HIP(hipEventRecord(t->ev_start, s));
    mark(t, 2, s);
    if (fork) {
        // Queued after P2M so that P2M's workgroups are dispatched first: clear L
        // and form the X pairs on side[1] (they need only the gathered weights).
        // The near field, which shares the GPU with the latency-bound shifts
        // and translations, is forked below.
        IMQ_HIP(hipStreamWaitEvent(t->side[1], t->ev_start, 0));
        imq_status st = prep_locals<T>(t, nrhs, t->side[1]);
        if (st != IMQ_OK) return st;
        IMQ_HIP(hipEventRecord(t->ev_prep, t->side[1]));
    }
    // The near field is forked once the finest upward shift level is queued:
    // it slows every latency-bound shift launch it runs beside, and the finest
    // level is the widest.  Measured on the 1M mixture (product ms, alternating
    // runs on one GPU) by the number of shift levels queued before the fork:
    // FP32 (an earlier kernel set) 0: 0.289-0.296, 1: 0.292-0.295, 2:
    // 0.297-0.298, 3: 0.304, all eight: 0.374; FP64 with the tuned orders,
    // best of five batches of 40, two or three alternations each: 0: 0.454,
    // 1: 0.414-0.416, 2: 0.419-0.420, 3: 0.456-0.457 (FP32 0.276-0.286 for
    // all four).
    constexpr int P2P_FORK_AFTER = 1;
    int nshift = 0;
    bool forked = !fork;
    for (int l = h.nlev - 2; l >= h.need_m; --l) {
        if (!forked && nshift == P2P_FORK_AFTER) {
            imq_status st = fork_p2p<T>(t, nrhs, s);
            if (st != IMQ_OK) return st;
            forked = true;
        }
        const int p0 = h.sh_level_begin[l], np = h.sh_level_begin[l + 1] - p0;
        launch_shift<T>(s, true, t->kcfg.shift_cols, np, nrhs, t->sh_par.as<int32_t>() + p0,
                        t->sh_kids.as<int32_t>() + 4 * size_t(p0), pd.m2m.as<T>(), t->KP, K, K, t->cut_m2m, M,
                        KS, M, KS);
        ++nshift;
    }
    if (!forked) {
        imq_status st = fork_p2p<T>(t, nrhs, s);
        if (st != IMQ_OK) return st;
    }
    IMQ_HIP(hipGetLastError());
    return IMQ_OK;
}

// Translations and downward pass into L (stages M2L, P2L, L2L).
// Clear L and form the X-list pair expansions (they need only the gathered
// weights); on side[1] when the product overlaps its stages.
template <typename T>
imq_status prep_locals(imq_tree_s *t, int nrhs, hipStream_t s)
{
    const HostTree &h = t->h;
    PrecData &pd = prec_data<T>(t);
    const int K = h.K, KS = coef_stride(K), ld = K | 1;
    const size_t nL = size_t(h.level.size()) * nrhs * KS;
    hipLaunchKernelGGL(k_fill<T>, dim3(unsigned((nL + 255) / 256)), dim3(256), 0, s, nL, pd.L.as<T>(), T(0));
    if (t->nxpairs > 0) {
        hipLaunchKernelGGL(k_p2l_pairs<T>, dim3(t->nxpairs), dim3(64), (size_t(64) * ld + 64) * sizeof(T), s,
                           make_view<T>(t), t->x_tgt.as<int32_t>(), pd.us.as<T>(), nrhs, pd.wx.as<T>(),
                           pd.Lx.as<T>(), ld, t->nxpairs);
        hipLaunchKernelGGL(k_p2l_reduce<T>, dim3(t->nxboxes), dim3(64), 0, s, make_view<T>(t),
                           t->x_boxes.as<int32_t>(), nrhs, pd.Lx.as<T>(), t->nxpairs, pd.L.as<T>());
    }
    IMQ_HIP(hipGetLastError());
    return IMQ_OK;
}

// Translations and downward pass into L (stages M2L, L2L; the X lists were
// added into the cleared L by prep_locals, so every M2L launch adds).
// overlap: the prep ran on side[1] (ev_prep); the M2L level groups run on
// side[1] and side[2], the W-list pair evaluations (M2P, which need only M)
// on side[2] ahead of its groups, and the L2L chain on the caller's stream
// starts as soon as the groups of the levels it reaches are done, beside the
// (larger) groups of the deeper levels.
template <typename T>
imq_status fmm_translate(imq_tree_s *t, int nrhs, hipStream_t s, bool overlap)
{
    const HostTree &h = t->h;
    PrecData &pd = prec_data<T>(t);
    DTree<T> v = make_view<T>(t);
    const int K = h.K, KP = t->KP, KS = coef_stride(K);
    T *M = pd.M.as<T>(), *L = pd.L.as<T>();
    const imq_kernel_config &kc = t->kcfg;
    mark(t, 3, s);
    imq_status st;
    if (!overlap) {
        if ((st = prep_locals<T>(t, nrhs, s)) != IMQ_OK) return st;
        mark(t, 4, s);
    } else {
        if ((st = t->ensure_side()) != IMQ_OK) return st;
        IMQ_HIP(hipEventRecord(t->ev_tfork, s));                  // multipoles complete
        for (int i = 1; i < imq_tree_s::NSIDE; ++i) IMQ_HIP(hipStreamWaitEvent(t->side[i], t->ev_tfork, 0));
        if (t->nwpairs > 0)
            hipLaunchKernelGGL(k_m2p_pairs<T>, dim3(t->nwpairs), dim3(64), 0, t->side[2], v, t->w_tgt.as<int32_t>(),
                               t->w_scr.as<int32_t>(), M, pd.wx.as<T>(), nrhs, t->Pw.as<double>(), t->nwscr);
        IMQ_HIP(hipStreamWaitEvent(s, t->ev_prep, 0));              // L cleared, X lists added
        IMQ_HIP(hipStreamWaitEvent(t->side[2], t->ev_prep, 0));
    }
    // Per level: the register-streaming kernel (modes 0 and 2, up to 80
    // coefficients; mode 2 runs the FP32 products on the BF16 matrix cores
    // from three-part operands) or the staged GEMM; consecutive levels of one
    // kind and row-block count share a launch (a group).
    std::vector<int> group_of(h.nlev, -1);
    {
        const DevGemm &g = t->g_m2l;
        // streamed up to 80 coefficients (modes 0, 2) or 160 (mode 3)
        const int smax = kc.m2l_mode == 3 ? 10 : 5;
        const auto kind = [&](int l) {
            const int nrb = (h.Klev[l] + 15) / 16;
            return (kc.m2l_mode != 1 && nrb <= smax) ? nrb : 0;
        };
        int ngroup = 0;
        for (int l = 0; l < h.nlev;) {
            const int t0 = g.level_task_begin[l];
            if (g.level_task_begin[l + 1] == t0) { ++l; continue; }
            const bool own_ev = overlap && ngroup < imq_tree_s::NGROUP_EV;
            hipStream_t gs = own_ev ? t->side[1 + ngroup % (imq_tree_s::NSIDE - 1)] : s;
            const int k = kind(l);
            int l2 = l + 1, kmax = h.Klev[l];
            while (l2 < h.nlev && (g.level_task_begin[l2 + 1] == g.level_task_begin[l2] || kind(l2) == k)) {
                kmax = std::max(kmax, h.Klev[l2]);
                ++l2;
            }
            const int nt = g.level_task_begin[l2] - t0;
            bool done = false;
            const uint16_t *abf = (sizeof(T) == 4 && kc.m2l_mode == 2) ? pd.m2l_bf3.as<uint16_t>() : nullptr;
            if (k > 0)
                done = launch_m2l_stream<T>(gs, 1, kmax, nt, t0, nrhs, g.tasks.as<GemmTask>(), g.tbox.as<int32_t>(),
                                            g.tab.as<int32_t>(), g.src.as<int32_t>(), pd.m2l_pk.as<T>(), abf, KP, KS, M,
                                            L);
            if (!done)
                launch_gemm<T>(gs, kc.m2l_kc > 0 ? kc.m2l_kc : 32, kc.m2l_split > 0 ? kc.m2l_split : 1, nt, nrhs,
                               g.tasks.as<GemmTask>(), t0, g.tbox.as<int32_t>(), g.tab.as<int32_t>(),
                               g.src.as<int32_t>(), pd.m2l.as<T>(), KP, KS, M, L, 1, 0, 0);
            if (own_ev) {
                IMQ_HIP(hipEventRecord(t->ev_grp[ngroup], gs));
                for (int ll = l; ll < l2; ++ll) group_of[ll] = ngroup;
            }
            ++ngroup;
            l = l2;
        }
    }
    IMQ_HIP(hipGetLastError());
    mark(t, 5, s);
    int waited = -1;                                               // groups are waited for in order
    auto wait_level = [&](int l) -> imq_status {
        if (l < h.nlev && group_of[l] > waited) {
            for (int gi = waited + 1; gi <= group_of[l]; ++gi) IMQ_HIP(hipStreamWaitEvent(s, t->ev_grp[gi], 0));
            waited = group_of[l];
        }
        return IMQ_OK;
    };
    for (int l = std::max(h.need_l, 0); l + 1 < h.nlev; ++l) {      // parents at level l
        if ((st = wait_level(l)) != IMQ_OK || (st = wait_level(l + 1)) != IMQ_OK) return st;
        const int p0 = h.sh_level_begin[l], np = h.sh_level_begin[l + 1] - p0;
        launch_shift<T>(s, false, kc.shift_cols, np, nrhs, t->sh_par.as<int32_t>() + p0,
                        t->sh_kids.as<int32_t>() + 4 * size_t(p0), pd.l2l.as<T>(), KP, h.Klev[l], h.Klev[l + 1],
                        t->cut_l2l, L, KS, L, KS);
    }
    if (overlap)
        for (int i = 1; i < imq_tree_s::NSIDE; ++i) {
            IMQ_HIP(hipEventRecord(t->ev_tjoin[i], t->side[i]));
            IMQ_HIP(hipStreamWaitEvent(s, t->ev_tjoin[i], 0));
        }
    IMQ_HIP(hipGetLastError());
    return IMQ_OK;
}

// The near field (P2P) depends only on the gathered charges, so it runs on a
// second stream of the tree, concurrently with the latency-bound shifts and
// translations (it is forked after P2M, which competes with it for the
// vector ALUs, and the finest upward shift level), and initialises bs;
// L2P and M2P then add to it.  With stage
// timing on, every stage runs on the caller's stream in order.
template <typename T>
imq_status fmm_sorted(imq_tree_s *t, int nrhs, hipStream_t s, const UserVec *io)
{
    const HostTree &h = t->h;
    PrecData &pd = prec_data<T>(t);
    DTree<T> v = make_view<T>(t);
    const int nleaves = int(h.leaves.size());
    const int32_t *leaves = t->leaves.as<int32_t>();
    double *bs = t->bs.as<double>();
    imq_status st;
    const bool overlap = g_cur_events == nullptr && !g_serial;
    if (io && !overlap) { set_error("internal: caller-order I/O needs the overlapped product"); return IMQ_EINVAL; }
    if ((st = fmm_upward<T>(t, nrhs, s, overlap, io)) != IMQ_OK) return st;
    if ((st = fmm_translate<T>(t, nrhs, s, overlap)) != IMQ_OK) return st;
    mark(t, 6, s);
    if (overlap) {
        IMQ_HIP(hipStreamWaitEvent(s, t->ev_join, 0));
    } else {
        launch_p2p<T, false>(s, unsigned(t->nnear), v, t->nnear, pd.us.as<T>(), nrhs, bs, t->kcfg.p2p_mode == 1);
        IMQ_HIP(hipGetLastError());
    }
    mark(t, 7, s);
    const UserVec uv = io ? *io : UserVec();
    const auto m2p = [&]() -> imq_status {
        if (t->nwpairs > 0) {
            double *Pw = t->Pw.as<double>();
            if (!overlap)        // else already run on side[2], joined after the translations
                hipLaunchKernelGGL(k_m2p_pairs<T>, dim3(t->nwpairs), dim3(64), 0, s, v, t->w_tgt.as<int32_t>(),
                                   t->w_scr.as<int32_t>(), pd.M.as<T>(), pd.wx.as<T>(), nrhs, Pw, t->nwscr);
            hipLaunchKernelGGL(k_m2p_reduce<T>, dim3(t->nwleaves), dim3(64), 0, s, v, t->w_leaves.as<int32_t>(),
                               t->w_scr.as<int32_t>(), nrhs, Pw, t->nwscr, bs);
        }
        IMQ_HIP(hipGetLastError());
        return IMQ_OK;
    };
    // Overlapped product with the result in caller order: L2P writes it last
    // and adds the W-list evaluations itself (one launch fewer on the chain).
    M2PParts wp;
    if (uv.out && t->nwpairs > 0) {
        if (!overlap) {
            set_error("internal: caller-order output needs the overlapped product");
            return IMQ_EINVAL;
        }
        wp.w_scr = t->w_scr.as<int32_t>();
        wp.Pw = t->Pw.as<double>();
        wp.nscr = t->nwscr;
    }
    LevelK lk = {};
    for (int l = 0; l < h.nlev && l < 32; ++l) lk.K[l] = h.Klev[l];
    constexpr int RB = sizeof(T) == 4 ? 64 : 32;
    const dim3 gb(unsigned(nleaves), unsigned((nrhs + RB - 1) / RB));
#define IMQ_L2P(PP)                                                                                    \
    if (nrhs >= BATCH_RHS_MIN)                                                                         \
        hipLaunchKernelGGL((k_l2p_mfma<T, PP, RB>), gb, dim3(64), 0, s, v, leaves, pd.L.as<T>(), nrhs, bs); \
    else                                                                                               \
        launch_l2p<T, PP>(s, nleaves, t->max_leaf, v, lk, pd.L.as<T>(), nrhs, bs, uv, wp)
    IMQ_DISPATCH_P(h.p, IMQ_L2P)
#undef IMQ_L2P
    IMQ_HIP(hipGetLastError());
    mark(t, 8, s);
    if (!uv.out && (st = m2p()) != IMQ_OK) return st;
    mark(t, 9, s);
    return IMQ_OK;
}

// Algorithm 1 (Sec. 2.2) on sorted, gathered vectors: P2M for every box at
// the levels that have V lists, the direct near field (which writes bs), then
// the direct multipole evaluations of k_alg1_far.  In order on s.
template <typename T>
imq_status alg1_sorted(imq_tree_s *t, int nrhs, hipStream_t s)
{
    const HostTree &h = t->h;
    if (t->nwpairs > 0 || t->nxpairs > 0) {
        set_error("Algorithm 1 mode needs the adaptive W/X interactions summed directly (build with a larger direct_max)");
        return IMQ_EUNSUPPORTED;
    }
    PrecData &pd = prec_data<T>(t);
    DTree<T> v = make_view<T>(t);
    const int nleaves = int(h.leaves.size());
    const int K = h.K, ld = K | 1;
    double *bs = t->bs.as<double>();
    mark(t, 1, s);
    const size_t lds_p2m = (size_t(P2M_CHUNK) * ld + P2M_CHUNK) * sizeof(T);
    if (t->nboxrec > 0) {
#define IMQ_P2M_ALL(PP)                                                                                  \
        hipLaunchKernelGGL((k_p2m_box<T, PP>), dim3(unsigned(t->nboxrec)), dim3(64), lds_p2m, s, v,       \
                           t->boxrec.as<BoxRec>(), t->boxleaf.as<int32_t>(), pd.us.as<T>(), nrhs, pd.M.as<T>(), ld)
        IMQ_DISPATCH_P(h.p, IMQ_P2M_ALL)
#undef IMQ_P2M_ALL
        IMQ_HIP(hipGetLastError());
    }
    mark(t, 2, s);
    mark(t, 3, s);
    mark(t, 4, s);
    mark(t, 5, s);
    mark(t, 6, s);
    launch_p2p<T, false>(s, unsigned(t->nnear), v, t->nnear, pd.us.as<T>(), nrhs, bs, false);
    IMQ_HIP(hipGetLastError());
    mark(t, 7, s);
    hipLaunchKernelGGL(k_alg1_far<T>, dim3(unsigned(nleaves)), dim3(64), 0, s, v, pd.M.as<T>(), pd.wx.as<T>(),
                       nrhs, bs);
    IMQ_HIP(hipGetLastError());
    mark(t, 8, s);
    mark(t, 9, s);
    return IMQ_OK;
}

template void launch_gemm<double>(hipStream_t, int, int, int, int, const GemmTask *, int, const int32_t *,
                                  const int32_t *, const int32_t *, const double *, int, int,
                                  const double *, double *, int, int, int);
template void launch_gemm<float>(hipStream_t, int, int, int, int, const GemmTask *, int, const int32_t *,
                                 const int32_t *, const int32_t *, const float *, int, int, const float *,
                                 float *, int, int, int);
template imq_status fmm_upward<double>(imq_tree_s *, int, hipStream_t, bool, const UserVec *);
template imq_status fmm_upward<float>(imq_tree_s *, int, hipStream_t, bool, const UserVec *);
template imq_status fmm_translate<double>(imq_tree_s *, int, hipStream_t, bool);
template imq_status fmm_translate<float>(imq_tree_s *, int, hipStream_t, bool);
template imq_status fmm_sorted<double>(imq_tree_s *, int, hipStream_t, const UserVec *);
template imq_status fmm_sorted<float>(imq_tree_s *, int, hipStream_t, const UserVec *);
template imq_status ensure_workspace<double>(imq_tree_s *, int);
template imq_status ensure_workspace<float>(imq_tree_s *, int);
template DTree<double> make_view<double>(const imq_tree_s *);
template DTree<float> make_view<float>(const imq_tree_s *);

template <typename Tin, typename T>
imq_status launch_gather(imq_tree_s *t, int nrhs, const Tin *u, int64_t ldu, hipStream_t s)
{
    const int64_t N = t->h.N;
    hipLaunchKernelGGL((k_gather<Tin, T>), dim3(unsigned((N + 255) / 256), nrhs), dim3(256), 0, s, N,
                       t->perm.as<int32_t>(), u, ldu, prec_data<T>(t).us.template as<T>());
    IMQ_HIP(hipGetLastError());
    return IMQ_OK;
}

template <typename Tout>
imq_status launch_scatter(imq_tree_s *t, int nrhs, Tout *b, int64_t ldb, hipStream_t s)
{
    const int64_t N = t->h.N;
    hipLaunchKernelGGL((k_scatter<Tout>), dim3(unsigned((N + 255) / 256), nrhs), dim3(256), 0, s, N,
                       t->perm.as<int32_t>(), t->pt_scale.as<double>(), t->bs.as<double>(), b, ldb);
    IMQ_HIP(hipGetLastError());
    return IMQ_OK;
}

template <typename T, typename Tio>
imq_status matvec_typed(imq_tree_s *t, int nrhs, const Tio *u, int64_t ldu, Tio *b, int64_t ldb,
                        hipStream_t s)
{
    imq_status st = ensure_workspace<T>(t, nrhs);
    if (st != IMQ_OK) return st;
    g_cur_events = t->stage_events();
    mark(t, 0, s);
    if (t->kcfg.far_field == 1) {
        if ((st = launch_gather<Tio, T>(t, nrhs, u, ldu, s)) == IMQ_OK && (st = alg1_sorted<T>(t, nrhs, s)) == IMQ_OK &&
            (st = launch_scatter<Tio>(t, nrhs, b, ldb, s)) == IMQ_OK)
            mark(t, 10, s);
    } else if (!g_cur_events && !g_serial && nrhs < BATCH_RHS_MIN) {
        // overlapped product: L2P, the last stage, writes b in caller order (no
        // separate scatter).  Reading u through the permutation inside P2M
        // instead of gathering it first was measured slower: it puts a second
        // dependent load in P2M, which is on the critical path.
        UserVec io;
        io.out = b;
        io.ldb = ldb;
        io.f32 = sizeof(Tio) == 4;
        io.perm = t->perm.as<int32_t>();
        io.scale = t->pt_scale.as<double>();
        if ((st = launch_gather<Tio, T>(t, nrhs, u, ldu, s)) == IMQ_OK) st = fmm_sorted<T>(t, nrhs, s, &io);
    } else if ((st = launch_gather<Tio, T>(t, nrhs, u, ldu, s)) == IMQ_OK &&
               (st = fmm_sorted<T>(t, nrhs, s, nullptr)) == IMQ_OK &&
               (st = launch_scatter<Tio>(t, nrhs, b, ldb, s)) == IMQ_OK)
        mark(t, 10, s);
    g_cur_events = nullptr;
    return st;
}

template imq_status matvec_typed<double, double>(imq_tree_s *, int, const double *, int64_t, double *, int64_t, hipStream_t);
template imq_status matvec_typed<double, float>(imq_tree_s *, int, const float *, int64_t, float *, int64_t, hipStream_t);
template imq_status matvec_typed<float, double>(imq_tree_s *, int, const double *, int64_t, double *, int64_t, hipStream_t);
template imq_status matvec_typed<float, float>(imq_tree_s *, int, const float *, int64_t, float *, int64_t, hipStream_t);

imq_status rows_exact(imq_tree_s *t, int nrhs, const double *u, int64_t ldu, int64_t nrows,
                      const int64_t *rows, double *b, int64_t ldb, hipStream_t s)
{
    if (nrows == 0) return IMQ_OK;
    hipLaunchKernelGGL(k_rows_exact, dim3(unsigned(nrows), nrhs), dim3(256), 0, s, t->h.nsets,
                       t->set_off.as<int64_t>(), t->cn.as<double>() + t->h.nsets, t->xy_user.as<double>(),
                       t->h.N, u, ldu, rows, b, ldb);
    IMQ_HIP(hipGetLastError());
    return IMQ_OK;
}

}  // namespace imq
