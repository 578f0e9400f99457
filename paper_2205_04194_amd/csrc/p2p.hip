// Near field (P2P, the U lists): the direct sums of the kernel over each
// leaf's adjacent leaves, in a vector form and, for one right-hand side, a
// matrix-core form (FP32 or FP64 matrix cores).
#include "device.h"
#include "mfma.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

namespace imq {

namespace {

// Reciprocal square root for the direct sums: the hardware estimate in
// FP32; in FP64 the hardware estimate (relative error below 2^-22) refined
// by one step of the third-order iteration for x^(-1/2): with
// e = 1 - x y^2, y <- y (1 + e/2 + 3 e^2 / 8), whose truncation error is
// about (5/16) |e|^3, below 1e-19 here (five operations; two Newton steps
// take seven).
__device__ __forceinline__ float rsqrt_fast(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double rsqrt_fast(double x)
{
    const double y = __builtin_amdgcn_rsq(x);
    const double e = fma(-x * y, y, 1.0);
    return fma(y * e, fma(e, 0.375, 0.5), y);
}

template <typename T> struct Vec4;
template <> struct Vec4<float> { typedef float type __attribute__((ext_vector_type(4))); };
template <> struct Vec4<double> { typedef double type __attribute__((ext_vector_type(4))); };

constexpr int P2P_CHUNK = 128;                 // sources staged per round (a small stage leaves LDS
                                               // to the tree passes running alongside)
constexpr int P2P_LDS = P2P_CHUNK + 64;        // + padding to a multiple of 4 per lane group
constexpr int P2P_MF_LD = P2P_CHUNK + 16;      // row stride of the matrix-core stage (bank offset)

// One U-list entry as the staging reads it back from LDS (one load): the
// offset from a chunk slot number to the source's point index, and the
// centre offset.
template <typename T>
struct alignas(16) SRec {
    int jo;
    T ox, oy;
};

// LDS of one workgroup.  MF: the kernel instance that also has the
// matrix-core form; a leaf uses one form, so the two forms' source stages
// share their memory.
template <typename T, int NR>
struct alignas(32) P2PVecStage {               // every array starts on a 32-byte boundary
    // vector form: the chunk's sources (and |x|^2 for the expanded
    // distances), read back four at a time
    T x[P2P_LDS], y[P2P_LDS], w[P2P_LDS], u[NR][P2P_LDS];
};
template <typename T>
struct alignas(32) P2PMfStage {
    // matrix-core form (one right-hand side): per source |x|^2, x, y and a
    // row of zeros (written once per leaf), and the weights in the order the
    // matrix-core result holds the sources
    T B[4][P2P_MF_LD];
    T U[P2P_CHUNK];
};
template <typename T, int NR, bool MF>
struct alignas(32) P2PStage {
    union {
        P2PVecStage<T, NR> v;
        P2PMfStage<T> m;
    };
    // staging: 1 + the entry that starts at each slot of the chunk (else 0),
    // and per entry of the batch the offset from slot number to point index
    // and the centre offset
    int mk[P2P_CHUNK];
    SRec<T> rec[64];
};

// Inclusive running maximum over the 64 lanes of a wave (values >= 0): a
// Hillis-Steele scan inside each row of 16 lanes (row shifts by 1, 2, 4, 8),
// then the last lane of rows 0 and 2 into rows 1 and 3, then lane 31 into
// rows 2 and 3 (row broadcasts).  Lanes with no source lane keep 0.
__device__ __forceinline__ int wave_max_scan(int v)
{
    v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, false));   // row_shr:1
    v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, false));   // row_shr:2
    v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, false));   // row_shr:4
    v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, false));   // row_shr:8
    v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, false));   // row_bcast:15
    v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x143, 0xc, 0xf, false));   // row_bcast:31
    return v;
}

// The sources of a target leaf (U-list entries [u0, u1)), staged a chunk of
// up to P2P_CHUNK at a time.  The entry records are read 64 at a time, one per
// lane, and a wave prefix sum numbers the batch's sources consecutively.
// Lane l gathers slots l, l + 64, ... of a chunk (each load of
// the wave covers consecutive points), with every load of the chunk in flight
// at once.  A slot's entry comes from marking each entry's first slot in LDS
// and a running maximum over the slots (across the wave for each group of
// 64 slots, carried from group to group).  store(e, x, y, u) puts the source of chunk slot e into
// the stage (coordinates relative to the target leaf's centre, zero past the
// chunk's n sources); consume(n) then runs once per chunk, in source order.
template <typename T, int NR, bool MF, typename S, typename F>
__device__ __forceinline__ void p2p_sources(const DTree<T> &t, int u0, int u1, const T *__restrict__ us, int r0,
                                            int nr, P2PStage<T, NR, MF> &sh, S &&store, F &&consume)
{
    constexpr int SPL = P2P_CHUNK / 64;              // chunk slots per lane
    const int lane = threadIdx.x;
    const int64_t N = t.N;
    for (int ub = u0; ub < u1; ub += 64) {
        const int nb = min(64, u1 - ub);
        URec<T> ur{0, 0, T(0), T(0)};
        if (lane < nb) ur = t.urec[ub + lane];
        int incl = ur.cnt;                           // inclusive prefix sum over the wave
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const int v = __shfl_up(incl, d);
            if (lane >= d) incl += v;
        }
        const int total = __shfl(incl, 63);
        const int off = incl - ur.cnt;               // first slot of this lane's entry
        __syncthreads();                             // previous batch's records no longer read
        sh.rec[lane] = SRec<T>{ur.beg - off, ur.ox, ur.oy};
        int carry = 0;                               // 1 + entry of the slot before the group
        for (int c0 = 0; c0 < total; c0 += P2P_CHUNK) {
            const int n = min(P2P_CHUNK, total - c0);
            if (4 * lane < P2P_CHUNK) *reinterpret_cast<int4 *>(&sh.mk[4 * lane]) = make_int4(0, 0, 0, 0);
            __syncthreads();
            if (ur.cnt > 0 && off >= c0 && off < c0 + P2P_CHUNK) sh.mk[off - c0] = lane + 1;
            __syncthreads();
            int ent[SPL];
#pragma unroll
            for (int k = 0; k < SPL; ++k) {
                const int m = max(wave_max_scan(sh.mk[lane + 64 * k]), carry);
                carry = __builtin_amdgcn_readlane(m, 63);
                ent[k] = max(m - 1, 0);
            }
            T vx[SPL], vy[SPL], vu[SPL][NR];
#pragma unroll
            for (int k = 0; k < SPL; ++k) {
                const int sl = c0 + lane + 64 * k;
                vx[k] = vy[k] = T(0);
#pragma unroll
                for (int q = 0; q < NR; ++q) vu[k][q] = T(0);
                if (sl < total) {
                    const SRec<T> rc = sh.rec[ent[k]];
                    const int j = sl + rc.jo;
                    vx[k] = t.xl[j] + rc.ox;
                    vy[k] = t.yl[j] + rc.oy;
#pragma unroll
                    for (int q = 0; q < NR; ++q)
                        if (q < nr) vu[k][q] = us[(r0 + q) * N + j];
                }
            }
#pragma unroll
            for (int k = 0; k < SPL; ++k) store(lane + 64 * k, vx[k], vy[k], vu[k]);
            consume(n);
        }
    }
}

// P2P: b_i += sum over U-list leaves a of sum_j u_j / sqrt(|x_i - x_j|^2 + c^2).
// One wave per target leaf at a time; with a grid smaller than the leaf count
// a workgroup walks several leaves (leaving wave slots free for kernels
// running alongside).
// SIDE only tells the two launch forms apart in profiles: alongside the tree
// passes (true) or alone on the caller's stream (false).
// Vector form, one block of up to 128 targets of a leaf (R per lane): lane l
// takes targets ti and ti + TP of group g (l = g TP + ti, TP = ceil(ntc / R)
// rounded up to 4 at least, G = 64 / TP groups; lanes past G TP idle).  R is
// chosen per leaf to keep the most lanes busy (e.g. 40 points: R = 2, 60 of 64
// lanes instead of 40).  Each chunk of sources is padded with zero weights to
// a multiple of 4 G; each group sums a contiguous run of it, 4 sources per
// step, in a loop whose trip count is the same for every lane.  Partial sums
// over one chunk are kept in T, the running sums in FP64, and the G group sums
// of a target are added with lane shuffles in group order.
// EXP: the squared distance plus c^2 as (|x_i|^2 + c^2 + |x_j|^2) - 2 x_i . x_j
// (one add and two fused multiply-adds instead of two subtractions and two
// fused multiply-adds), for leaves whose neighbourhood is small against c.
template <typename T, int NR, int R, bool MF, bool EXP>
__device__ __forceinline__ void p2p_block(const DTree<T> &t, const NearLeaf &nl, int t0, int ntc,
                                          const T *__restrict__ us, int nrhs, double *__restrict__ bs, int add,
                                          P2PStage<T, NR, MF> &sh)
{
    using V4 = typename Vec4<T>::type;
    const int lane = threadIdx.x;
    const int64_t N = t.N;
    const T c2 = T(nl.c2);
    const int TP = max(4, (ntc + R - 1) / R);
    const int G = 64 / TP, grp = lane / TP, ti = lane % TP;
    bool valid[R];
    T xi[R], yi[R], ai[R];
#pragma unroll
    for (int rr = 0; rr < R; ++rr) {
        valid[rr] = grp < G && ti + rr * TP < ntc;
        const int i = t0 + (valid[rr] ? ti + rr * TP : 0);
        xi[rr] = t.xl[i];
        yi[rr] = t.yl[i];
        if constexpr (EXP) {
            ai[rr] = fma(xi[rr], xi[rr], fma(yi[rr], yi[rr], c2));
            xi[rr] *= T(-2);
            yi[rr] *= T(-2);
        }
    }
    for (int r0 = 0; r0 < nrhs; r0 += NR) {          // NR right-hand sides per pass
        const int nr = min(NR, nrhs - r0);
        double acc[R][NR];
#pragma unroll
        for (int rr = 0; rr < R; ++rr)
#pragma unroll
            for (int q = 0; q < NR; ++q) acc[rr][q] = 0.0;
        auto store = [&](int e, T x, T y, const T (&u)[NR]) {
            sh.v.x[e] = x;
            sh.v.y[e] = y;
            if constexpr (EXP) sh.v.w[e] = fma(x, x, y * y);
#pragma unroll
            for (int q = 0; q < NR; ++q) sh.v.u[q][e] = u[q];
        };
        auto consume = [&](int n) {
            const int per = ((n + G - 1) / G + 3) & ~3;   // sources per group, multiple of 4
            for (int e = P2P_CHUNK / 4 + lane; e < per * G / 4; e += 64) {
                reinterpret_cast<V4 *>(sh.v.x)[e] = V4{T(0), T(0), T(0), T(0)};
                reinterpret_cast<V4 *>(sh.v.y)[e] = V4{T(0), T(0), T(0), T(0)};
                if constexpr (EXP) reinterpret_cast<V4 *>(sh.v.w)[e] = V4{T(0), T(0), T(0), T(0)};
#pragma unroll
                for (int q = 0; q < NR; ++q) reinterpret_cast<V4 *>(sh.v.u[q])[e] = V4{T(0), T(0), T(0), T(0)};
            }
            __syncthreads();
            if (grp < G) {
                T part[R][NR];
#pragma unroll
                for (int rr = 0; rr < R; ++rr)
#pragma unroll
                    for (int q = 0; q < NR; ++q) part[rr][q] = T(0);
                const int nq = __builtin_amdgcn_readfirstlane(per >> 2);   // the same in every lane
                const V4 *px = reinterpret_cast<const V4 *>(sh.v.x) + grp * nq;
                const V4 *py = reinterpret_cast<const V4 *>(sh.v.y) + grp * nq;
                const V4 *pw = reinterpret_cast<const V4 *>(sh.v.w) + grp * nq;
                for (int it = 0; it < nq; ++it) {
                    const V4 X = px[it], Y = py[it];
                    V4 W;
                    if constexpr (EXP) W = pw[it];
#pragma unroll
                    for (int rr = 0; rr < R; ++rr) {
                        T kv[4];
#pragma unroll
                        for (int k = 0; k < 4; ++k) {
                            if constexpr (EXP) {
                                kv[k] = rsqrt_fast(fma(xi[rr], X[k], fma(yi[rr], Y[k], ai[rr] + W[k])));
                            } else {
                                const T dx = xi[rr] - X[k], dy = yi[rr] - Y[k];
                                kv[k] = rsqrt_fast(fma(dx, dx, fma(dy, dy, c2)));
                            }
                        }
#pragma unroll
                        for (int q = 0; q < NR; ++q) {
                            const V4 U = reinterpret_cast<const V4 *>(sh.v.u[q])[grp * nq + it];
#pragma unroll
                            for (int k = 0; k < 4; ++k) part[rr][q] += U[k] * kv[k];
                        }
                    }
                }
#pragma unroll
                for (int rr = 0; rr < R; ++rr)
#pragma unroll
                    for (int q = 0; q < NR; ++q) acc[rr][q] += double(part[rr][q]);
            }
            __syncthreads();
        };
        p2p_sources<T, NR, MF>(t, nl.u0, nl.u1, us, r0, nr, sh, store, consume);
        // group sums in group order; group 0 writes
#pragma unroll
        for (int rr = 0; rr < R; ++rr)
#pragma unroll
            for (int q = 0; q < NR; ++q) {
                double aq = acc[rr][q];
                for (int g = 1; g < G; ++g) aq += __shfl(acc[rr][q], ti + g * TP);
                if (q < nr && grp == 0 && valid[rr]) {
                    double &dst = bs[(r0 + q) * N + t0 + ti + rr * TP];
                    dst = add ? dst + aq : aq;
                }
            }
    }
}

// Matrix-core form (one right-hand side), up to 16 TT targets.  With
// every coordinate relative to the target leaf's centre,
//     |x_i - x_j|^2 + c^2 = (|x_i|^2 + c^2) + |x_j|^2 - 2 x_i . x_j,
// so the squared distances of 16 sources x 16 targets are one matrix-core
// step: the source matrix with rows [|x_j|^2, x_j, y_j, 0] times the target
// matrix with columns [1, -2 x_i, -2 y_i, 0], accumulated onto |x_i|^2 + c^2.
// The vector unit is left with the reciprocal square roots and the weights.
// The expansion loses about (|x_i|^2 + |x_j|^2) / c^2 units of rounding to
// cancellation, so the host sends a leaf here only when its neighbourhood is
// small against c.
// Lane l (q = l / 16, c16 = l % 16) supplies entry (c16, q) of the source
// matrix and (q, c16) of the target matrix; item v of the result is the pair
// (source 16 s + row(q, v), target 16 tt + c16) (row = 4 q + v in FP32,
// 4 v + q in FP64), so a lane sums its target over four sources per tile and
// the four lane groups are added at the end.
// Padding sources have weight 0 and padding targets |x_i|^2 + c^2 = 1, so
// every squared distance stays positive.
template <typename T, int TT>
__device__ __forceinline__ void p2p_block_mf(const DTree<T> &t, const NearLeaf &nl, int t0, int ntc,
                                             const T *__restrict__ us, double *__restrict__ bs, int add,
                                             P2PStage<T, 1, true> &sh)
{
    using acc_t = typename Mfma<T>::acc_t;
    const int lane = threadIdx.x, q = lane >> 4, c16 = lane & 15;
    const T c2 = T(nl.c2);
    T bt[TT];
    acc_t ci[TT];
    double acc[TT];
#pragma unroll
    for (int tt = 0; tt < TT; ++tt) {
        const int i = 16 * tt + c16;
        T xi = T(0), yi = T(0), ai = T(1);
        if (i < ntc) {
            xi = t.xl[t0 + i];
            yi = t.yl[t0 + i];
            ai = fma(xi, xi, fma(yi, yi, c2));
        }
        bt[tt] = q == 0 ? T(1) : q == 1 ? T(-2) * xi : q == 2 ? T(-2) * yi : T(0);
        ci[tt] = acc_t{ai, ai, ai, ai};
        acc[tt] = 0.0;
    }
    // the zero row of the source matrix (the stage is shared with the vector
    // form, which may have used it since)
    for (int e = threadIdx.x; e < P2P_MF_LD; e += 64) sh.m.B[3][e] = T(0);
    // item v of a lane's result holds source Mfma<T>::row(q, v) of the tile:
    // the weights are stored so that four consecutive ones are those
    auto upos = [](int e) {
        const int sl = e & 15;
        int pos = sl;
        for (int qq = 0; qq < 4; ++qq)
            for (int v = 0; v < 4; ++v)
                if (Mfma<T>::row(qq, v) == sl) pos = 4 * qq + v;
        return (e & ~15) + pos;
    };
    auto store = [&](int e, T x, T y, const T (&u)[1]) {
        sh.m.B[0][e] = fma(x, x, y * y);
        sh.m.B[1][e] = x;
        sh.m.B[2][e] = y;
        sh.m.U[upos(e)] = u[0];
    };
    auto consume = [&](int n) {
        const int nt = __builtin_amdgcn_readfirstlane((n + 15) >> 4);   // 16-source tiles
        __syncthreads();
        T part[TT];
#pragma unroll
        for (int tt = 0; tt < TT; ++tt) part[tt] = T(0);
        // Software pipelined: while the vector unit works on tile s, the
        // matrix-core step of tile s + 1 and the LDS reads of tile s + 2
        // (source entries) and s + 1 (weights) are in flight; indices past the
        // last tile re-read it.  The scheduling barriers keep the compiler from
        // sinking the reads back next to their use.
        auto lda = [&](int s) { return sh.m.B[q][16 * min(s, nt - 1) + c16]; };
        auto ldu = [&](int s) { return *reinterpret_cast<const acc_t *>(&sh.m.U[16 * min(s, nt - 1) + 4 * q]); };
        auto mma = [&](T a, acc_t (&r)[TT]) {
#pragma unroll
            for (int tt = 0; tt < TT; ++tt) r[tt] = Mfma<T>::mac(a, bt[tt], ci[tt]);
        };
        auto use = [&](const acc_t (&r)[TT], const acc_t &u) {
#pragma unroll
            for (int tt = 0; tt < TT; ++tt)
#pragma unroll
                for (int v = 0; v < 4; ++v) part[tt] = fma(u[v], rsqrt_fast(r[tt][v]), part[tt]);
        };
        // two tiles per trip with the registers of the two in alternation
        acc_t rA[TT], rB[TT];
        mma(lda(0), rA);
        T aA, aB = lda(1);
        acc_t uA = ldu(0), uB;
        for (int s = 0; s < nt; s += 2) {
            mma(aB, rB);                         // tile s + 1
            __builtin_amdgcn_sched_barrier(0);
            aA = lda(s + 2);
            uB = ldu(s + 1);
            __builtin_amdgcn_sched_barrier(0);
            use(rA, uA);                         // tile s
            if (s + 1 >= nt) break;
            mma(aA, rA);                         // tile s + 2
            __builtin_amdgcn_sched_barrier(0);
            aB = lda(s + 3);
            uA = ldu(s + 2);
            __builtin_amdgcn_sched_barrier(0);
            use(rB, uB);                         // tile s + 1
        }
#pragma unroll
        for (int tt = 0; tt < TT; ++tt) acc[tt] += double(part[tt]);
        __syncthreads();
    };
    p2p_sources<T, 1, true>(t, nl.u0, nl.u1, us, 0, 1, sh, store, consume);
#pragma unroll
    for (int tt = 0; tt < TT; ++tt) {
        double s = acc[tt];
        s += __shfl_xor(s, 16);
        s += __shfl_xor(s, 32);
        const int i = 16 * tt + c16;
        if (q == 0 && i < ntc) {
            double &dst = bs[t0 + i];
            dst = add ? dst + s : s;
        }
    }
}

// MF (one right-hand side only): leaves flagged in the NearLeaf records take
// the matrix-core form.
template <typename T, bool SIDE, int NR, bool MF>
__global__ __launch_bounds__(64) void k_p2p(DTree<T> t, int nleaves, const T *__restrict__ us, int nrhs,
                                            double *__restrict__ bs, int add)
{
    static_assert(!MF || NR == 1, "matrix-core form: one right-hand side");
    __shared__ P2PStage<T, NR, MF> sh;
    // Leaf records are dealt round robin, as the hardware deals workgroups to
    // the XCDs: record lf runs on XCD lf mod 8 when the grid is a multiple of
    // 8, and the host arranges the records for that (equal-cost runs of the
    // Morton order, one per XCD; empty records have no targets).
    for (int lf = blockIdx.x; lf < nleaves; lf += gridDim.x) {
        const NearLeaf nl = t.nleaf[lf];
        if constexpr (MF) {
            if (nl.expand) {
                for (int t0 = nl.begin; t0 < nl.end; t0 += 64) {
                    const int ntc = min(64, nl.end - t0);
                    switch ((ntc + 15) >> 4) {
                    case 1: p2p_block_mf<T, 1>(t, nl, t0, ntc, us, bs, add, sh); break;
                    case 2: p2p_block_mf<T, 2>(t, nl, t0, ntc, us, bs, add, sh); break;
                    case 3: p2p_block_mf<T, 3>(t, nl, t0, ntc, us, bs, add, sh); break;
                    default: p2p_block_mf<T, 4>(t, nl, t0, ntc, us, bs, add, sh); break;
                    }
                }
                continue;
            }
        }
        auto blocks = [&](auto exp) {
            constexpr bool E = decltype(exp)::value;
            for (int t0 = nl.begin; t0 < nl.end; t0 += 128) {
                const int ntc = min(128, nl.end - t0);
                // targets per lane: the choice that keeps the most lanes busy
                const int g1 = ntc <= 64 ? 64 / max(4, ntc) : 0;
                const int g2 = 64 / max(4, (ntc + 1) / 2);
                if (NR <= 4 && g2 * ntc > 2 * g1 * ntc)
                    p2p_block<T, NR, (NR <= 4 ? 2 : 1), MF, E>(t, nl, t0, ntc, us, nrhs, bs, add, sh);
                else if (ntc <= 64)
                    p2p_block<T, NR, 1, MF, E>(t, nl, t0, ntc, us, nrhs, bs, add, sh);
                else {       // 65..128 targets with 16 right-hand sides: two blocks of one per lane
                    p2p_block<T, NR, 1, MF, E>(t, nl, t0, 64, us, nrhs, bs, add, sh);
                    p2p_block<T, NR, 1, MF, E>(t, nl, t0 + 64, ntc - 64, us, nrhs, bs, add, sh);
                }
            }
        };
        if (nl.expand)
            blocks(std::true_type{});
        else
            blocks(std::false_type{});
    }
}

}  // namespace

// Near-field launch: NR right-hand sides share each kernel value.
template <typename T, bool SIDE>
void launch_p2p(hipStream_t s, unsigned grid, const DTree<T> &v, int nleaves, const T *us, int nrhs, double *bs,
                bool mf)
{
    if (nrhs == 1 && mf) {
        hipLaunchKernelGGL((k_p2p<T, SIDE, 1, true>), dim3(grid), dim3(64), 0, s, v, nleaves, us, nrhs, bs, 0);
        return;
    }
    if (nrhs == 1)
        hipLaunchKernelGGL((k_p2p<T, SIDE, 1, false>), dim3(grid), dim3(64), 0, s, v, nleaves, us, nrhs, bs, 0);
    else if (nrhs <= 4)
        hipLaunchKernelGGL((k_p2p<T, SIDE, 4, false>), dim3(grid), dim3(64), 0, s, v, nleaves, us, nrhs, bs, 0);
    else
        hipLaunchKernelGGL((k_p2p<T, SIDE, 16, false>), dim3(grid), dim3(64), 0, s, v, nleaves, us, nrhs, bs, 0);
}

template void launch_p2p<float, true>(hipStream_t, unsigned, const DTree<float> &, int, const float *, int, double *,
                                      bool);
template void launch_p2p<float, false>(hipStream_t, unsigned, const DTree<float> &, int, const float *, int, double *,
                                       bool);
template void launch_p2p<double, true>(hipStream_t, unsigned, const DTree<double> &, int, const double *, int,
                                       double *, bool);
template void launch_p2p<double, false>(hipStream_t, unsigned, const DTree<double> &, int, const double *, int,
                                        double *, bool);

}  // namespace imq
