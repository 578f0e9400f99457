// Level-by-level expansion shifts on the matrix cores.
//
//   M2M (upward):  M[parent] = sum over the four quadrants q of T_q M[child_q]
//   L2L (downward): L[child_q] += T_q L[parent]
//
// T_q is the shift of the expansion centre from the parent's to the child's
// (or back) for the child in quadrant q (Sec. 2.2: the addition theorem of the
// solid harmonics; the lifted planes z = -c/2 and z = +c/2 stay fixed, so the
// shift is horizontal and its table depends on the quadrant only).  One
// launch per level.  Each workgroup loads its slice of the tables into
// registers at the start and stages the source expansions of its tile in LDS
// once, so a launch costs two dependent memory round trips (the quadrant map,
// then the expansions) plus the matrix-core work.
#include "device.h"
#include "mfma.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

namespace imq {

namespace {

// Workgroup = 4 waves; wave w owns quadrant w.  A tile is TC = 16*NCB columns
// (parent box, right-hand side) times RBS row blocks of 16 output coefficients
// (blockIdx.y picks the row blocks).  Packed table layout: element j of lane l of
// (quadrant, row block rb, chunk ch) is T[16 rb + l%16][16 ch + 4 (l/16) + j],
// so one load of four values per lane feeds four 16x16x4 steps, and the
// source coefficients a lane feeds in them are four consecutive ones.
// M2M: each wave reads its quadrant's children straight into registers (no
// source is shared between waves), and the four partial results are summed
// in LDS; L2L: the parents, which all four waves read, are staged in LDS.
template <typename T, int NRB, int NCB, int RBS, bool UP>
__global__ __launch_bounds__(256) void k_shift(const int32_t *__restrict__ par,
                                               const int32_t *__restrict__ kids, int npar, int nrhs,
                                               const T *__restrict__ Apk, int kin, int kout, ShiftCuts cuts,
                                               const T *__restrict__ in, int ldin, T *__restrict__ out,
                                               int ldout)
{
    tree_pass_priority();
    constexpr int TC = 16 * NCB;
    constexpr int KPC = NRB * 16;
    constexpr int LD = KPC + (sizeof(T) == 4 ? 2 : 1);     // LDS row stride of the staged parents
    constexpr int RLD = RBS * 16 + 1;                       // row stride of the quadrant sums
    constexpr int NBT = TC * KPC / 256;                     // staged values per thread
    constexpr int BATCH = sizeof(T) == 4 ? 32 : 16;
    using acc_t = typename Mfma<T>::acc_t;
    using Q = Quad<T>;
    __shared__ T Bs[UP ? 4 * TC * RLD : TC * LD];
    __shared__ int s_ci[4][TC];     // column of the child in quadrant q (-1: none)
    __shared__ int s_pc[TC];        // column of the parent

    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int i16 = lane & 15, q = lane >> 4;
    const int ncols = npar * nrhs;
    const int col0 = blockIdx.x * TC;

    if (tid < 4 * TC) {
        const int sl = tid / TC, c = tid - sl * TC;
        const int gc = col0 + c;
        int ci = -1, pc = -1;
        if (gc < ncols) {
            const int pl = gc / nrhs, r = gc - pl * nrhs;
            const int kid = kids[4 * pl + sl];
            if (kid >= 0) ci = kid * nrhs + r;
            pc = par[pl] * nrhs + r;
        }
        s_ci[sl][c] = ci;
        if (sl == 0) s_pc[c] = pc;
    }

    // This workgroup's row blocks rb0 + [0, RBS): their whole table slice is
    // loaded into registers up front (it does not depend on the columns), so
    // the matrix-core loop never waits on memory for it.
    const int rb0 = blockIdx.y * RBS;
    const int nrb = min((kout + 15) >> 4, rb0 + RBS) - rb0;
    const int nchk = (kin + 15) >> 4;
    int lo[RBS], hi[RBS];
#pragma unroll
    for (int r = 0; r < RBS; ++r) {
        lo[r] = r < nrb ? cuts.lo[rb0 + r] : 0;
        hi[r] = r < nrb ? min(cuts.hi[rb0 + r], nchk) : 0;
    }
    const T *Aw = Apk + (size_t(w) * NRB + rb0) * NRB * 256 + lane * 4;
    Q a[RBS][NRB];
#pragma unroll
    for (int r = 0; r < RBS; ++r)
#pragma unroll
        for (int ch = 0; ch < NRB; ++ch)
            if (ch >= lo[r] && ch < hi[r]) a[r][ch] = *reinterpret_cast<const Q *>(Aw + (r * NRB + ch) * 256);
    __syncthreads();

    if constexpr (!UP) {
        // stage the parents: row = column, k fastest
        constexpr int TPR = 256 / TC;                       // threads per staged row
        constexpr int FPT = KPC / TPR;                      // values per thread
        if constexpr (sizeof(T) == 4 && 256 % TC == 0 && FPT % 4 == 0) {
            // one row per TPR threads, FPT/4 four-value loads each (a missing
            // parent reads column 0, coefficients past kin read coefficient 0;
            // both are zeroed): no branch around the loads
            const int row = tid / TPR, k0 = (tid % TPR) * FPT;
            const int col = s_pc[row];
            const T *base = in + size_t(col >= 0 ? col : 0) * ldin;
            Q v[FPT / 4];
#pragma unroll
            for (int j = 0; j < FPT / 4; ++j) {
                const int k = k0 + 4 * j;
                // k + 3 < ldin when k < kin: the stride is a multiple of 4 and covers kin
                v[j] = *reinterpret_cast<const Q *>(base + (k < kin ? k : 0));
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    if (col < 0 || k + e >= kin) v[j].v[e] = T(0);
            }
#pragma unroll
            for (int j = 0; j < FPT / 4; ++j)
#pragma unroll
                for (int e = 0; e < 4; ++e) Bs[row * LD + k0 + 4 * j + e] = v[j].v[e];
        } else
#pragma unroll
        for (int j0 = 0; j0 < NBT; j0 += BATCH) {
            T v[BATCH];
#pragma unroll
            for (int j = 0; j < BATCH; ++j)
                if (j0 + j < NBT) {
                    const int e = tid + 256 * (j0 + j);
                    const int row = e / KPC, k = e - row * KPC;
                    const int col = s_pc[row];
                    v[j] = (col >= 0 && k < kin) ? in[size_t(col) * ldin + k] : T(0);
                }
#pragma unroll
            for (int j = 0; j < BATCH; ++j)
                if (j0 + j < NBT) {
                    const int e = tid + 256 * (j0 + j);
                    const int row = e / KPC, k = e - row * KPC;
                    Bs[row * LD + k] = v[j];
                }
        }
    }

    // wave-uniform: does quadrant w have a child in this tile?
    const bool on = __ballot(lane < TC && s_ci[w][lane] >= 0) != 0;
    acc_t acc[RBS][NCB];
#pragma unroll
    for (int rb = 0; rb < RBS; ++rb)
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[rb][cb][v] = T(0);
    if (!UP && on) {            // L2L adds to what the translations left in L
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) {
            const int ci = s_ci[w][cb * 16 + i16];
            if (ci < 0) continue;
#pragma unroll
            for (int rb = 0; rb < RBS; ++rb)
                if (rb < nrb)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int row = (rb0 + rb) * 16 + Mfma<T>::row(q, v);
                        if (row < kout) acc[rb][cb][v] = out[size_t(ci) * ldout + row];
                    }
        }
    }

    if constexpr (UP) {
        if (on) {
            // the children of this quadrant, every chunk requested at once
            // (a missing child reads column 0, coefficients past kin read
            // coefficient 0; both are zeroed)
            Q b[NRB][NCB];
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) {
                const int ci = s_ci[w][cb * 16 + i16];
                const T *src = in + size_t(ci >= 0 ? ci : 0) * ldin;
#pragma unroll
                for (int ch = 0; ch < NRB; ++ch) {
                    const int k0 = 16 * ch + 4 * q;
                    // k0 + 3 < ldin when k0 < kin: the stride is a multiple of 4 and covers kin
                    b[ch][cb] = *reinterpret_cast<const Q *>(src + (k0 < kin ? k0 : 0));
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        if (ci < 0 || k0 + e >= kin) b[ch][cb].v[e] = T(0);
                }
            }
#pragma unroll
            for (int ch = 0; ch < NRB; ++ch)
#pragma unroll
                for (int r = 0; r < RBS; ++r)
                    if (ch >= lo[r] && ch < hi[r])
#pragma unroll
                        for (int j = 0; j < 4; ++j)
#pragma unroll
                            for (int cb = 0; cb < NCB; ++cb)
                                acc[r][cb] = Mfma<T>::mac(a[r][ch].v[j], b[ch][cb].v[j], acc[r][cb]);
        }
        // sum the four quadrants' partial results in LDS (fixed order)
        T *red = Bs;
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
            for (int rb = 0; rb < RBS; ++rb)
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    red[(w * TC + cb * 16 + i16) * RLD + rb * 16 + Mfma<T>::row(q, v)] = acc[rb][cb][v];
        __syncthreads();
        const int row0 = rb0 * 16, nrow = min(kout - row0, nrb * 16);
        constexpr int NR = RBS * 16;                         // rows of a tile: the index math is by a constant
        for (int e = tid; e < TC * NR; e += 256) {
            const int c = e / NR, k = e - c * NR;
            const int pc = s_pc[c];
            if (pc < 0 || k >= nrow) continue;
            out[size_t(pc) * ldout + row0 + k] = ((red[c * RLD + k] + red[(TC + c) * RLD + k]) +
                                                  red[(2 * TC + c) * RLD + k]) + red[(3 * TC + c) * RLD + k];
        }
    } else {
        __syncthreads();
        if (on) {
            const T *Bw = Bs + i16 * LD + 4 * q;
#pragma unroll
            for (int ch = 0; ch < NRB; ++ch) {
                bool use = false;
#pragma unroll
                for (int r = 0; r < RBS; ++r) use |= ch >= lo[r] && ch < hi[r];
                if (!use) continue;
                T b[NCB][4];
#pragma unroll
                for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
                    for (int j = 0; j < 4; ++j) b[cb][j] = Bw[cb * 16 * LD + ch * 16 + j];
#pragma unroll
                for (int r = 0; r < RBS; ++r)
                    if (ch >= lo[r] && ch < hi[r])
#pragma unroll
                        for (int j = 0; j < 4; ++j)
#pragma unroll
                            for (int cb = 0; cb < NCB; ++cb)
                                acc[r][cb] = Mfma<T>::mac(a[r][ch].v[j], b[cb][j], acc[r][cb]);
            }
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) {
                const int ci = s_ci[w][cb * 16 + i16];
                if (ci < 0) continue;
#pragma unroll
                for (int rb = 0; rb < RBS; ++rb)
                    if (rb < nrb)
#pragma unroll
                        for (int v = 0; v < 4; ++v) {
                            const int row = (rb0 + rb) * 16 + Mfma<T>::row(q, v);
                            if (row < kout) out[size_t(ci) * ldout + row] = acc[rb][cb][v];
                        }
            }
        }
    }
}

}  // namespace

void pack_shift_tables(const std::vector<double> &tabs, int KP, std::vector<double> &packed, ShiftCuts &cuts)
{
    const int nrb = KP / 16;
    const size_t PP = size_t(KP) * KP;
    const size_t ntab = tabs.size() / PP;
    packed.assign(tabs.size(), 0.0);
    for (int rb = 0; rb < SHIFT_MAXRB; ++rb) { cuts.lo[rb] = 0; cuts.hi[rb] = 0; }
    for (int rb = 0; rb < nrb; ++rb) {
        int lo = nrb, hi = 0;
        for (size_t tb = 0; tb < ntab; ++tb)
            for (int ch = 0; ch < nrb; ++ch)
                for (int l = 0; l < 64; ++l)
                    for (int j = 0; j < 4; ++j) {
                        const double x = tabs[tb * PP + size_t(rb * 16 + l % 16) * KP + ch * 16 + 4 * (l / 16) + j];
                        packed[tb * PP + ((size_t(rb) * nrb + ch) * 64 + l) * 4 + j] = x;
                        if (x != 0.0) { lo = std::min(lo, ch); hi = std::max(hi, ch + 1); }
                    }
        if (lo < hi) { cuts.lo[rb] = lo; cuts.hi[rb] = hi; }
    }
}

template <typename T>
void launch_shift(hipStream_t s, bool up, int cols, int npar, int nrhs, const int32_t *par,
                  const int32_t *kids, const T *Apk, int KP, int kin, int kout, const ShiftCuts &cuts,
                  const T *in, int ldin, T *out, int ldout)
{
    const int ncols = npar * nrhs;
    const int nrb = (kout + 15) / 16;
    if (ncols <= 0 || nrb <= 0) return;
    // 32-column tiles halve the table traffic but need enough columns to fill the chip
    const bool wide = sizeof(T) == 4 && (cols == 32 || (cols == 0 && ncols >= 16 * 1024));
    // row blocks per workgroup: their table slice is held in registers
    constexpr int RBS = sizeof(T) == 4 ? 2 : 1;
    const unsigned gy = unsigned((nrb + RBS - 1) / RBS);
#define IMQ_SHIFT(NRB, NCB)                                                                                  \
    do {                                                                                                     \
        const dim3 grid(unsigned((ncols + 16 * NCB - 1) / (16 * NCB)), gy);                                  \
        if (up)                                                                                              \
            hipLaunchKernelGGL((k_shift<T, NRB, NCB, RBS, true>), grid, dim3(256), 0, s, par, kids, npar,    \
                               nrhs, Apk, kin, kout, cuts, in, ldin, out, ldout);                            \
        else                                                                                                 \
            hipLaunchKernelGGL((k_shift<T, NRB, NCB, RBS, false>), grid, dim3(256), 0, s, par, kids, npar,   \
                               nrhs, Apk, kin, kout, cuts, in, ldin, out, ldout);                            \
    } while (0)
#define IMQ_SHIFT_NRB(NRB)                                       \
    case NRB:                                                    \
        if constexpr (sizeof(T) == 4) {                          \
            if (wide) IMQ_SHIFT(NRB, 2); else IMQ_SHIFT(NRB, 1); \
        } else {                                                 \
            IMQ_SHIFT(NRB, 1);                                   \
        }                                                        \
        break;
    switch (KP / 16) {
        IMQ_SHIFT_NRB(1) IMQ_SHIFT_NRB(2) IMQ_SHIFT_NRB(3) IMQ_SHIFT_NRB(4) IMQ_SHIFT_NRB(5)
        IMQ_SHIFT_NRB(6) IMQ_SHIFT_NRB(7) IMQ_SHIFT_NRB(8) IMQ_SHIFT_NRB(9) IMQ_SHIFT_NRB(10)
        default: break;
    }
#undef IMQ_SHIFT_NRB
#undef IMQ_SHIFT
    (void)wide;
}

template void launch_shift<float>(hipStream_t, bool, int, int, int, const int32_t *, const int32_t *,
                                  const float *, int, int, int, const ShiftCuts &, const float *, int, float *,
                                  int);
template void launch_shift<double>(hipStream_t, bool, int, int, int, const int32_t *, const int32_t *,
                                   const double *, int, int, int, const ShiftCuts &, const double *, int,
                                   double *, int);

}  // namespace imq
