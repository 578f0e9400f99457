// Expansion-to-local translations (V lists) with every operand streamed
// through registers.
//
// L[target] = sum over the (up to 27) occupied V-list classes s of
// T_{level, set, class(s)} M[source_s]  (Sec. 2.2: the lifted translation from
// the source plane z = -c/2 to the target plane z = +c/2).
//
// The batched GEMM of fmm.hip stages one class per step through LDS, so a
// workgroup pays one memory round trip per class and coefficient chunk.
// Here the NW waves of a workgroup (4 or 8) split the classes (wave w takes
// classes w, w + NW, ...); each wave loads its table slices and source
// expansions straight from memory in the matrix-core lane order (16 bytes per
// lane and load), one class ahead of the matrix cores, and the partial results
// of the waves are summed in LDS in a fixed order.
#include "device.h"
#include "mfma.h"

#include <hip/hip_runtime.h>

#include <type_traits>

namespace imq {

namespace {


// Task = GemmTask of the translation batches (<= 64 targets sharing level,
// set and child position).  blockIdx.y picks TC = 16*NCB of its columns
// (target, rhs).  Packed table layout (ntab x nrbT x nrbT chunks of 64 lanes x
// 4): element j of lane l of (row block rb, input chunk ci) is
// T[16 rb + l%16][16 ci + 4 (l/16) + j], so a lane's four values of a chunk
// match four consecutive source coefficients.
//
// Wave w walks its classes w, w+NW, ...
// For class k the source expansions of class k+1 and, row block by row
// block as soon as each is consumed, the table of class k+1 are requested
// while the matrix cores work on class k; the source indices run one class
// further ahead.  blockIdx.z picks the RBW output row blocks (of NRB) that the
// workgroup computes: small levels spread over NRB / RBW times more
// workgroups, each reading only its rows of every table.  Register use:
// RBW*NRB + 2*NCB*NRB four-value quads.
// BF (FP32 products): the table is read as three BF16 parts per entry (hi,
// mid, lo: hi = bf16(t), mid = bf16(t - hi), lo = bf16(t - hi - mid), 24
// significant bits in all), the source quads are split the same way in
// registers, and each four-coefficient step is six BF16 matrix-core
// products (v_mfma_f32_16x16x16_bf16: the quad of a lane is exactly its A or
// B operand) accumulated in FP32: hi.hi + hi.mid + mid.hi + hi.lo + lo.hi +
// mid.mid, the dropped products being below 2^-24 of the result.  Split
// table records: per (table, row block, input chunk, lane) 12 BF16 values,
// hi[4] mid[4] lo[4].
typedef __bf16 bf4 __attribute__((ext_vector_type(4)));
typedef float fv4 __attribute__((ext_vector_type(4)));
struct BfQ {
    bf4 h, m, l;
};

__device__ __forceinline__ BfQ split3(const Quad<float> &x)
{
    const fv4 v{x.v[0], x.v[1], x.v[2], x.v[3]};
    BfQ o;
    o.h = __builtin_convertvector(v, bf4);
    const fv4 r1 = v - __builtin_convertvector(o.h, fv4);
    o.m = __builtin_convertvector(r1, bf4);
    const fv4 r2 = r1 - __builtin_convertvector(o.m, fv4);
    o.l = __builtin_convertvector(r2, bf4);
    return o;
}

__device__ __forceinline__ f32x4 mac_bf3(const BfQ &a, const BfQ &b, f32x4 c)
{
    c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a.m, b.m, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a.l, b.h, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a.h, b.l, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a.m, b.h, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a.h, b.m, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a.h, b.h, c, 0, 0, 0);
    return c;
}

template <typename T, int NRB, int NCB, int NW, int RBW, bool BF = false>
__global__ __launch_bounds__(64 * NW) void k_m2l_stream(const GemmTask *__restrict__ tasks, int task0,
                                                    const int32_t *__restrict__ tbox,
                                                    const int32_t *__restrict__ tab,
                                                    const int32_t *__restrict__ src, const T *__restrict__ Apk,
                                                    const uint16_t *__restrict__ Abf,
                                                    int nrbT, int nrhs, int KS, const T *__restrict__ in,
                                                    T *__restrict__ out, int add, int ntask, int kout_ovr)
{
    tree_pass_priority();
    static_assert(NRB % RBW == 0, "whole row-block groups");
    static_assert(!BF || sizeof(T) == 4, "BF16 parts of FP32 operands");
    constexpr int TC = 16 * NCB;
    constexpr int LDR = RBW * 16 + 1;
    using acc_t = typename Mfma<T>::acc_t;
    using Q = Quad<T>;
    constexpr int SPW = (GEMM_MAXSLOT + NW - 1) / NW;  // classes per wave
    __shared__ T red[NW * TC * LDR];
    __shared__ int s_out[TC];

    // Workgroups are dealt to the eight XCDs in turn (workgroup b to XCD b mod
    // 8; gridDim.x is a multiple of 8, so the row-block and column splits of a
    // task share its XCD).  XCD x takes the x-th contiguous range of tasks:
    // neighbouring tasks (one set and level, other child positions) read the
    // same translation tables, which then stay in that XCD's L2.  With many
    // sets, each with its own tables, this cut the M2L stage of a 256-set
    // forest from 0.92 to 0.78 ms.
    const int per_xcd = gridDim.x / 8;
    const int ti = (blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
    if (ti >= ntask) return;                         // padding of the grid
    const GemmTask tk = tasks[task0 + ti];
    const int ncols = tk.nbox * nrhs;
    const int col0 = blockIdx.y * TC;
    if (col0 >= ncols) return;                       // uniform over the workgroup
    // the wave index as a scalar: the class tables' indices are then scalar loads
    const int tid = threadIdx.x, lane = tid & 63, w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int i16 = lane & 15, q = lane >> 4;
    const int kin = tk.kin, kout = kout_ovr > 0 ? kout_ovr : tk.kout;   // override: other tables' output rows
    const int rb0 = blockIdx.z * RBW;                // first output row block of the workgroup
    if (rb0 * 16 >= kout) return;                    // uniform over the workgroup
    const int nslot = tk.nslot;
    if (tid < TC) {
        const int gc = col0 + tid;
        int o = -1;
        if (gc < ncols) {
            const int bl = gc / nrhs, r = gc - bl * nrhs;
            o = tbox[tk.box0 + bl] * nrhs + r;
        }
        s_out[tid] = o;
    }
    int bl[NCB], rr[NCB];
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) {
        const int gc = col0 + cb * 16 + i16;
        bl[cb] = gc < ncols ? gc / nrhs : -1;
        rr[cb] = gc < ncols ? gc - bl[cb] * nrhs : 0;
    }
    // source box of class k of this wave for each column (-1: none); the load
    // is unconditional (entry 0 of the task where there is no source) so that
    // no branch separates the loads of the classes
    auto source = [&](int k, int *sb) {
        const int sl = w + NW * k;
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) {
            const bool ok = k < SPW && sl < nslot && bl[cb] >= 0;
            const int v = src[tk.src0 + (ok ? bl[cb] * nslot + sl : 0)];
            sb[cb] = ok ? v : -1;
        }
    };
    // Every lane loads every quad (a missing source or a coefficient past kin
    // reads box 0 or coefficient 0 and is zeroed after the load): no branch
    // around the loads, which matters where the vector units are shared.
    auto load_b = [&](const int *sb, Q (*dst)[NRB]) {
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) {
            const bool okc = sb[cb] >= 0;
            const T *base = in + (size_t(okc ? sb[cb] : 0) * nrhs + rr[cb]) * KS;
#pragma unroll
            for (int ci = 0; ci < NRB; ++ci) {
                const int k0 = ci * 16 + 4 * q;
                // k0 + 3 < KS when k0 < kin: KS is a multiple of 4 and kin <= KS
                Q x = *reinterpret_cast<const Q *>(base + (k0 < kin ? k0 : 0));
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    if (!okc || k0 + j >= kin) x.v[j] = T(0);
                dst[cb][ci] = x;
            }
        }
    };
    // class k of this wave exists (wave-uniform)
    auto has = [&](int k) { return k < SPW && w + NW * k < nslot; };
    // table index of class k (the task's first class where the wave has no
    // class k: loaded all the same, and not used)
    auto tindex = [&](int k) { return tab[tk.tab0 + (has(k) ? w + NW * k : 0)]; };
    auto table = [&](int k) -> const T * {
        return Apk + (size_t(tindex(k)) * nrbT + rb0) * nrbT * 256 + lane * 4;
    };
    auto table_bf = [&](int k) -> const uint16_t * {
        return Abf + ((size_t(tindex(k)) * nrbT + rb0) * nrbT * 64 + lane) * 12;
    };
    using AQ = typename std::conditional<BF, BfQ, Q>::type;
    // the table operand of row block rb, input chunk ci
    auto load_a = [&](const void *A, int rb, int ci) -> AQ {
        if constexpr (BF) {
            const uint2 *r = reinterpret_cast<const uint2 *>(static_cast<const uint16_t *>(A) +
                                                             size_t(rb * nrbT + ci) * 64 * 12);
            BfQ o;
            o.h = __builtin_bit_cast(bf4, r[0]);
            o.m = __builtin_bit_cast(bf4, r[1]);
            o.l = __builtin_bit_cast(bf4, r[2]);
            return o;
        } else {
            return *reinterpret_cast<const Q *>(static_cast<const T *>(A) + (rb * nrbT + ci) * 256);
        }
    };
    auto table_any = [&](int k) -> const void * {
        if constexpr (BF) return table_bf(k);
        else return table(k);
    };

    acc_t acc[RBW][NCB];
#pragma unroll
    for (int rb = 0; rb < RBW; ++rb)
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[rb][cb][v] = T(0);

    // Loads run PD classes ahead of the matrix cores (as many as about 128
    // registers of operands allow, all of the wave's classes where they fit):
    // the source indices of every class first, then the table slices and
    // source expansions of classes 0 .. PD-1, and the slot of class k is
    // refilled with class k + PD as soon as class k is consumed.  A wave
    // thus waits about two memory latencies in all instead of one per class.
    constexpr int QV = int(sizeof(T));                 // registers per quad: 4 (FP32), 8 (FP64)
    constexpr int AV = BF ? 6 : QV;
    constexpr int STEPV = RBW * NRB * AV + NCB * NRB * QV;
    constexpr int PD = STEPV * SPW <= 128 ? SPW : (128 / STEPV < 1 ? 1 : 128 / STEPV);
    int sidx[SPW][NCB];
#pragma unroll
    for (int k = 0; k < SPW; ++k) source(k, sidx[k]);
    // the class tables of the wave: scalar loads, all issued before the first wait
    const void *tptr[SPW];
#pragma unroll
    for (int k = 0; k < SPW; ++k) tptr[k] = table_any(k);
    AQ a[PD][RBW][NRB];
    Q b[PD][NCB][NRB];
    auto issue = [&](int k, int d) {
        const void *A = tptr[k];
#pragma unroll
        for (int rb = 0; rb < RBW; ++rb)
#pragma unroll
            for (int ci = 0; ci < NRB; ++ci) a[d][rb][ci] = load_a(A, rb, ci);
        load_b(sidx[k], b[d]);
    };
#pragma unroll
    for (int d = 0; d < PD; ++d) issue(d, d);
#pragma unroll
    for (int k = 0; k < SPW; ++k) {
        const int d = k % PD;
        if (has(k)) {                                  // wave-uniform
            if constexpr (BF) {
                BfQ bs[NCB][NRB];
#pragma unroll
                for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
                    for (int ci = 0; ci < NRB; ++ci) bs[cb][ci] = split3(b[d][cb][ci]);
#pragma unroll
                for (int rb = 0; rb < RBW; ++rb)
#pragma unroll
                    for (int ci = 0; ci < NRB; ++ci)
#pragma unroll
                        for (int cb = 0; cb < NCB; ++cb)
                            acc[rb][cb] = mac_bf3(a[d][rb][ci], bs[cb][ci], acc[rb][cb]);
            } else {
#pragma unroll
                for (int rb = 0; rb < RBW; ++rb)
#pragma unroll
                    for (int ci = 0; ci < NRB; ++ci)
#pragma unroll
                        for (int j = 0; j < 4; ++j)
#pragma unroll
                            for (int cb = 0; cb < NCB; ++cb)
                                acc[rb][cb] = Mfma<T>::mac(a[d][rb][ci].v[j], b[d][cb][ci].v[j], acc[rb][cb]);
            }
        }
        if (k + PD < SPW) issue(k + PD, d);
    }

#pragma unroll
    for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
        for (int rb = 0; rb < RBW; ++rb)
#pragma unroll
            for (int v = 0; v < 4; ++v)
                red[(w * TC + cb * 16 + i16) * LDR + rb * 16 + Mfma<T>::row(q, v)] = acc[rb][cb][v];
    __syncthreads();
    const int nk = min(kout - rb0 * 16, RBW * 16);   // output rows of the workgroup
    constexpr int NKM = RBW * 16;                     // at most: the index math is by a constant
    for (int e = tid; e < TC * NKM; e += 64 * NW) {
        const int c = e / NKM, kk = e - c * NKM;
        const int o = s_out[c];
        if (o < 0 || kk >= nk) continue;
        T sum = red[c * LDR + kk];
#pragma unroll
        for (int ww = 1; ww < NW; ++ww) sum += red[(ww * TC + c) * LDR + kk];
        T &dst = out[size_t(o) * KS + rb0 * 16 + kk];
        dst = add ? dst + sum : sum;
    }
}

}  // namespace

template <typename T>
bool launch_m2l_stream(hipStream_t s, int acc, int kmax, int ntask, int task0, int nrhs, const GemmTask *tasks,
                       const int32_t *tbox, const int32_t *tab, const int32_t *src, const T *Apk,
                       const uint16_t *Abf, int KP, int KS, const T *in, T *out, int kout_ovr)
{
    const int nrb = (kmax + 15) / 16;
    if (ntask <= 0) return true;
    // 4 waves per workgroup everywhere: 8 (a class chain half as long) was
    // measured slower on the mixture workload, in particular beside the near
    // field, whose small workgroups leave few CUs with 8 wave slots free
    // Levels too small to give every CU a few workgroups split the output rows
    // (one row block per workgroup).  16 target columns per workgroup
    // everywhere: at the fine levels (up to 48 coefficients) 32 columns gave
    // half the workgroups and a 7% slower M2L stage.
#define IMQ_M2LS_BF(NRB, NCB, NW, BF)                                                                      \
    do {                                                                                                   \
        const unsigned ny = unsigned((GEMM_TILE * nrhs + 16 * NCB - 1) / (16 * NCB));                      \
        if (NRB > 1 && size_t(ntask) * ny < 512)                                                           \
            hipLaunchKernelGGL((k_m2l_stream<T, NRB, NCB, NW, 1, BF>), dim3((ntask + 7) & ~7, ny, NRB), dim3(64 * NW), 0, \
                               s, tasks, task0, tbox, tab, src, Apk, Abf, KP / 16, nrhs, KS, in, out, acc, ntask, kout_ovr);     \
        else                                                                                               \
            hipLaunchKernelGGL((k_m2l_stream<T, NRB, NCB, NW, NRB, BF>), dim3((ntask + 7) & ~7, ny, 1), dim3(64 * NW), 0,  \
                               s, tasks, task0, tbox, tab, src, Apk, Abf, KP / 16, nrhs, KS, in, out, acc, ntask, kout_ovr);     \
    } while (0)
#define IMQ_M2LS(NRB, NCB, NW)                                                                             \
    do {                                                                                                   \
        if constexpr (sizeof(T) == 4) {                                                                    \
            if (Abf) { IMQ_M2LS_BF(NRB, NCB, NW, true); break; }                                           \
        }                                                                                                  \
        IMQ_M2LS_BF(NRB, NCB, NW, false);                                                                  \
    } while (0)
    // 96 to 160 coefficients (m2l_mode 3): one row block per workgroup, the
    // FP32 and FP64 products on their own matrix cores
#define IMQ_M2LS_ROW(NRB)                                                                                  \
    case NRB:                                                                                              \
        hipLaunchKernelGGL((k_m2l_stream<T, NRB, 1, 4, 1>),                                                \
                           dim3((ntask + 7) & ~7, unsigned((GEMM_TILE * nrhs + 15) / 16), NRB), dim3(256), 0, s, \
                           tasks, task0, tbox, tab, src, Apk, nullptr, KP / 16, nrhs, KS, in, out, acc, ntask, kout_ovr); \
        return true;
    if constexpr (sizeof(T) == 4) {
        switch (nrb) {
        case 1: IMQ_M2LS(1, 1, 4); return true;
        case 2: IMQ_M2LS(2, 1, 4); return true;
        case 3: IMQ_M2LS(3, 1, 4); return true;
        case 4: IMQ_M2LS(4, 1, 4); return true;
        case 5: IMQ_M2LS(5, 1, 4); return true;
        IMQ_M2LS_ROW(6) IMQ_M2LS_ROW(7) IMQ_M2LS_ROW(8) IMQ_M2LS_ROW(9) IMQ_M2LS_ROW(10)
        default: return false;
        }
    } else {
        switch (nrb) {
        case 1: IMQ_M2LS(1, 1, 4); return true;
        case 2: IMQ_M2LS(2, 1, 4); return true;
        case 3: IMQ_M2LS(3, 1, 4); return true;
        case 4: IMQ_M2LS(4, 1, 4); return true;
        case 5:      // one row block per workgroup: a whole-row tile would not fit the registers
            hipLaunchKernelGGL((k_m2l_stream<T, 5, 1, 4, 1>),
                               dim3((ntask + 7) & ~7, unsigned((GEMM_TILE * nrhs + 15) / 16), 5), dim3(256), 0, s, tasks,
                               task0, tbox, tab, src, Apk, nullptr, KP / 16, nrhs, KS, in, out, acc, ntask, kout_ovr);
            return true;
        IMQ_M2LS_ROW(6) IMQ_M2LS_ROW(7) IMQ_M2LS_ROW(8) IMQ_M2LS_ROW(9) IMQ_M2LS_ROW(10)
        default: return false;
        }
    }
#undef IMQ_M2LS_ROW
#undef IMQ_M2LS
#undef IMQ_M2LS_BF
}

template bool launch_m2l_stream<float>(hipStream_t, int, int, int, int, int, const GemmTask *, const int32_t *,
                                       const int32_t *, const int32_t *, const float *, const uint16_t *, int, int,
                                       const float *, float *, int);
template bool launch_m2l_stream<double>(hipStream_t, int, int, int, int, int, const GemmTask *, const int32_t *,
                                        const int32_t *, const int32_t *, const double *, const uint16_t *, int, int,
                                        const double *, double *, int);

}  // namespace imq
