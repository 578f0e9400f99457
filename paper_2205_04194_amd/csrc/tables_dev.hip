// Expansion-to-local (M2L) translation tables generated on the device.
//
// The table of (set, level, class) is the translation operator of
// harmonics.cpp (make_m2l_table): with I_n^m the irregular solid harmonics
// of the displacement t = (dx, dy, c_set / s_l) between the source and the
// target centres in units of the box edge s_l (the lifted planes put the
// target c above the source, Sec. 2.2), the local coefficient (j, k)
// receives sum_(n,m) (-1)^(j+k) I_(n+j)^(m-k)(t) M_n^m, written as a real
// matrix on the stored n+m-even coefficients.  One workgroup per table:
// the harmonics up to degree 2p by the same recurrences (one thread per
// order m after the diagonal), then one thread per (output, input)
// coefficient pair writes its 2 x 2 real block into the layouts the
// translation kernels read: FP64 and FP32, row-major zero-padded to KP x KP
// (staged GEMM) and in the lane order of the register-streaming kernel, and
// the FP32 lane order once more as three BF16 parts per entry.
// A forest of many sets has one table set per set (its own c): generating
// them here takes milliseconds where the host took seconds, and nothing is
// uploaded.  The arithmetic repeats the host's operations in its order
// (compiled without contraction), so the tables agree with the host's to
// the last bits.
#include "device.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <vector>

namespace imq {

namespace {

struct Cx {
    double re, im;
};
__device__ __forceinline__ Cx cmul(Cx a, Cx b) { return Cx{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ __forceinline__ Cx cscale(double s, Cx a) { return Cx{s * a.re, s * a.im}; }

__device__ __forceinline__ int tri_d(int n, int m) { return n * (n + 1) / 2 + m; }
__device__ __forceinline__ int ire_d(int n, int m) { return n * (n + 1) / 2 + (m > 0 ? m - 1 : 0); }

constexpr int NH = (2 * PMAX + 1) * (2 * PMAX + 2) / 2;   // harmonics up to degree 2 PMAX

// I_n^m for |m| <= n <= N from the m >= 0 table
__device__ __forceinline__ Cx harm(const Cx *H, int N, int n, int m)
{
    if (n < 0 || n > N || m > n || -m > n) return Cx{0.0, 0.0};
    if (m >= 0) return H[tri_d(n, m)];
    const Cx v = H[tri_d(n, -m)];
    return (m & 1) ? Cx{-v.re, v.im} : Cx{v.re, -v.im};      // (-1)^m conj
}

// Real coefficient index -> (n, m, sine part): n + 1 entries per degree n,
// m = 0, 2, 4, ... (n even) or 1, 3, ... (n odd), cosine then sine part for
// m > 0 (the stored layout, ire).
__device__ __forceinline__ void decode(int r, int &n, int &m, bool &im)
{
    n = 0;
    while ((n + 1) * (n + 2) / 2 <= r) ++n;
    const int o = r - n * (n + 1) / 2;
    m = (n & 1) ? 2 * (o / 2) + 1 : 2 * ((o + 1) / 2);
    im = m > 0 && o == ire_d(n, m) - n * (n + 1) / 2 + 1;
}

// cnm: P_n^m(0) / (n+m)!, (n, m) at tri_d(n, m), n <= p (host-computed)
__global__ __launch_bounds__(256) void k_m2l_tables(int p, int nlev, const double *__restrict__ cn,
                                                    const double *__restrict__ cnm, int KP,
                                                    double *__restrict__ t64, double *__restrict__ pk64,
                                                    float *__restrict__ t32, float *__restrict__ pk32,
                                                    uint16_t *__restrict__ bf3)
{
    __shared__ Cx H[NH];
    __shared__ Cx diag[2 * PMAX + 1];
    const int id = blockIdx.x;
    const int cls = id % NCLASS, l = (id / NCLASS) % nlev, s = id / NCLASS / nlev;
    const int dx = cls / 7 - 3, dy = cls % 7 - 3;
    if (l < 2 || (abs(dx) <= 1 && abs(dy) <= 1)) return;    // no table (zeros)
    const int N = 2 * p;
    const double scale = ldexp(1.0, l);
    const double x = double(dx), y = double(dy), z = cn[s] * scale;
    const double r2 = x * x + y * y + z * z;
    const double inv_r2 = 1.0 / r2;
    const Cx xy{x, y};
    if (threadIdx.x == 0) {
        Cx imm{1.0 / sqrt(r2), 0.0};
        for (int m = 0; m <= N; ++m) {
            if (m > 0) imm = cmul(cscale(inv_r2, cscale(-(2.0 * m - 1), xy)), imm);
            diag[m] = imm;
        }
    }
    __syncthreads();
    for (int m = threadIdx.x; m <= N; m += blockDim.x) {
        const Cx imm = diag[m];
        H[tri_d(m, m)] = imm;
        if (m + 1 <= N) H[tri_d(m + 1, m)] = cscale((2.0 * m + 1) * z * inv_r2, imm);
        for (int n = m + 2; n <= N; ++n) {
            const Cx a = cscale((2.0 * n - 1) * z, H[tri_d(n - 1, m)]);
            const Cx b = cscale(double((n + m - 1) * (n - m - 1)), H[tri_d(n - 2, m)]);
            H[tri_d(n, m)] = cscale(inv_r2, Cx{a.re - b.re, a.im - b.im});
        }
    }
    __syncthreads();
    const int PP = KP * KP, nrb = KP / 16;
    double *T64 = t64 + size_t(id) * PP;
    double *P64 = pk64 + size_t(id) * PP;
    float *T32 = t32 + size_t(id) * PP;
    float *P32 = pk32 + size_t(id) * PP;
    uint16_t *B3 = bf3 + size_t(id) * PP * 3;
    auto store = [&](int r, int c, double v) {
        const size_t rec = (size_t(r / 16) * nrb + c / 16) * 64 + ((c % 16) / 4) * 16 + r % 16;
        const size_t pkx = rec * 4 + c % 4;
        T64[size_t(r) * KP + c] = v;
        P64[pkx] = v;
        const float f = float(v);
        T32[size_t(r) * KP + c] = f;
        P32[pkx] = f;
        // the FP32 value as three BF16 parts (each difference exact in FP32)
        const __bf16 hi = __bf16(f);
        const float r1 = f - float(hi);
        const __bf16 mid = __bf16(r1);
        const __bf16 lo = __bf16(r1 - float(mid));
        B3[rec * 12 + c % 4] = __builtin_bit_cast(uint16_t, hi);
        B3[rec * 12 + 4 + c % 4] = __builtin_bit_cast(uint16_t, mid);
        B3[rec * 12 + 8 + c % 4] = __builtin_bit_cast(uint16_t, lo);
    };
    const int K = (p + 1) * (p + 2) / 2;
    // one thread per real entry (r, c): output coefficient (j, k) (cosine or
    // sine part), input coefficient (n, m)
    for (int item = threadIdx.x; item < K * K; item += blockDim.x) {
        const int r = item / K, c = item % K;
        int j, k, n, m;
        bool rim, cim;
        decode(r, j, k, rim);
        decode(c, n, m, cim);
        const double so = (k == 0 ? 1.0 : 2.0) * cnm[tri_d(j, k)] * scale;
        const double si = cnm[tri_d(n, m)] * (((j + k) & 1) ? -1.0 : 1.0);
        const Cx A1 = cscale(si, harm(H, N, n + j, m - k));
        const Cx A2 = m > 0 ? cscale(((m & 1) ? -1.0 : 1.0) * si, harm(H, N, n + j, -m - k)) : Cx{0.0, 0.0};
        const Cx sum{A1.re + A2.re, A1.im + A2.im}, dif{A1.re - A2.re, A1.im - A2.im};
        double v;
        if (!rim && !cim) v = so * sum.re;
        else if (!rim && cim) v = -so * dif.im;
        else if (rim && !cim) v = so * sum.im;
        else v = so * dif.re;
        store(r, c, v);
    }
}

}  // namespace

// Every M2L table of the tree, in the four layouts, on the device: the
// buffers of both precisions (zero-filled first; the padding and the
// levels and classes without translations stay zero).
imq_status make_m2l_tables_device(imq_tree_s *t, int KP)
{
    const HostTree &h = t->h;
    const int p = h.p;
    const size_t ntab = size_t(h.nsets) * h.nlev * NCLASS, PP = size_t(KP) * KP;
    std::vector<double> cnm(size_t(p + 1) * (p + 2) / 2, 0.0);
    for (int n = 0; n <= p; ++n)
        for (int m = 0; m <= n; ++m) cnm[size_t(n) * (n + 1) / 2 + m] = legendre_coef(n, m);
    DevBuf d_cnm, d_cn;
    struct Free {
        DevBuf &a, &b;
        ~Free() { dev_free(a); dev_free(b); }
    } fr{d_cnm, d_cn};
    IMQ_HIP(dev_alloc(d_cnm, sizeof(double) * cnm.size()));
    IMQ_HIP(hipMemcpy(d_cnm.p, cnm.data(), sizeof(double) * cnm.size(), hipMemcpyHostToDevice));
    IMQ_HIP(dev_alloc(d_cn, sizeof(double) * h.cn.size()));
    IMQ_HIP(hipMemcpy(d_cn.p, h.cn.data(), sizeof(double) * h.cn.size(), hipMemcpyHostToDevice));
    IMQ_HIP(dev_alloc(t->f64.m2l, sizeof(double) * ntab * PP));
    IMQ_HIP(dev_alloc(t->f64.m2l_pk, sizeof(double) * ntab * PP));
    IMQ_HIP(dev_alloc(t->f32.m2l, sizeof(float) * ntab * PP));
    IMQ_HIP(dev_alloc(t->f32.m2l_pk, sizeof(float) * ntab * PP));
    IMQ_HIP(hipMemset(t->f64.m2l.p, 0, sizeof(double) * ntab * PP));
    IMQ_HIP(hipMemset(t->f64.m2l_pk.p, 0, sizeof(double) * ntab * PP));
    IMQ_HIP(hipMemset(t->f32.m2l.p, 0, sizeof(float) * ntab * PP));
    IMQ_HIP(hipMemset(t->f32.m2l_pk.p, 0, sizeof(float) * ntab * PP));
    IMQ_HIP(dev_alloc(t->f32.m2l_bf3, sizeof(uint16_t) * 3 * ntab * PP));
    IMQ_HIP(hipMemset(t->f32.m2l_bf3.p, 0, sizeof(uint16_t) * 3 * ntab * PP));
    if (ntab > 0)
        hipLaunchKernelGGL(k_m2l_tables, dim3(unsigned(ntab)), dim3(256), 0, 0, p, h.nlev, d_cn.as<double>(),
                           d_cnm.as<double>(), KP, t->f64.m2l.as<double>(), t->f64.m2l_pk.as<double>(),
                           t->f32.m2l.as<float>(), t->f32.m2l_pk.as<float>(), t->f32.m2l_bf3.as<uint16_t>());
    IMQ_HIP(hipGetLastError());
    IMQ_HIP(hipDeviceSynchronize());
    return IMQ_OK;
}

}  // namespace imq
