// Adjoint of the fast product b = A(c, X) v for a scalar loss with upstream
// gradient g = dL/db.  From the entries of eq. IMQ_def,
//     phi = (r^2 + c^2)^(-1/2),  grad_x phi = -(x_i - x_j) (r^2+c^2)^(-3/2),
//     d phi / dc = -c (r^2 + c^2)^(-3/2),
// and, with the fields F_w(x) = sum_j w_j grad_x phi(x - x_j) and
// Z_w(x) = sum_j w_j dphi/dc(x - x_j),
//     dL/dv   = A g                          (A is symmetric)
//     dL/dx_k = g_k F_v(x_k) + v_k F_g(x_k)
//     dL/dc   = sum_i g_i Z_v(x_i).
// All of it comes from one expansion pass over the two weight vectors v and
// g: the n+m-even local coefficients give the potential and its in-plane
// gradient, the n+m-odd ones (extra translation tables) the vertical
// derivative, which is d/dc in the lifted picture.  The near field is summed
// directly with the same formulas, each neighbour leaf's points staged
// through LDS 64 at a time.
//
// Adaptive lists.  An X-list leaf's points enter the target box's even local
// coefficients with the forward pass (P2L) and its odd ones here, from the
// n+m-odd irregular harmonics of the points.  A W-list box's multipole is
// evaluated at the leaf's points with its derivatives, from the ladder
// relations of the irregular solid harmonics (normalisation of the table
// generator): with d+ = d/dx + i d/dy,
//     d+ I_n^m = I_{n+1}^{m+1},   d/dz I_n^m = -I_{n+1}^m   (every m),
// so for a real field sum_{n,m} M_n^m I_n^m (all m, M_n^{-m} = (-1)^m conj M_n^m)
//     d+ phi   = sum_{n, m>=0} M_n^m I_{n+1}^{m+1} - sum_{n, m>=1} conj(M_n^m I_{n+1}^{m-1})
//     dphi/dz  = -sum_{n, m>=0} eps_m Re(M_n^m I_{n+1}^m),
// the gradient being (Re d+ phi, Im d+ phi); the harmonics are needed to
// order P+1, both parities.
#include "device.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

namespace imq {

template <typename T> imq_status fmm_upward(imq_tree_s *t, int nrhs, hipStream_t s, bool fork, const UserVec *io);
template <typename T> imq_status fmm_translate(imq_tree_s *t, int nrhs, hipStream_t s, bool overlap);

namespace {

__device__ __forceinline__ int cidx_e(int n, int m) { return n * (n + 1) / 2 + (m > 0 ? m - 1 : 0); }
__device__ __forceinline__ int cidx_o(int j, int k) { return j * (j - 1) / 2 + (k > 0 ? k - 1 : 0); }

template <typename T> __device__ __forceinline__ T rsqrt_a(T x) { return T(1) / sqrt(x); }

// Reciprocal square root of the near-field sums: the hardware estimate (FP32:
// as is; FP64: relative error below 2^-22) refined in FP64 by one step of the
// third-order iteration y (1 + e/2 + 3e^2/8), e = 1 - x y^2, whose truncation
// error, about (5/16)|e|^3, is below 1e-19 here.
__device__ __forceinline__ float rsqrt_near(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double rsqrt_near(double x)
{
    const double y = __builtin_amdgcn_rsq(x);
    const double e = fma(-x * y, y, 1.0);
    return fma(y * e, fma(e, 0.375, 0.5), y);
}

// Irregular solid harmonics I_n^m(v), 0 <= m <= n <= NMAX, both parities:
// I_0^0 = 1/|v|, I_m^m = -(2m-1)(vx + i vy)/|v|^2 I_{m-1}^{m-1} and
// |v|^2 I_n^m = (2n-1) vz I_{n-1}^m - (n+m-1)(n-m-1) I_{n-2}^m; f(n, m, re, im).
template <typename T, typename F>
__device__ __forceinline__ void irregular_all(int NMAX, T vx, T vy, T vz, F &&f)
{
    const T r2 = vx * vx + vy * vy + vz * vz;
    const T inv_r2 = T(1) / r2;
    T mr = rsqrt_a(r2), mi = T(0);
    for (int m = 0; m <= NMAX; ++m) {
        if (m > 0) {
            const T a = -T(2 * m - 1) * inv_r2;
            const T nr = a * (vx * mr - vy * mi);
            mi = a * (vx * mi + vy * mr);
            mr = nr;
        }
        T p2r = 0, p2i = 0, p1r = mr, p1i = mi;
        f(m, m, mr, mi);
        for (int n = m + 1; n <= NMAX; ++n) {
            const T a = T(2 * n - 1) * vz;
            const T b = T((n + m - 1) * (n - m - 1));
            const T cr = (a * p1r - b * p2r) * inv_r2;
            const T ci = (a * p1i - b * p2i) * inv_r2;
            f(n, m, cr, ci);
            p2r = p1r; p2i = p1i; p1r = cr; p1i = ci;
        }
    }
}

// Odd local coefficients of the v weights from the X lists: one workgroup
// per target box b, its X-list leaves in list order,
//     Lo[b][j,k] += (1/s^2) eps_k c_{j-1,k} sum_i v_i conj(I_j^k((y_i - z_b)/s)),
// j+k odd, with the sources c below the target plane (vz = -c/s); wxo holds
// eps_k c_{j-1,k} in the odd layout.  Points go through LDS in chunks of 32.
constexpr int X_CH = 32;
constexpr int KODD_MAX = PMAX * (PMAX + 1) / 2;

template <typename T>
__global__ __launch_bounds__(64) void k_p2l_odd(DTree<T> t, const int32_t *__restrict__ xboxes,
                                                const T *__restrict__ us, const T *__restrict__ wxo, int Ko,
                                                T *__restrict__ Lo)
{
    __shared__ T mono[X_CH][KODD_MAX | 1];
    __shared__ T su[X_CH];
    const int b = xboxes[blockIdx.x];
    const int P = t.P, lane = threadIdx.x;
    const double inv_sd = ldexp(1.0, t.level[b]);
    const T inv_s = T(inv_sd);
    const T vz = T(-t.cn[t.set[b]] * inv_sd);
    T acc[(KODD_MAX + 63) / 64] = {};
    for (int kp = t.x_off[b]; kp < t.x_off[b + 1]; ++kp) {
        const int a = t.x_idx[kp];
        const T ox = T((t.cx[a] - t.cx[b]) * inv_sd), oy = T((t.cy[a] - t.cy[b]) * inv_sd);
        for (int c0 = t.begin[a]; c0 < t.end[a]; c0 += X_CH) {
            const int n = min(X_CH, t.end[a] - c0);
            __syncthreads();                       // the previous chunk is no longer read
            if (lane < n) {
                T *row = mono[lane];
                irregular_all<T>(P, t.xl[c0 + lane] * inv_s + ox, t.yl[c0 + lane] * inv_s + oy, vz,
                                 [&](int j, int k, T re, T im) {
                                     if ((j + k) & 1) {
                                         const int o = cidx_o(j, k);
                                         row[o] = re;
                                         if (k > 0) row[o + 1] = -im;
                                     }
                                 });
                su[lane] = us[c0 + lane];
            }
            __syncthreads();
#pragma unroll
            for (int q = 0; q < (KODD_MAX + 63) / 64; ++q) {
                const int o = lane + 64 * q;
                if (o < Ko) {
                    T s = T(0);
                    for (int i = 0; i < n; ++i) s += mono[i][o] * su[i];
                    acc[q] += s;
                }
            }
        }
    }
#pragma unroll
    for (int q = 0; q < (KODD_MAX + 63) / 64; ++q) {
        const int o = lane + 64 * q;
        if (o < Ko) Lo[size_t(b) * 2 * t.KS + o] += acc[q] * wxo[o] * inv_s * inv_s;
    }
}

template <typename T>
__global__ void k_zero(size_t n, T *__restrict__ p)
{
    const size_t i = blockIdx.x * size_t(blockDim.x) + threadIdx.x;
    if (i < n) p[i] = T(0);
}

template <typename Tin, typename T>
__global__ void k_gather2(int64_t N, const int32_t *__restrict__ perm, const Tin *__restrict__ v,
                          const Tin *__restrict__ g, T *__restrict__ us)
{
    const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (i < N) {
        us[i] = T(v[perm[i]]);
        us[N + i] = T(g[perm[i]]);
    }
}

// Per target (normalised units): out[0] = potential of g, out[1..2] = grad of
// the v field, out[3..4] = grad of the g field, out[5] = d/dc of the v field.
// M (premultiplied by wx = eps_m c_{nm}) feeds the W-list evaluations.
template <typename T>
__global__ __launch_bounds__(64) void k_adjoint_eval(DTree<T> t, const int32_t *__restrict__ leaves,
                                                     const T *__restrict__ L, const T *__restrict__ Lo,
                                                     const T *__restrict__ M, const T *__restrict__ wx,
                                                     const T *__restrict__ us, double *__restrict__ out)
{
    const int b = leaves[blockIdx.x];
    const int P = t.P;
    const double inv_sd = ldexp(1.0, t.level[b]);
    const T inv_s = T(inv_sd);
    const double cnd = t.cn[t.set[b]];
    const T cc = T(cnd), c2 = T(cnd * cnd);
    const T *Lv = L + (size_t(b) * 2 + 0) * t.KS;
    const T *Lg = L + (size_t(b) * 2 + 1) * t.KS;
    const T *Lov = Lo + (size_t(b) * 2 + 0) * t.KS;
    const int64_t N = t.N;
    // the near field's sources, staged 64 points at a time; a W-list box's
    // multipoles of v and g
    __shared__ T sx[64], sy[64], sv[64], sg[64];
    __shared__ T mwv[KMAX + 1], mwg[KMAX + 1];
    const int K = t.K;
    for (int i0 = t.begin[b]; i0 < t.end[b]; i0 += 64) {
        const int i = i0 + threadIdx.x;
        const bool ok = i < t.end[b];
        const T xi = ok ? t.xl[i] : T(0), yi = ok ? t.yl[i] : T(0);
        double o0 = 0, o1 = 0, o2 = 0, o3 = 0, o4 = 0, o5 = 0;
        if (ok) {
            // far field from the local expansions
            const T wx = xi * inv_s, wy = yi * inv_s;
            const T r2 = wx * wx + wy * wy;
            T potg = 0, gvx = 0, gvy = 0, ggx = 0, ggy = 0, dzv = 0;
            T pmr = 1, pmi = 0, p1r = 0, p1i = 0;              // W^m, W^(m-1)
            for (int m = 0; m <= P; ++m) {
                T tr = pmr, ti = pmi;                            // r2^q W^m
                T sr = p1r, si = p1i;                            // r2^q W^(m-1)
                T qr = 0, qi = 0;                                // r2^(q-1) W^m
                for (int n = m, q = 0; n <= P; n += 2, ++q) {
                    const int k = cidx_e(n, m);
                    const T dxr = T(2 * q) * wx * qr + T(m) * sr, dxi = T(2 * q) * wx * qi + T(m) * si;
                    const T dyr = T(2 * q) * wy * qr - T(m) * si, dyi = T(2 * q) * wy * qi + T(m) * sr;
                    const T lvr = Lv[k], lvi = m > 0 ? Lv[k + 1] : T(0);
                    const T lgr = Lg[k], lgi = m > 0 ? Lg[k + 1] : T(0);
                    potg += lgr * tr - lgi * ti;
                    ggx += lgr * dxr - lgi * dxi;
                    ggy += lgr * dyr - lgi * dyi;
                    gvx += lvr * dxr - lvi * dxi;
                    gvy += lvr * dyr - lvi * dyi;
                    if (n + 1 <= P) {
                        const int ko = cidx_o(n + 1, m);
                        const T lor = Lov[ko], loi = m > 0 ? Lov[ko + 1] : T(0);
                        dzv += lor * tr - loi * ti;
                    }
                    qr = tr; qi = ti;
                    tr *= r2; ti *= r2;
                    sr *= r2; si *= r2;
                }
                p1r = pmr; p1i = pmi;
                const T nr = pmr * wx - pmi * wy;
                pmi = pmr * wy + pmi * wx;
                pmr = nr;
            }
            o0 = double(potg); o1 = double(gvx * inv_s); o2 = double(gvy * inv_s);
            o3 = double(ggx * inv_s); o4 = double(ggy * inv_s); o5 = double(dzv);
        }
        // W list: each box's multipole expansions at the leaf's points
        for (int ww = t.w_off[b]; ww < t.w_off[b + 1]; ++ww) {
            const int a = t.w_idx[ww];
            __syncthreads();                             // the previous box is no longer read
            for (int k = threadIdx.x; k < K; k += 64) {
                mwv[k] = M[(size_t(a) * 2 + 0) * t.KS + k] * wx[k];
                mwg[k] = M[(size_t(a) * 2 + 1) * t.KS + k] * wx[k];
            }
            __syncthreads();
            if (ok) {
                const double ia_d = ldexp(1.0, t.level[a]);
                const T ia = T(ia_d);
                const T vx = xi * ia + T((t.cx[b] - t.cx[a]) * ia_d);
                const T vy = yi * ia + T((t.cy[b] - t.cy[a]) * ia_d);
                T pg = 0, dz = 0, dvr = 0, dvi = 0, dgr = 0, dgi = 0;
                irregular_all<T>(P + 1, vx, vy, T(cnd * ia_d), [&](int n, int m, T re, T im) {
                    if (((n + m) & 1) == 0) {
                        if (n <= P) {                        // potential of g
                            const int k = cidx_e(n, m);
                            pg += mwg[k] * re - (m > 0 ? mwg[k + 1] * im : T(0));
                        }
                        if (m >= 1) {                        // M_{n-1}^{m-1} I_n^m
                            const int k = cidx_e(n - 1, m - 1);
                            const T h = m == 1 ? T(1) : T(0.5);
                            const T vr = h * mwv[k], vi = m > 1 ? h * mwv[k + 1] : T(0);
                            const T gr = h * mwg[k], gi = m > 1 ? h * mwg[k + 1] : T(0);
                            dvr += vr * re - vi * im; dvi += vr * im + vi * re;
                            dgr += gr * re - gi * im; dgi += gr * im + gi * re;
                        }
                        if (m + 2 <= n) {                    // -conj(M_{n-1}^{m+1} I_n^m)
                            const int k = cidx_e(n - 1, m + 1);
                            const T vr = T(0.5) * mwv[k], vi = T(0.5) * mwv[k + 1];
                            const T gr = T(0.5) * mwg[k], gi = T(0.5) * mwg[k + 1];
                            dvr -= vr * re - vi * im; dvi += vr * im + vi * re;
                            dgr -= gr * re - gi * im; dgi += gr * im + gi * re;
                        }
                    } else {                                 // -eps_m Re(M_{n-1}^m I_n^m)
                        const int k = cidx_e(n - 1, m);
                        dz -= mwv[k] * re - (m > 0 ? mwv[k + 1] * im : T(0));
                    }
                });
                const double ia2 = ia_d * ia_d;
                o0 += double(pg) * ia_d;
                o1 += double(dvr) * ia2; o2 += double(dvi) * ia2;
                o3 += double(dgr) * ia2; o4 += double(dgi) * ia2;
                o5 += double(dz) * ia2;
            }
        }
        // near field, summed directly: each U-list leaf's points through LDS
        for (int uu = t.u_off[b]; uu < t.u_off[b + 1]; ++uu) {
            const int a = t.u_idx[uu];
            const T px = xi + T(t.cx[b] - t.cx[a]), py = yi + T(t.cy[b] - t.cy[a]);
            T s0 = 0, s1 = 0, s2 = 0, s3 = 0, s4 = 0, s5 = 0;
            for (int j0 = t.begin[a]; j0 < t.end[a]; j0 += 64) {
                const int nj = min(64, t.end[a] - j0);
                __syncthreads();                         // the previous chunk is no longer read
                if (threadIdx.x < nj) {
                    const int j = j0 + threadIdx.x;
                    sx[threadIdx.x] = t.xl[j];
                    sy[threadIdx.x] = t.yl[j];
                    sv[threadIdx.x] = us[j];
                    sg[threadIdx.x] = us[N + j];
                }
                __syncthreads();
                if (ok)
                    for (int jj = 0; jj < nj; ++jj) {
                        const T dx = px - sx[jj], dy = py - sy[jj];
                        const T ir = rsqrt_near(dx * dx + dy * dy + c2);
                        const T ir3 = ir * ir * ir;
                        const T vj = sv[jj], gj = sg[jj];
                        s0 += gj * ir;
                        s1 -= vj * dx * ir3;
                        s2 -= vj * dy * ir3;
                        s3 -= gj * dx * ir3;
                        s4 -= gj * dy * ir3;
                        s5 -= cc * vj * ir3;
                    }
            }
            o0 += double(s0); o1 += double(s1); o2 += double(s2);
            o3 += double(s3); o4 += double(s4); o5 += double(s5);
        }
        if (ok) {
            out[0 * N + i] = o0;
            out[1 * N + i] = o1;
            out[2 * N + i] = o2;
            out[3 * N + i] = o3;
            out[4 * N + i] = o4;
            out[5 * N + i] = o5;
        }
    }
}

template <typename T, typename Tout>
__global__ void k_adjoint_final(int64_t N, const int32_t *__restrict__ perm, const double *__restrict__ scale,
                                const T *__restrict__ us, const double *__restrict__ out,
                                Tout *__restrict__ dv, double *__restrict__ dxy, double *__restrict__ dcpart,
                                int accumulate)
{
    const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (i >= N) return;
    const double s1 = scale[i], s2 = s1 * s1;
    const double v = double(us[i]), g = double(us[N + i]);
    const int32_t k = perm[i];
    dv[k] = Tout(out[i] * s1);
    const double gx = (g * out[1 * N + i] + v * out[3 * N + i]) * s2;
    const double gy = (g * out[2 * N + i] + v * out[4 * N + i]) * s2;
    dxy[k] = accumulate ? dxy[k] + gx : gx;
    dxy[N + k] = accumulate ? dxy[N + k] + gy : gy;
    dcpart[i] = g * out[5 * N + i] * s2;
}

// dc[s] = sum of dcpart over the set's points, in a fixed order: SETSUM_NB
// contiguous slices of each set summed by as many workgroups, then the
// slices' sums in slice order.
constexpr int SETSUM_NB = 64;

__global__ __launch_bounds__(256) void k_set_partial(const int64_t *__restrict__ set_off,
                                                     const double *__restrict__ part, double *__restrict__ partial)
{
    __shared__ double red[256];
    const int s = blockIdx.x, blk = blockIdx.y;
    const int64_t a = set_off[s], n = set_off[s + 1] - a;
    const int64_t lo = a + n * blk / SETSUM_NB, hi = a + n * (blk + 1) / SETSUM_NB;
    double acc = 0.0;
    for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) acc += part[i];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[size_t(s) * SETSUM_NB + blk] = red[0];
}

__global__ void k_set_final(int nsets, const double *__restrict__ partial, double *__restrict__ dc, int accumulate)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nsets) return;
    double acc = 0.0;
    for (int b = 0; b < SETSUM_NB; ++b) acc += partial[size_t(s) * SETSUM_NB + b];
    dc[s] = accumulate ? dc[s] + acc : acc;
}

template <typename V>
imq_status upload_vec(DevBuf &d, const std::vector<V> &h)
{
    IMQ_HIP(dev_alloc(d, sizeof(V) * h.size()));
    if (!h.empty()) IMQ_HIP(hipMemcpy(d.p, h.data(), sizeof(V) * h.size(), hipMemcpyHostToDevice));
    return IMQ_OK;
}

// Odd-coefficient tables, generated once per tree on first use.
imq_status ensure_odd_tables(imq_tree_s *t)
{
    if (t->odd_ready) return IMQ_OK;
    const HostTree &h = t->h;
    const int K = h.K, KP = t->KP, p = h.p;
    const size_t KK = size_t(K) * K, PP = size_t(KP) * KP;
    const size_t ntab = size_t(h.nsets) * h.nlev * NCLASS;
    std::vector<double> m2l(ntab * PP, 0.0), l2l(4 * PP, 0.0), tmp(KK);
    auto pad_into = [&](const std::vector<double> &src, double *dst) {
        for (int r = 0; r < K; ++r) std::copy(src.begin() + size_t(r) * K, src.begin() + size_t(r + 1) * K, dst + size_t(r) * KP);
    };
    for (int pos = 0; pos < 4; ++pos) {
        make_l2l_odd_table(p, pos, tmp.data());
        pad_into(tmp, l2l.data() + pos * PP);
    }
    {
        std::vector<double> pk;
        pack_shift_tables(l2l, KP, pk, t->cut_l2l_odd);
        l2l.swap(pk);
    }
    for (int s = 0; s < h.nsets; ++s)
        for (int l = 2; l < h.nlev; ++l)
            for (int cls = 0; cls < NCLASS; ++cls) {
                const int dx = cls / 7 - 3, dy = cls % 7 - 3;
                if (std::abs(dx) <= 1 && std::abs(dy) <= 1) continue;
                make_m2l_odd_table(p, l, dx, dy, h.cn[s], tmp.data());
                pad_into(tmp, m2l.data() + ((size_t(s) * h.nlev + l) * NCLASS + cls) * PP);
            }
    // eps_k c_{j-1,k} per odd coefficient (the X-list odd P2L)
    std::vector<double> wxo(std::max(Kodd(p), 1), 0.0);
    for (int j = 1; j <= p; ++j)
        for (int k = (j + 1) & 1; k <= j - 1; k += 2) {
            const int o = j * (j - 1) / 2 + (k > 0 ? k - 1 : 0);
            const double v = (k == 0 ? 1.0 : 2.0) * legendre_coef(j - 1, k);
            wxo[o] = v;
            if (k > 0) wxo[o + 1] = v;
        }
    // the translation tables also in the streamed kernel's lane order: entry
    // (r, c) of a table at record (r/16 * nrb + c/16) * 64 + (c%16)/4 * 16 + r%16,
    // element c%4
    std::vector<double> m2l_pk(m2l.size(), 0.0);
    {
        const int nrb = KP / 16;
        for (size_t tb = 0; tb < ntab; ++tb)
            for (int r = 0; r < KP; ++r)
                for (int c = 0; c < KP; ++c) {
                    const size_t rec = (size_t(r / 16) * nrb + c / 16) * 64 + size_t((c % 16) / 4) * 16 + r % 16;
                    m2l_pk[tb * PP + rec * 4 + c % 4] = m2l[tb * PP + size_t(r) * KP + c];
                }
    }
    std::vector<float> m2l32(m2l.begin(), m2l.end()), l2l32(l2l.begin(), l2l.end()), wxo32(wxo.begin(), wxo.end());
    std::vector<float> m2l_pk32(m2l_pk.begin(), m2l_pk.end());
    imq_status st;
    if ((st = upload_vec(t->f64.m2l_odd_pk, m2l_pk)) != IMQ_OK) return st;
    if ((st = upload_vec(t->f32.m2l_odd_pk, m2l_pk32)) != IMQ_OK) return st;
    if ((st = upload_vec(t->f64.wxo, wxo)) != IMQ_OK) return st;
    if ((st = upload_vec(t->f32.wxo, wxo32)) != IMQ_OK) return st;
    if ((st = upload_vec(t->f64.m2l_odd, m2l)) != IMQ_OK) return st;
    if ((st = upload_vec(t->f64.l2l_odd, l2l)) != IMQ_OK) return st;
    if ((st = upload_vec(t->f32.m2l_odd, m2l32)) != IMQ_OK) return st;
    if ((st = upload_vec(t->f32.l2l_odd, l2l32)) != IMQ_OK) return st;
    t->odd_ready = true;
    return IMQ_OK;
}

inline dim3 grid1(int64_t n) { return dim3(unsigned((n + 255) / 256)); }

}  // namespace

template <typename T, typename Tio>
imq_status backward_typed(imq_tree_s *t, const Tio *v, const Tio *g, Tio *dv, double *dc, double *dxy,
                          int accumulate, hipStream_t s)
{
    const HostTree &h = t->h;
    const int64_t N = h.N;
    const int K = h.K, KP = t->KP, KS = coef_stride(K);
    const int nbox = int(h.level.size());
    imq_status st;
    if ((st = ensure_workspace<T>(t, 2)) != IMQ_OK) return st;
    if ((st = ensure_odd_tables(t)) != IMQ_OK) return st;
    PrecData &pd = prec_data<T>(t);
    const size_t lo_bytes = sizeof(T) * size_t(nbox) * 2 * KS;
    if (pd.Lodd.bytes < lo_bytes) IMQ_HIP(dev_alloc(pd.Lodd, lo_bytes));
    const size_t adj_bytes = sizeof(double) * (7 * size_t(N) + size_t(h.nsets) * SETSUM_NB);
    if (t->adj.bytes < adj_bytes) IMQ_HIP(dev_alloc(t->adj, adj_bytes));
    T *us = pd.us.as<T>();
    double *out = t->adj.as<double>();
    double *dcpart = out + 6 * N;
    double *dcslice = out + 7 * N;

    hipLaunchKernelGGL((k_gather2<Tio, T>), grid1(N), dim3(256), 0, s, N, t->perm.as<int32_t>(), v, g, us);
    IMQ_HIP(hipGetLastError());
    if ((st = fmm_upward<T>(t, 2, s, false, nullptr)) != IMQ_OK) return st;
    if ((st = fmm_translate<T>(t, 2, s, false)) != IMQ_OK) return st;
    // odd (vertical-derivative) coefficients: same batches, other tables
    T *Lo = pd.Lodd.as<T>();
    const int Ko = Kodd(h.p);
    {
        const size_t n = size_t(nbox) * 2 * KS;
        hipLaunchKernelGGL(k_zero<T>, dim3(unsigned((n + 255) / 256)), dim3(256), 0, s, n, Lo);
    }
    // streamed when the tree's kernel choice streams every level (m2l_mode 3;
    // output rows: the odd coefficients), else the staged GEMM
    bool streamed = false;
    if (t->g_m2l.ntasks > 0 && t->kcfg.m2l_mode == 3)
        streamed = launch_m2l_stream<T>(s, 0, K, t->g_m2l.ntasks, 0, 2, t->g_m2l.tasks.as<GemmTask>(),
                                        t->g_m2l.tbox.as<int32_t>(), t->g_m2l.tab.as<int32_t>(),
                                        t->g_m2l.src.as<int32_t>(), pd.m2l_odd_pk.as<T>(), nullptr, KP, KS,
                                        pd.M.as<T>(), Lo, Ko);
    if (t->g_m2l.ntasks > 0 && !streamed)
        launch_gemm<T>(s, 32, 1, t->g_m2l.ntasks, 2, t->g_m2l.tasks.as<GemmTask>(), 0, t->g_m2l.tbox.as<int32_t>(),
                       t->g_m2l.tab.as<int32_t>(), t->g_m2l.src.as<int32_t>(), pd.m2l_odd.as<T>(), KP, KS,
                       pd.M.as<T>(), Lo, 0, 0, Ko);
    if (t->nxboxes > 0)
        hipLaunchKernelGGL(k_p2l_odd<T>, dim3(unsigned(t->nxboxes)), dim3(64), 0, s, make_view<T>(t),
                           t->x_boxes.as<int32_t>(), us, pd.wxo.as<T>(), Ko, Lo);
    for (int l = std::max(h.need_l, 0); l + 1 < h.nlev; ++l) {
        const int p0 = h.sh_level_begin[l], np = h.sh_level_begin[l + 1] - p0;
        launch_shift<T>(s, false, t->kcfg.shift_cols, np, 2, t->sh_par.as<int32_t>() + p0,
                        t->sh_kids.as<int32_t>() + 4 * size_t(p0), pd.l2l_odd.as<T>(), KP, Ko, Ko,
                        t->cut_l2l_odd, Lo, KS, Lo, KS);
    }
    IMQ_HIP(hipGetLastError());
    DTree<T> view = make_view<T>(t);
    hipLaunchKernelGGL(k_adjoint_eval<T>, dim3(unsigned(h.leaves.size())), dim3(64), 0, s, view,
                       t->leaves.as<int32_t>(), pd.L.as<T>(), Lo, pd.M.as<T>(), pd.wx.as<T>(), us, out);
    hipLaunchKernelGGL((k_adjoint_final<T, Tio>), grid1(N), dim3(256), 0, s, N, t->perm.as<int32_t>(),
                       t->pt_scale.as<double>(), us, out, dv, dxy, dcpart, accumulate);
    hipLaunchKernelGGL(k_set_partial, dim3(h.nsets, SETSUM_NB), dim3(256), 0, s, t->set_off.as<int64_t>(), dcpart,
                       dcslice);
    hipLaunchKernelGGL(k_set_final, dim3(unsigned((h.nsets + 255) / 256)), dim3(256), 0, s, h.nsets, dcslice, dc,
                       accumulate);
    IMQ_HIP(hipGetLastError());
    return IMQ_OK;
}

template imq_status backward_typed<double, double>(imq_tree_s *, const double *, const double *, double *,
                                                   double *, double *, int, hipStream_t);
template imq_status backward_typed<double, float>(imq_tree_s *, const float *, const float *, float *,
                                                  double *, double *, int, hipStream_t);
template imq_status backward_typed<float, double>(imq_tree_s *, const double *, const double *, double *,
                                                  double *, double *, int, hipStream_t);
template imq_status backward_typed<float, float>(imq_tree_s *, const float *, const float *, float *,
                                                 double *, double *, int, hipStream_t);

}  // namespace imq
