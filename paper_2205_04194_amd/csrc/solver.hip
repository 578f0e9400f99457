// Iterative solution of A a = f (Sec. 2, eq. interp_system) on the fast
// product: restarted GMRES with the Krylov basis, the orthogonalisation and
// every vector update on the device, and mixed-precision iterative
// refinement around an FP32-product GMRES.
//
// The paper only names an iterative method as the use of the product; the
// solver is the textbook one: Arnoldi with classical Gram-Schmidt applied
// twice (CGS2) for stability, Givens rotations on the small Hessenberg
// matrix (host), residual estimate |g_{j+1}|, explicit residual f - A x at
// every restart.  All vectors stay in the tree's Morton order.
//
// Precision: the FP64 solver keeps its basis in FP64; the inner solver of
// the refinement (FP32 products, inner tolerance >= 1e-6) keeps its basis in
// FP32, which halves the memory traffic of the orthogonalisation.  Dot
// products, the Hessenberg matrix and the rotations are FP64 in both.
//
// The host reads one Hessenberg column per step.  To keep the GPU busy
// meanwhile, the product of step j+1 is queued before the host waits for
// column j (it is discarded if step j ends the cycle).
#include "device.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

namespace imq {

template <typename T>
imq_status fmm_sorted(imq_tree_s *t, int nrhs, hipStream_t s, const UserVec *io);
template <typename T>
imq_status ensure_workspace(imq_tree_s *t, int nrhs);

namespace {

constexpr int RED_BLOCKS = 512;       // partial sums per dot product

template <typename A, typename B>
__global__ void k_convert(int64_t n, const A *__restrict__ x, B *__restrict__ y)
{
    const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (i < n) y[i] = B(x[i]);
}

template <typename V>
__global__ void k_fill0(int64_t n, V *__restrict__ y)
{
    const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (i < n) y[i] = V(0);
}

// y = scale .* bs  (normalised-unit product -> caller units), in the type of y
template <typename V>
__global__ void k_scale(int64_t n, const double *__restrict__ bs, const double *__restrict__ sc,
                        V *__restrict__ y)
{
    const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (i < n) y[i] = V(bs[i] * sc[i]);
}

// part[v * RED_BLOCKS + blk] = partial sum over the block's slice of V_v . w
template <typename V, typename W>
__global__ __launch_bounds__(256) void k_dots(int64_t n, const V *__restrict__ Vb, int64_t ldv,
                                              const W *__restrict__ w, double *__restrict__ part)
{
    __shared__ double red[256];
    const int v = blockIdx.y;
    const V *x = Vb + v * ldv;
    double s = 0.0;
    for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
        s += double(x[i]) * double(w[i]);
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[v * RED_BLOCKS + blockIdx.x] = red[0];
}

// h[v] (+)= sum over blocks of part[v]; fixed order, so deterministic
__global__ void k_dots_final(const double *__restrict__ part, double *__restrict__ h, int accumulate)
{
    __shared__ double red[256];
    const int v = blockIdx.x;
    double s = 0.0;
    for (int b = threadIdx.x; b < RED_BLOCKS; b += blockDim.x) s += part[v * RED_BLOCKS + b];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) h[v] = accumulate ? h[v] + red[0] : red[0];
}

// w -= sum_v V_v h[v]
template <typename V>
__global__ void k_sub_Vh(int64_t n, int nv, const V *__restrict__ Vb, int64_t ldv, const double *__restrict__ h,
                         V *__restrict__ w)
{
    const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
    for (int v = 0; v < nv; ++v) s += double(Vb[v * ldv + i]) * h[v];
    w[i] = V(double(w[i]) - s);
}

// y = x / norm, norm = sqrt(*nrm2)
template <typename A, typename B>
__global__ void k_normalize(int64_t n, const A *__restrict__ x, const double *__restrict__ nrm2, B *__restrict__ y)
{
    const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    const double nr = sqrt(*nrm2);
    if (i < n) y[i] = B(nr > 0.0 ? double(x[i]) / nr : 0.0);
}

// z = a*x + b*y
__global__ void k_axpby(int64_t n, double a, const double *__restrict__ x, double b,
                        const double *__restrict__ y, double *__restrict__ z)
{
    const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (i < n) z[i] = a * x[i] + b * y[i];
}

// x += V y (first k columns)
template <typename V>
__global__ void k_add_Vy(int64_t n, int k, const V *__restrict__ Vb, int64_t ldv, const double *__restrict__ y,
                         double *__restrict__ x)
{
    const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
    for (int v = 0; v < k; ++v) s += double(Vb[v * ldv + i]) * y[v];
    x[i] += s;
}

__global__ void k_gather_f64(int64_t n, const int32_t *__restrict__ perm, const double *__restrict__ x,
                             double *__restrict__ y)
{
    const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (i < n) y[i] = x[perm[i]];
}

__global__ void k_scatter_f64(int64_t n, const int32_t *__restrict__ perm, const double *__restrict__ x,
                              double *__restrict__ y)
{
    const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (i < n) y[perm[i]] = x[i];
}

inline dim3 grid1(int64_t n) { return dim3(unsigned((n + 255) / 256)); }

struct Solver {
    imq_tree_s *t;
    hipStream_t s;
    int64_t N;
    int m;
    void *Vraw, *wraw;                 // basis (m+1) x N and two product vectors, FP64-sized
    double *tmp, *r, *x, *f, *h, *part;
    double *hh = nullptr;              // pinned host copy of one Hessenberg column
    hipEvent_t ev_h = nullptr;
    double *hist = nullptr;            // host residual history (optional)
    int hist_cap = 0, hist_n = 0;
    double hist_scale = 1.0;           // 1 / ||f|| of the outer system

    // y = A x in Morton order, product arithmetic T, vectors of type V
    template <typename T, typename V>
    imq_status apply(const V *xin, V *yout)
    {
        imq_status st = ensure_workspace<T>(t, 1);
        if (st != IMQ_OK) return st;
        T *us = prec_data<T>(t).us.template as<T>();
        hipLaunchKernelGGL((k_convert<V, T>), grid1(N), dim3(256), 0, s, N, xin, us);
        if ((st = fmm_sorted<T>(t, 1, s, nullptr)) != IMQ_OK) return st;
        hipLaunchKernelGGL(k_scale<V>, grid1(N), dim3(256), 0, s, N, t->bs.as<double>(), t->pt_scale.as<double>(),
                           yout);
        IMQ_HIP(hipGetLastError());
        return IMQ_OK;
    }

    // h[0..nv) = V[0..nv)^T w
    template <typename V, typename W>
    imq_status dots(const V *Vb, int nv, const W *wv, double *hout)
    {
        hipLaunchKernelGGL((k_dots<V, W>), dim3(RED_BLOCKS, nv), dim3(256), 0, s, N, Vb, N, wv, part);
        hipLaunchKernelGGL(k_dots_final, dim3(nv), dim3(256), 0, s, part, hout, 0);
        IMQ_HIP(hipGetLastError());
        return IMQ_OK;
    }

    imq_status norm(const double *v, double &out)
    {
        imq_status st = dots(v, 1, v, h + m + 1);
        if (st != IMQ_OK) return st;
        IMQ_HIP(hipMemcpyAsync(hh, h + m + 1, sizeof(double), hipMemcpyDeviceToHost, s));
        IMQ_HIP(hipStreamSynchronize(s));
        out = std::sqrt(hh[0]);
        return IMQ_OK;
    }

    // Restarted GMRES on the product in arithmetic T for A x = rhs; x in/out
    // (FP64).  Stops when the estimate falls to tol*||rhs|| (checked every
    // step) or after maxit products; the explicit residual is recomputed at
    // every restart.
    template <typename T, typename V>
    imq_status gmres(const double *rhs, double *xs, double tol, int maxit, int &its, double &relres)
    {
        imq_status st;
        V *Vb = static_cast<V *>(Vraw);
        V *w[2] = {static_cast<V *>(wraw), static_cast<V *>(wraw) + N};
        double nf;
        if ((st = norm(rhs, nf)) != IMQ_OK) return st;
        if (nf == 0.0) {
            hipLaunchKernelGGL(k_fill0<double>, grid1(N), dim3(256), 0, s, N, xs);
            IMQ_HIP(hipGetLastError());
            relres = 0.0;
            return IMQ_OK;
        }
        std::vector<double> H(size_t(m + 1) * m, 0.0), cs(m), sn(m), g(m + 1), y(m);
        its = 0;
        for (;;) {
            if ((st = apply<T, double>(xs, tmp)) != IMQ_OK) return st;
            hipLaunchKernelGGL(k_axpby, grid1(N), dim3(256), 0, s, N, 1.0, rhs, -1.0, tmp, r);
            double beta;
            if ((st = norm(r, beta)) != IMQ_OK) return st;
            relres = beta / nf;
            if (relres <= tol || its >= maxit) return IMQ_OK;
            hipLaunchKernelGGL((k_normalize<double, V>), grid1(N), dim3(256), 0, s, N, r, h + m + 1, Vb);
            std::fill(g.begin(), g.end(), 0.0);
            g[0] = beta;
            int k = 0, cur = 0;
            if ((st = apply<T, V>(Vb, w[cur])) != IMQ_OK) return st;
            for (int j = 0; j < m && its < maxit; ++j) {
                V *wj = w[cur];
                V *vn = Vb + size_t(j + 1) * N;
                // CGS2: two passes of classical Gram-Schmidt
                if ((st = dots(Vb, j + 1, wj, h)) != IMQ_OK) return st;
                hipLaunchKernelGGL(k_sub_Vh<V>, grid1(N), dim3(256), 0, s, N, j + 1, Vb, N, h, wj);
                if ((st = dots(Vb, j + 1, wj, h + m + 2)) != IMQ_OK) return st;
                hipLaunchKernelGGL(k_sub_Vh<V>, grid1(N), dim3(256), 0, s, N, j + 1, Vb, N, h + m + 2, wj);
                hipLaunchKernelGGL(k_axpby, grid1(j + 1), dim3(256), 0, s, int64_t(j + 1), 1.0, h, 1.0, h + m + 2,
                                   h);
                if ((st = dots(wj, 1, wj, h + j + 1)) != IMQ_OK) return st;
                hipLaunchKernelGGL((k_normalize<V, V>), grid1(N), dim3(256), 0, s, N, wj, h + j + 1, vn);
                IMQ_HIP(hipGetLastError());
                IMQ_HIP(hipMemcpyAsync(hh, h, sizeof(double) * (j + 2), hipMemcpyDeviceToHost, s));
                IMQ_HIP(hipEventRecord(ev_h, s));
                // the next step's product runs while the host waits for this column
                if (j + 1 < m && its + 1 < maxit)
                    if ((st = apply<T, V>(vn, w[1 - cur])) != IMQ_OK) return st;
                IMQ_HIP(hipEventSynchronize(ev_h));
                hh[j + 1] = std::sqrt(std::max(hh[j + 1], 0.0));
                ++its;
                // Givens rotations on column j of the Hessenberg matrix
                double *col = &H[size_t(j) * (m + 1)];
                for (int i = 0; i <= j + 1; ++i) col[i] = hh[i];
                for (int i = 0; i < j; ++i) {
                    const double a = cs[i] * col[i] + sn[i] * col[i + 1];
                    col[i + 1] = -sn[i] * col[i] + cs[i] * col[i + 1];
                    col[i] = a;
                }
                const double den = std::hypot(col[j], col[j + 1]);
                cs[j] = den > 0 ? col[j] / den : 1.0;
                sn[j] = den > 0 ? col[j + 1] / den : 0.0;
                col[j] = den;
                col[j + 1] = 0.0;
                g[j + 1] = -sn[j] * g[j];
                g[j] = cs[j] * g[j];
                if (hist && hist_n < hist_cap) hist[hist_n++] = std::fabs(g[j + 1]) * hist_scale;
                k = j + 1;
                cur = 1 - cur;
                if (std::fabs(g[j + 1]) <= tol * nf || col[j] == 0.0 || hh[j + 1] == 0.0) break;
            }
            // back substitution and update x += V y
            for (int i = k - 1; i >= 0; --i) {
                double sum = g[i];
                for (int l = i + 1; l < k; ++l) sum -= H[size_t(l) * (m + 1) + i] * y[l];
                const double d = H[size_t(i) * (m + 1) + i];
                y[i] = d != 0.0 ? sum / d : 0.0;
            }
            for (int i = 0; i < k; ++i) hh[i] = y[i];
            IMQ_HIP(hipMemcpyAsync(h, hh, sizeof(double) * k, hipMemcpyHostToDevice, s));
            hipLaunchKernelGGL(k_add_Vy<V>, grid1(N), dim3(256), 0, s, N, k, Vb, N, h, xs);
            IMQ_HIP(hipGetLastError());
            IMQ_HIP(hipStreamSynchronize(s));            // hh is reused by the next norm
        }
    }
};

}  // namespace

imq_status solve_one(imq_tree_s *t, const double *f_user, double *a_user, const imq_solve_opts &o,
                     imq_solve_stats &stats, double *history, hipStream_t s)
{
    Solver S;
    S.t = t;
    S.s = s;
    S.N = t->h.N;
    S.m = o.restart;
    const int64_t N = S.N;
    const int m = o.restart;
    // workspace: basis (m+1) and two product vectors (FP64-sized); tmp, r, x,
    // f; d, e (refinement); small vectors and reduction partials
    const size_t need = sizeof(double) * (size_t(m + 3) * N + 6 * size_t(N) + 2 * (m + 2) +
                                          size_t(RED_BLOCKS) * (m + 2));
    if (t->sol_bytes < need) {
        IMQ_HIP(dev_alloc(t->sol, need));
        t->sol_bytes = need;
    }
    double *base = t->sol.as<double>();
    S.Vraw = base;
    S.wraw = base + size_t(m + 1) * N;
    S.tmp = base + size_t(m + 3) * N;
    S.r = S.tmp + N;
    S.x = S.r + N;
    S.f = S.x + N;
    double *d = S.f + N;
    double *e = d + N;
    S.h = e + N;
    S.part = S.h + 2 * (m + 2);
    IMQ_HIP(hipHostMalloc(reinterpret_cast<void **>(&S.hh), sizeof(double) * (m + 2), hipHostMallocDefault));
    struct Release {
        Solver &S;
        ~Release()
        {
            if (S.hh) (void)hipHostFree(S.hh);
            if (S.ev_h) (void)hipEventDestroy(S.ev_h);
        }
    } release{S};
    IMQ_HIP(hipEventCreateWithFlags(&S.ev_h, hipEventDisableTiming));

    const int32_t *perm = t->perm.as<int32_t>();
    hipLaunchKernelGGL(k_gather_f64, grid1(N), dim3(256), 0, s, N, perm, f_user, S.f);
    hipLaunchKernelGGL(k_gather_f64, grid1(N), dim3(256), 0, s, N, perm, a_user, S.x);
    IMQ_HIP(hipGetLastError());

    imq_status st;
    int its = 0;
    double rel = 0.0;
    stats = imq_solve_stats{0, 0, 0, 0.0};
    S.hist = history;
    S.hist_cap = history ? o.max_iters : 0;
    {
        double nf0;
        if ((st = S.norm(S.f, nf0)) != IMQ_OK) return st;
        S.hist_scale = nf0 > 0.0 ? 1.0 / nf0 : 0.0;
    }
    if (!o.mixed_ir) {
        if ((st = S.gmres<double, double>(S.f, S.x, o.tol, o.max_iters, its, rel)) != IMQ_OK) return st;
        stats.iters = its;
        stats.outer_iters = 1;
    } else {
        // refinement: r = f - A64 a in FP64, correction from FP32-product GMRES
        double nf;
        if ((st = S.norm(S.f, nf)) != IMQ_OK) return st;
        const int max_outer = o.max_outer > 0 ? o.max_outer : 10;
        int total = 0, outer = 0;
        for (; outer < max_outer; ++outer) {
            // residual d = f - A64 a (e is scratch here)
            if ((st = S.apply<double, double>(S.x, e)) != IMQ_OK) return st;
            hipLaunchKernelGGL(k_axpby, grid1(N), dim3(256), 0, s, N, 1.0, S.f, -1.0, e, d);
            double nr;
            if ((st = S.norm(d, nr)) != IMQ_OK) return st;
            rel = nr / nf;
            if (rel <= o.tol || total >= o.max_iters) break;
            // correction A32 e = d, to the relative accuracy the FP32 product can reach
            const double inner_tol = std::max(o.tol * nf / nr, 1e-6);
            hipLaunchKernelGGL(k_fill0<double>, grid1(N), dim3(256), 0, s, N, e);
            int inner_its = 0;
            double inner_rel = 0.0;
            if ((st = S.gmres<float, float>(d, e, inner_tol, o.max_iters - total, inner_its, inner_rel)) != IMQ_OK)
                return st;
            total += inner_its;
            hipLaunchKernelGGL(k_axpby, grid1(N), dim3(256), 0, s, N, 1.0, S.x, 1.0, e, S.x);
            IMQ_HIP(hipGetLastError());
        }
        stats.iters = total;
        stats.outer_iters = outer;
    }
    // final explicit residual with the FP64 product
    double nf, nr;
    if ((st = S.norm(S.f, nf)) != IMQ_OK) return st;
    if ((st = S.apply<double, double>(S.x, S.tmp)) != IMQ_OK) return st;
    hipLaunchKernelGGL(k_axpby, grid1(N), dim3(256), 0, s, N, 1.0, S.f, -1.0, S.tmp, S.r);
    if ((st = S.norm(S.r, nr)) != IMQ_OK) return st;
    stats.relres_fast64 = nf > 0 ? nr / nf : 0.0;
    stats.converged = stats.relres_fast64 <= o.tol;
    hipLaunchKernelGGL(k_scatter_f64, grid1(N), dim3(256), 0, s, N, perm, S.x, a_user);
    IMQ_HIP(hipGetLastError());
    return IMQ_OK;
}

}  // namespace imq
