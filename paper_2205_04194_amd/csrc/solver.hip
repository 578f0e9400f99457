// Iterative solution of A a = f (Sec. 2, eq. interp_system) on the fast
// product: restarted GMRES with the Krylov basis, the orthogonalisation and
// every vector update in FP64 on the device, and mixed-precision iterative
// refinement around an FP32-product GMRES.
//
// The paper only names an iterative method as the use of the product; the
// solver is the textbook one: Arnoldi with classical Gram-Schmidt applied
// twice (CGS2) for stability, Givens rotations on the small Hessenberg
// matrix (host), residual estimate |g_{j+1}|, explicit residual f - A x at
// every restart.  All vectors stay in the tree's Morton order.
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

__global__ void k_to_type_f(int64_t n, const double *__restrict__ x, float *__restrict__ y)
{
    const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (i < n) y[i] = float(x[i]);
}
__global__ void k_to_type_d(int64_t n, const double *__restrict__ x, double *__restrict__ y)
{
    const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (i < n) y[i] = x[i];
}

// y = scale .* bs  (normalised-unit product -> caller units)
__global__ void k_scale(int64_t n, const double *__restrict__ bs, const double *__restrict__ sc,
                        double *__restrict__ y)
{
    const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (i < n) y[i] = bs[i] * sc[i];
}

// part[v * RED_BLOCKS + blk] = partial sum over the block's slice of V_v . w
__global__ __launch_bounds__(256) void k_dots(int64_t n, const double *__restrict__ V, int64_t ldv,
                                              const double *__restrict__ w, double *__restrict__ part)
{
    __shared__ double red[256];
    const int v = blockIdx.y;
    const double *x = V + v * ldv;
    double s = 0.0;
    for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
        s += x[i] * w[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[v * RED_BLOCKS + blockIdx.x] = red[0];
}

// h[v] (+)= sum over blocks of part[v]; fixed order, so deterministic
__global__ void k_dots_final(int nv, const double *__restrict__ part, double *__restrict__ h, int accumulate)
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
    (void)nv;
}

// w -= sum_v V_v h[v]
__global__ void k_sub_Vh(int64_t n, int nv, const double *__restrict__ V, int64_t ldv,
                         const double *__restrict__ h, double *__restrict__ w)
{
    const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
    for (int v = 0; v < nv; ++v) s += V[v * ldv + i] * h[v];
    w[i] -= s;
}

// y = x / norm, norm = sqrt(*nrm2)
__global__ void k_normalize(int64_t n, const double *__restrict__ x, const double *__restrict__ nrm2,
                            double *__restrict__ y)
{
    const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    const double nr = sqrt(*nrm2);
    if (i < n) y[i] = nr > 0.0 ? x[i] / nr : 0.0;
}

// z = a*x + b*y
__global__ void k_axpby(int64_t n, double a, const double *__restrict__ x, double b,
                        const double *__restrict__ y, double *__restrict__ z)
{
    const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (i < n) z[i] = a * x[i] + b * y[i];
}

// x += V y (first k columns)
__global__ void k_add_Vy(int64_t n, int k, const double *__restrict__ V, int64_t ldv,
                         const double *__restrict__ y, double *__restrict__ x)
{
    const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
    for (int v = 0; v < k; ++v) s += V[v * ldv + i] * y[v];
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
    double *V, *w, *tmp, *r, *x, *f, *h, *part;
    std::vector<double> hh;

    // y = A x in Morton order, FP64 vectors, product arithmetic T
    template <typename T>
    imq_status apply(const double *xin, double *yout)
    {
        imq_status st = ensure_workspace<T>(t, 1);
        if (st != IMQ_OK) return st;
        T *us = prec_data<T>(t).us.template as<T>();
        if constexpr (sizeof(T) == 4)
            hipLaunchKernelGGL(k_to_type_f, grid1(N), dim3(256), 0, s, N, xin, us);
        else
            hipLaunchKernelGGL(k_to_type_d, grid1(N), dim3(256), 0, s, N, xin, us);
        if ((st = fmm_sorted<T>(t, 1, s, nullptr)) != IMQ_OK) return st;
        hipLaunchKernelGGL(k_scale, grid1(N), dim3(256), 0, s, N, t->bs.as<double>(),
                           t->pt_scale.as<double>(), yout);
        IMQ_HIP(hipGetLastError());
        return IMQ_OK;
    }

    imq_status apply_prec(int prec, const double *xin, double *yout)
    {
        return prec == IMQ_PREC_FP32 ? apply<float>(xin, yout) : apply<double>(xin, yout);
    }

    // h[0..nv) (+)= V[0..nv)^T w
    imq_status dots(const double *Vb, int nv, const double *wv, double *hout, int accumulate)
    {
        hipLaunchKernelGGL(k_dots, dim3(RED_BLOCKS, nv), dim3(256), 0, s, N, Vb, N, wv, part);
        hipLaunchKernelGGL(k_dots_final, dim3(nv), dim3(256), 0, s, nv, part, hout, accumulate);
        IMQ_HIP(hipGetLastError());
        return IMQ_OK;
    }

    imq_status norm(const double *v, double &out)
    {
        imq_status st = dots(v, 1, v, h + m + 1, 0);
        if (st != IMQ_OK) return st;
        double n2 = 0;
        IMQ_HIP(hipMemcpyAsync(&n2, h + m + 1, sizeof(double), hipMemcpyDeviceToHost, s));
        IMQ_HIP(hipStreamSynchronize(s));
        out = std::sqrt(n2);
        return IMQ_OK;
    }

    // Restarted GMRES on A_prec for A x = rhs; x in/out.  Stops when the
    // estimate falls to tol*||rhs|| (checked every step) or after maxit
    // products; the explicit residual is recomputed at every restart.
    imq_status gmres(int prec, const double *rhs, double *xs, double tol, int maxit, int &its,
                     double &relres)
    {
        imq_status st;
        double nf;
        if ((st = norm(rhs, nf)) != IMQ_OK) return st;
        if (nf == 0.0) {
            IMQ_HIP(hipMemsetAsync(xs, 0, sizeof(double) * N, s));
            relres = 0.0;
            return IMQ_OK;
        }
        std::vector<double> H(size_t(m + 1) * m, 0.0), cs(m), sn(m), g(m + 1), y(m);
        its = 0;
        for (;;) {
            if ((st = apply_prec(prec, xs, tmp)) != IMQ_OK) return st;
            hipLaunchKernelGGL(k_axpby, grid1(N), dim3(256), 0, s, N, 1.0, rhs, -1.0, tmp, r);
            double beta;
            if ((st = norm(r, beta)) != IMQ_OK) return st;
            relres = beta / nf;
            if (relres <= tol || its >= maxit) return IMQ_OK;
            hipLaunchKernelGGL(k_axpby, grid1(N), dim3(256), 0, s, N, 1.0 / beta, r, 0.0, r, V);
            std::fill(g.begin(), g.end(), 0.0);
            g[0] = beta;
            int k = 0;
            for (int j = 0; j < m && its < maxit; ++j) {
                double *vj = V + size_t(j) * N, *vn = V + size_t(j + 1) * N;
                if ((st = apply_prec(prec, vj, w)) != IMQ_OK) return st;
                // CGS2: two passes of classical Gram-Schmidt
                if ((st = dots(V, j + 1, w, h, 0)) != IMQ_OK) return st;
                hipLaunchKernelGGL(k_sub_Vh, grid1(N), dim3(256), 0, s, N, j + 1, V, N, h, w);
                if ((st = dots(V, j + 1, w, h + m + 2, 0)) != IMQ_OK) return st;
                hipLaunchKernelGGL(k_sub_Vh, grid1(N), dim3(256), 0, s, N, j + 1, V, N, h + m + 2, w);
                hipLaunchKernelGGL(k_axpby, grid1(j + 1), dim3(256), 0, s, int64_t(j + 1), 1.0, h, 1.0,
                                   h + m + 2, h);
                if ((st = dots(w, 1, w, h + j + 1, 0)) != IMQ_OK) return st;
                hipLaunchKernelGGL(k_normalize, grid1(N), dim3(256), 0, s, N, w, h + j + 1, vn);
                IMQ_HIP(hipGetLastError());
                hh.resize(j + 2);
                IMQ_HIP(hipMemcpyAsync(hh.data(), h, sizeof(double) * (j + 2), hipMemcpyDeviceToHost, s));
                IMQ_HIP(hipStreamSynchronize(s));
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
                k = j + 1;
                if (std::fabs(g[j + 1]) <= tol * nf || hh[j + 1] == 0.0) break;
            }
            // back substitution and update x += V y
            for (int i = k - 1; i >= 0; --i) {
                double sum = g[i];
                for (int l = i + 1; l < k; ++l) sum -= H[size_t(l) * (m + 1) + i] * y[l];
                const double d = H[size_t(i) * (m + 1) + i];
                y[i] = d != 0.0 ? sum / d : 0.0;
            }
            IMQ_HIP(hipMemcpyAsync(h, y.data(), sizeof(double) * k, hipMemcpyHostToDevice, s));
            hipLaunchKernelGGL(k_add_Vy, grid1(N), dim3(256), 0, s, N, k, V, N, h, xs);
            IMQ_HIP(hipGetLastError());
        }
    }
};

}  // namespace

imq_status solve_one(imq_tree_s *t, const double *f_user, double *a_user, const imq_solve_opts &o,
                     imq_solve_stats &stats, hipStream_t s)
{
    Solver S;
    S.t = t;
    S.s = s;
    S.N = t->h.N;
    S.m = o.restart;
    const int64_t N = S.N;
    const int m = o.restart;
    // workspace: basis (m+1); w, tmp, r (inside GMRES); x, f; d, e (refinement);
    // small vectors and reduction partials
    const size_t need = sizeof(double) * (size_t(m + 1) * N + 7 * size_t(N) + 2 * (m + 2) +
                                          size_t(RED_BLOCKS) * (m + 2));
    if (t->sol_bytes < need) {
        IMQ_HIP(dev_alloc(t->sol, need));
        t->sol_bytes = need;
    }
    double *base = t->sol.as<double>();
    S.V = base;
    S.w = S.V + size_t(m + 1) * N;
    S.tmp = S.w + N;
    S.r = S.tmp + N;
    S.x = S.r + N;
    S.f = S.x + N;
    double *d = S.f + N;
    double *e = d + N;
    S.h = e + N;
    S.part = S.h + 2 * (m + 2);

    const int32_t *perm = t->perm.as<int32_t>();
    hipLaunchKernelGGL(k_gather_f64, grid1(N), dim3(256), 0, s, N, perm, f_user, S.f);
    hipLaunchKernelGGL(k_gather_f64, grid1(N), dim3(256), 0, s, N, perm, a_user, S.x);
    IMQ_HIP(hipGetLastError());

    imq_status st;
    int its = 0;
    double rel = 0.0;
    stats = imq_solve_stats{0, 0, 0, 0.0};
    if (!o.mixed_ir) {
        if ((st = S.gmres(IMQ_PREC_FP64, S.f, S.x, o.tol, o.max_iters, its, rel)) != IMQ_OK) return st;
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
            if ((st = S.apply<double>(S.x, e)) != IMQ_OK) return st;
            hipLaunchKernelGGL(k_axpby, grid1(N), dim3(256), 0, s, N, 1.0, S.f, -1.0, e, d);
            double nr;
            if ((st = S.norm(d, nr)) != IMQ_OK) return st;
            rel = nr / nf;
            if (rel <= o.tol || total >= o.max_iters) break;
            // correction A32 e = d, to the relative accuracy the FP32 product can reach
            const double inner_tol = std::max(o.tol * nf / nr, 1e-6);
            IMQ_HIP(hipMemsetAsync(e, 0, sizeof(double) * N, s));
            int inner_its = 0;
            double inner_rel = 0.0;
            if ((st = S.gmres(IMQ_PREC_FP32, d, e, inner_tol, o.max_iters - total, inner_its, inner_rel)) != IMQ_OK)
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
    if ((st = S.apply<double>(S.x, S.tmp)) != IMQ_OK) return st;
    hipLaunchKernelGGL(k_axpby, grid1(N), dim3(256), 0, s, N, 1.0, S.f, -1.0, S.tmp, S.r);
    if ((st = S.norm(S.r, nr)) != IMQ_OK) return st;
    stats.relres = nf > 0 ? nr / nf : 0.0;
    stats.converged = stats.relres <= o.tol;
    hipLaunchKernelGGL(k_scatter_f64, grid1(N), dim3(256), 0, s, N, perm, S.x, a_user);
    IMQ_HIP(hipGetLastError());
    return IMQ_OK;
}

}  // namespace imq
