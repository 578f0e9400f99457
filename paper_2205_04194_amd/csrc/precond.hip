// Leaf block-Jacobi preconditioner for the GMRES solves.
//
// The paper leaves a preconditioner built from the structure of A as future
// work (Sec. 4) and points to preconditioned GMRES for radial-basis fitting
// (Sec. 1).  This is the simplest member of that family that the quadtree
// gives for free: M = blockdiag(A_bb) over runs of at most 64 consecutive
// points (in the tree's point order) of every leaf, so M^-1 applies the exact
// inverse of the interactions inside each run.  The solver uses it as a
// right preconditioner, A M^-1 y = f, a = M^-1 y: the residual it monitors
// stays that of A a = f.
//
// Setup: one workgroup per run forms A_bb in LDS from the caller's FP64
// coordinates and c of the run's set (eq. IMQ_def) and inverts it in place by
// Gauss-Jordan elimination with partial pivoting (row swaps recorded, undone
// on the columns at the end); the inverse is stored row-major per run.
// Apply: one workgroup per (run, right-hand side), lane i forms row i of the
// run's inverse times the run's slice of the vector, in FP64.
#include "device.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

namespace imq {

namespace {

constexpr int BJ_MAX = 64;     // points per run

__global__ __launch_bounds__(256) void k_bj_setup(const BJRun *__restrict__ runs, const int32_t *__restrict__ perm,
                                                  const double *__restrict__ xy, int64_t N,
                                                  const double *__restrict__ c, double *__restrict__ inv)
{
    __shared__ double A[BJ_MAX][BJ_MAX + 1];
    __shared__ double px[BJ_MAX], py[BJ_MAX];
    __shared__ int ipiv[BJ_MAX];
    __shared__ double col[BJ_MAX];
    const BJRun rn = runs[blockIdx.x];
    const int n = rn.n, tid = threadIdx.x;
    const double cc = c[rn.set] * c[rn.set];
    if (tid < n) {
        const int j = perm[rn.begin + tid];
        px[tid] = xy[j];
        py[tid] = xy[N + j];
    }
    __syncthreads();
    for (int e = tid; e < n * n; e += 256) {
        const int i = e / n, j = e - i * n;
        const double dx = px[i] - px[j], dy = py[i] - py[j];
        A[i][j] = 1.0 / sqrt(dx * dx + dy * dy + cc);
    }
    __syncthreads();
    for (int k = 0; k < n; ++k) {
        // pivot: the largest |A[i][k]|, i >= k (first of equals), by wave 0
        if (tid < 64) {
            const int i = k + tid;
            double v = i < n ? fabs(A[i][k]) : -1.0;
            int idx = i;
            for (int d = 32; d > 0; d >>= 1) {
                const double ov = __shfl_down(v, d);
                const int oi = __shfl_down(idx, d);
                if (ov > v || (ov == v && oi < idx)) { v = ov; idx = oi; }
            }
            if (tid == 0) ipiv[k] = idx;
        }
        __syncthreads();
        const int p = ipiv[k];
        if (p != k)
            for (int j = tid; j < n; j += 256) {
                const double t = A[k][j];
                A[k][j] = A[p][j];
                A[p][j] = t;
            }
        __syncthreads();
        const double piv = A[k][k];
        __syncthreads();
        // row k /= pivot, with A[k][k] replaced by 1 first (in-place inverse)
        if (tid < n) A[k][tid] = (tid == k ? 1.0 : A[k][tid]) / piv;
        __syncthreads();
        // eliminate column k from every other row (its entries read first);
        // column k of row i becomes -A[i][k] / piv, the inverse's entry
        if (tid < n) col[tid] = A[tid][k];
        __syncthreads();
        for (int e = tid; e < n * n; e += 256) {
            const int i = e / n, j = e - i * n;
            if (i == k) continue;
            A[i][j] = (j == k ? 0.0 : A[i][j]) - col[i] * A[k][j];
        }
        __syncthreads();
    }
    // undo the row interchanges on the columns, last first
    for (int k = n - 1; k >= 0; --k) {
        const int p = ipiv[k];
        if (p != k)
            for (int i = tid; i < n; i += 256) {
                const double t = A[i][k];
                A[i][k] = A[i][p];
                A[i][p] = t;
            }
        __syncthreads();
    }
    double *out = inv + rn.off;
    for (int e = tid; e < n * n; e += 256) out[e] = A[e / n][e % n];
}

template <typename V>
__global__ __launch_bounds__(64) void k_bj_apply(const BJRun *__restrict__ runs, const double *__restrict__ inv,
                                                 int64_t N, const V *__restrict__ in, V *__restrict__ out)
{
    __shared__ double v[BJ_MAX];
    const BJRun rn = runs[blockIdx.x];
    const int r = blockIdx.y, i = threadIdx.x, n = rn.n;
    if (i < n) v[i] = double(in[r * N + rn.begin + i]);
    __syncthreads();
    if (i < n) {
        const double *a = inv + rn.off + size_t(i) * n;
        double acc = 0.0;
        for (int j = 0; j < n; ++j) acc += a[j] * v[j];
        out[r * N + rn.begin + i] = V(acc);
    }
}

}  // namespace

// The runs of every leaf and their inverses, once per tree.
imq_status precond_setup(imq_tree_s *t, hipStream_t s)
{
    if (t->nbj > 0) return IMQ_OK;
    const HostTree &h = t->h;
    std::vector<BJRun> runs;
    int64_t off = 0;
    for (int b : h.leaves)
        for (int i0 = h.begin[b]; i0 < h.end[b]; i0 += BJ_MAX) {
            const int n = std::min(BJ_MAX, h.end[b] - i0);
            runs.push_back(BJRun{i0, n, h.set[b], 0, off});
            off += int64_t(n) * n;
        }
    IMQ_HIP(dev_alloc(t->bj_runs, sizeof(BJRun) * runs.size()));
    IMQ_HIP(hipMemcpy(t->bj_runs.p, runs.data(), sizeof(BJRun) * runs.size(), hipMemcpyHostToDevice));
    IMQ_HIP(dev_alloc(t->bj_inv, sizeof(double) * size_t(std::max<int64_t>(off, 1))));
    if (!runs.empty())
        hipLaunchKernelGGL(k_bj_setup, dim3(unsigned(runs.size())), dim3(256), 0, s, t->bj_runs.as<BJRun>(),
                           t->perm.as<int32_t>(), t->xy_user.as<double>(), h.N,
                           t->cn.as<double>() + h.nsets, t->bj_inv.as<double>());
    IMQ_HIP(hipGetLastError());
    IMQ_HIP(hipStreamSynchronize(s));
    t->nbj = int(runs.size());
    return IMQ_OK;
}

// out = M^-1 in for nrhs columns of length N (tree point order); in != out.
template <typename V>
imq_status precond_apply(imq_tree_s *t, int nrhs, const V *in, V *out, hipStream_t s)
{
    if (t->nbj <= 0) return IMQ_OK;
    hipLaunchKernelGGL(k_bj_apply<V>, dim3(unsigned(t->nbj), unsigned(nrhs)), dim3(64), 0, s,
                       t->bj_runs.as<BJRun>(), t->bj_inv.as<double>(), t->h.N, in, out);
    IMQ_HIP(hipGetLastError());
    return IMQ_OK;
}

template imq_status precond_apply<float>(imq_tree_s *, int, const float *, float *, hipStream_t);
template imq_status precond_apply<double>(imq_tree_s *, int, const double *, double *, hipStream_t);

}  // namespace imq
