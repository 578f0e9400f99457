// Iterative solution of A a = f (Sec. 2, eq. interp_system) on the fast
// product: restarted GMRES for nrhs right-hand sides at once, and
// mixed-precision iterative refinement around an FP32-product GMRES.
//
// The paper only names an iterative method as the use of the product; the
// solver is the textbook one, batched over the columns: every Arnoldi step
// applies the fast product to all nrhs basis vectors in one call (the
// product carries nrhs columns through every stage), orthogonalises each
// column against its own basis with classical Gram-Schmidt applied twice
// (CGS2), and updates each column's Hessenberg matrix and Givens rotations
// on the device; the cycle ends for a column when its residual estimate
// |g_(j+1)| falls to tol ||f|| (the column is then frozen: later steps leave
// it untouched), and for all at the restart length.  The back-substitution
// and the update x += V y run on the device too; the explicit residual
// f - A x is recomputed at every restart.  All vectors stay in the tree's
// Morton order.
//
// Host synchronisation: one 4-byte copy per Arnoldi step (the number of
// columns still active), read one step late: the product of step j + 1 is
// queued before the host waits for step j's count, so the device never
// waits for the host inside a cycle; a step queued after every column
// converged changes nothing.  One synchronisation per restart reads the
// number of columns still to solve.
//
// Preconditioning (optional): the leaf block-Jacobi M of precond.hip on the
// right, A M^-1 y = f with x = M^-1 y, so the residual estimates and the
// explicit residuals stay those of A x = f.
//
// Precision: the FP64 solver keeps its basis in FP64; the inner solver of
// the refinement (FP32 products, inner tolerance >= 1e-6) keeps its basis in
// FP32, which halves the memory traffic of the orthogonalisation.  Dot
// products, the Hessenberg matrices and the rotations are FP64 in both.
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

constexpr int TPB = 256;

inline unsigned blocks_for(int64_t n) { return unsigned((n + TPB - 1) / TPB); }

// Vectors of nrhs columns: column c of x is x + c * n.
template <typename A, typename B>
__global__ void k_convert(int64_t n, const A *__restrict__ x, B *__restrict__ y)
{
    const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    const int64_t o = blockIdx.y * n;
    if (i < n) y[o + i] = B(x[o + i]);
}

// y = scale .* bs  (normalised-unit product -> caller units), in the type of y
template <typename V>
__global__ void k_scale(int64_t n, const double *__restrict__ bs, const double *__restrict__ sc,
                        V *__restrict__ y)
{
    const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    const int64_t o = blockIdx.y * n;
    if (i < n) y[o + i] = V(bs[o + i] * sc[i]);
}

// part[(c * nv + v) * nb + blk] = the block's share of V_v[c] . w[c], for
// the active columns; V_v[c] at Vb + (v * nrhs + c) * n.
template <typename V, typename W>
__global__ __launch_bounds__(TPB) void k_dots(int64_t n, int nrhs, int nv, const V *__restrict__ Vb,
                                              const W *__restrict__ w, const int *__restrict__ active,
                                              double *__restrict__ part)
{
    __shared__ double red[TPB];
    const int v = blockIdx.y, c = blockIdx.z;
    if (!active[c]) return;                          // uniform over the block
    const V *x = Vb + (size_t(v) * nrhs + c) * n;
    const W *y = w + size_t(c) * n;
    double s = 0.0;
    for (int64_t i = blockIdx.x * int64_t(TPB) + threadIdx.x; i < n; i += int64_t(gridDim.x) * TPB)
        s += double(x[i]) * double(y[i]);
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = TPB / 2; k > 0; k >>= 1) {
        if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[(size_t(c) * nv + v) * gridDim.x + blockIdx.x] = red[0];
}

// h[c * ldh + v] = sum of the partials of (c, v), in a fixed order
__global__ __launch_bounds__(TPB) void k_dots_final(int nv, int nb, const int *__restrict__ active,
                                                    const double *__restrict__ part, double *__restrict__ h,
                                                    int ldh)
{
    __shared__ double red[TPB];
    const int v = blockIdx.x, c = blockIdx.y;
    if (!active[c]) return;
    double s = 0.0;
    for (int b = threadIdx.x; b < nb; b += TPB) s += part[(size_t(c) * nv + v) * nb + b];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = TPB / 2; k > 0; k >>= 1) {
        if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) h[size_t(c) * ldh + v] = red[0];
}

// w[c] -= sum_v V_v[c] h[c * ldh + v]  (active columns)
template <typename V>
__global__ void k_sub_Vh(int64_t n, int nrhs, int nv, const V *__restrict__ Vb, const double *__restrict__ h,
                         int ldh, const int *__restrict__ active, V *__restrict__ w)
{
    const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    const int c = blockIdx.y;
    if (i >= n || !active[c]) return;
    double s = 0.0;
    for (int v = 0; v < nv; ++v) s += double(Vb[(size_t(v) * nrhs + c) * n + i]) * h[size_t(c) * ldh + v];
    w[size_t(c) * n + i] = V(double(w[size_t(c) * n + i]) - s);
}

// y[c] = x[c] / sqrt(nrm2[c])  (active columns; zero for a zero norm)
template <typename A, typename B>
__global__ void k_normalize(int64_t n, const A *__restrict__ x, const double *__restrict__ nrm2,
                            const int *__restrict__ active, B *__restrict__ y)
{
    const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    const int c = blockIdx.y;
    if (i >= n || !active[c]) return;
    const double nr = sqrt(nrm2[c]);
    y[size_t(c) * n + i] = B(nr > 0.0 ? double(x[size_t(c) * n + i]) / nr : 0.0);
}

// z[c] = x[c] - y[c]  (every column)
__global__ void k_sub(int64_t n, const double *__restrict__ x, const double *__restrict__ y, double *__restrict__ z)
{
    const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    const int64_t o = blockIdx.y * n;
    if (i < n) z[o + i] = x[o + i] - y[o + i];
}

// x[c] += y[c]
__global__ void k_add(int64_t n, const double *__restrict__ y, double *__restrict__ x)
{
    const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    const int64_t o = blockIdx.y * n;
    if (i < n) x[o + i] += y[o + i];
}

template <typename V>
__global__ void k_fill0(int64_t n, V *__restrict__ y)
{
    const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (i < n) y[blockIdx.y * n + i] = V(0);
}

// Per-column state of the solver (device).
struct ColState {
    double nf;       // ||rhs|| of the current system
    double thr;      // stop when the residual (estimate) falls to thr
    int k;           // basis vectors in use (steps taken this cycle)
    int iters;       // inner iterations of the current system
    int done;        // converged (or the rhs is zero)
    int hist0;       // history entries written by earlier systems (refinement)
};

// x[c] += sum_{v < k_c} V_v[c] y[c * ldy + v]
template <typename V>
__global__ void k_add_Vy(int64_t n, int nrhs, const V *__restrict__ Vb, const double *__restrict__ y, int ldy,
                         const ColState *__restrict__ st, double *__restrict__ x)
{
    const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    const int c = blockIdx.y;
    if (i >= n) return;
    const int kc = st[c].k;
    double s = 0.0;
    for (int v = 0; v < kc; ++v) s += double(Vb[(size_t(v) * nrhs + c) * n + i]) * y[size_t(c) * ldy + v];
    x[size_t(c) * n + i] += s;
}

__global__ void k_gather(int64_t n, const int32_t *__restrict__ perm, const double *__restrict__ x, int64_t ldx,
                         double *__restrict__ y)
{
    const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (i < n) y[blockIdx.y * n + i] = x[blockIdx.y * ldx + perm[i]];
}

__global__ void k_scatter(int64_t n, const int32_t *__restrict__ perm, const double *__restrict__ x,
                          double *__restrict__ y, int64_t ldy)
{
    const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (i < n) y[blockIdx.y * ldy + perm[i]] = x[blockIdx.y * n + i];
}

// Column state for a new system rhs: nf = ||rhs||, thr = tol_c nf, done
// when rhs = 0; the earlier systems' iterations move to hist0.
__global__ void k_state_init(int nrhs, const double *__restrict__ nrm2, const double *__restrict__ tol,
                             ColState *__restrict__ st)
{
    for (int c = threadIdx.x; c < nrhs; c += blockDim.x) {
        const double nf = sqrt(nrm2[c]);
        ColState &s = st[c];
        s.hist0 += s.iters;
        s.iters = 0;
        s.nf = nf;
        s.thr = tol[c] * nf;
        s.done = nf == 0.0;
        s.k = 0;
    }
}

// Start of a cycle: beta = ||r|| (nrm2 = ||r||^2), g = (beta, 0, ...), the
// column active unless converged; counts the active columns.
__global__ void k_cycle_start(int nrhs, int m, const double *__restrict__ nrm2, ColState *__restrict__ st,
                              double *__restrict__ g, int *__restrict__ active, int *__restrict__ nactive)
{
    __shared__ int cnt;
    if (threadIdx.x == 0) cnt = 0;
    __syncthreads();
    for (int c = threadIdx.x; c < nrhs; c += blockDim.x) {
        ColState &s = st[c];
        const double beta = sqrt(nrm2[c]);
        s.k = 0;
        g[size_t(c) * (m + 1)] = beta;
        const bool act = !s.done && beta > s.thr && beta > 0.0;
        if (!act) s.done = 1;
        active[c] = act;
        if (act) atomicAdd(&cnt, 1);
    }
    __syncthreads();
    if (threadIdx.x == 0) *nactive = cnt;
}

// Step j of every active column: Hessenberg column j = h1 + h2 (the two
// Gram-Schmidt passes) with ||w|| below the diagonal, the earlier rotations
// applied, a new rotation that zeroes the subdiagonal, the residual estimate
// |g_(j+1)|; a column whose estimate reaches its threshold, whose Krylov
// space is exhausted or whose cycle is full is frozen with k = j + 1.  One
// thread per column.
__global__ void k_givens(int nrhs, int m, int mc, int j, const double *__restrict__ h1,
                         const double *__restrict__ h2, const double *__restrict__ nrm2, double *__restrict__ H,
                         double *__restrict__ cs_, double *__restrict__ sn_, double *__restrict__ g,
                         ColState *__restrict__ st, int *__restrict__ active, double *__restrict__ hist,
                         int hist_cap, int *__restrict__ nactive)
{
    __shared__ int cnt;
    if (threadIdx.x == 0) cnt = 0;
    __syncthreads();
    for (int c = threadIdx.x; c < nrhs; c += blockDim.x) {
        if (!active[c]) continue;
        ColState &s = st[c];
        double *col = H + (size_t(c) * m + j) * (m + 1);
        double *cs = cs_ + size_t(c) * m, *sn = sn_ + size_t(c) * m, *gc = g + size_t(c) * (m + 1);
        for (int i = 0; i <= j; ++i) col[i] = h1[size_t(c) * (m + 1) + i] + h2[size_t(c) * (m + 1) + i];
        const double hn = sqrt(fmax(nrm2[c], 0.0));
        col[j + 1] = hn;
        for (int i = 0; i < j; ++i) {
            const double a = cs[i] * col[i] + sn[i] * col[i + 1];
            col[i + 1] = -sn[i] * col[i] + cs[i] * col[i + 1];
            col[i] = a;
        }
        const double den = hypot(col[j], col[j + 1]);
        cs[j] = den > 0 ? col[j] / den : 1.0;
        sn[j] = den > 0 ? col[j + 1] / den : 0.0;
        col[j] = den;
        col[j + 1] = 0.0;
        gc[j + 1] = -sn[j] * gc[j];
        gc[j] = cs[j] * gc[j];
        const double res = fabs(gc[j + 1]);
        const int it = s.hist0 + s.iters;
        if (hist && it < hist_cap) hist[size_t(c) * hist_cap + it] = s.nf > 0 ? res / s.nf : 0.0;
        s.iters += 1;
        s.k = j + 1;
        if (res <= s.thr || den == 0.0 || hn == 0.0 || j + 1 == mc)
            active[c] = 0;
        else
            atomicAdd(&cnt, 1);
    }
    __syncthreads();
    if (threadIdx.x == 0) *nactive = cnt;
}

// Back-substitution R y = g for each column (R the rotated Hessenberg
// matrix, k_c steps), one workgroup per column.
__global__ __launch_bounds__(TPB) void k_backsub(int m, const double *__restrict__ H, const double *__restrict__ g,
                                                 const ColState *__restrict__ st, double *__restrict__ y)
{
    __shared__ double red[TPB];
    const int c = blockIdx.x;
    const int k = st[c].k;
    const double *Hc = H + size_t(c) * m * (m + 1);
    const double *gc = g + size_t(c) * (m + 1);
    double *yc = y + size_t(c) * m;
    for (int i = k - 1; i >= 0; --i) {
        double s = 0.0;
        for (int l = i + 1 + threadIdx.x; l < k; l += TPB) s += Hc[size_t(l) * (m + 1) + i] * yc[l];
        red[threadIdx.x] = s;
        __syncthreads();
        for (int w = TPB / 2; w > 0; w >>= 1) {
            if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            const double d = Hc[size_t(i) * (m + 1) + i];
            yc[i] = d != 0.0 ? (gc[i] - red[0]) / d : 0.0;
        }
        __syncthreads();
    }
}

struct Solver {
    imq_tree_s *t;
    hipStream_t s;
    int64_t N;
    int nrhs, m, nb;
    void *Vraw, *wraw;                 // basis (m+1) x nrhs x N and one product block, FP64-sized
    double *tmp, *r, *x, *f, *d, *e;   // nrhs x N each
    void *zraw;                        // M^-1 of a basis vector (right preconditioning), FP64-sized
    bool pc = false;                   // leaf block-Jacobi right preconditioner
    double *h1, *h2, *nrm, *part, *H, *csn, *snn, *g, *y, *tolv;
    ColState *st;
    int *active, *active_all, *nact;
    double *hist = nullptr;            // device history (nrhs x hist_cap) or null
    int hist_cap = 0;
    int *hcount = nullptr;             // pinned host: active counts of two steps
    hipEvent_t ev[2] = {nullptr, nullptr};

    dim3 grid2() const { return dim3(blocks_for(N), unsigned(nrhs)); }

    // y = A x for the nrhs columns, product arithmetic T, vectors of type V
    template <typename T, typename V>
    imq_status apply(const V *xin, V *yout)
    {
        imq_status st_ = ensure_workspace<T>(t, nrhs);
        if (st_ != IMQ_OK) return st_;
        T *us = prec_data<T>(t).us.template as<T>();
        hipLaunchKernelGGL((k_convert<V, T>), grid2(), dim3(TPB), 0, s, N, xin, us);
        if ((st_ = fmm_sorted<T>(t, nrhs, s, nullptr)) != IMQ_OK) return st_;
        hipLaunchKernelGGL(k_scale<V>, grid2(), dim3(TPB), 0, s, N, t->bs.as<double>(), t->pt_scale.as<double>(),
                           yout);
        IMQ_HIP(hipGetLastError());
        return IMQ_OK;
    }

    // y = A M^-1 x (y = A x without the preconditioner)
    template <typename T, typename V>
    imq_status apply_pc(const V *xin, V *yout)
    {
        if (!pc) return apply<T, V>(xin, yout);
        V *z = static_cast<V *>(zraw);
        imq_status st_ = precond_apply<V>(t, nrhs, xin, z, s);
        if (st_ != IMQ_OK) return st_;
        return apply<T, V>(z, yout);
    }

    // hout[c * ldh + v] = V_v[c] . w[c], v < nv, for the columns act marks
    template <typename V, typename W>
    imq_status dots(const V *Vb, int nv, const W *w, double *hout, int ldh, const int *act)
    {
        hipLaunchKernelGGL((k_dots<V, W>), dim3(nb, nv, nrhs), dim3(TPB), 0, s, N, nrhs, nv, Vb, w, act, part);
        hipLaunchKernelGGL(k_dots_final, dim3(nv, nrhs), dim3(TPB), 0, s, nv, nb, act, part, hout, ldh);
        IMQ_HIP(hipGetLastError());
        return IMQ_OK;
    }

    // nrm[c] = ||v[c]||^2 for every column
    imq_status norms2(const double *v) { return dots<double, double>(v, 1, v, nrm, 1, active_all); }

    // Restarted GMRES for A_T x = rhs (nrhs columns, thresholds in st), x
    // in/out (FP64); at most maxit steps.
    template <typename T, typename V>
    imq_status gmres(const double *rhs, double *xs, int maxit, int &steps)
    {
        imq_status st_;
        V *Vb = static_cast<V *>(Vraw);
        V *w = static_cast<V *>(wraw);
        steps = 0;
        for (;;) {
            // r = rhs - A x, beta = ||r||, V_0 = r / beta
            if ((st_ = apply<T, double>(xs, tmp)) != IMQ_OK) return st_;
            hipLaunchKernelGGL(k_sub, grid2(), dim3(TPB), 0, s, N, rhs, tmp, r);
            if ((st_ = norms2(r)) != IMQ_OK) return st_;
            hipLaunchKernelGGL(k_cycle_start, dim3(1), dim3(TPB), 0, s, nrhs, m, nrm, st, g, active, nact);
            IMQ_HIP(hipGetLastError());
            IMQ_HIP(hipMemcpyAsync(hcount, nact, sizeof(int), hipMemcpyDeviceToHost, s));
            IMQ_HIP(hipStreamSynchronize(s));
            if (hcount[0] == 0 || steps >= maxit) return IMQ_OK;
            hipLaunchKernelGGL((k_normalize<double, V>), grid2(), dim3(TPB), 0, s, N, r, nrm, active, Vb);
            const int mc = std::min(m, maxit - steps);      // steps of this cycle
            if ((st_ = apply_pc<T, V>(Vb, w)) != IMQ_OK) return st_;
            int j = 0;
            while (j < mc) {
                V *vn = Vb + size_t(j + 1) * nrhs * N;
                // CGS2: two passes of classical Gram-Schmidt
                if ((st_ = dots(Vb, j + 1, w, h1, m + 1, active)) != IMQ_OK) return st_;
                hipLaunchKernelGGL(k_sub_Vh<V>, grid2(), dim3(TPB), 0, s, N, nrhs, j + 1, Vb, h1, m + 1, active, w);
                if ((st_ = dots(Vb, j + 1, w, h2, m + 1, active)) != IMQ_OK) return st_;
                hipLaunchKernelGGL(k_sub_Vh<V>, grid2(), dim3(TPB), 0, s, N, nrhs, j + 1, Vb, h2, m + 1, active, w);
                if ((st_ = dots(w, 1, w, nrm, 1, active)) != IMQ_OK) return st_;
                hipLaunchKernelGGL((k_normalize<V, V>), grid2(), dim3(TPB), 0, s, N, w, nrm, active, vn);
                hipLaunchKernelGGL(k_givens, dim3(1), dim3(TPB), 0, s, nrhs, m, mc, j, h1, h2, nrm, H, csn, snn, g,
                                   st, active, hist, hist_cap, nact);
                IMQ_HIP(hipGetLastError());
                IMQ_HIP(hipMemcpyAsync(hcount + (j & 1), nact, sizeof(int), hipMemcpyDeviceToHost, s));
                IMQ_HIP(hipEventRecord(ev[j & 1], s));
                // the next step's product runs while the host waits for this step's count
                if (j + 1 < mc)
                    if ((st_ = apply_pc<T, V>(vn, w)) != IMQ_OK) return st_;
                IMQ_HIP(hipEventSynchronize(ev[j & 1]));
                ++j;
                if (hcount[(j - 1) & 1] == 0) break;
            }
            steps += j;
            hipLaunchKernelGGL(k_backsub, dim3(nrhs), dim3(TPB), 0, s, m, H, g, st, y);
            if (!pc) {
                hipLaunchKernelGGL(k_add_Vy<V>, grid2(), dim3(TPB), 0, s, N, nrhs, Vb, y, m, st, xs);
            } else {                               // x += M^-1 (V y), through tmp and r (free here)
                hipLaunchKernelGGL(k_fill0<double>, grid2(), dim3(TPB), 0, s, N, tmp);
                hipLaunchKernelGGL(k_add_Vy<V>, grid2(), dim3(TPB), 0, s, N, nrhs, Vb, y, m, st, tmp);
                if ((st_ = precond_apply<double>(t, nrhs, tmp, r, s)) != IMQ_OK) return st_;
                hipLaunchKernelGGL(k_add, grid2(), dim3(TPB), 0, s, N, r, xs);
            }
            IMQ_HIP(hipGetLastError());
        }
    }

    // a new system rhs: per-column thresholds tolv_c ||rhs_c||
    imq_status set_system(const double *rhs)
    {
        imq_status st_ = norms2(rhs);
        if (st_ != IMQ_OK) return st_;
        hipLaunchKernelGGL(k_state_init, dim3(1), dim3(TPB), 0, s, nrhs, nrm, tolv, st);
        IMQ_HIP(hipGetLastError());
        return IMQ_OK;
    }
};

}  // namespace

imq_status solve_batched(imq_tree_s *t, int nrhs, const double *f_user, int64_t ldf, double *a_user, int64_t lda,
                         const imq_solve_opts &o, imq_solve_stats *stats, hipStream_t s)
{
    Solver S;
    S.t = t;
    S.s = s;
    S.N = t->h.N;
    S.nrhs = nrhs;
    S.m = o.restart;
    const int64_t N = S.N;
    const int m = o.restart;
    S.nb = int(std::min<int64_t>(512, std::max<int64_t>(1, (N + 4095) / 4096)));
    const size_t vecs = size_t(nrhs) * N;
    const size_t hist_cap = o.history ? size_t(o.max_iters) : 0;
    // device workspace: basis (m+1) blocks and one product block
    // (FP64-sized), six nrhs x N vectors, the per-column arrays, the
    // reduction partials, the history, the states and flags
    const size_t nsmall = size_t(nrhs) * (2 * size_t(m + 1) + 1 + size_t(m) * (m + 1) + 2 * size_t(m) + (m + 1) +
                                          m + 1) +
                          size_t(nrhs) * (m + 1) * S.nb + nrhs * hist_cap;
    const size_t need = sizeof(double) * (size_t(m + 2) * vecs + 7 * vecs + nsmall) + sizeof(ColState) * nrhs +
                        sizeof(int) * (2 * size_t(nrhs) + 2) + 256;
    if (t->sol_bytes < need) {
        IMQ_HIP(dev_alloc(t->sol, need));
        t->sol_bytes = need;
    }
    double *base = t->sol.as<double>();
    S.Vraw = base;
    S.wraw = base + size_t(m + 1) * vecs;
    S.tmp = base + size_t(m + 2) * vecs;
    S.r = S.tmp + vecs;
    S.x = S.r + vecs;
    S.f = S.x + vecs;
    S.d = S.f + vecs;
    S.e = S.d + vecs;
    S.zraw = S.e + vecs;
    double *p = S.e + 2 * vecs;
    S.h1 = p; p += size_t(nrhs) * (m + 1);
    S.h2 = p; p += size_t(nrhs) * (m + 1);
    S.nrm = p; p += nrhs;
    S.H = p; p += size_t(nrhs) * m * (m + 1);
    S.csn = p; p += size_t(nrhs) * m;
    S.snn = p; p += size_t(nrhs) * m;
    S.g = p; p += size_t(nrhs) * (m + 1);
    S.y = p; p += size_t(nrhs) * m;
    S.tolv = p; p += nrhs;
    S.part = p; p += size_t(nrhs) * (m + 1) * S.nb;
    if (hist_cap) {
        S.hist = p;
        S.hist_cap = int(hist_cap);
        p += nrhs * hist_cap;
    }
    S.st = reinterpret_cast<ColState *>(p);
    S.active = reinterpret_cast<int *>(S.st + nrhs);
    S.active_all = S.active + nrhs;
    S.nact = S.active_all + nrhs;

    IMQ_HIP(hipHostMalloc(reinterpret_cast<void **>(&S.hcount), sizeof(int) * 2, hipHostMallocDefault));
    struct Release {
        Solver &S;
        ~Release()
        {
            if (S.hcount) (void)hipHostFree(S.hcount);
            for (hipEvent_t e : S.ev)
                if (e) (void)hipEventDestroy(e);
        }
    } release{S};
    for (hipEvent_t &e : S.ev) IMQ_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));

    // host staging: ones (every column), a clean state, the tolerance
    {
        std::vector<int> ones(nrhs, 1);
        std::vector<ColState> st0(nrhs, ColState{0.0, 0.0, 0, 0, 0, 0});
        std::vector<double> tol(nrhs, o.tol);
        IMQ_HIP(hipMemcpyAsync(S.active_all, ones.data(), sizeof(int) * nrhs, hipMemcpyHostToDevice, s));
        IMQ_HIP(hipMemcpyAsync(S.st, st0.data(), sizeof(ColState) * nrhs, hipMemcpyHostToDevice, s));
        IMQ_HIP(hipMemcpyAsync(S.tolv, tol.data(), sizeof(double) * nrhs, hipMemcpyHostToDevice, s));
        IMQ_HIP(hipStreamSynchronize(s));    // the host vectors go out of scope
    }
    const int32_t *perm = t->perm.as<int32_t>();
    const dim3 g2 = S.grid2();
    if (hist_cap)
        hipLaunchKernelGGL(k_fill0<double>, dim3(blocks_for(int64_t(hist_cap)), unsigned(nrhs)), dim3(TPB), 0, s,
                           int64_t(hist_cap), S.hist);
    hipLaunchKernelGGL(k_gather, g2, dim3(TPB), 0, s, N, perm, f_user, ldf, S.f);
    hipLaunchKernelGGL(k_gather, g2, dim3(TPB), 0, s, N, perm, a_user, lda, S.x);
    IMQ_HIP(hipGetLastError());

    imq_status st;
    if (o.precond == 1) {
        if ((st = precond_setup(t, s)) != IMQ_OK) return st;
        S.pc = true;
    }
    int steps = 0, outer = 0;
    std::vector<double> nf(nrhs), nr(nrhs);
    if (!o.mixed_ir) {
        if ((st = S.set_system(S.f)) != IMQ_OK) return st;
        if ((st = S.gmres<double, double>(S.f, S.x, o.max_iters, steps)) != IMQ_OK) return st;
        outer = 1;
    } else {
        // refinement: d = f - A64 a in FP64, the correction e from FP32-product
        // GMRES to the relative accuracy the FP32 product can reach
        if ((st = S.norms2(S.f)) != IMQ_OK) return st;
        IMQ_HIP(hipMemcpyAsync(nf.data(), S.nrm, sizeof(double) * nrhs, hipMemcpyDeviceToHost, s));
        IMQ_HIP(hipStreamSynchronize(s));
        const int max_outer = o.max_outer > 0 ? o.max_outer : 10;
        std::vector<double> tol(nrhs);
        for (; outer < max_outer; ++outer) {
            if ((st = S.apply<double, double>(S.x, S.e)) != IMQ_OK) return st;
            hipLaunchKernelGGL(k_sub, g2, dim3(TPB), 0, s, N, S.f, S.e, S.d);
            if ((st = S.norms2(S.d)) != IMQ_OK) return st;
            IMQ_HIP(hipMemcpyAsync(nr.data(), S.nrm, sizeof(double) * nrhs, hipMemcpyDeviceToHost, s));
            IMQ_HIP(hipStreamSynchronize(s));
            bool all = true;
            for (int c = 0; c < nrhs; ++c) {
                const double a = std::sqrt(nf[c]), b = std::sqrt(nr[c]);
                const bool ok = a == 0.0 || b <= o.tol * a;
                all = all && ok;
                // a converged column gets threshold 1 (relative): no step is taken for it
                tol[c] = ok ? 1.0 : std::max(o.tol * a / b, 1e-6);
            }
            if (all || steps >= o.max_iters) break;
            IMQ_HIP(hipMemcpyAsync(S.tolv, tol.data(), sizeof(double) * nrhs, hipMemcpyHostToDevice, s));
            if ((st = S.set_system(S.d)) != IMQ_OK) return st;
            hipLaunchKernelGGL(k_fill0<double>, g2, dim3(TPB), 0, s, N, S.e);
            int inner = 0;
            if ((st = S.gmres<float, float>(S.d, S.e, o.max_iters - steps, inner)) != IMQ_OK) return st;
            steps += inner;
            hipLaunchKernelGGL(k_add, g2, dim3(TPB), 0, s, N, S.e, S.x);
            IMQ_HIP(hipGetLastError());
        }
    }
    // final explicit residual with the FP64 product
    if ((st = S.norms2(S.f)) != IMQ_OK) return st;
    IMQ_HIP(hipMemcpyAsync(nf.data(), S.nrm, sizeof(double) * nrhs, hipMemcpyDeviceToHost, s));
    if ((st = S.apply<double, double>(S.x, S.tmp)) != IMQ_OK) return st;
    hipLaunchKernelGGL(k_sub, g2, dim3(TPB), 0, s, N, S.f, S.tmp, S.r);
    if ((st = S.norms2(S.r)) != IMQ_OK) return st;
    IMQ_HIP(hipMemcpyAsync(nr.data(), S.nrm, sizeof(double) * nrhs, hipMemcpyDeviceToHost, s));
    std::vector<ColState> fin(nrhs);
    IMQ_HIP(hipMemcpyAsync(fin.data(), S.st, sizeof(ColState) * nrhs, hipMemcpyDeviceToHost, s));
    hipLaunchKernelGGL(k_scatter, g2, dim3(TPB), 0, s, N, perm, S.x, a_user, lda);
    IMQ_HIP(hipGetLastError());
    if (hist_cap)
        IMQ_HIP(hipMemcpyAsync(o.history, S.hist, sizeof(double) * nrhs * hist_cap, hipMemcpyDeviceToHost, s));
    IMQ_HIP(hipStreamSynchronize(s));
    for (int c = 0; c < nrhs; ++c) {
        imq_solve_stats &x = stats[c];
        x.iters = fin[c].hist0 + fin[c].iters;
        x.outer_iters = outer;
        x.relres_fast64 = nf[c] > 0 ? std::sqrt(nr[c] / nf[c]) : 0.0;
        x.converged = x.relres_fast64 <= o.tol;
    }
    return IMQ_OK;
}

}  // namespace imq
