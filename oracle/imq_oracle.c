/*
 * FP64 dense CPU oracle for the inverse-multiquadric (IMQ) interpolation
 * matrix.  TEST INFRASTRUCTURE ONLY: it is called by the test-suite, by the
 * smoke check and by the CPU-baseline leg of the benchmark, never by the
 * library.  It shares no code, header or table with the GPU path.
 *
 * What it computes is the plain definition of the operator, evaluated
 * entry by entry:
 *
 *   A_ij = 1 / sqrt(|x_i - y_j|^2 + c^2)           (Sec. 2, eq. IMQ_def;
 *                                                    entries of eq. interp_system)
 *   b_i  = sum_j A_ij u_j                            (the product b = A u that
 *                                                    Algorithm 1 approximates)
 *
 * Each entry is evaluated in IEEE double precision in exactly the order
 * dx*dx + dy*dy + c*c, then sqrt, then a division (build with
 * -ffp-contract=off so no fused multiply-add changes the rounding).  The
 * row sums use Neumaier's compensated summation in ascending j; a second,
 * pairwise summation order is provided so the two can be compared.
 *
 * The gradient routine differentiates the scalar loss
 *   L(v, c, X) = || A(c, X) v - f ||^2,  g = dL/d(Av) = 2 (A v - f)
 * from the entry formula above:
 *   dL/dv   = A g                               (A is symmetric)
 *   dL/dc   = -c sum_ij g_i v_j (r_ij^2 + c^2)^(-3/2)
 *   dL/dx_k = -sum_j (g_k v_j + v_k g_j) (x_k - x_j) (r_kj^2 + c^2)^(-3/2)
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct { double s, comp; } neumaier;

static inline void nm_add(neumaier *a, double t)
{
    double tmp = a->s + t;
    if (fabs(a->s) >= fabs(t))
        a->comp += (a->s - tmp) + t;
    else
        a->comp += (t - tmp) + a->s;
    a->s = tmp;
}

static inline double nm_val(const neumaier *a) { return a->s + a->comp; }

/* One matrix entry, in the documented order of operations. */
static inline double imq_entry(double xi, double yi, double xj, double yj, double c)
{
    double dx = xi - xj;
    double dy = yi - yj;
    double s = dx * dx + dy * dy + c * c;
    return 1.0 / sqrt(s);
}

int imq_oracle_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads of the following parallel loops (n >= 1); the arithmetic of every
 * row is the same whatever the count. */
void imq_oracle_set_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/*
 * b[r*ldb + i] = sum_j A(t_i, s_j) u[r*ldu + j]  for i < nt, r < nrhs.
 * Targets (xt, yt) and sources (xs, ys) may be the same arrays.
 */
void imq_oracle_matvec(int64_t nt, const double *xt, const double *yt,
                       int64_t ns, const double *xs, const double *ys,
                       int nrhs, const double *u, int64_t ldu, double c,
                       double *b, int64_t ldb)
{
    #pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < nt; ++i) {
        for (int r = 0; r < nrhs; ++r) {
            const double *ur = u + (int64_t)r * ldu;
            neumaier acc = {0.0, 0.0};
            for (int64_t j = 0; j < ns; ++j)
                nm_add(&acc, imq_entry(xt[i], yt[i], xs[j], ys[j], c) * ur[j]);
            b[(int64_t)r * ldb + i] = nm_val(&acc);
        }
    }
}

/* Plain pairwise (recursive halving) summation of the same products. */
static double pairwise_row(double xi, double yi, const double *xs, const double *ys,
                           const double *u, int64_t lo, int64_t hi, double c)
{
    if (hi - lo <= 8) {
        double s = 0.0;
        for (int64_t j = lo; j < hi; ++j)
            s += imq_entry(xi, yi, xs[j], ys[j], c) * u[j];
        return s;
    }
    int64_t mid = lo + (hi - lo) / 2;
    return pairwise_row(xi, yi, xs, ys, u, lo, mid, c) +
           pairwise_row(xi, yi, xs, ys, u, mid, hi, c);
}

void imq_oracle_matvec_pairwise(int64_t n, const double *xs, const double *ys,
                                const double *u, double c, double *b)
{
    #pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; ++i)
        b[i] = pairwise_row(xs[i], ys[i], xs, ys, u, 0, n, c);
}

/*
 * Gradient of L = ||A v - f||^2 given g = 2 (A v - f):
 *   dv[k] = (A g)_k,  *dc = dL/dc,  dx[k], dy[k] = dL/dx_k.
 */
void imq_oracle_grad(int64_t n, const double *xs, const double *ys, double c,
                     const double *v, const double *g,
                     double *dv, double *dc, double *dx, double *dy)
{
    double *rowc = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    #pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < n; ++k) {
        neumaier ag = {0, 0}, vw = {0, 0};
        neumaier vx = {0, 0}, vy = {0, 0}, gx = {0, 0}, gy = {0, 0};
        for (int64_t j = 0; j < n; ++j) {
            double ddx = xs[k] - xs[j];
            double ddy = ys[k] - ys[j];
            double s = ddx * ddx + ddy * ddy + c * c;
            double q = sqrt(s);
            double a = 1.0 / q;            /* A_kj          */
            double w = 1.0 / (s * q);      /* (r^2+c^2)^-3/2 */
            nm_add(&ag, a * g[j]);
            nm_add(&vw, v[j] * w);
            nm_add(&vx, v[j] * ddx * w);
            nm_add(&vy, v[j] * ddy * w);
            nm_add(&gx, g[j] * ddx * w);
            nm_add(&gy, g[j] * ddy * w);
        }
        dv[k] = nm_val(&ag);
        rowc[k] = g[k] * nm_val(&vw);
        dx[k] = -(g[k] * nm_val(&vx) + v[k] * nm_val(&gx));
        dy[k] = -(g[k] * nm_val(&vy) + v[k] * nm_val(&gy));
    }
    neumaier tot = {0, 0};
    for (int64_t k = 0; k < n; ++k)
        nm_add(&tot, rowc[k]);
    *dc = -c * nm_val(&tot);
    free(rowc);
}
