// FP64 generation of the translation tables of the lifted-Laplace expansion.
//
// Solid harmonics (Sec. 2.1, eq. GreenDecompositionG, written with complex
// exponentials): with P_n^m the unnormalised associated Legendre function
// (Condon-Shortley sign included) and r = (rho, theta, omega),
//     R_n^m(r) = rho^n P_n^m(cos theta) e^{i m omega} / (n+m)!      (regular)
//     I_n^m(r) = (n-m)! P_n^m(cos theta) e^{i m omega} / rho^(n+1)  (irregular)
// and R_n^{-m} = (-1)^m conj(R_n^m), I_n^{-m} = (-1)^m conj(I_n^m).  Summing
// conj(R_n^m(y)) I_n^m(x) over -n <= m <= n gives, term by term in n, the
// m >= 0 sum of eq. GreenDecompositionG with the Neumann factor eps_m and
// d_{n,m} = (n-m)!/(n+m)! (eq. dec_separata); so 1/|x - y| is
// sum_{n,m} conj(R_n^m(y)) I_n^m(x) for |y| < |x|.
//
// From this addition theorem and the corresponding shift identities for
// solid harmonics (the standard ones of the fast multipole literature the
// paper builds on, Greengard-Rokhlin), for centres z:
//     multipole  M_n^m = sum_j u_j conj(R_n^m(y_j - z))
//     shift      M'_n^m = sum_{j,k} M_j^k conj(R_{n-j}^{m-k}(z - z'))
//     translate  L_j^k  = sum_{n,m} (-1)^(j+k) I_{n+j}^{m-k}(z_t - z_s) M_n^m
//     shift      L'_j^k = sum_{n,m} L_n^m R_{n-j}^{m-k}(z' - z)
//     evaluate   phi(x) = sum_{j,k} L_j^k R_j^k(x - z_t)
// The tables below are these maps written as real matrices on the stored
// n+m-even coefficients (see imq_internal.h for the layout and scaling).
#include "imq_internal.h"

#include <cmath>
#include <complex>
#include <vector>

namespace imq {

using cplx = std::complex<double>;

static inline int tri(int n, int m) { return n * (n + 1) / 2 + m; }
static inline int ire(int n, int m) { return n * (n + 1) / 2 + (m > 0 ? m - 1 : 0); }

double legendre_at_zero(int n, int m)
{
    if (m < 0 || m > n || ((n + m) & 1)) return 0.0;
    double num = 1.0, den = 1.0;
    for (int k = n + m - 1; k > 1; k -= 2) num *= k;   // (n+m-1)!!
    for (int k = n - m; k > 1; k -= 2) den *= k;       // (n-m)!!
    double v = num / den;
    return (((n + m) / 2) & 1) ? -v : v;
}

static double factorial(int n)
{
    double f = 1.0;
    for (int k = 2; k <= n; ++k) f *= k;
    return f;
}

// c_{n,m} = P_n^m(0) / (n+m)!
static double cnm(int n, int m) { return legendre_at_zero(n, m) / factorial(n + m); }
static double eps(int m) { return m == 0 ? 1.0 : 2.0; }
double legendre_coef(int n, int m) { return cnm(n, m); }

// Regular solid harmonics R_n^m, 0 <= m <= n <= N, by the Cartesian
// recurrences R_m^m = -(x+iy)/(2m) R_{m-1}^{m-1},
// (n+m)(n-m) R_n^m = (2n-1) z R_{n-1}^m - |r|^2 R_{n-2}^m.
static void regular_all(int N, double x, double y, double z, std::vector<cplx> &R)
{
    R.assign((N + 1) * (N + 2) / 2, cplx(0, 0));
    const double r2 = x * x + y * y + z * z;
    const cplx xy(x, y);
    cplx rmm(1, 0);
    for (int m = 0; m <= N; ++m) {
        if (m > 0) rmm = -xy * rmm / (2.0 * m);
        R[tri(m, m)] = rmm;
        if (m + 1 <= N) R[tri(m + 1, m)] = z * rmm;
        for (int n = m + 2; n <= N; ++n)
            R[tri(n, m)] = ((2.0 * n - 1) * z * R[tri(n - 1, m)] - r2 * R[tri(n - 2, m)]) /
                           (double((n + m) * (n - m)));
    }
}

// Irregular solid harmonics I_n^m by I_0^0 = 1/|r|,
// I_m^m = -(2m-1)(x+iy)/|r|^2 I_{m-1}^{m-1},
// |r|^2 I_n^m = (2n-1) z I_{n-1}^m - (n+m-1)(n-m-1) I_{n-2}^m.
static void irregular_all(int N, double x, double y, double z, std::vector<cplx> &I)
{
    I.assign((N + 1) * (N + 2) / 2, cplx(0, 0));
    const double r2 = x * x + y * y + z * z;
    const double inv_r2 = 1.0 / r2;
    const cplx xy(x, y);
    cplx imm(1.0 / std::sqrt(r2), 0);
    for (int m = 0; m <= N; ++m) {
        if (m > 0) imm = -(2.0 * m - 1) * xy * inv_r2 * imm;
        I[tri(m, m)] = imm;
        if (m + 1 <= N) I[tri(m + 1, m)] = (2.0 * m + 1) * z * inv_r2 * imm;
        for (int n = m + 2; n <= N; ++n)
            I[tri(n, m)] = ((2.0 * n - 1) * z * I[tri(n - 1, m)] -
                            double((n + m - 1) * (n - m - 1)) * I[tri(n - 2, m)]) * inv_r2;
    }
}

// Value at any order m (|m| <= n) from the m >= 0 table.
static cplx at(const std::vector<cplx> &H, int N, int n, int m)
{
    if (n < 0 || n > N || m > n || -m > n) return cplx(0, 0);
    if (m >= 0) return H[tri(n, m)];
    cplx v = std::conj(H[tri(n, -m)]);
    return (m & 1) ? -v : v;
}

static inline double sgn(int k) { return (k & 1) ? -1.0 : 1.0; }

// Write the four real entries that a complex-linear coefficient pair
// (A1 acting on M, A2 acting on conj(M)) contributes for output (jo, ko)
// and input (ni, mi), with output scale so.
static void put(double *T, int K, int jo, int ko, int ni, int mi, cplx A1, cplx A2, double so)
{
    const int r = ire(jo, ko), c = ire(ni, mi);
    const cplx sum = A1 + A2, dif = A1 - A2;
    T[r * K + c] += so * sum.real();
    if (mi > 0) T[r * K + c + 1] += -so * dif.imag();
    if (ko > 0) {
        T[(r + 1) * K + c] += so * sum.imag();
        if (mi > 0) T[(r + 1) * K + c + 1] += so * dif.real();
    }
}

static void child_offset(int pos, double &dx, double &dy)
{
    dx = (pos & 1) ? 0.25 : -0.25;
    dy = (pos & 2) ? 0.25 : -0.25;
}

void make_m2m_table(int p, int pos, double *T)
{
    const int K = Kof(p);
    for (int i = 0; i < K * K; ++i) T[i] = 0.0;
    double dx, dy;
    child_offset(pos, dx, dy);
    std::vector<cplx> R;
    regular_all(p, dx, dy, 0.0, R);              // d = child - parent, parent edge 1
    for (int n = 0; n <= p; ++n)
        for (int m = n & 1; m <= n; m += 2) {
            const double so = 1.0 / cnm(n, m);
            for (int j = 0; j <= n; ++j)
                for (int k = j & 1; k <= j; k += 2) {
                    const double si = cnm(j, k) * std::ldexp(1.0, -j);   // child edge 1/2
                    cplx B1 = si * std::conj(at(R, p, n - j, m - k));
                    cplx B2 = (k > 0) ? sgn(k) * si * std::conj(at(R, p, n - j, m + k)) : cplx(0, 0);
                    put(T, K, n, m, j, k, B1, B2, so);
                }
        }
}

void make_l2l_table(int p, int pos, double *T)
{
    const int K = Kof(p);
    for (int i = 0; i < K * K; ++i) T[i] = 0.0;
    double dx, dy;
    child_offset(pos, dx, dy);
    std::vector<cplx> R;
    regular_all(p, dx, dy, 0.0, R);
    for (int j = 0; j <= p; ++j)
        for (int k = j & 1; k <= j; k += 2) {
            const double so = eps(k) * cnm(j, k) * std::ldexp(1.0, -j);
            for (int n = j; n <= p; ++n)
                for (int m = n & 1; m <= n; m += 2) {
                    const double si = 1.0 / (eps(m) * cnm(n, m));
                    cplx C1 = si * at(R, p, n - j, m - k);
                    cplx C2 = (m > 0) ? sgn(m) * si * at(R, p, n - j, -m - k) : cplx(0, 0);
                    put(T, K, j, k, n, m, C1, C2, so);
                }
        }
}

void make_m2l_table(int p, int level, int dx, int dy, double cnorm, double *T)
{
    const int K = Kof(p);
    for (int i = 0; i < K * K; ++i) T[i] = 0.0;
    const double scale = std::ldexp(1.0, level);     // 1/s at this level
    std::vector<cplx> I;
    // target centre minus source centre, in units of the box edge: the
    // lifted planes put the target c above the source.
    irregular_all(2 * p, double(dx), double(dy), cnorm * scale, I);
    for (int j = 0; j <= p; ++j)
        for (int k = j & 1; k <= j; k += 2) {
            const double so = eps(k) * cnm(j, k) * scale;
            for (int n = 0; n <= p; ++n)
                for (int m = n & 1; m <= n; m += 2) {
                    const double si = cnm(n, m) * sgn(j + k);
                    cplx A1 = si * at(I, 2 * p, n + j, m - k);
                    cplx A2 = (m > 0) ? sgn(m) * si * at(I, 2 * p, n + j, -m - k) : cplx(0, 0);
                    put(T, K, j, k, n, m, A1, A2, so);
                }
        }
}

void make_wx_consts(int p, double *w)
{
    for (int n = 0; n <= p; ++n)
        for (int m = n & 1; m <= n; m += 2) {
            const double v = eps(m) * cnm(n, m);
            w[ire(n, m)] = v;
            if (m > 0) w[ire(n, m) + 1] = v;
        }
}

// ---- vertical derivative (adjoint with respect to the shape parameter)
//
// Moving a target vertically changes its lifted separation from the sources,
// so d/dc of the potential is the z-derivative of the local expansion at the
// target plane.  With d/dz R_j^k = R_{j-1}^k, only the n+m-odd local
// coefficients contribute there:
//     dphi/dz (x) = sum_{j+k odd} Re(Lo[j,k] |w|^(j-1-k) w^k),  w = (x - z)/s,
// stored in the odd layout  idx_odd(j, k) = j(j-1)/2 + max(k-1, 0)  (j >= 1),
// p(p+1)/2 real numbers.  Rows of these tables are odd coefficients; the
// K x K buffers are filled in their first p(p+1)/2 rows (and, for the local
// shift, columns).
static inline int iro(int j, int k) { return j * (j - 1) / 2 + (k > 0 ? k - 1 : 0); }

static void put2(double *T, int K, int r, bool rim, int c, bool cim, cplx A1, cplx A2, double so)
{
    const cplx sum = A1 + A2, dif = A1 - A2;
    T[r * K + c] += so * sum.real();
    if (cim) T[r * K + c + 1] += -so * dif.imag();
    if (rim) {
        T[(r + 1) * K + c] += so * sum.imag();
        if (cim) T[(r + 1) * K + c + 1] += so * dif.real();
    }
}

void make_m2l_odd_table(int p, int level, int dx, int dy, double cnorm, double *T)
{
    const int K = Kof(p);
    for (int i = 0; i < K * K; ++i) T[i] = 0.0;
    const double scale = std::ldexp(1.0, level);
    std::vector<cplx> I;
    irregular_all(2 * p, double(dx), double(dy), cnorm * scale, I);
    for (int j = 1; j <= p; ++j)
        for (int k = (j + 1) & 1; k <= j - 1; k += 2) {
            const double so = eps(k) * cnm(j - 1, k) * scale * scale;
            for (int n = 0; n <= p; ++n)
                for (int m = n & 1; m <= n; m += 2) {
                    const double si = cnm(n, m) * sgn(j + k);
                    cplx A1 = si * at(I, 2 * p, n + j, m - k);
                    cplx A2 = (m > 0) ? sgn(m) * si * at(I, 2 * p, n + j, -m - k) : cplx(0, 0);
                    put2(T, K, iro(j, k), k > 0, ire(n, m), m > 0, A1, A2, so);
                }
        }
}

void make_l2l_odd_table(int p, int pos, double *T)
{
    const int K = Kof(p);
    for (int i = 0; i < K * K; ++i) T[i] = 0.0;
    double dx, dy;
    child_offset(pos, dx, dy);
    std::vector<cplx> R;
    regular_all(p, dx, dy, 0.0, R);
    for (int j = 1; j <= p; ++j)
        for (int k = (j + 1) & 1; k <= j - 1; k += 2) {
            const double so = eps(k) * cnm(j - 1, k) * std::ldexp(1.0, -(j - 1));
            for (int n = j; n <= p; ++n)
                for (int m = (n + 1) & 1; m <= n - 1; m += 2) {
                    const double si = 1.0 / (eps(m) * cnm(n - 1, m));
                    cplx C1 = si * at(R, p, n - j, m - k);
                    cplx C2 = (m > 0) ? sgn(m) * si * at(R, p, n - j, -m - k) : cplx(0, 0);
                    put2(T, K, iro(j, k), k > 0, iro(n, m), m > 0, C1, C2, so);
                }
        }
}

}  // namespace imq
