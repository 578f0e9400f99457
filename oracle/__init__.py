"""Plain FP64 CPU oracle for the IMQ interpolation matrix and its product.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this package.  The GPU
library never uses it, and it shares no code with the GPU library: it
neither imports the library nor is imported by it.

Contents (each follows the passage of the paper named in its docstring):

* O1 ``dense_matrix``      entries of A, eq. (IMQ_def) / eq. (interp_system)
* O2 ``matvec``            b = A u, compensated FP64 row sums (C, OpenMP)
* O3 ``solve_dense``       direct solve of A a = f (eq. interp_system)
* O4 ``relres``            true relative residual ||f - A a|| / ||f||
* O5 ``series_truncated``  the truncated spectral series, eq. (serieTroncata)
     ``legendre_table``    unnormalised associated Legendre functions P_n^m
     ``thm21_bound``       the truncation bound of Theorem 2.1
* O6 ``grad``              dense gradient of ||A(c,X) v - f||^2
* O7 ``gmres``             plain restarted GMRES (textbook Arnoldi + Givens)

Everything is FP64.  Functions the C library provides fall back to nothing:
if gcc is unavailable they raise.
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

from . import build as _build

_lib = None


def _load():
    global _lib
    if _lib is None:
        path = _build.LIB
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_build.SRC):
            _build.build()
        lib = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        i64 = ctypes.c_int64
        lib.imq_oracle_matvec.argtypes = [i64, dp, dp, i64, dp, dp, ctypes.c_int, dp, i64,
                                          ctypes.c_double, dp, i64]
        lib.imq_oracle_matvec.restype = None
        lib.imq_oracle_matvec_pairwise.argtypes = [i64, dp, dp, dp, ctypes.c_double, dp]
        lib.imq_oracle_matvec_pairwise.restype = None
        lib.imq_oracle_grad.argtypes = [i64, dp, dp, ctypes.c_double, dp, dp, dp, dp, dp, dp]
        lib.imq_oracle_grad.restype = None
        lib.imq_oracle_threads.argtypes = []
        lib.imq_oracle_threads.restype = ctypes.c_int
        lib.imq_oracle_set_threads.argtypes = [ctypes.c_int]
        lib.imq_oracle_set_threads.restype = None
        _lib = lib
    return _lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def threads() -> int:
    """Number of OpenMP threads the C oracle runs with."""
    return int(_load().imq_oracle_threads())


def set_threads(n: int) -> None:
    """Run the C oracle's loops on n threads (results do not depend on n)."""
    _load().imq_oracle_set_threads(int(n))


# ----------------------------------------------------------------------------
# O1, O2, O4: the matrix and its product
# ----------------------------------------------------------------------------

def dense_matrix(xy, c: float, xy_targets=None) -> np.ndarray:
    """Explicit A with A_ij = 1/sqrt(|x_i - x_j|^2 + c^2).

    Sec. 2, eq. (IMQ_def) for phi and eq. (interp_system) for the entries.
    Rows are targets (default: the data sites), columns the centres.
    """
    xy = _f64(xy)
    t = xy if xy_targets is None else _f64(xy_targets)
    dx = t[:, 0][:, None] - xy[:, 0][None, :]
    dy = t[:, 1][:, None] - xy[:, 1][None, :]
    s = dx * dx + dy * dy + c * c
    return 1.0 / np.sqrt(s)


def matvec(xy, c: float, u, xy_targets=None) -> np.ndarray:
    """b = A u by compensated row sums (C, OpenMP).

    ``u`` is (N,) or (nrhs, N); ``b`` has the matching shape.  Targets
    default to the data sites (the square interpolation matrix, Sec. 2).
    """
    xy = _f64(xy)
    t = xy if xy_targets is None else _f64(xy_targets)
    u = _f64(u)
    one = u.ndim == 1
    u2 = u[None, :] if one else u
    nrhs, ns = u2.shape
    if ns != len(xy):
        raise ValueError("u has the wrong length")
    xs, ys = _f64(xy[:, 0]), _f64(xy[:, 1])
    xt, yt = _f64(t[:, 0]), _f64(t[:, 1])
    b = np.empty((nrhs, len(t)))
    _load().imq_oracle_matvec(len(t), _dp(xt), _dp(yt), ns, _dp(xs), _dp(ys),
                              nrhs, _dp(u2), ns, float(c), _dp(b), len(t))
    return b[0] if one else b


def matvec_pairwise(xy, c: float, u) -> np.ndarray:
    """b = A u with plain pairwise summation (a second summation order)."""
    xy = _f64(xy)
    u = _f64(u)
    xs, ys = _f64(xy[:, 0]), _f64(xy[:, 1])
    b = np.empty(len(xy))
    _load().imq_oracle_matvec_pairwise(len(xy), _dp(xs), _dp(ys), _dp(u), float(c), _dp(b))
    return b


def relres(xy, c: float, a, f) -> float:
    """True relative residual ||f - A a||_2 / ||f||_2 (O4)."""
    r = _f64(f) - matvec(xy, c, a)
    return float(np.linalg.norm(r) / np.linalg.norm(f))


# ----------------------------------------------------------------------------
# O3: direct solve
# ----------------------------------------------------------------------------

def solve_dense(xy, c: float, f):
    """Solve A a = f (eq. interp_system) directly.

    Cholesky first (A is symmetric positive definite for distinct points);
    if the factorisation fails in floating point, LU with partial pivoting.
    Returns (a, method).
    """
    A = dense_matrix(xy, c)
    f = _f64(f)
    try:
        L = np.linalg.cholesky(A)
        y = _lower_solve(L, f)
        a = _lower_solve(L, y, transpose=True)
        return a, "cholesky"
    except np.linalg.LinAlgError:
        return np.linalg.solve(A, f), "lu"


def _lower_solve(L, b, transpose=False):
    import scipy.linalg
    return scipy.linalg.solve_triangular(L, b, lower=True, trans=1 if transpose else 0)


# ----------------------------------------------------------------------------
# O5: the truncated spectral series of Sec. 2.1
# ----------------------------------------------------------------------------

def legendre_table(nmax: int, x: float) -> np.ndarray:
    """Unnormalised associated Legendre functions P_n^m(x), 0 <= m <= n <= nmax.

    Standard upward recurrence in n at fixed m, seeded at
    P_m^m(x) = (-1)^m (2m-1)!! (1-x^2)^(m/2) and
    P_{m+1}^m(x) = (2m+1) x P_m^m(x), then
    (n-m) P_n^m = (2n-1) x P_{n-1}^m - (n+m-1) P_{n-2}^m.
    (The Condon-Shortley sign (-1)^m cancels in every product P_n^m P_n^m
    of the series.)  Returns an (nmax+1, nmax+1) array, zero above m > n.
    """
    P = np.zeros((nmax + 1, nmax + 1))
    s = math.sqrt(max(0.0, 1.0 - x * x))
    pmm = 1.0
    for m in range(nmax + 1):
        if m > 0:
            pmm = -pmm * (2 * m - 1) * s
        P[m, m] = pmm
        if m + 1 <= nmax:
            P[m + 1, m] = (2 * m + 1) * x * pmm
        for n in range(m + 2, nmax + 1):
            P[n, m] = ((2 * n - 1) * x * P[n - 1, m] - (n + m - 1) * P[n - 2, m]) / (n - m)
    return P


def spherical(X):
    """(rho, theta, omega) of a point of R^3; theta from the third axis.

    At rho = 0 the angles are taken as theta = 0, omega = 0.
    """
    x, y, z = (float(v) for v in X)
    rho = math.sqrt(x * x + y * y + z * z)
    if rho == 0.0:
        return 0.0, 0.0, 0.0
    theta = math.acos(max(-1.0, min(1.0, z / rho)))
    omega = math.atan2(y, x) % (2 * math.pi)
    return rho, theta, omega


def neumann(m: int) -> float:
    """Neumann factor: 1 for m = 0, 2 for m > 0."""
    return 1.0 if m == 0 else 2.0


def series_truncated(X, Y, M: int) -> float:
    """Sum of eq. (serieTroncata) for n = 0..M (Sec. 2.1).

    G(X;Y) ~ sum_n sum_{m<=n} eps_m (n-m)!/(n+m)! P_n^m(cos th_y) P_n^m(cos th_x)
             cos(m (om_x - om_y)) * (rho_<^n / rho_>^(n+1)),
    with the branch chosen by which of rho_x, rho_y is larger.
    """
    rx, tx, ox = spherical(X)
    ry, ty, oy = spherical(Y)
    if rx == ry:
        raise ValueError("series undefined for rho_x == rho_y")
    Px = legendre_table(M, math.cos(tx))
    Py = legendre_table(M, math.cos(ty))
    rin, rout = (ry, rx) if ry < rx else (rx, ry)
    total = 0.0
    for n in range(M + 1):
        radial = rin ** n / rout ** (n + 1)
        for m in range(n + 1):
            d = neumann(m) * math.factorial(n - m) / math.factorial(n + m)
            total += d * Py[n, m] * Px[n, m] * math.cos(m * (ox - oy)) * radial
    return total


def addition_theorem_term(X, Y, n: int) -> float:
    """sum_m eps_m (n-m)!/(n+m)! P_n^m(cos th_y) P_n^m(cos th_x) cos(m dw).

    The addition theorem (used in the proof of Theorem 2.1) says this equals
    the Legendre polynomial P_n(cos alpha), alpha the angle between X and Y.
    """
    _, tx, ox = spherical(X)
    _, ty, oy = spherical(Y)
    Px = legendre_table(n, math.cos(tx))
    Py = legendre_table(n, math.cos(ty))
    return sum(neumann(m) * math.factorial(n - m) / math.factorial(n + m)
               * Py[n, m] * Px[n, m] * math.cos(m * (ox - oy)) for m in range(n + 1))


def thm21_bound(rho_x: float, rho_y: float, M: int) -> float:
    """Theorem 2.1: E <= (1/rho_>) r^(M+1) / (1 - r), r = rho_< / rho_>."""
    rin, rout = min(rho_x, rho_y), max(rho_x, rho_y)
    r = rin / rout
    return r ** (M + 1) / ((1.0 - r) * rout)


# ----------------------------------------------------------------------------
# O6: gradients of L = ||A(c, X) v - f||^2
# ----------------------------------------------------------------------------

def loss(xy, c: float, v, f) -> float:
    r = matvec(xy, c, v) - _f64(f)
    return float(r @ r)


def grad(xy, c: float, v, f):
    """(dL/dv, dL/dc, dL/dX) for L = ||A(c,X) v - f||^2, dense FP64 (C).

    With g = 2 (A v - f): dL/dv = A g; dL/dc = -c sum_ij g_i v_j s_ij^(-3/2);
    dL/dx_k = -sum_j (g_k v_j + v_k g_j)(x_k - x_j) s_kj^(-3/2), where
    s_ij = |x_i - x_j|^2 + c^2 (derivatives of eq. IMQ_def).
    """
    xy = _f64(xy)
    v = _f64(v)
    g = 2.0 * (matvec(xy, c, v) - _f64(f))
    return grad_given_g(xy, c, v, g)


def grad_given_g(xy, c: float, v, g):
    """Same as :func:`grad` but with the upstream g = dL/d(Av) given."""
    xy = _f64(xy)
    v, g = _f64(v), _f64(g)
    n = len(xy)
    xs, ys = _f64(xy[:, 0]), _f64(xy[:, 1])
    dv = np.empty(n)
    dx = np.empty(n)
    dy = np.empty(n)
    dc = np.zeros(1)
    _load().imq_oracle_grad(n, _dp(xs), _dp(ys), float(c), _dp(v), _dp(g),
                            _dp(dv), _dp(dc), _dp(dx), _dp(dy))
    return dv, float(dc[0]), np.stack([dx, dy], axis=1)


def grad_numpy(xy, c: float, v, f):
    """Tiny-N NumPy form of :func:`grad`, written from the same formulas."""
    xy = _f64(xy)
    A = dense_matrix(xy, c)
    g = 2.0 * (A @ _f64(v) - _f64(f))
    dX = xy[:, None, :] - xy[None, :, :]
    s = (dX ** 2).sum(-1) + c * c
    W = s ** -1.5
    dv = A @ g
    dc = -c * float(g @ W @ v)
    gx = -(g[:, None, None] * (W * v[None, :])[:, :, None] * dX).sum(1) \
         - (v[:, None, None] * (W * g[None, :])[:, :, None] * dX).sum(1)
    return dv, dc, gx


# ----------------------------------------------------------------------------
# O7: restarted GMRES
# ----------------------------------------------------------------------------

def gmres(apply, f, restart: int = 50, tol: float = 1e-10, maxiter: int = 1000,
          x0=None):
    """Restarted GMRES(m), x0 = 0 by default.

    Arnoldi with modified Gram-Schmidt, Givens rotations on the Hessenberg
    matrix, stop when the rotated residual estimate falls to tol*||f||; at
    each restart the residual is recomputed explicitly.  Returns
    (x, iterations, estimate_history, explicit_restart_residuals).
    """
    f = _f64(f)
    n = len(f)
    x = np.zeros(n) if x0 is None else _f64(x0).copy()
    nf = np.linalg.norm(f)
    hist, explicit = [], []
    its = 0
    while True:
        r = f - apply(x)
        beta = np.linalg.norm(r)
        explicit.append(beta / nf)
        if beta <= tol * nf or its >= maxiter:
            break
        m = min(restart, maxiter - its)
        V = np.zeros((m + 1, n))
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        gvec = np.zeros(m + 1)
        gvec[0] = beta
        V[0] = r / beta
        k_used = 0
        for k in range(m):
            w = apply(V[k])
            for i in range(k + 1):
                H[i, k] = w @ V[i]
                w = w - H[i, k] * V[i]
            H[k + 1, k] = np.linalg.norm(w)
            if H[k + 1, k] != 0.0:
                V[k + 1] = w / H[k + 1, k]
            for i in range(k):
                t = cs[i] * H[i, k] + sn[i] * H[i + 1, k]
                H[i + 1, k] = -sn[i] * H[i, k] + cs[i] * H[i + 1, k]
                H[i, k] = t
            den = math.hypot(H[k, k], H[k + 1, k])
            cs[k] = H[k, k] / den
            sn[k] = H[k + 1, k] / den
            H[k, k] = den
            H[k + 1, k] = 0.0
            gvec[k + 1] = -sn[k] * gvec[k]
            gvec[k] = cs[k] * gvec[k]
            its += 1
            k_used = k + 1
            hist.append(abs(gvec[k + 1]) / nf)
            if abs(gvec[k + 1]) <= tol * nf:
                break
        y = np.zeros(k_used)
        for i in range(k_used - 1, -1, -1):
            y[i] = (gvec[i] - H[i, i + 1:k_used] @ y[i + 1:]) / H[i, i]
        x = x + V[:k_used].T @ y
    return x, its, np.array(hist), np.array(explicit)
