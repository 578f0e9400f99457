"""Pins of the FP64 oracle against what the paper and the mathematics fix.

None of these re-types an oracle formula: each compares the oracle with a
closed form, an invariant, a brute-force computation, a library routine on a
special case, or a value printed in the paper (tests/golden/).
"""
import math
import os

import numpy as np
import pytest
import scipy.special

import oracle
import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _ulps(a, b):
    return np.abs(np.asarray(a) - np.asarray(b)) / np.spacing(np.abs(np.asarray(b)))


# ---------------------------------------------------------------- O1 entries

@pytest.mark.parametrize("c", [0.02, 0.1, 1.0, 3.7])
def test_entry_at_zero_distance_is_one_over_c(c):
    """phi(0) = 1/|t| (eq. IMQ_def at r = 0): the diagonal of A."""
    xy = W.uniform_points(5, W.rng(99, 0))
    A = oracle.dense_matrix(xy, c)
    assert np.all(_ulps(np.diag(A), 1.0 / c) <= 1)
    b = oracle.matvec(xy[:1], c, np.array([1.0]))
    assert _ulps(b[0], 1.0 / c) <= 1


@pytest.mark.parametrize("c", [0.05, 0.3, 2.0])
def test_entry_at_distance_c_sqrt3_is_half(c):
    """phi(c sqrt 3) = 1/sqrt(3c^2 + c^2) = 1/(2c)."""
    xy = np.array([[0.0, 0.0], [c * math.sqrt(3.0), 0.0], [0.0, c * math.sqrt(3.0)]])
    A = oracle.dense_matrix(xy, c)
    assert _ulps(A[0, 1], 0.5 / c) <= 3
    assert _ulps(A[0, 2], 0.5 / c) <= 3


def test_lifting_identity_to_an_ulp():
    """Sec. 2.2, eq. (G_eq_phi): phi(|x-y|) = 1/|X - Y| with X=(x, t/2), Y=(y, -t/2)."""
    g = W.rng(99, 1)
    xy = g.random((40, 2))
    for c in (0.02, 0.5, 1.0):
        A = oracle.dense_matrix(xy, c)
        X = np.concatenate([xy, np.full((40, 1), c / 2)], axis=1)
        Y = np.concatenate([xy, np.full((40, 1), -c / 2)], axis=1)
        G = 1.0 / np.linalg.norm(X[:, None, :] - Y[None, :, :], axis=-1)
        assert np.max(_ulps(A, G)) <= 4


def test_matrix_is_bitwise_symmetric():
    """A_ij = A_ji exactly: (x_i - x_j)^2 = (x_j - x_i)^2 in IEEE arithmetic."""
    xy = W.uniform_points(300, W.rng(99, 2))
    A = oracle.dense_matrix(xy, 0.07)
    assert np.array_equal(A, A.T)


@pytest.mark.parametrize("c", [0.02, 0.1])
def test_tiny_matrix_is_positive_definite(c):
    """IMQ matrices of distinct points are positive definite (Micchelli 1986)."""
    xy = W.uniform_points(150, W.rng(99, 3))
    A = oracle.dense_matrix(xy, c)
    np.linalg.cholesky(A)
    assert np.linalg.eigvalsh(A).min() > 0


# ---------------------------------------------------------------- O2 product

def test_matvec_matches_exactly_rounded_row_sums():
    """Brute force: each row sum against math.fsum of the same products."""
    d = W.small(300)
    xy, c, u = d["xy"], d["c"], d["u"]
    b = oracle.matvec(xy, c, u)
    for i in range(0, 300, 7):
        dx = xy[i, 0] - xy[:, 0]
        dy = xy[i, 1] - xy[:, 1]
        terms = [(1.0 / math.sqrt(dx[j] * dx[j] + dy[j] * dy[j] + c * c)) * u[j] for j in range(300)]
        ex = math.fsum(terms)
        assert abs(b[i] - ex) <= 2.3e-16 * abs(ex) + 1e-28 * sum(abs(t) for t in terms)


def test_matvec_two_summation_orders_and_dgemv_agree():
    d = W.small()
    xy, c, u = d["xy"], d["c"], d["u"]
    b = oracle.matvec(xy, c, u)
    b2 = oracle.matvec_pairwise(xy, c, u)
    b3 = oracle.dense_matrix(xy, c) @ u
    nb = np.linalg.norm(b)
    assert np.linalg.norm(b - b2) / nb < 1e-13
    assert np.linalg.norm(b - b3) / nb < 1e-13


def test_matvec_rectangular_targets_and_many_rhs():
    """Transposed-operand and column-layout mistakes: separate target set, 3 RHS."""
    g = W.rng(99, 4)
    xs = g.random((200, 2))
    xt = g.random((77, 2)) * 1.5 - 0.25
    U = g.standard_normal((3, 200))
    B = oracle.matvec(xs, 0.3, U, xy_targets=xt)
    assert B.shape == (3, 77)
    ref = np.array([[math.fsum(U[r, j] / math.sqrt((xt[i, 0] - xs[j, 0]) ** 2
                                                   + (xt[i, 1] - xs[j, 1]) ** 2 + 0.09)
                               for j in range(200)) for i in range(0, 77, 11)]
                    for r in range(3)])
    assert np.allclose(B[:, ::11], ref, rtol=1e-13, atol=1e-13)


def test_matvec_linear_in_u():
    d = W.small(500)
    xy, c = d["xy"], d["c"]
    g = W.rng(99, 5)
    u1, u2 = g.standard_normal(500), g.standard_normal(500)
    lhs = oracle.matvec(xy, c, 2.0 * u1 - 3.0 * u2)
    rhs = 2.0 * oracle.matvec(xy, c, u1) - 3.0 * oracle.matvec(xy, c, u2)
    assert np.linalg.norm(lhs - rhs) / np.linalg.norm(lhs) < 1e-14


# ---------------------------------------------------------------- O3 / O4

def test_direct_solve_reproduces_data_values():
    """Sec. 2, eq. (P_fiEqfi): the interpolant reproduces f at the data sites."""
    d = W.small()
    a, method = oracle.solve_dense(d["xy"], d["c"], d["f"])
    assert method == "cholesky"
    assert oracle.relres(d["xy"], d["c"], a, d["f"]) < 1e-11


def test_direct_solve_against_library_on_well_conditioned_case():
    xy = W.uniform_points(120, W.rng(99, 6))
    f = W.franke(xy[:, 0], xy[:, 1])
    a, _ = oracle.solve_dense(xy, 0.02, f)
    ref = scipy.linalg.solve(oracle.dense_matrix(xy, 0.02), f, assume_a="sym")
    assert np.linalg.norm(a - ref) / np.linalg.norm(ref) < 1e-10


# ---------------------------------------------------------------- O5 series

def test_legendre_table_matches_scipy_lpmv():
    for x in (-0.93, -0.2, 0.0, 0.37, 0.999):
        P = oracle.legendre_table(20, x)
        for n in range(21):
            for m in range(n + 1):
                ref = scipy.special.lpmv(m, n, x)
                # compare on the normalised scale: sqrt((n-m)!/(n+m)!) |P_n^m| <= 1
                nrm = math.sqrt(math.factorial(n - m) / math.factorial(n + m))
                assert abs(P[n, m] - ref) * nrm <= 1e-13, (n, m, x)


def test_legendre_at_zero_golden():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "legendre_at_zero.txt"))
            if l.strip() and not l.startswith("#")]
    P = oracle.legendre_table(6, 0.0)
    for n, m, v in rows:
        assert P[int(n), int(m)] == pytest.approx(float(v), rel=1e-15, abs=1e-15)


def _sph(rho, th, om):
    return np.array([rho * math.sin(th) * math.cos(om), rho * math.sin(th) * math.sin(om),
                     rho * math.cos(th)])


@pytest.mark.parametrize("n", [0, 1, 2, 5, 9, 14, 20])
def test_addition_theorem_against_legendre_polynomial(n):
    """The identity in the proof of Theorem 2.1, against scipy's P_n(cos alpha)."""
    g = W.rng(99, 7)
    for _ in range(20):
        X = g.standard_normal(3)
        Y = g.standard_normal(3)
        cosa = X @ Y / (np.linalg.norm(X) * np.linalg.norm(Y))
        assert oracle.addition_theorem_term(X, Y, n) == pytest.approx(
            scipy.special.eval_legendre(n, cosa), abs=1e-12)


@pytest.mark.parametrize("M", [5, 10, 20])
@pytest.mark.parametrize("rho_x", [1.1, 1.5, 2.0, 5.0, 21.0])
def test_error_equals_bound_when_points_are_aligned(M, rho_x):
    """Fig. 1(a) angles (all pi/3, so alpha = 0): every tail term is r^n/rho_x,
    so the truncation error equals the Theorem 2.1 bound exactly."""
    a = math.pi / 3
    X = _sph(rho_x, a, a)
    Y = _sph(1.0, a, a)
    exact = 1.0 / np.linalg.norm(X - Y)
    err = abs(exact - oracle.series_truncated(X, Y, M))
    bound = oracle.thm21_bound(rho_x, 1.0, M)
    # rounding of the partial sums limits the check to ~64 ulps of G
    assert err == pytest.approx(bound, rel=1e-9, abs=64 * 2.2e-16 * exact)


@pytest.mark.parametrize("M", [5, 10, 20])
def test_error_below_bound_for_fig1b_angles(M):
    """Fig. 1(b) angles: theta_x = pi, theta_y = pi/4, omega_x = pi/3, omega_y = pi/2."""
    for rho_x in np.linspace(1.1, 21.0, 25):
        X = _sph(rho_x, math.pi, math.pi / 3)
        Y = _sph(1.0, math.pi / 4, math.pi / 2)
        err = abs(1.0 / np.linalg.norm(X - Y) - oracle.series_truncated(X, Y, M))
        assert err <= oracle.thm21_bound(rho_x, 1.0, M) * (1 + 1e-12) + 1e-16


def test_series_geometric_decay_random_pairs():
    """log E falls with slope at least log r in M; both branches of the series."""
    g = W.rng(99, 8)
    for _ in range(10):
        X = g.standard_normal(3) * 3
        Y = g.standard_normal(3)
        for P, Q in ((X, Y), (Y, X)):
            exact = 1.0 / np.linalg.norm(P - Q)
            rp, rq = np.linalg.norm(P), np.linalg.norm(Q)
            if abs(rp - rq) < 0.5:
                continue
            for M in (2, 4, 8, 12):
                err = abs(exact - oracle.series_truncated(P, Q, M))
                assert err <= oracle.thm21_bound(rp, rq, M) * (1 + 1e-9) + 1e-15


def test_worked_example_golden():
    """Sec. 2.2: t=1, unit square, M=10 -> E < 2.86e-9, M=20 -> E < 4.41e-17."""
    vals = dict(l.split()[:2] for l in open(os.path.join(GOLDEN, "worked_example.txt"))
                if l.strip() and not l.startswith("#"))
    rho_y = math.sqrt(2) / 8
    rho_x = math.sqrt(73) / 8
    # the geometric facts behind the example: half-diagonal of a 1/4 block,
    # and in-plane distance 3/8 to a non-adjacent block at vertical offset t.
    assert rho_y == pytest.approx(math.hypot(0.125, 0.125), rel=1e-15)
    assert rho_x == pytest.approx(math.hypot(0.375, 1.0), rel=1e-15)
    r = round(rho_y / rho_x, 4)
    assert r == float(vals["ratio_printed"])
    # the paper rounds the ratio to 0.1655 before evaluating the bound
    assert float(f"{r ** 11 / ((1 - r) * rho_x):.2e}") == float(vals["bound_M10_printed"])
    assert float(f"{r ** 21 / ((1 - r) * rho_x):.2e}") == float(vals["bound_M20_printed"])
    assert float(f"{oracle.thm21_bound(rho_x, r * rho_x, 10):.2e}") == float(vals["bound_M10_printed"])


def test_worked_example_brute_force_ratio_and_error():
    """Brute force over the 4x4 partition of Sec. 2.2: sources in a block,
    targets in non-adjacent blocks, t = 1; the worst ratio is <= 0.1655 and
    the M=10 series error stays below 2.86e-9."""
    t = 1.0
    g = W.rng(99, 9)
    worst = 0.0
    worst_err = 0.0
    bi, bj = 1, 1                                   # an interior source block
    z = np.array([(bi + 0.5) / 4, (bj + 0.5) / 4])
    src = z + (g.random((64, 2)) - 0.5) / 4
    corners = z + np.array([[-1, -1], [-1, 1], [1, -1], [1, 1]]) / 8
    src = np.concatenate([src, corners])
    for ti in range(4):
        for tj in range(4):
            if max(abs(ti - bi), abs(tj - bj)) <= 1:
                continue
            tz = np.array([(ti + 0.5) / 4, (tj + 0.5) / 4])
            tgt = tz + (g.random((16, 2)) - 0.5) / 4
            for y in src[::4]:
                Y = np.array([y[0] - z[0], y[1] - z[1], 0.0])
                for x in tgt:
                    X = np.array([x[0] - z[0], x[1] - z[1], t])
                    worst = max(worst, np.linalg.norm(Y) / np.linalg.norm(X))
                    e = abs(1 / np.linalg.norm(X - Y) - oracle.series_truncated(X, Y, 10))
                    worst_err = max(worst_err, e)
            # nearest possible target point to the block corner
    for y in corners:
        Y = np.array([y[0] - z[0], y[1] - z[1], 0.0])
        worst = max(worst, np.linalg.norm(Y) / math.hypot(0.375, t))
    assert worst <= math.sqrt(2) / math.sqrt(73) + 1e-15
    assert worst > 0.16
    assert worst_err < 2.86e-9


# ---------------------------------------------------------------- O6 gradient

def _fd_setup(n=60, seed=10):
    g = W.rng(99, seed)
    xy = g.random((n, 2))
    v = g.standard_normal(n)
    f = g.standard_normal(n)
    return xy, 0.07, v, f


def _richardson(fun, h):
    """Central difference at h and h/2 combined to cancel the O(h^2) term."""
    d1 = (fun(h) - fun(-h)) / (2 * h)
    d2 = (fun(h / 2) - fun(-h / 2)) / h
    return (4 * d2 - d1) / 3


def test_gradient_against_central_differences():
    xy, c, v, f = _fd_setup()
    dv, dc, dX = oracle.grad(xy, c, v, f)
    h = 1e-4
    fd_c = _richardson(lambda e: oracle.loss(xy, c + e, v, f), h)
    assert dc == pytest.approx(fd_c, rel=1e-7)
    for k in (0, 7, 33, 59):
        for ax in (0, 1):
            def lk(e):
                p = xy.copy()
                p[k, ax] += e
                return oracle.loss(p, c, v, f)
            fd = _richardson(lk, h)
            assert dX[k, ax] == pytest.approx(fd, rel=1e-6, abs=1e-7 * np.abs(dX).max())
    g = W.rng(99, 11)
    for _ in range(3):
        d = g.standard_normal(len(v))
        fd = _richardson(lambda e: oracle.loss(xy, c, v + e * d, f), h)
        assert dv @ d == pytest.approx(fd, rel=1e-7)


def test_gradient_invariants():
    """Translation invariance: sum_k dL/dx_k = 0.  Homogeneity phi(lr, lc) = phi/l:
    c dL/dc + sum_k x_k . dL/dx_k = -g^T A v with g = 2(Av - f)."""
    xy, c, v, f = _fd_setup(200, 12)
    dv, dc, dX = oracle.grad(xy, c, v, f)
    scale = np.abs(dX).sum()
    assert np.abs(dX.sum(0)).max() < 1e-12 * scale
    Av = oracle.matvec(xy, c, v)
    g = 2 * (Av - f)
    lhs = c * dc + float((xy * dX).sum())
    assert lhs == pytest.approx(-(g @ Av), rel=1e-10)


def test_gradient_c_and_numpy_forms_agree():
    xy, c, v, f = _fd_setup(50, 13)
    a = oracle.grad(xy, c, v, f)
    b = oracle.grad_numpy(xy, c, v, f)
    assert np.allclose(a[0], b[0], rtol=1e-12)
    assert a[1] == pytest.approx(b[1], rel=1e-11)
    assert np.allclose(a[2], b[2], rtol=1e-10, atol=1e-12 * np.abs(b[2]).max())


# ---------------------------------------------------------------- O7 GMRES

def test_gmres_solves_small_system_like_a_library():
    xy = W.uniform_points(100, W.rng(99, 14))
    A = oracle.dense_matrix(xy, 0.3)
    f = W.franke(xy[:, 0], xy[:, 1])
    x, its, hist, expl = oracle.gmres(lambda z: A @ z, f, restart=100, tol=1e-12, maxiter=100)
    assert expl[-1] <= 1e-12
    assert its <= 100
    assert np.all(np.diff(hist) <= 1e-15)          # minimal residual: non-increasing
    ref = np.linalg.solve(A, f)
    assert np.linalg.norm(A @ x - f) <= 1e-12 * np.linalg.norm(f)
    assert np.linalg.norm(x - ref) / np.linalg.norm(ref) < 1e-3


def test_gmres_identity_and_diagonal_finite_termination():
    d = np.arange(1.0, 11.0)
    f = np.ones(10)
    x, its, hist, expl = oracle.gmres(lambda z: d * z, f, restart=10, tol=1e-14, maxiter=50)
    assert its <= 10
    assert np.allclose(x, 1.0 / d, rtol=1e-12)
    x, its, _, _ = oracle.gmres(lambda z: z, f, restart=5, tol=1e-14)
    assert its == 1 and np.allclose(x, f)


def test_gmres_restarted_estimates_track_explicit_residual():
    xy = W.uniform_points(300, W.rng(99, 15))
    A = oracle.dense_matrix(xy, 0.05)
    f = W.franke(xy[:, 0], xy[:, 1])
    x, its, hist, expl = oracle.gmres(lambda z: A @ z, f, restart=20, tol=1e-8, maxiter=400)
    true = np.linalg.norm(A @ x - f) / np.linalg.norm(f)
    assert true == pytest.approx(expl[-1], rel=1e-6)
    assert hist[-1] == pytest.approx(true, rel=1e-2, abs=1e-12)
