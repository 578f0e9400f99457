"""CPU tests of the FP64 translation tables (host logic, no GPU).

The stored representation is re-derived here from its definition (raw
moments of the complex coordinate, see tests/_hostlib.py), and each table
is checked against the kernel itself: the shifts must be exact, the
translations must reproduce the dense IMQ sums of the oracle with an error
that falls geometrically in the order p.
"""
import math

import numpy as np
import pytest
import scipy.special

import oracle
import workloads as W
from tests import _hostlib as H


@pytest.mark.parametrize("p", [4, 10, 16])
@pytest.mark.parametrize("pos", [0, 1, 2, 3])
def test_m2m_shift_is_exact(p, pos):
    g = W.rng(88, p * 4 + pos)
    zc = np.array([0.25 if pos & 1 else -0.25, 0.25 if pos & 2 else -0.25])
    pts = zc + (g.random((30, 2)) - 0.5) * 0.5
    u = g.uniform(-1, 1, 30)
    T = H.table(0, p, pos=pos)
    child = H.moments(p, pts, u, zc, 0.5)
    parent = H.moments(p, pts, u, np.zeros(2), 1.0)
    assert np.allclose(T @ child, parent, rtol=1e-12, atol=1e-13 * np.abs(parent).max())


@pytest.mark.parametrize("p", [4, 10, 16])
@pytest.mark.parametrize("pos", [0, 3])
def test_l2l_shift_is_exact_on_the_plane(p, pos):
    g = W.rng(88, 100 + p + pos)
    K = (p + 1) * (p + 2) // 2
    lay = H.layout(p)
    Lp = g.standard_normal(K) * np.array([0.5 ** n for n, m, ri in lay])
    zc = np.array([0.25 if pos & 1 else -0.25, 0.25 if pos & 2 else -0.25])
    pts = zc + (g.random((25, 2)) - 0.5) * 0.5
    T = H.table(1, p, pos=pos)
    a = H.local_eval(p, Lp, pts, np.zeros(2), 1.0)
    b = H.local_eval(p, T @ Lp, pts, zc, 0.5)
    assert np.allclose(a, b, rtol=1e-12, atol=1e-12 * np.abs(a).max())


def _m2l_error(p, level, dx, dy, cn, seed=0):
    g = W.rng(89, seed)
    s = 2.0 ** -level
    zs = np.array([3.5, 4.5]) * s
    zt = zs + np.array([dx, dy]) * s
    src = zs + (g.random((40, 2)) - 0.5) * s
    tgt = zt + (g.random((30, 2)) - 0.5) * s
    u = g.uniform(-1, 1, 40)
    T = H.table(2, p, level=level, dx=dx, dy=dy, cnorm=cn)
    phi = H.local_eval(p, T @ H.moments(p, src, u, zs, s), tgt, zt, s)
    exact = oracle.matvec(src, cn, u, xy_targets=tgt)
    return np.abs(phi - exact).max() / np.abs(exact).max()


@pytest.mark.parametrize("level,dx,dy,cn", [(2, 2, 0, 0.02), (3, -3, 2, 0.05), (5, 2, 2, 0.02),
                                            (7, 3, -3, 0.02), (9, 0, -2, 0.02), (4, -2, -1, 1.0)])
def test_m2l_matches_dense_sum_and_decays_in_p(level, dx, dy, cn):
    errs = [_m2l_error(p, level, dx, dy, cn, seed=level) for p in (2, 4, 8, 12, 16)]
    s = 2.0 ** -level
    # separation ratio of the lifted boxes: radii s/sqrt2 each, distance |(d s, c)|
    rho = math.sqrt(2) * s / math.hypot(math.hypot(dx, dy) * s, cn)
    for p, e in zip((2, 4, 8, 12, 16), errs):
        assert e <= 4 * rho ** (p + 1) / (1 - rho) + 1e-13, (p, e)
    assert errs[-1] < 1e-5
    assert errs[2] < errs[0]


def _irregular(n, m, v):
    """I_n^m(v) = (n-m)! P_n^m(cos th) e^{i m om} / rho^(n+1) via scipy's lpmv."""
    rho = np.linalg.norm(v)
    return (math.factorial(n - m) * scipy.special.lpmv(m, n, v[2] / rho)
            * np.exp(1j * m * math.atan2(v[1], v[0])) / rho ** (n + 1))


@pytest.mark.parametrize("p", [6, 12])
def test_point_evaluation_constants_multipole_to_point(p):
    """(1/s) sum Re(Mt eps_m P_n^m(0)/(n+m)! I_n^m((x - z)/s)) = sum_j u_j phi(x - y_j)."""
    g = W.rng(90, p)
    s, cn = 0.125, 0.03
    zs = np.array([0.3, 0.4])
    src = zs + (g.random((20, 2)) - 0.5) * s
    u = g.uniform(-1, 1, 20)
    Mt = H.moments(p, src, u, zs, s)
    wx = H.table(3, p)
    lay = H.layout(p)
    for x in (zs + np.array([0.3, 0.05]), zs + np.array([-0.2, -0.25])):
        v = np.array([(x[0] - zs[0]) / s, (x[1] - zs[1]) / s, cn / s])
        tot = 0.0
        for i, (n, m, ri) in enumerate(lay):
            if ri:
                continue
            I = _irregular(n, m, v)
            mt = Mt[i] + (1j * Mt[i + 1] if m > 0 else 0)
            tot += wx[i] * (mt * I).real
        tot /= s
        ex = oracle.matvec(src, cn, u, xy_targets=x[None, :])[0]
        assert tot == pytest.approx(ex, rel=10 * 0.45 ** (p + 1))


@pytest.mark.parametrize("p", [6, 12])
def test_point_evaluation_constants_point_to_local(p):
    """Lt = (1/s) sum_j u_j eps_k P_j^k(0)/(j+k)! conj(I_j^k((y_j - z)/s)) evaluated locally."""
    g = W.rng(91, p)
    s, cn = 0.125, 0.03
    zt = np.array([0.5, 0.5])
    src = zt + np.array([0.35, -0.3]) + (g.random((15, 2)) - 0.5) * 0.1
    tgt = zt + (g.random((10, 2)) - 0.5) * s
    u = g.uniform(-1, 1, 15)
    wx = H.table(3, p)
    lay = H.layout(p)
    Lt = np.zeros(len(lay))
    for y, uj in zip(src, u):
        v = np.array([(y[0] - zt[0]) / s, (y[1] - zt[1]) / s, -cn / s])
        for i, (n, m, ri) in enumerate(lay):
            val = uj * wx[i] * np.conj(_irregular(n, m, v)) / s
            Lt[i] += val.real if ri == 0 else val.imag
    phi = H.local_eval(p, Lt, tgt, zt, s)
    ex = oracle.matvec(src, cn, u, xy_targets=tgt)
    assert np.abs(phi - ex).max() / np.abs(ex).max() < 10 * 0.4 ** (p + 1)


@pytest.mark.parametrize("p", [4, 10, 16])
@pytest.mark.parametrize("pos", [1, 2])
def test_l2l_odd_shift_is_exact_on_the_plane(p, pos):
    g = W.rng(88, 200 + p + pos)
    Ko = p * (p + 1) // 2
    lay = H.odd_layout(p)
    Lo = g.standard_normal(Ko) * np.array([0.5 ** j for j, k, ri in lay])
    zc = np.array([0.25 if pos & 1 else -0.25, 0.25 if pos & 2 else -0.25])
    pts = zc + (g.random((25, 2)) - 0.5) * 0.5
    T = H.table(5, p, pos=pos)[:Ko, :Ko]
    a = H.vertical_eval(p, Lo, pts, np.zeros(2), 1.0)
    b = H.vertical_eval(p, T @ Lo, pts, zc, 0.5)
    assert np.allclose(a, b, rtol=1e-12, atol=1e-12 * np.abs(a).max())


@pytest.mark.parametrize("level,dx,dy,cn", [(3, 2, 1, 0.05), (6, -3, 3, 0.02), (9, 2, -2, 0.02)])
def test_m2l_odd_gives_the_vertical_derivative(level, dx, dy, cn):
    """d/dc of sum_j u_j / sqrt(r^2 + c^2) is -c sum_j u_j (r^2 + c^2)^(-3/2)."""
    g = W.rng(92, level)
    s = 2.0 ** -level
    zs = np.array([3.5, 4.5]) * s
    zt = zs + np.array([dx, dy]) * s
    src = zs + (g.random((40, 2)) - 0.5) * s
    tgt = zt + (g.random((30, 2)) - 0.5) * s
    u = g.uniform(-1, 1, 40)
    d2 = ((tgt[:, None, :] - src[None, :, :]) ** 2).sum(-1)
    exact = -cn * (u[None, :] * (d2 + cn * cn) ** -1.5).sum(1)
    errs = []
    for p in (4, 8, 12, 16):
        Ko = p * (p + 1) // 2
        T = H.table(4, p, level=level, dx=dx, dy=dy, cnorm=cn)[:Ko, :]
        dz = H.vertical_eval(p, T @ H.moments(p, src, u, zs, s), tgt, zt, s)
        errs.append(np.abs(dz - exact).max() / np.abs(exact).max())
    assert errs[-1] < 1e-6
    assert errs[-1] < errs[0]
