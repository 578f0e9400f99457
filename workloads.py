"""Seeded synthetic inputs for the IMQ interpolation problem.

This module only *draws* inputs: point sets, right-hand sides and vectors.
It contains none of the method's arithmetic (no kernel evaluation, no
expansions, no tree), so both the FP64 oracle and the GPU library can take
their inputs from here without sharing any computation.

Every generator takes a ``numpy.random.Generator`` made by :func:`rng` from a
workload id and a stream id, so that each array of each workload is
reproducible on its own.

Workloads (problem statement: Sec. 2, interpolation system ``A a = f`` with
the IMQ kernel of eq. (IMQ_def); sizes and distributions are the ones the
benchmarks below use):

* ``small``      N=2,000 uniform points in [0,1)^2, c=0.1, f = Franke.
* ``uniform100k`` N=100,000 uniform, c=0.05, f = sin(2 pi x) cos(2 pi y) + noise.
* ``mixture1m``  N=1,000,000 from an 8-component Gaussian mixture, c=0.02.
* ``batched``    N=200,000 uniform with 64 random Fourier right-hand sides,
                 and 256 independent sets with log-uniform sizes.
* ``grad``       N=100,000 (and 5,000) uniform, c=0.05, v, f ~ N(0,1) in FP32.
* ``halton``     the quasi-random Halton points of the paper's experiment
                 (Sec. 3), bases (2, 3), indices 1..N.
"""
from __future__ import annotations

import numpy as np

WORKLOAD_IDS = {
    "small": 1,
    "uniform100k": 2,
    "mixture1m": 3,
    "batched": 4,
    "grad": 5,
    "halton": 6,
}


def rng(workload: str | int, stream: int) -> np.random.Generator:
    """Generator seeded by (workload id, stream id)."""
    wid = WORKLOAD_IDS[workload] if isinstance(workload, str) else int(workload)
    return np.random.default_rng([wid, int(stream)])


# ----------------------------------------------------------------------------
# point sets (returned as an (N, 2) float64 array, one row per point)
# ----------------------------------------------------------------------------

def uniform_points(n: int, g: np.random.Generator) -> np.ndarray:
    """N i.i.d. points, uniform in [0,1)^2."""
    return g.random((n, 2))


def mixture_params(g: np.random.Generator, k: int = 8,
                   sigma_range=(0.01, 0.1), centre_range=(0.1, 0.9)):
    """Parameters of an isotropic, equally weighted Gaussian mixture."""
    centres = g.uniform(centre_range[0], centre_range[1], size=(k, 2))
    sigmas = g.uniform(sigma_range[0], sigma_range[1], size=k)
    return centres, sigmas


def mixture_points(n: int, g_params: np.random.Generator,
                   g_draw: np.random.Generator, k: int = 8,
                   sigma_range=(0.01, 0.1)) -> np.ndarray:
    """N points from a k-component Gaussian mixture restricted to [0,1)^2.

    Draws that fall outside the unit square are re-drawn (rejection) rather
    than clamped: clamping would stack points on the edges and corners and
    create exact duplicates, which make the interpolation matrix singular.
    """
    centres, sigmas = mixture_params(g_params, k, sigma_range)
    out = np.empty((n, 2))
    filled = 0
    while filled < n:
        m = n - filled
        comp = g_draw.integers(0, k, size=m)
        pts = centres[comp] + sigmas[comp, None] * g_draw.standard_normal((m, 2))
        ok = np.all((pts >= 0.0) & (pts < 1.0), axis=1)
        pts = pts[ok]
        out[filled:filled + len(pts)] = pts
        filled += len(pts)
    return out


def halton_points(n: int, bases=(2, 3), start: int = 1) -> np.ndarray:
    """First n Halton points (radical inverses of start..start+n-1)."""
    idx = np.arange(start, start + n, dtype=np.int64)
    out = np.empty((n, len(bases)))
    for d, b in enumerate(bases):
        f = np.ones(n)
        r = np.zeros(n)
        i = idx.copy()
        while np.any(i > 0):
            f = f / b
            r = r + f * (i % b)
            i = i // b
        out[:, d] = r
    return out


def log_uniform_sizes(count: int, lo: int, hi: int, g: np.random.Generator) -> np.ndarray:
    """Set sizes floor(exp(U[ln lo, ln hi]))."""
    return np.floor(np.exp(g.uniform(np.log(lo), np.log(hi), size=count))).astype(np.int64)


def assert_distinct(xy: np.ndarray) -> None:
    """Raise if two points coincide exactly (the system would be singular)."""
    v = np.ascontiguousarray(xy).view([("x", xy.dtype), ("y", xy.dtype)]).ravel()
    if len(np.unique(v)) != len(v):
        raise ValueError("point set has exact duplicates")


# ----------------------------------------------------------------------------
# data values / vectors
# ----------------------------------------------------------------------------

def franke(x: np.ndarray, y: np.ndarray) -> np.ndarray:
    """Franke's bivariate test function (the standard four-Gaussian form)."""
    t1 = 0.75 * np.exp(-((9 * x - 2) ** 2 + (9 * y - 2) ** 2) / 4)
    t2 = 0.75 * np.exp(-((9 * x + 1) ** 2) / 49 - (9 * y + 1) / 10)
    t3 = 0.5 * np.exp(-((9 * x - 7) ** 2 + (9 * y - 3) ** 2) / 4)
    t4 = -0.2 * np.exp(-(9 * x - 4) ** 2 - (9 * y - 7) ** 2)
    return t1 + t2 + t3 + t4


def sincos(x: np.ndarray, y: np.ndarray) -> np.ndarray:
    return np.sin(2 * np.pi * x) * np.cos(2 * np.pi * y)


def sincos_noisy(x, y, g: np.random.Generator, sigma: float = 1e-3) -> np.ndarray:
    """sin(2 pi x) cos(2 pi y) plus Gaussian noise of standard deviation sigma."""
    return sincos(x, y) + sigma * g.standard_normal(len(x))


def fourier_rhs(x, y, nrhs: int, g: np.random.Generator, modes: int = 4) -> np.ndarray:
    """nrhs random cosine series with modes x modes terms, N(0,1) coefficients.

    Returned as (nrhs, N): one right-hand side per row.
    """
    coef = g.standard_normal((nrhs, modes, modes))
    cx = np.cos(np.pi * np.arange(modes)[:, None] * x[None, :])   # (modes, N)
    cy = np.cos(np.pi * np.arange(modes)[:, None] * y[None, :])
    return np.einsum("rab,an,bn->rn", coef, cx, cy)


def uniform_vector(n: int, g: np.random.Generator, nrhs: int | None = None) -> np.ndarray:
    """i.i.d. U(-1,1) entries; shape (n,) or (nrhs, n)."""
    shape = (n,) if nrhs is None else (nrhs, n)
    return g.uniform(-1.0, 1.0, size=shape)


def normal_vector_f32(n: int, g: np.random.Generator) -> np.ndarray:
    """N(0,1) entries drawn in FP32 and promoted exactly to FP64."""
    return g.standard_normal(n, dtype=np.float32).astype(np.float64)


# ----------------------------------------------------------------------------
# named workloads
# ----------------------------------------------------------------------------

def small(n: int = 2000):
    """N=2000 uniform points, c=0.1, f = Franke, u ~ U(-1,1)."""
    xy = uniform_points(n, rng("small", 0))
    assert_distinct(xy)
    return dict(name="small", xy=xy, c=0.1, f=franke(xy[:, 0], xy[:, 1]),
                u=uniform_vector(n, rng("small", 2)), leaf=32, p=10)


def uniform100k(n: int = 100_000):
    """N=100,000 uniform points, c=0.05, f = sin cos + N(0, sigma=1e-3)."""
    xy = uniform_points(n, rng("uniform100k", 0))
    assert_distinct(xy)
    f = sincos_noisy(xy[:, 0], xy[:, 1], rng("uniform100k", 1))
    return dict(name="uniform100k", xy=xy, c=0.05, f=f,
                u=uniform_vector(n, rng("uniform100k", 2)), leaf=64, p=12)


def mixture1m(n: int = 1_000_000):
    """N=1e6 points, 8-component Gaussian mixture, c=0.02."""
    xy = mixture_points(n, rng("mixture1m", 3), rng("mixture1m", 0))
    assert_distinct(xy)
    return dict(name="mixture1m", xy=xy, c=0.02, f=sincos(xy[:, 0], xy[:, 1]),
                u=uniform_vector(n, rng("mixture1m", 2)), leaf=64, p=12)


def batched_rhs(n: int = 200_000, nrhs: int = 64):
    """N=2e5 uniform points, c=0.05, nrhs random Fourier right-hand sides."""
    xy = uniform_points(n, rng("batched", 0))
    assert_distinct(xy)
    f = fourier_rhs(xy[:, 0], xy[:, 1], nrhs, rng("batched", 1))
    u = uniform_vector(n, rng("batched", 2), nrhs=nrhs)
    return dict(name="batched_rhs", xy=xy, c=0.05, f=f, u=u, leaf=64, p=12)


def batched_sets(count: int = 256, lo: int = 1000, hi: int = 20000):
    """count independent uniform sets, N_i log-uniform in [lo, hi], c_i ~ U[0.02,0.2]."""
    sizes = log_uniform_sizes(count, lo, hi, rng("batched", 3))
    cs = rng("batched", 4).uniform(0.02, 0.2, size=count)
    g = rng("batched", 5)
    sets = []
    for i in range(count):
        xy = uniform_points(int(sizes[i]), g)
        assert_distinct(xy)
        sets.append(xy)
    offsets = np.concatenate([[0], np.cumsum(sizes)])
    xy = np.concatenate(sets, axis=0)
    f = franke(xy[:, 0], xy[:, 1])
    u = uniform_vector(len(xy), rng("batched", 6))
    return dict(name="batched_sets", xy=xy, offsets=offsets, c=cs, f=f, u=u,
                leaf=32, p=12)


def grad(n: int = 100_000):
    """Uniform points, c=0.05, v and f ~ N(0,1) drawn in FP32."""
    xy = uniform_points(n, rng("grad", n))
    assert_distinct(xy)
    return dict(name=f"grad{n}", xy=xy, c=0.05,
                v=normal_vector_f32(n, rng("grad", 1)),
                f=normal_vector_f32(n, rng("grad", 2)))


def halton(n: int):
    """The paper's experiment: Halton points, c=1, u ~ U(-1,1), M=10."""
    xy = halton_points(n)
    return dict(name=f"halton{n}", xy=xy, c=1.0,
                u=uniform_vector(n, rng("halton", 2)), p=10)
