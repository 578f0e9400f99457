"""Input generators: determinism, ranges, distinctness, closed forms."""
import numpy as np

import workloads as W


def test_seeding_is_reproducible_and_streams_differ():
    a = W.uniform_points(100, W.rng("small", 0))
    b = W.uniform_points(100, W.rng("small", 0))
    c = W.uniform_points(100, W.rng("small", 1))
    assert np.array_equal(a, b)
    assert not np.array_equal(a, c)


def test_halton_first_points():
    """Radical inverses in bases 2 and 3 of 1, 2, 3, 4."""
    h = W.halton_points(4)
    assert np.allclose(h, [[1 / 2, 1 / 3], [1 / 4, 2 / 3], [3 / 4, 1 / 9], [1 / 8, 4 / 9]])


def test_mixture_points_stay_in_unit_square_and_are_distinct():
    xy = W.mixture_points(50_000, W.rng("mixture1m", 3), W.rng("mixture1m", 0))
    assert xy.shape == (50_000, 2)
    assert np.all(xy >= 0.0) and np.all(xy < 1.0)
    W.assert_distinct(xy)
    centres, sigmas = W.mixture_params(W.rng("mixture1m", 3))
    assert np.all((sigmas >= 0.01) & (sigmas <= 0.1))
    assert np.all((centres >= 0.1) & (centres <= 0.9))


def test_assert_distinct_detects_duplicates():
    xy = np.array([[0.1, 0.2], [0.3, 0.4], [0.1, 0.2]])
    try:
        W.assert_distinct(xy)
    except ValueError:
        return
    raise AssertionError("duplicate not detected")


def test_named_workloads_shapes():
    d = W.small()
    assert d["xy"].shape == (2000, 2) and d["c"] == 0.1 and d["f"].shape == (2000,)
    s = W.batched_sets(count=8, lo=100, hi=400)
    assert len(s["offsets"]) == 9 and s["offsets"][-1] == len(s["xy"])
    assert np.all((s["c"] >= 0.02) & (s["c"] <= 0.2))
    r = W.fourier_rhs(np.array([0.0, 1.0]), np.array([0.0, 0.0]), 3, W.rng(1, 1))
    assert r.shape == (3, 2)


def test_fp32_normal_vectors_are_exact_in_fp64():
    v = W.normal_vector_f32(1000, W.rng("grad", 1))
    assert np.array_equal(v.astype(np.float32).astype(np.float64), v)
