"""GPU parity of the interpolant evaluation at new points (Sec. 2, eq.
interp_eq) against the FP64 oracle, through the C ABI.

The evaluation tree holds the data sites and the evaluation points; the
evaluation points carry weight zero, so the product read at them is the
interpolant.  Tolerances as for the product: 1e-6 with FP64 expansions at
p = 12, 1e-5 on the FP32 path (relative 2-norm over the evaluation points).
"""
import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def imq():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2205_04194_amd as m
    from paper_2205_04194_amd import _lib
    _lib.load()
    return m


def _dev(a):
    return torch.tensor(a, device="cuda:0")


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - b) / np.linalg.norm(b))


def _points(seed, n, m):
    g = W.rng(96, seed)
    xs = np.concatenate([W.mixture_points(n - n // 4, W.rng(96, seed + 1), g), W.uniform_points(n // 4, g)])
    # fresh points (some outside the data sites' square), points on data sites, repeats
    fresh = W.uniform_points(m, g) * 1.2 - 0.1
    xt = np.concatenate([fresh, xs[::97], fresh[::13], [[xs[0, 0], xs[0, 1]]]])
    return xs, xt


@pytest.mark.parametrize("n,m", [(6000, 3000), (3000, 1), (500, 20000)])
def test_evaluation_matches_the_oracle(imq, n, m):
    xs, xt = _points(n % 7 + 1, n, m)
    c = 0.03
    lam = W.uniform_vector(n, W.rng(97, n), nrhs=3)
    tree = imq.build_eval_tree(_dev(xs), c, _dev(xt), leaf=32, p=12)
    ref = oracle.matvec(xs, c, lam, xy_targets=xt)
    s64 = tree.evaluate(_dev(lam), "fp64").cpu().numpy()
    s32 = tree.evaluate(_dev(lam.astype(np.float32)), "fp32").cpu().numpy()
    assert s64.shape == (3, len(xt)) and s32.dtype == np.float32
    for r in range(3):
        e64, e32 = _rel(s64[r], ref[r]), _rel(s32[r], ref[r])
        print(f"n={n} m={len(xt)} rhs {r}: rel err fp64 {e64:.2e} fp32 {e32:.2e}")
        assert e64 < 1e-6 and e32 < 1e-5
    # a repeated evaluation point reads the same tree point: equal values
    k = m + len(xs[::97])
    assert np.array_equal(s64[:, k:k + len(xt[k:-1])], s64[:, 0:m:13][:, :len(xt[k:-1])])
    # one column alone gives its column of the batch
    one = tree.evaluate(_dev(lam[1]), "fp64").cpu().numpy()
    assert _rel(one, s64[1]) < 1e-12


def test_solve_then_evaluate_at_the_data_sites_returns_the_data(imq):
    """With lambda from the solve of A lambda = f, the interpolant at the data
    sites is f (eq. P_fiEqfi) to the solve's residual; evaluated at the data
    sites every evaluation point coincides with a site, so the evaluation
    tree holds the sites only."""
    g = W.rng(98, 1)
    xs = W.uniform_points(3000, g)
    c = 0.004                                    # below the spacing: a well-conditioned system
    f = W.uniform_vector(3000, W.rng(98, 2))
    tree = imq.build_tree(_dev(xs), c, leaf=32, p=16)
    lam, st = tree.solve(_dev(f), tol=1e-9, restart=60, max_iters=3000)
    assert st["converged"]
    ev = imq.build_eval_tree(_dev(xs), c, _dev(xs[::-1].copy()), leaf=32, p=16)
    assert ev.n == len(xs)
    s = ev.evaluate(lam, "fp64").cpu().numpy()[::-1]
    err = _rel(s, f)
    print(f"solve relres {st['relres_fast64']:.2e}, interpolant at the sites vs data {err:.2e}")
    assert err < 10 * max(st["relres_fast64"], 1e-9)


def test_evaluation_arguments(imq):
    xs, xt = _points(3, 800, 100)
    tree = imq.build_eval_tree(_dev(xs), 0.05, _dev(xt), leaf=16, p=8)
    with pytest.raises(ValueError):
        tree.evaluate(_dev(np.zeros((1, 801))))
    with pytest.raises(imq.IMQError):
        imq.build_eval_tree(_dev(np.concatenate([xs, xs[:1]])), 0.05, _dev(xt))
    plain = imq.build_tree(_dev(xs), 0.05, leaf=16, p=8)
    plain.n_src, plain.m_eval = len(xs), 10
    with pytest.raises(imq.IMQError):
        plain.evaluate(_dev(np.ones(len(xs))))     # not an evaluation tree
    empty = imq.build_eval_tree(_dev(xs), 0.05, _dev(np.zeros((0, 2))), leaf=16, p=8)
    assert empty.evaluate(_dev(np.ones(len(xs)))).shape == (0,)
