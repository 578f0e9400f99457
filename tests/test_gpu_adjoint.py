"""GPU adjoint of the fast product against the dense FP64 oracle gradient.

Loss L = ||A(c, X) v - f||^2 with v, f ~ N(0,1) drawn in FP32 (promoted
exactly to FP64).  The oracle gradient is itself pinned by finite
differences in tests/test_oracle_pins.py; here the GPU result is compared
with it (relative 2-norm 1e-6 with FP64 expansions at p = 16) and, for c,
also with Richardson-extrapolated central differences of the oracle loss.
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
    return m


def _dev(a):
    return torch.tensor(a, device="cuda:0")


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - b) / np.linalg.norm(b))


@pytest.mark.parametrize("n,c", [(2000, 0.05), (5000, 0.05)])
def test_adjoint_matches_dense_gradient(imq, n, c):
    d = W.grad(n)
    xy, v, f = d["xy"], d["v"], d["f"]
    g = 2.0 * (oracle.matvec(xy, c, v) - f)
    ref_dv, ref_dc, ref_dX = oracle.grad_given_g(xy, c, v, g)
    tree = imq.build_tree(_dev(xy), c, leaf=64, p=16, direct_max=1 << 30)
    dv, dc, dX = tree.backward(_dev(v), _dev(g), prec="fp64")
    assert _rel(dv.cpu().numpy(), ref_dv) < 1e-6
    assert abs(float(dc[0]) - ref_dc) / abs(ref_dc) < 1e-6
    assert _rel(dX.cpu().numpy(), ref_dX) < 1e-6
    # FP32 arithmetic inside, same entry point
    dv32, dc32, dX32 = tree.backward(_dev(v), _dev(g), prec="fp32")
    assert _rel(dv32.cpu().numpy(), ref_dv) < 1e-5
    assert abs(float(dc32[0]) - ref_dc) / abs(ref_dc) < 1e-4
    assert _rel(dX32.cpu().numpy(), ref_dX) < 1e-4


def test_dc_against_finite_differences_of_the_oracle_loss(imq):
    d = W.grad(2000)
    xy, v, f = d["xy"], d["v"], d["f"]
    c, h = 0.05, 1e-4
    fd1 = (oracle.loss(xy, c + h, v, f) - oracle.loss(xy, c - h, v, f)) / (2 * h)
    fd2 = (oracle.loss(xy, c + h / 2, v, f) - oracle.loss(xy, c - h / 2, v, f)) / h
    fd = (4 * fd2 - fd1) / 3
    g = 2.0 * (oracle.matvec(xy, c, v) - f)
    tree = imq.build_tree(_dev(xy), c, leaf=64, p=16, direct_max=1 << 30)
    _, dc, _ = tree.backward(_dev(v), _dev(g))
    assert float(dc[0]) == pytest.approx(fd, rel=1e-6)


def test_autograd_function_end_to_end(imq):
    d = W.grad(3000)
    xy, v, f = d["xy"], d["v"], d["f"]
    c = 0.05
    X = _dev(xy).requires_grad_(True)
    cc = torch.tensor(c, dtype=torch.float64, device="cuda:0", requires_grad=True)
    V = _dev(v).requires_grad_(True)
    b = imq.IMQMatvec.apply(X, cc, V, 64, 16, "fp64")
    loss = ((b - _dev(f)) ** 2).sum()
    loss.backward()
    ref_dv, ref_dc, ref_dX = oracle.grad(xy, c, v, f)
    assert _rel(V.grad.cpu().numpy(), ref_dv) < 1e-6
    assert abs(float(cc.grad) - ref_dc) / abs(ref_dc) < 1e-6
    assert _rel(X.grad.cpu().numpy(), ref_dX) < 1e-6


def test_several_sets_get_their_own_dc(imq):
    g0 = W.rng(55, 1)
    sets = [W.uniform_points(k, g0) for k in (700, 1300)]
    cs = [0.05, 0.12]
    xy = np.concatenate(sets)
    v = g0.standard_normal(len(xy))
    gg = g0.standard_normal(len(xy))
    tree = imq.build_tree(_dev(xy), cs, leaf=32, p=16, set_offsets=[0, 700, 2000],
                          direct_max=1 << 30)
    dv, dc, dX = tree.backward(_dev(v), _dev(gg))
    for s, (a, e) in enumerate(((0, 700), (700, 2000))):
        rdv, rdc, rdX = oracle.grad_given_g(xy[a:e], cs[s], v[a:e], gg[a:e])
        assert _rel(dv.cpu().numpy()[a:e], rdv) < 1e-6
        assert abs(float(dc[s]) - rdc) / abs(rdc) < 1e-6
        assert _rel(dX.cpu().numpy()[a:e], rdX) < 1e-6


def test_tree_with_expansion_w_lists_is_refused(imq):
    xy = W.mixture_points(20000, W.rng("mixture1m", 3), W.rng(55, 2))
    tree = imq.build_tree(_dev(xy), 0.02, leaf=64, p=8, direct_max=-1)
    assert tree.info()["m2p_evals"] > 0
    with pytest.raises(imq.IMQError):
        tree.backward(_dev(np.ones(20000)), _dev(np.ones(20000)))
