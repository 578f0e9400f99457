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


@pytest.mark.parametrize("direct_max", [-1, 0])
def test_adjoint_with_expansion_w_and_x_lists(imq, direct_max):
    """Clustered points: the adaptive W/X interactions go through expansions
    (all of them with direct_max = -1, the large ones with the default), so
    the W-list derivative evaluations and the X-list odd coefficients are
    exercised; the result must match the dense gradient as on uniform trees."""
    n, c = 20000, 0.02
    xy = W.mixture_points(n, W.rng("mixture1m", 3), W.rng(55, 2))
    gen = np.random.default_rng(21)
    v, g = gen.standard_normal(n), gen.standard_normal(n)
    ref_dv, ref_dc, ref_dX = oracle.grad_given_g(xy, c, v, g)
    tree = imq.build_tree(_dev(xy), c, leaf=64, p=16, direct_max=direct_max)
    info = tree.info()
    assert info["m2p_evals"] > 0 and info["p2l_evals"] > 0
    dv, dc, dX = tree.backward(_dev(v), _dev(g), prec="fp64")
    print(f"direct_max {direct_max}: m2p {info['m2p_evals']} p2l {info['p2l_evals']}: "
          f"dv {_rel(dv.cpu().numpy(), ref_dv):.2e} dc {abs(float(dc[0]) - ref_dc) / abs(ref_dc):.2e} "
          f"dX {_rel(dX.cpu().numpy(), ref_dX):.2e}")
    assert _rel(dv.cpu().numpy(), ref_dv) < 1e-6
    assert abs(float(dc[0]) - ref_dc) / abs(ref_dc) < 1e-6
    assert _rel(dX.cpu().numpy(), ref_dX) < 1e-6
    dv32, dc32, dX32 = tree.backward(_dev(v), _dev(g), prec="fp32")
    assert _rel(dv32.cpu().numpy(), ref_dv) < 1e-5
    assert abs(float(dc32[0]) - ref_dc) / abs(ref_dc) < 1e-4
    assert _rel(dX32.cpu().numpy(), ref_dX) < 1e-4


def test_autograd_with_float_c_and_several_columns(imq):
    """c passed as a Python float gets no gradient (and no error); a 2-D v of
    nrhs columns gets dv per column and dX summed over the columns."""
    d = W.grad(2500)
    xy, c = d["xy"], d["c"]
    gen = np.random.default_rng(8)
    V2 = gen.standard_normal((3, len(xy)))
    F2 = gen.standard_normal((3, len(xy)))
    X = _dev(xy).requires_grad_(True)
    V = _dev(V2).requires_grad_(True)
    b = imq.IMQMatvec.apply(X, c, V, 64, 16, "fp64")
    assert b.shape == (3, len(xy))
    loss = ((b - _dev(F2)) ** 2).sum()
    loss.backward()
    dX_ref = np.zeros_like(xy)
    for r in range(3):
        rdv, _, rdX = oracle.grad(xy, c, V2[r], F2[r])
        assert _rel(V.grad.cpu().numpy()[r], rdv) < 1e-6
        dX_ref += rdX
    assert _rel(X.grad.cpu().numpy(), dX_ref) < 1e-6


def test_backward_columns_match_single_column_calls(imq):
    d = W.grad(3000)
    xy, c = d["xy"], d["c"]
    gen = np.random.default_rng(9)
    V2, G2 = gen.standard_normal((2, len(xy))), gen.standard_normal((2, len(xy)))
    tree = imq.build_tree(_dev(xy), c, leaf=64, p=16, direct_max=1 << 30)
    dv, dc, dX = tree.backward(_dev(V2), _dev(G2))
    parts = [tree.backward(_dev(V2[r]), _dev(G2[r])) for r in range(2)]
    for r in range(2):
        assert torch.equal(dv[r], parts[r][0])
    assert float(dc[0]) == pytest.approx(float(parts[0][1][0] + parts[1][1][0]), rel=1e-14)
    assert torch.allclose(dX, parts[0][2] + parts[1][2], rtol=1e-13, atol=0)
    with pytest.raises(ValueError):
        tree.backward(_dev(V2), _dev(G2[0]))               # g of another shape
    with pytest.raises(ValueError):
        tree.backward(_dev(V2[0][:-1]), _dev(G2[0][:-1]))   # short vectors
    with pytest.raises(ValueError):
        tree.backward(torch.tensor(V2[0]), torch.tensor(G2[0]))   # host tensors


def test_adjoint_with_streamed_translations(imq):
    """m2l_mode 3 streams both the even and the odd (vertical-derivative)
    translations through registers at p = 16; the gradients equal those of
    the staged GEMM to rounding and the dense oracle's."""
    d = W.grad(5000)
    xy, v, f = d["xy"], d["v"], d["f"]
    c = 0.05
    g = 2.0 * (oracle.matvec(xy, c, v) - f)
    ref_dv, ref_dc, ref_dX = oracle.grad_given_g(xy, c, v, g)
    tree = imq.build_tree(_dev(xy), c, leaf=64, p=16, direct_max=1 << 30)
    out = {}
    for mode in (0, 3):
        tree.set_kernel_config(m2l_mode=mode)
        for prec in ("fp64", "fp32"):
            out[mode, prec] = [x.cpu().numpy() for x in tree.backward(_dev(v), _dev(g), prec=prec)]
    for k in range(3):
        assert _rel(out[3, "fp64"][k], out[0, "fp64"][k]) < 1e-12
        assert _rel(out[3, "fp32"][k], out[0, "fp64"][k]) < 2e-5
    dv, dc, dX = out[3, "fp64"]
    assert _rel(dv, ref_dv) < 1e-6
    assert abs(float(dc[0]) - ref_dc) / abs(ref_dc) < 1e-6
    assert _rel(dX, ref_dX) < 1e-6
