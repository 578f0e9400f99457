"""GPU parity of the paper's Algorithm 1 far field (far_field = 1) against the
FP64 oracle, through the C ABI.

Algorithm 1 (Sec. 2.2) forms every box's multipole from its own points and
evaluates it directly at the points of the boxes of its V list, level by
level, plus the direct near field.  On the paper's experiment (Halton
points, t = c = 1, M = 10, a uniform partition of L levels starting from
4 x 4 blocks) the relative error in the infinity norm is of order 1e-9
(Sec. 3, Table 1; the worked example's bound for the ratio 0.1655 is
2.86e-9); the bar here is 1e-8.  On an adaptive tree whose W/X interactions
are summed directly the product must meet the usual targets (1e-6 FP64 at
p = 12, 1e-5 FP32).
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


@pytest.mark.parametrize("L", [1, 2, 3])
def test_paper_experiment_error_magnitude(imq, L):
    d = W.halton(20000)
    xy, c, u = d["xy"], d["c"], d["u"]
    # uniform partition: every box splits down to level L + 1 (the paper's
    # level 1 is the 4 x 4 partition, two levels below the square)
    tree = imq.build_tree(_dev(xy), c, leaf=1, p=10, max_level=L + 1)
    assert tree.info()["depth"] == L + 1
    ref = oracle.matvec(xy, c, u)
    tree.set_kernel_config(far_field=1)
    b1 = tree.matvec(_dev(u), "fp64").cpu().numpy()
    tree.set_kernel_config(far_field=0)
    b0 = tree.matvec(_dev(u), "fp64").cpu().numpy()
    e1 = float(np.abs(b1 - ref).max() / np.abs(ref).max())
    e0 = float(np.abs(b0 - ref).max() / np.abs(ref).max())
    print(f"Halton N=20000 L={L} M=10: E (inf) Algorithm 1 {e1:.2e}, tree passes {e0:.2e}")
    assert e1 < 1e-8
    assert e0 < 1e-8


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-6), ("fp32", 1e-5)])
def test_adaptive_tree_with_direct_w_x(imq, prec, tol):
    g = W.rng(99, 1)
    n = 12000
    xy = np.concatenate([W.mixture_points(n - 3000, W.rng(99, 2), g), W.uniform_points(3000, g)])
    U = W.uniform_vector(n, W.rng(99, 3), nrhs=3)
    tree = imq.build_tree(_dev(xy), 0.02, leaf=32, p=12, direct_max=1 << 30)
    tree.set_kernel_config(far_field=1)
    dt = np.float64 if prec == "fp64" else np.float32
    B = tree.matvec(_dev(U.astype(dt)), prec).cpu().numpy()
    ref = oracle.matvec(xy, 0.02, U)
    for r in range(3):
        err = _rel(B[r], ref[r])
        print(f"adaptive, {prec}, rhs {r}: rel err {err:.2e}")
        assert err < tol
    one = tree.matvec(_dev(U[2].astype(dt)), prec).cpu().numpy()
    assert _rel(one, B[2]) < (1e-12 if prec == "fp64" else 1e-6)


def test_w_x_expansions_are_refused(imq):
    g = W.rng(99, 4)
    xy = np.concatenate([W.mixture_points(6000, W.rng(99, 5), g), W.uniform_points(500, g)])
    tree = imq.build_tree(_dev(xy), 0.02, leaf=16, p=8, direct_max=-1)
    inf = tree.info()
    tree.set_kernel_config(far_field=1)
    if inf["m2p_evals"] == 0 and inf["p2l_evals"] == 0:
        pytest.skip("this tree has no W/X expansions")
    with pytest.raises(imq.IMQError) as e:
        tree.matvec(_dev(W.uniform_vector(len(xy), g)))
    assert e.value.status == -5


def test_forest_many_rhs_and_stage_timing(imq):
    """Several sets (each with its own c), 9 right-hand sides (the batched
    near field), and the stage-timed pass: every set's columns match the
    oracle and the timed pass gives the same numbers."""
    g = W.rng(99, 7)
    sizes = [3000, 40, 2500]
    cs = [0.05, 0.2, 0.01]
    sets = [W.uniform_points(k, g) * (i + 1) for i, k in enumerate(sizes)]
    xy = np.concatenate(sets)
    offs = np.concatenate([[0], np.cumsum(sizes)])
    U = W.uniform_vector(len(xy), g, nrhs=9)
    tree = imq.build_tree(_dev(xy), cs, leaf=16, p=12, set_offsets=list(offs), direct_max=1 << 30)
    tree.set_kernel_config(far_field=1)
    B = tree.matvec(_dev(U), "fp64").cpu().numpy()
    for s in range(3):
        a, e = offs[s], offs[s + 1]
        ref = oracle.matvec(xy[a:e], cs[s], U[:, a:e])
        err = _rel(B[:, a:e], ref)
        print(f"set {s} (N={e - a}, c={cs[s]}): rel err {err:.2e}")
        assert err < 1e-6
    tree.set_stage_timing(True)
    Bt = tree.matvec(_dev(U), "fp64").cpu().numpy()
    st = tree.stage_times()
    tree.set_stage_timing(False)
    assert np.array_equal(Bt, B)
    assert all(v >= 0 for v in st.values()) and st["p2p"] > 0
