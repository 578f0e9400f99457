"""GPU parity of the fast product against the FP64 oracle (through the C ABI).

Tolerances (relative 2-norm over the compared entries):
  FP64 expansions: 1e-6   FP32 path: 1e-5      (the targets of the method)
  a tree with a single leaf is the plain dense product: 1e-13 (FP64) and
  1e-6 (FP32: one rounding per entry and per partial sum).
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


def test_single_leaf_tree_is_the_dense_product(imq):
    d = W.small(700)
    tree = imq.build_tree(_dev(d["xy"]), d["c"], leaf=1000, p=4)
    assert tree.info()["nboxes"] == 1
    ref = oracle.matvec(d["xy"], d["c"], d["u"])
    u = _dev(d["u"])
    assert _rel(tree.matvec(u, "fp64").cpu().numpy(), ref) < 1e-13
    assert _rel(tree.matvec(u, "fp32").cpu().numpy(), ref) < 1e-6


@pytest.mark.parametrize("p,tol64", [(8, 1e-5), (10, 1e-6), (12, 2e-7)])
def test_small_workload_fp64_and_fp32(imq, p, tol64):
    d = W.small()
    tree = imq.build_tree(_dev(d["xy"]), d["c"], leaf=32, p=p)
    ref = oracle.matvec(d["xy"], d["c"], d["u"])
    u = _dev(d["u"])
    e64 = _rel(tree.matvec(u, "fp64").cpu().numpy(), ref)
    e32 = _rel(tree.matvec(u, "fp32").cpu().numpy(), ref)
    assert e64 < tol64
    assert e32 < max(tol64, 1e-5)


@pytest.mark.parametrize("n", [1, 2, 3, 17, 65, 129, 1000])
def test_ragged_sizes_and_tiny_sets(imq, n):
    xy = W.uniform_points(n, W.rng(66, n))
    u = W.uniform_vector(n, W.rng(66, n + 1))
    tree = imq.build_tree(_dev(xy), 0.05, leaf=8, p=10)
    ref = oracle.matvec(xy, 0.05, u)
    assert _rel(tree.matvec(_dev(u), "fp64").cpu().numpy(), ref) < 1e-6


def test_many_rhs_and_fp32_io(imq):
    d = W.small(3000)
    U = W.uniform_vector(3000, W.rng(66, 5), nrhs=5)
    tree = imq.build_tree(_dev(d["xy"]), d["c"], leaf=32, p=12)
    ref = oracle.matvec(d["xy"], d["c"], U)
    B = tree.matvec(_dev(U), "fp64").cpu().numpy()
    for r in range(5):
        assert _rel(B[r], ref[r]) < 1e-6
    B32 = tree.matvec(_dev(U).float(), "fp32").cpu().numpy().astype(np.float64)
    assert B32.dtype == np.float64
    for r in range(5):
        assert _rel(B32[r], ref[r]) < 1e-5


def test_several_sets_in_one_forest(imq):
    g = W.rng(66, 9)
    sizes = [500, 1, 1800, 37]
    cs = [0.1, 0.05, 0.02, 0.2]
    sets = [W.uniform_points(k, g) * (i + 1) for i, k in enumerate(sizes)]
    xy = np.concatenate(sets)
    offs = np.concatenate([[0], np.cumsum(sizes)])
    u = W.uniform_vector(len(xy), g)
    tree = imq.build_tree(_dev(xy), cs, leaf=16, p=12, set_offsets=list(offs))
    b = tree.matvec(_dev(u), "fp64").cpu().numpy()
    for s in range(4):
        a, e = offs[s], offs[s + 1]
        ref = oracle.matvec(xy[a:e], cs[s], u[a:e])
        assert _rel(b[a:e], ref) < 1e-6, s


@pytest.mark.parametrize("direct_max", [-1, 0])
def test_clustered_points(imq, direct_max):
    xy = W.mixture_points(20000, W.rng("mixture1m", 3), W.rng(66, 11))
    u = W.uniform_vector(20000, W.rng(66, 12))
    tree = imq.build_tree(_dev(xy), 0.02, leaf=64, p=12, direct_max=direct_max)
    inf = tree.info()
    if direct_max < 0:
        assert inf["m2p_evals"] > 0 and inf["p2l_evals"] > 0   # W/X through expansions
    ref = oracle.matvec(xy, 0.02, u)
    assert _rel(tree.matvec(_dev(u), "fp64").cpu().numpy(), ref) < 1e-6
    assert _rel(tree.matvec(_dev(u), "fp32").cpu().numpy(), ref) < 1e-5


def test_exact_rows_match_the_oracle(imq):
    d = W.uniform100k()
    tree = imq.build_tree(_dev(d["xy"]), d["c"], leaf=64, p=12)
    rows = np.sort(W.rng(66, 13).choice(len(d["xy"]), 300, replace=False))
    ex = tree.rows_exact(_dev(d["u"]), _dev(rows)).cpu().numpy()
    ref = oracle.matvec(d["xy"], d["c"], d["u"], xy_targets=d["xy"][rows])
    assert _rel(ex, ref) < 1e-13
    b = tree.matvec(_dev(d["u"]), "fp64").cpu().numpy()
    assert _rel(b[rows], ref) < 1e-6
    b32 = tree.matvec(_dev(d["u"]), "fp32").cpu().numpy()
    assert _rel(b32[rows], ref) < 1e-5


def test_invalid_arguments_raise(imq):
    xy = W.uniform_points(10, W.rng(66, 14))
    with pytest.raises(imq.IMQError):
        imq.build_tree(_dev(np.concatenate([xy, xy[:1]])), 0.1, leaf=4, p=4)
    with pytest.raises(imq.IMQError):
        imq.build_tree(_dev(xy), -1.0, leaf=4, p=4)
    tree = imq.build_tree(_dev(xy), 0.1, leaf=4, p=4)
    with pytest.raises(ValueError):
        tree.matvec(_dev(np.zeros(11)))


@pytest.mark.parametrize("p", [3, 4, 6, 9, 12, 16])
def test_translation_kernels_agree_and_match_the_oracle(imq, p):
    """The M2L kernels (operands streamed through registers, staged GEMM, and
    the streamed FP32 products on the BF16 matrix cores from three-part
    operands) compute the same truncated sums, so they differ by rounding
    only; all stay within the truncation error of order p against the
    oracle."""
    d = W.small(6000)
    U = W.uniform_vector(6000, W.rng(67, p), nrhs=3)
    tree = imq.build_tree(_dev(d["xy"]), d["c"], leaf=16, p=p)
    ref = oracle.matvec(d["xy"], d["c"], U)
    out = {}
    for mode in (0, 1, 2, 3):
        tree.set_kernel_config(m2l_mode=mode)
        out[mode, "fp64"] = tree.matvec(_dev(U), "fp64").cpu().numpy()
        out[mode, "fp32"] = tree.matvec(_dev(U), "fp32").cpu().numpy()
    for r in range(3):
        assert _rel(out[0, "fp64"][r], out[1, "fp64"][r]) < 1e-12
        assert _rel(out[2, "fp64"][r], out[0, "fp64"][r]) < 1e-13
        assert _rel(out[3, "fp64"][r], out[1, "fp64"][r]) < 1e-12
        for mode in (0, 1, 2, 3):
            assert _rel(out[mode, "fp32"][r], out[1, "fp64"][r]) < 2e-6
        err = _rel(out[0, "fp64"][r], ref[r])
        print(f"p={p} rhs {r}: rel err vs oracle {err:.3e}")
        assert err < {3: 1e-2, 4: 3e-3, 6: 3e-4, 9: 2e-5, 12: 1e-6, 16: 1e-7}[p]


@pytest.mark.parametrize("nrhs", [1, 2, 70])
def test_streamed_translations_up_to_80_coefficients(imq, nrhs):
    """The register-streaming M2L kernel at every row-block count (1 to 5: up to
    80 coefficients per box; FP64, FP32, and FP32 on the BF16 matrix cores) on
    a deep tree with per-level orders from 12 down to 1 and several
    right-hand sides, against the staged GEMM."""
    d = W.small(30000)
    U = _dev(W.uniform_vector(30000, W.rng(68, nrhs), nrhs=nrhs))
    tree = imq.build_tree(_dev(d["xy"]), d["c"], leaf=8, p=11)
    nlev = tree.info()["nlevels"]
    orders = [max(1, 11 - 2 * max(0, l - 2)) for l in range(nlev)]
    tree.set_level_orders(orders)
    tree.set_kernel_config(m2l_mode=1)
    ref = tree.matvec(U, "fp64")
    for mode, prec, tol in ((0, "fp64", 1e-13), (0, "fp32", 2e-6), (2, "fp32", 2e-6), (3, "fp64", 1e-13),
                            (3, "fp32", 2e-6)):
        tree.set_kernel_config(m2l_mode=mode)
        b = tree.matvec(U, prec)
        e = float(torch.linalg.norm(b - ref) / torch.linalg.norm(ref))
        print(f"orders {orders}, nrhs {nrhs}, mode {mode} {prec}: streamed vs staged GEMM {e:.2e}")
        assert e < tol


def test_mixed_level_orders_use_both_kernels(imq):
    d = W.small(20000)
    u = _dev(d["u"])
    tree = imq.build_tree(_dev(d["xy"]), d["c"], leaf=16, p=12)
    nlev = tree.info()["nlevels"]
    orders = [12] * nlev
    for l in range(nlev - 3, nlev):
        orders[l] = {nlev - 3: 6, nlev - 2: 4, nlev - 1: 3}[l]
    tree.set_level_orders(orders)
    res = {}
    for mode in (0, 1):
        tree.set_kernel_config(m2l_mode=mode)
        res[mode] = tree.matvec(u, "fp64").cpu().numpy()
    assert _rel(res[0], res[1]) < 1e-12
    rows = np.arange(0, 20000, 37)
    exact = oracle.matvec(d["xy"], d["c"], d["u"], xy_targets=d["xy"][rows])
    err = _rel(res[0][rows], exact)
    print(f"mixed orders {orders}: rel err {err:.3e}")
    assert err < 1e-3


@pytest.mark.parametrize("nrhs", [8, 70])
def test_batched_right_hand_sides_match_single_products(imq, nrhs):
    """From 8 right-hand sides on, P2M and L2P run as matrix-core products
    over (points x coefficients x rhs) and the near field shares each kernel
    value across the block; every column must equal its own single-RHS
    product up to rounding and the oracle within the FP64/FP32 targets."""
    d = W.small(3000)
    U = W.uniform_vector(3000, W.rng(68, nrhs), nrhs=nrhs)
    tree = imq.build_tree(_dev(d["xy"]), d["c"], leaf=32, p=12)
    B64 = tree.matvec(_dev(U), "fp64").cpu().numpy()
    B32 = tree.matvec(_dev(U), "fp32").cpu().numpy()
    cols = sorted({0, 1, nrhs // 2, nrhs - 1})
    ref = oracle.matvec(d["xy"], d["c"], U[cols])
    for k, r in enumerate(cols):
        single = tree.matvec(_dev(U[r]), "fp64").cpu().numpy()
        assert _rel(B64[r], single) < 1e-12
        assert _rel(B64[r], ref[k]) < 1e-6
        assert _rel(B32[r], ref[k]) < 1e-5


@pytest.mark.parametrize("c", [0.03, 0.3])
def test_near_field_forms_match_the_oracle(imq, c):
    """The near field takes, per leaf, direct differences or the expansion of
    the squared distance about the leaf's centre (where its rounding bound
    allows), on the vector unit (default) or, with p2p_mode = 1 and one
    right-hand side, as a rank-4 product on the FP32 or FP64 matrix cores.
    Both kernels must give the product to the precision's target and agree
    with each other to rounding; the mixture at c = 0.03 has leaves of both
    kinds, at c = 0.3 nearly all expand."""
    n = 20000
    g = W.rng(92, 3)
    xy = W.mixture_points(n, W.rng(92, 1), g)
    u = W.uniform_vector(n, W.rng(92, 2))
    tree = imq.build_tree(_dev(xy), c, leaf=32, p=12)
    rows = np.arange(0, n, 41)
    exact = oracle.matvec(xy, c, u, xy_targets=xy[rows])
    for prec, tol, agree in (("fp32", 1e-5, 1e-6), ("fp64", 1e-6, 1e-13)):
        out = {}
        for mode in (0, 1):
            tree.set_kernel_config(p2p_mode=mode)
            out[mode] = tree.matvec(_dev(u), prec).cpu().numpy()
            err = _rel(out[mode][rows], exact)
            print(f"c={c} {prec} p2p_mode={mode}: rel err vs oracle {err:.3e}")
            assert err < tol
        d = _rel(out[1], out[0])
        print(f"c={c} {prec}: forms differ by {d:.2e}")
        assert d < agree
    tree.set_kernel_config()


def test_near_field_workgroup_count_does_not_change_the_product(imq):
    """The near field's leaf records are arranged for eight XCDs (runs of
    equal cost of the Morton order, empty records padding the shorter runs)
    and walked by however many workgroups the launch has.  Each leaf's sums
    are made by one workgroup in a fixed order, so the product is the same
    bit for bit at any workgroup count, including counts that are not a
    multiple of 8 and counts above the number of records, and matches the
    oracle."""
    n = 20000
    xy = W.mixture_points(n, W.rng(97, 1), W.rng(97, 3))
    u = W.uniform_vector(n, W.rng(97, 2))
    c = 0.03
    tree = imq.build_tree(_dev(xy), c, leaf=32, p=12)
    rows = np.arange(0, n, 53)
    exact = oracle.matvec(xy, c, u, xy_targets=xy[rows])
    for prec, tol in (("fp64", 1e-6), ("fp32", 1e-5)):
        out = {}
        for wg in (0, 8, 100, 1 << 16):
            tree.set_kernel_config(p2p_wg=wg)
            out[wg] = tree.matvec(_dev(u), prec).cpu().numpy()
            assert _rel(out[wg][rows], exact) < tol, (prec, wg)
        for wg in (8, 100, 1 << 16):
            assert np.array_equal(out[wg], out[0]), (prec, wg)
    tree.set_kernel_config()


def test_caller_allocator_gives_the_same_products(imq):
    """A tree whose device memory comes from PyTorch's caching allocator
    (imq_build_tree_alloc) computes exactly what the default tree computes;
    its buffers are visible to PyTorch's memory accounting and are returned
    when the tree is freed."""
    d = W.small(6000)
    U = W.uniform_vector(6000, W.rng(69, 1), nrhs=2)
    base = imq.build_tree(_dev(d["xy"]), d["c"], leaf=32, p=10)
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    tree = imq.build_tree(_dev(d["xy"]), d["c"], leaf=32, p=10, allocator="torch")
    held = torch.cuda.memory_allocated() - before
    for prec in ("fp64", "fp32"):
        b0 = base.matvec(_dev(U), prec).cpu().numpy()
        b1 = tree.matvec(_dev(U), prec).cpu().numpy()
        assert np.array_equal(b0, b1), prec
    a0, _ = base.solve(_dev(d["u"]), tol=1e-6, max_iters=60)
    a1, _ = tree.solve(_dev(d["u"]), tol=1e-6, max_iters=60)
    assert torch.equal(a0, a1)
    grown = torch.cuda.memory_allocated() - before
    print(f"caller allocator: {held} bytes after the build, {grown} with workspaces")
    assert held > 0 and grown >= held
    tree.close()
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() <= before + (1 << 20)   # tensors of this test aside
    # the last call before the free was on the caller-allocated tree: a build
    # after it allocates with hipMalloc again, never through the freed tree
    src, tgt = d["xy"][:3000], d["xy"][3000:3400]
    ev = imq.build_eval_tree(_dev(src), d["c"], _dev(tgt), leaf=32, p=10)
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() <= before + (1 << 20)
    s = ev.evaluate(_dev(d["u"][:3000])).cpu().numpy()
    exact = oracle.matvec(src, d["c"], d["u"][:3000], xy_targets=tgt)
    assert _rel(s, exact) < 1e-6
    ev.close()
    base.close()


def test_shift_column_tiles_give_the_same_products(imq):
    """The FP32 shift kernels take parents in 16- or 32-column tiles
    (shift_cols); the tile width only regroups parents among workgroups, so
    both give the product to the FP32 target and agree to rounding."""
    d = W.small(6000)
    U = W.uniform_vector(6000, W.rng(70, 1), nrhs=3)
    tree = imq.build_tree(_dev(d["xy"]), d["c"], leaf=16, p=10)
    rows = np.arange(0, 6000, 37)
    exact = oracle.matvec(d["xy"], d["c"], U, xy_targets=d["xy"][rows])
    out = {}
    for cols in (16, 32):
        tree.set_kernel_config(shift_cols=cols)
        out[cols] = tree.matvec(_dev(U), "fp32").cpu().numpy()
        assert _rel(out[cols][:, rows], exact) < 1e-5, cols
    assert _rel(out[32], out[16]) < 1e-6
    tree.set_kernel_config()


def test_short_or_host_vectors_and_freed_handles_are_rejected(imq):
    import ctypes
    from paper_2205_04194_amd import _lib
    d = W.small(1000)
    tree = imq.build_tree(_dev(d["xy"]), d["c"], leaf=32, p=8)
    with pytest.raises(ValueError):
        tree.matvec(_dev(np.ones(999)))
    with pytest.raises(ValueError):
        tree.matvec(torch.ones(1000, dtype=torch.float64))          # host memory
    with pytest.raises(ValueError):
        tree.solve(_dev(np.ones(999)))
    with pytest.raises(ValueError):
        tree.solve(_dev(np.ones(1000)), a0=_dev(np.ones(999)))
    with pytest.raises(ValueError):
        tree.rows_exact(_dev(np.ones(1000)), torch.tensor([0, 1000], device="cuda:0"))
    u = _dev(np.ones(1000))
    b = torch.empty_like(u)
    h = tree._h
    tree.close()
    st = _lib.load().imq_matvec(h, 1, _lib.F64, ctypes.c_void_p(u.data_ptr()), 1000,
                                ctypes.c_void_p(b.data_ptr()), 1000, 0, None)
    assert st == -1 and "freed" in _lib.load().imq_last_error().decode()
