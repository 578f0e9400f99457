"""GPU GMRES with the leaf block-Jacobi right preconditioner, against the oracle.

Right preconditioning leaves the system A a = f unchanged, so the solves are
judged as the unpreconditioned ones are: by the oracle's residual with the
dense FP64 product and, on a well-conditioned system, by the direct solution.
The preconditioner's own effect is judged by the iteration count (fewer) and,
on the ill-conditioned 2 000-point workload where restarted GMRES stalls, by
the residual reached within a fixed budget of iterations (lower).
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


def _clustered(seed=3):
    """40 tight clusters of 20 points on a coarse grid, c below the clusters'
    scale: A is dominated by its within-cluster blocks, which are the
    preconditioner's runs."""
    g = W.rng(95, seed)
    centres = np.stack(np.meshgrid(np.arange(8), np.arange(5)), -1).reshape(-1, 2) * 0.12 + 0.06
    xy = np.concatenate([ctr + 0.004 * (g.random((20, 2)) - 0.5) for ctr in centres])
    W.assert_distinct(xy)
    f = W.franke(xy[:, 0], xy[:, 1])
    return xy, 0.0002, f


@pytest.mark.parametrize("case", ["clustered", "uniform"])
def test_preconditioned_solve_matches_the_direct_solution_in_fewer_iterations(imq, case):
    if case == "clustered":
        xy, c, f = _clustered()
        leaf, p = 32, 16
    else:
        xy = W.uniform_points(2000, W.rng(44, 1))
        c, f = 0.001, W.franke(xy[:, 0], xy[:, 1])
        leaf, p = 32, 16
    tree = imq.build_tree(_dev(xy), c, leaf=leaf, p=p)
    a0, st0 = tree.solve(_dev(f), tol=1e-10, restart=30, max_iters=600)
    a1, st1 = tree.solve(_dev(f), tol=1e-10, restart=30, max_iters=600, precond="block_jacobi")
    print(f"{case}: iterations {st0['iters']} without, {st1['iters']} with the preconditioner")
    assert st1["converged"] and st1["relres_fast64"] <= 1e-10
    a1 = a1.cpu().numpy()
    assert oracle.relres(xy, c, a1, f) < 1e-7
    ref, _ = oracle.solve_dense(xy, c, f)
    assert np.linalg.norm(a1 - ref) / np.linalg.norm(ref) < 1e-6
    assert st1["iters"] < st0["iters"]
    if case == "clustered":
        assert st1["iters"] <= st0["iters"] // 3


def test_preconditioned_mixed_refinement_and_several_columns(imq):
    xy, c, f = _clustered(seed=5)
    tree = imq.build_tree(_dev(xy), c, leaf=32, p=16)
    F = np.stack([f, np.cos(3 * xy[:, 0]) * xy[:, 1]])
    a, sts = tree.solve(_dev(F), tol=1e-10, restart=30, max_iters=600, mixed_ir=True, precond="block_jacobi")
    for r in range(2):
        assert sts[r]["converged"], sts[r]
        assert oracle.relres(xy, c, a[r].cpu().numpy(), F[r]) < 1e-7


def test_preconditioner_lowers_the_stalled_residual_of_an_ill_conditioned_system(imq):
    """N=2000 uniform, c=0.1 (kappa ~ 2e14): restarted GMRES stalls far above
    1e-10; within the same budget the preconditioned solve ends lower, and the
    residual it reports is the one the fast product gives for its solution."""
    d = W.small(2000)
    xy, c, f = d["xy"], d["c"], d["f"]
    tree = imq.build_tree(_dev(xy), c, leaf=32, p=14)
    res = {}
    for pc in ("none", "block_jacobi"):
        a, st = tree.solve(_dev(f), tol=1e-12, restart=50, max_iters=1500, precond=pc)
        b = tree.matvec(a, "fp64").cpu().numpy()
        rr = np.linalg.norm(f - b) / np.linalg.norm(f)
        assert abs(rr - st["relres_fast64"]) <= 1e-3 * st["relres_fast64"] + 1e-14
        res[pc] = st["relres_fast64"]
        print(f"{pc}: relres {st['relres_fast64']:.3e} after {st['iters']} iterations, "
              f"oracle {oracle.relres(xy, c, a.cpu().numpy(), f):.3e}")
    assert res["block_jacobi"] < res["none"]


def test_unknown_preconditioner_is_rejected(imq):
    xy, c, f = _clustered()
    tree = imq.build_tree(_dev(xy), c, leaf=32, p=8)
    with pytest.raises(ValueError):
        tree.solve(_dev(f), precond="ilu")
