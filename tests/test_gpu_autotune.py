"""GPU tests of the autotuner: the configuration it returns meets its error
target against the dense FP64 oracle, and the tree is left configured with it."""
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


@pytest.mark.parametrize("target", [1e-5, 1e-6])
def test_tuned_configuration_meets_the_target_against_the_oracle(imq, target):
    from paper_2205_04194_amd import autotune
    d = W.uniform100k()
    xy, u = d["xy"][:30000], d["u"][:30000]
    tree = imq.build_tree(_dev(xy), d["c"], leaf=64, p=12)
    res = autotune.tune(tree, _dev(u), target=target, nrows=500)
    assert res.error <= 0.8 * target
    assert len(res.level_orders) == tree.info()["nlevels"]
    assert all(1 <= o <= 12 for o in res.level_orders)
    # the tree keeps the tuned configuration: an independent row sample
    rows = np.arange(7, 30000, 61)
    b = tree.matvec(_dev(u), res.precision).cpu().numpy()
    exact = oracle.matvec(xy, d["c"], u, xy_targets=xy[rows])
    err = float(np.linalg.norm(b[rows] - exact) / np.linalg.norm(exact))
    assert err <= target
    assert tree.info()["level_K"] == [(o + 1) * (o + 2) // 2 for o in res.level_orders]
