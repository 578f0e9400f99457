"""Parity at the headline size, in the configuration the benchmark times.

The 1M-point mixture (c = 0.02, leaf <= 64) is tuned exactly as bench.py
does it (autotuner to a 1e-6 sampled-row error, tree rebuilt at the highest
tuned order), then sampled rows of the product are compared with the FP64
oracle's rows computed one by one (direct compensated sums over all 1e6
sources).  The bar is the method's target: relative 2-norm error <= 1e-6.
The FP64 path at uniform p = 12 is held to the same bar.
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


def test_headline_configuration_matches_the_oracle_on_sampled_rows(imq):
    from paper_2205_04194_amd import autotune
    d = W.mixture1m()
    dev = torch.device("cuda:0")
    xy = torch.tensor(d["xy"], device=dev)
    u = torch.tensor(d["u"], device=dev)
    tree = imq.build_tree(xy, d["c"], leaf=64, p=12)
    rows = np.sort(np.random.default_rng(31).choice(len(d["xy"]), 256, replace=False))
    ref = oracle.matvec(d["xy"], d["c"], d["u"], xy_targets=d["xy"][rows])
    b64 = tree.matvec(u, "fp64").cpu().numpy()[rows]
    e64 = float(np.linalg.norm(b64 - ref) / np.linalg.norm(ref))
    res = autotune.tune(tree, u, target=1e-6, precisions=("fp32", "fp64"), seed=1)
    if max(res.level_orders) < 12:
        tree.close()
        tree = imq.build_tree(xy, d["c"], leaf=64, p=max(res.level_orders))
        tree.set_level_orders(res.level_orders)
        tree.set_kernel_config(m2l_kc=res.m2l_kc, m2l_split=res.m2l_split, m2l_mode=res.m2l_mode)
    b = tree.matvec(u, res.precision).cpu().numpy()[rows]
    err = float(np.linalg.norm(b - ref) / np.linalg.norm(ref))
    print(f"mixture1m: FP64 p=12 rel err {e64:.2e}; tuned {res.precision} {res.level_orders}: rel err {err:.2e}")
    assert e64 < 1e-6
    assert err < 1e-6
    tree.close()
