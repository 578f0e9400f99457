"""The device construction of the forest against the host construction,
array for array and bit for bit: point order, leaf-local coordinates, the
boxes, the U/V/W/X lists (after the moves of the small W/X interactions),
the shift lists, the translation batches' inputs and the near-field flags
(Sec. 2.2: the hierarchical partition and the well-separated / near
classification).  Inputs: uniform and clustered points, the 256-set forest,
every direct_max form, tiny and degenerate sets, and the 1M-point mixture."""
import numpy as np
import pytest

import workloads as W
from tests import _hostlib as H

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _same_trees(xy_list, c_list, leaf, **kw):
    hh, sh = H.host_tree(xy_list, c_list, leaf, **kw)
    hd, sd = H.device_tree(xy_list, c_list, leaf, **kw)
    assert sh == sd
    if sh != 0:
        return sh
    try:
        for f in H.FIELDS:
            a, b = H.get(hh, f), H.get(hd, f)
            assert a.dtype == b.dtype and a.shape == b.shape, f
            assert np.array_equal(a.view(np.uint8), b.view(np.uint8)), f
    finally:
        H.free(hh)
        H.free(hd)
    return 0


@pytest.mark.parametrize("n,leaf", [(20000, 32), (20000, 1), (5000, 200)])
def test_uniform_points(n, leaf):
    xy = W.uniform_points(n, W.rng(91, n))
    assert _same_trees([xy], [0.05], leaf, p=8) == 0


@pytest.mark.parametrize("direct_max", [0, -1, 5, 100000])
def test_clustered_points_every_direct_max(direct_max):
    xy = W.mixture_points(50000, W.rng("mixture1m", 3), W.rng(91, 7))
    assert _same_trees([xy], [0.02], 64, p=12, direct_max=direct_max) == 0


def test_the_256_set_forest():
    d = W.batched_sets()
    offs = d["offsets"]
    sets = [d["xy"][offs[s]:offs[s + 1]] for s in range(len(offs) - 1)]
    assert _same_trees(sets, list(d["c"]), d["leaf"], p=d["p"]) == 0


def test_tiny_and_degenerate_sets():
    g = W.rng(91, 11)
    line = np.stack([np.full(300, 0.25), g.uniform(0, 1, 300)], axis=1)      # one x: zero width
    grid = np.stack(np.meshgrid(np.arange(16) / 16, np.arange(16) / 16), -1).reshape(-1, 2)  # on box edges
    sets = [np.array([[0.3, 0.7]]), g.uniform(0, 1, (2, 2)), g.uniform(0, 1, (3, 2)), line, grid,
            g.uniform(-5e3, 5e3, (1000, 2))]
    assert _same_trees(sets, [0.1, 0.2, 0.3, 0.05, 0.01, 7.0], 4, p=6) == 0
    for s in sets:
        assert _same_trees([s], [0.1], 1, p=3, max_level=3) == 0


def test_errors_match():
    xy = W.uniform_points(100, W.rng(91, 12))
    dup = np.concatenate([xy, xy[5:6]])
    assert _same_trees([dup], [0.1], 8) == -2                    # IMQ_EDUPLICATE
    bad = xy.copy()
    bad[7, 1] = np.nan
    assert _same_trees([bad], [0.1], 8) == -1                    # IMQ_EINVAL


def test_mixture1m():
    d = W.mixture1m()
    assert _same_trees([d["xy"]], [d["c"]], 64, p=12) == 0


@pytest.mark.parametrize("p", [3, 8, 12, 16])
def test_device_translation_tables_equal_the_host_tables(p):
    """The M2L tables generated on the device (four layouts) against the host
    generation of the same operator, for a two-set forest with different c."""
    import ctypes
    from paper_2205_04194_amd import _lib
    import paper_2205_04194_amd as imq
    g = W.rng(92, p)
    sets = [W.uniform_points(3000, g), W.uniform_points(2000, g) * 3.0]
    cs = [0.05, 0.4]
    offs = [0, 3000, 5000]
    tree = imq.build_tree(torch.tensor(np.concatenate(sets), device="cuda:0"), cs, leaf=16, p=p,
                          set_offsets=offs)
    K = (p + 1) * (p + 2) // 2
    KP = (K + 15) // 16 * 16
    nlev = tree.info()["nlevels"]
    side = [np.ptp(s_, axis=0).max() * (1 + 2.0 ** -20) for s_ in sets]
    lib = _lib.load()
    checked = 0
    for s_ in range(2):
        cn = cs[s_] / side[s_]
        for l in (2, nlev - 1):
            for cls in (0, 3 * 7 + 1, 48, 2 * 7 + 5):
                dx, dy = cls // 7 - 3, cls % 7 - 3
                ref = H.table(2, p, level=l, dx=dx, dy=dy, cnorm=cn).reshape(K, K)
                refp = np.zeros((KP, KP))
                refp[:K, :K] = ref
                out = [np.empty(KP * KP, dtype=np.float64 if lay < 2 else np.float32) for lay in range(4)]
                for lay in range(4):
                    assert lib.imq_debug_tree_table(tree._h, s_, l, cls, lay,
                                                    out[lay].ctypes.data_as(ctypes.c_void_p)) == KP
                t64 = out[0].reshape(KP, KP)
                err = np.abs(t64 - refp).max() / np.abs(refp).max()
                assert err <= 1e-15, (s_, l, cls, err)
                assert np.array_equal(out[2].reshape(KP, KP), t64.astype(np.float32))
                # lane order: element j of lane q of chunk (rb, ci) is T[16 rb + q % 16][16 ci + 4 (q / 16) + j]
                pk = out[1].reshape(KP // 16, KP // 16, 64, 4)
                rb, ci, q, j = np.meshgrid(np.arange(KP // 16), np.arange(KP // 16), np.arange(64), np.arange(4),
                                           indexing="ij")
                assert np.array_equal(pk, t64[16 * rb + q % 16, 16 * ci + 4 * (q // 16) + j])
                assert np.array_equal(out[3], out[1].astype(np.float32))
                checked += 1
    assert checked == 16
    tree.close()
