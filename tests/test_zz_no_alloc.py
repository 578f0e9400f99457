"""imq_matvec_noalloc (the product that allocates nothing) against imq_matvec,
called through the C interface: two calls in a row on one device, the
second on a smaller input, each compared with the allocating product on
the same tree (same kernels, stages in another order: the FP64 results
agree to rounding) and with the oracle."""
import ctypes

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


def _noalloc(tree, u, prec):
    from paper_2205_04194_amd import _lib
    lib = _lib.load()
    u2 = (u.unsqueeze(0) if u.dim() == 1 else u).contiguous()
    b = torch.full_like(u2, float("nan"))
    dt = _lib.F64 if u2.dtype == torch.float64 else _lib.F32
    st = lib.imq_matvec_noalloc(tree._h, u2.shape[0], dt, ctypes.c_void_p(u2.data_ptr()), tree.n,
                                ctypes.c_void_p(b.data_ptr()), tree.n, _lib.PREC[prec],
                                ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    _lib.check(st, "imq_matvec_noalloc")
    return b[0] if u.dim() == 1 else b


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - b) / np.linalg.norm(b))


def test_noalloc_product_matches_the_allocating_product(imq):
    from paper_2205_04194_amd import _lib
    assert _lib.load().imq_matvec_noalloc_max_bytes() == 128 << 20
    cases = [  # (points, rhs, generator id): the second call is smaller
        (30000, 3, 61),
        (4000, 1, 62),
    ]
    for n, nrhs, gid in cases:
        xy = W.mixture_points(n, W.rng(gid, 3), W.rng(gid, 0))
        U = W.uniform_vector(n, W.rng(gid, 2), nrhs=nrhs)
        tree = imq.build_tree(torch.tensor(xy, device="cuda:0"), 0.02, leaf=64, p=12)
        u = torch.tensor(U, device="cuda:0")
        for prec, tol in (("fp64", 1e-12), ("fp32", 1e-5)):
            ref = tree.matvec(u, prec)
            b = _noalloc(tree, u, prec)
            torch.cuda.synchronize()
            assert not torch.isnan(b).any()
            e = float(torch.linalg.norm(b - ref) / torch.linalg.norm(ref))
            print(f"N={n} nrhs={nrhs} {prec}: no-alloc vs imq_matvec {e:.2e}", flush=True)
            assert e <= tol
            # the allocating product still works after the no-alloc call
            assert torch.equal(tree.matvec(u, prec), ref)
        rows = np.sort(np.random.default_rng(gid).choice(n, 200, replace=False))
        ref = oracle.matvec(xy, 0.02, U, xy_targets=xy[rows])
        b = _noalloc(tree, u, "fp64").cpu().numpy()
        assert _rel(b[..., rows], ref) <= 1e-6
        tree.close()


def test_noalloc_rejects_a_product_beyond_its_workspace(imq):
    from paper_2205_04194_amd import _lib
    xy = W.uniform_points(20000, W.rng(63, 0))
    tree = imq.build_tree(torch.tensor(xy, device="cuda:0"), 0.05, leaf=64, p=12)
    u = torch.zeros((1000, 20000), dtype=torch.float64, device="cuda:0")   # ~300 MB of workspace
    with pytest.raises(_lib.IMQError, match="workspace"):
        _noalloc(tree, u, "fp64")
    tree.close()
