"""MI355X (gfx950) fast product with the inverse-multiquadric interpolation matrix.

The method (arXiv 2205.04194, Sec. 2): A_ij = 1/sqrt(|x_i - x_j|^2 + c^2) is
the 3-D Laplace Green's function between the points lifted to z = -c/2 and
z = +c/2, so the product b = A u is evaluated with the truncated spectral
expansion of that Green's function on a quadtree (expansions, translations,
and a direct near field), all in HIP kernels behind the C interface of
include/imq.h.  This module only marshals torch tensors (device memory and
the current stream) into those calls.

    tree = build_tree(xy, c, leaf=64, p=12)     # xy: (N, 2) float64 on cuda
    b = tree.matvec(u, prec="fp64")             # u: (N,) or (nrhs, N)
"""
from __future__ import annotations

import ctypes
from typing import Optional, Sequence

import torch

from . import _lib
from ._lib import IMQError, PREC

__all__ = ["Tree", "build_tree", "build_eval_tree", "matvec", "solve", "IMQMatvec", "IMQError"]


def _stream_ptr(stream=None) -> ctypes.c_void_p:
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _dptr(t: torch.Tensor) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr())


def _check_vec(t: torch.Tensor, name: str, n: int, device, allow_2d: bool = True) -> None:
    """Reject a tensor that the library would read out of bounds or from host
    memory: it must be a float64/float32 tensor on the tree's device, of
    shape (n,) or (nrhs, n)."""
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if not t.is_cuda or t.device != device:
        raise ValueError(f"{name} must be on the tree's device {device} (got {t.device})")
    if t.dtype not in (torch.float64, torch.float32):
        raise ValueError(f"{name} must be float64 or float32 (got {t.dtype})")
    if t.dim() not in ((1, 2) if allow_2d else (1,)) or t.shape[-1] != n or (t.dim() == 2 and t.shape[0] < 1):
        want = f"({n},) or (nrhs, {n})" if allow_2d else f"({n},)"
        raise ValueError(f"{name} must have shape {want} (got {tuple(t.shape)})")


def _torch_allocator(device) -> "_lib.Allocator":
    """imq_allocator over PyTorch's caching allocator (the callbacks are kept
    alive by the returned structure's owner, the Tree)."""
    def alloc(nbytes, ctx):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), device=device)
        except Exception:          # out of memory: the library reports IMQ_ENOMEM
            return None

    def free(ptr, ctx):
        torch.cuda.caching_allocator_delete(ptr)

    a = _lib.Allocator(_lib.ALLOC_FN(alloc), _lib.FREE_FN(free), None)
    a._keep = (alloc, free)
    return a


class Tree:
    """A quadtree forest over one or more point sets, resident on the GPU.

    xy          (Ntot, 2) float64 cuda tensor, the sets concatenated
    c           shape parameter (float) or one per set
    set_offsets None (one set) or nsets+1 offsets into xy
    leaf        points per leaf before a box is split (leaf_max)
    p           truncation index of the expansions (1..16)
    level_order optional per-level truncation of the translations
    direct_max  W/X interactions with at most this many points in the finer
                box are summed directly (0: 2*leaf, negative: never)
    allocator   None (the library's hipMalloc) or "torch": the tree's device
                memory comes from PyTorch's caching allocator
    autotune    tune orders, precision and kernels in the library after the
                build for a sampled-row relative error <= autotune_tol (0:
                1e-6); info() then reports tuned_prec ("fp64"/"fp32"),
                tuned_err and tuned_ms, and `tuned_prec` holds the choice
    """

    def __init__(self, xy: torch.Tensor, c, leaf: int = 64, p: int = 12,
                 set_offsets: Optional[Sequence[int]] = None, level_order=None,
                 max_level: int = 0, direct_max: int = 0, stream=None, allocator=None,
                 autotune: bool = False, autotune_tol: float = 0.0):
        lib = _lib.load()
        if xy.dim() != 2 or xy.shape[1] != 2:
            raise ValueError("xy must have shape (N, 2)")
        if not xy.is_cuda:
            raise ValueError("xy must be a cuda tensor")
        xy64 = xy.detach().to(torch.float64)
        soa = xy64.t().contiguous()
        n = xy.shape[0]
        offs = [0, n] if set_offsets is None else [int(v) for v in set_offsets]
        nsets = len(offs) - 1
        cs = [float(c)] * nsets if not hasattr(c, "__len__") else [float(v) for v in c]
        if len(cs) != nsets:
            raise ValueError("need one shape parameter per set")
        self.n = n
        self.nsets = nsets
        self.offsets = offs
        self.c = cs
        self.leaf = leaf
        self.p = p
        self.device = xy.device
        self._xy = xy64
        off_arr = (ctypes.c_int64 * (nsets + 1))(*offs)
        c_arr = (ctypes.c_double * nsets)(*cs)
        prm = _lib.params(leaf, p, max_level, level_order, direct_max, autotune, autotune_tol)
        h = ctypes.c_void_p()
        self._alloc = None
        if allocator not in (None, "torch"):
            raise ValueError('allocator must be None or "torch"')
        with torch.cuda.device(self.device):
            if allocator == "torch":
                self._alloc = _torch_allocator(self.device)
                st = lib.imq_build_tree_alloc(nsets, off_arr, _dptr(soa), c_arr, ctypes.byref(prm),
                                              ctypes.byref(self._alloc), _stream_ptr(stream), ctypes.byref(h))
            else:
                st = lib.imq_build_tree(nsets, off_arr, _dptr(soa), c_arr, ctypes.byref(prm),
                                        _stream_ptr(stream), ctypes.byref(h))
        _lib.check(st, "imq_build_tree")
        self._h = h
        self.tuned_prec = None
        if autotune:
            self.tuned_prec = self.info()["tuned_prec"]

    # ------------------------------------------------------------ evaluation
    @classmethod
    def for_evaluation(cls, xy_src: torch.Tensor, c: float, xy_tgt: torch.Tensor, leaf: int = 64,
                       p: int = 12, level_order=None, max_level: int = 0, direct_max: int = 0,
                       stream=None) -> "Tree":
        """Tree over data sites and evaluation points together (imq_build_eval_tree)."""
        lib = _lib.load()
        for a in (xy_src, xy_tgt):
            if a.dim() != 2 or a.shape[1] != 2 or not a.is_cuda:
                raise ValueError("xy_src and xy_tgt must be cuda tensors of shape (n, 2)")
        self = cls.__new__(cls)
        # SoA copies held in locals for the duration of the call (a temporary
        # passed by pointer could be freed and its memory reused before the
        # library reads it)
        src = xy_src.detach().to(torch.float64).t().contiguous()
        tgt = xy_tgt.detach().to(torch.float64).t().contiguous()
        self.n_src, self.m_eval = xy_src.shape[0], xy_tgt.shape[0]
        self.nsets, self.c, self.leaf, self.p = 1, [float(c)], leaf, p
        self.device = xy_src.device
        prm = _lib.params(leaf, p, max_level, level_order, direct_max)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            st = lib.imq_build_eval_tree(_dptr(src), self.n_src, _dptr(tgt),
                                         self.m_eval, float(c), ctypes.byref(prm), _stream_ptr(stream),
                                         ctypes.byref(h))
        _lib.check(st, "imq_build_eval_tree")
        self._h = h
        self.n = int(self.info()["npoints"])
        self.offsets = [0, self.n]
        self._xy = None
        return self

    def evaluate(self, lam: torch.Tensor, prec: str = "fp64", stream=None) -> torch.Tensor:
        """Interpolant sum_j lam_j phi(|y_k - x_j|) at the evaluation points: (m,) or (nrhs, m)."""
        lib = _lib.load()
        _check_vec(lam, "lam", self.n_src, self.device)
        one = lam.dim() == 1
        l2 = (lam.unsqueeze(0) if one else lam).contiguous()
        s = torch.empty((l2.shape[0], self.m_eval), dtype=l2.dtype, device=self.device)
        dt = _lib.F64 if l2.dtype == torch.float64 else _lib.F32
        with torch.cuda.device(self.device):
            st = lib.imq_evaluate(self._h, l2.shape[0], dt, _dptr(l2), self.n_src, _dptr(s),
                                  max(self.m_eval, 1), PREC[prec], _stream_ptr(stream))
        _lib.check(st, "imq_evaluate")
        return s[0] if one else s

    # ----------------------------------------------------------------- product
    def matvec(self, u: torch.Tensor, prec: str = "fp64", stream=None) -> torch.Tensor:
        """b = A u; u is (N,) or (nrhs, N), float64 or float32, on the tree's device."""
        lib = _lib.load()
        _check_vec(u, "u", self.n, self.device)
        one = u.dim() == 1
        u2 = (u.unsqueeze(0) if one else u).contiguous()
        b = torch.empty_like(u2)
        dt = _lib.F64 if u2.dtype == torch.float64 else _lib.F32
        with torch.cuda.device(self.device):
            st = lib.imq_matvec(self._h, u2.shape[0], dt, _dptr(u2), self.n, _dptr(b), self.n,
                                PREC[prec], _stream_ptr(stream))
        _lib.check(st, "imq_matvec")
        return b[0] if one else b

    def rows_exact(self, u: torch.Tensor, rows: torch.Tensor, stream=None) -> torch.Tensor:
        """Exact FP64 rows of A u (direct sums) for the given row indices."""
        lib = _lib.load()
        _check_vec(u, "u", self.n, self.device)
        one = u.dim() == 1
        u2 = (u.unsqueeze(0) if one else u).to(torch.float64).contiguous()
        rows = rows.to(device=self.device, dtype=torch.int64).contiguous()
        if rows.dim() != 1:
            raise ValueError("rows must be a 1-D index tensor")
        if rows.numel() and (int(rows.min()) < 0 or int(rows.max()) >= self.n):
            raise ValueError("row index out of range")
        b = torch.empty((u2.shape[0], rows.numel()), dtype=torch.float64, device=self.device)
        with torch.cuda.device(self.device):
            st = lib.imq_rows_exact(self._h, u2.shape[0], _dptr(u2), self.n, rows.numel(),
                                    _dptr(rows), _dptr(b), rows.numel(), _stream_ptr(stream))
        _lib.check(st, "imq_rows_exact")
        return b[0] if one else b

    # ----------------------------------------------------------------- solve
    def solve(self, f: torch.Tensor, tol: float = 1e-10, restart: int = 50,
              max_iters: int = 2000, mixed_ir: bool = False, max_outer: int = 10,
              a0: Optional[torch.Tensor] = None, history: bool = False, precond: str = "none",
              stream=None):
        """GMRES on the fast product: returns (a, stats).  stats["relres_fast64"]
        is the final residual with the FP64 fast product (the operator the
        solver works with), not with the exact matrix.  precond: "none" or
        "block_jacobi" (leaf blocks, on the right)."""
        lib = _lib.load()
        _check_vec(f, "f", self.n, self.device)
        one = f.dim() == 1
        f2 = (f.unsqueeze(0) if one else f).to(torch.float64).contiguous()
        if a0 is None:
            a = torch.zeros_like(f2)
        else:
            _check_vec(a0, "a0", self.n, self.device)
            if a0.shape != f.shape:
                raise ValueError(f"a0 must have the shape of f {tuple(f.shape)} (got {tuple(a0.shape)})")
            a = (a0.unsqueeze(0) if one else a0).to(torch.float64).contiguous().clone()
        nrhs = f2.shape[0]
        hist = (ctypes.c_double * (nrhs * int(max_iters)))() if history else None
        pcs = {"none": 0, "block_jacobi": 1}
        if precond not in pcs:
            raise ValueError(f"precond must be one of {sorted(pcs)} (got {precond!r})")
        opts = _lib.SolveOpts(float(tol), int(restart), int(max_iters), int(bool(mixed_ir)),
                              int(max_outer), hist, pcs[precond])
        stats = (_lib.SolveStats * nrhs)()
        with torch.cuda.device(self.device):
            st = lib.imq_solve(self._h, nrhs, _dptr(f2), self.n, _dptr(a), self.n,
                               ctypes.byref(opts), stats, _stream_ptr(stream))
        _lib.check(st, "imq_solve", allow_not_converged=True)
        out = [dict(iters=s.iters, outer_iters=s.outer_iters, converged=bool(s.converged),
                    relres_fast64=s.relres_fast64) for s in stats]
        if history:
            for r, d in enumerate(out):
                d["history"] = list(hist[r * int(max_iters):r * int(max_iters) + min(d["iters"], int(max_iters))])
        return (a[0] if one else a), (out[0] if one else out)

    # ----------------------------------------------------------------- adjoint
    def backward(self, v: torch.Tensor, g: torch.Tensor, prec: str = "fp64", stream=None):
        """Adjoint of B = A(c, X) V for upstream G = dL/dB: returns
        (A G, dL/dc per set, dL/dxy), with v and g of shape (N,) or (nrhs, N)
        (the derivatives in c and xy summed over the columns)."""
        lib = _lib.load()
        _check_vec(v, "v", self.n, self.device)
        _check_vec(g, "g", self.n, self.device)
        if g.shape != v.shape:
            raise ValueError(f"g must have the shape of v {tuple(v.shape)} (got {tuple(g.shape)})")
        dt = _lib.F64 if v.dtype == torch.float64 else _lib.F32
        one = v.dim() == 1
        v2 = (v.unsqueeze(0) if one else v).contiguous()
        g2 = (g.unsqueeze(0) if one else g).to(v.dtype).contiguous()
        nrhs = v2.shape[0]
        dv = torch.empty_like(v2)
        dc = torch.zeros(self.nsets, dtype=torch.float64, device=self.device)
        dxy = torch.zeros((2, self.n), dtype=torch.float64, device=self.device)
        with torch.cuda.device(self.device):
            st = lib.imq_matvec_backward(self._h, nrhs, dt, _dptr(v2), self.n, _dptr(g2), self.n, _dptr(dv),
                                         self.n, _dptr(dc), _dptr(dxy), PREC[prec], _stream_ptr(stream))
        _lib.check(st, "imq_matvec_backward")
        return (dv[0] if one else dv), dc, dxy.t()

    # ----------------------------------------------------------------- info
    def info(self) -> dict:
        lib = _lib.load()
        inf = _lib.TreeInfo()
        _lib.check(lib.imq_get_tree_info(self._h, ctypes.byref(inf)), "imq_get_tree_info")
        out = {}
        for k, _ in _lib.TreeInfo._fields_:
            v = getattr(inf, k)
            out[k] = list(v)[:inf.nlevels] if k.startswith("level_") else v
        out["tuned_prec"] = {0: "fp64", 1: "fp32"}.get(out["tuned_prec"])   # None: not tuned
        return out

    def set_kernel_config(self, m2l_kc: int = 0, m2l_split: int = 0, shift_cols: int = 0,
                          m2l_mode: int = 0, p2p_wg: int = 0, p2p_mode: int = 0,
                          far_field: int = 0) -> None:
        """Launch shape of the batched translations and the near field (0 = default);
        far_field = 1 selects the paper's Algorithm 1 for the far field."""
        cfg = _lib.KernelConfig(m2l_kc, m2l_split, shift_cols, m2l_mode, p2p_wg, p2p_mode, far_field)
        _lib.check(_lib.load().imq_set_kernel_config(self._h, ctypes.byref(cfg)),
                   "imq_set_kernel_config")

    def set_level_orders(self, orders) -> None:
        """Per-level truncation of the translations (0 = order p)."""
        arr = (ctypes.c_int * max(1, len(orders)))(*[int(o) for o in orders])
        _lib.check(_lib.load().imq_set_level_orders(self._h, len(orders), arr), "imq_set_level_orders")

    def set_stage_timing(self, on: bool = True) -> None:
        _lib.check(_lib.load().imq_set_stage_timing(self._h, int(on)), "imq_set_stage_timing")

    def stage_times(self) -> dict:
        lib = _lib.load()
        arr = (ctypes.c_double * _lib.IMQ_NSTAGES)()
        _lib.check(lib.imq_get_stage_times(self._h, arr), "imq_get_stage_times")
        return {lib.imq_stage_name(k).decode(): arr[k] for k in range(_lib.IMQ_NSTAGES)}

    def close(self) -> None:
        if getattr(self, "_h", None):
            _lib.load().imq_tree_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def build_tree(xy, c, leaf: int = 64, p: int = 12, **kw) -> Tree:
    return Tree(xy, c, leaf=leaf, p=p, **kw)


def build_eval_tree(xy_src, c, xy_tgt, leaf: int = 64, p: int = 12, **kw) -> Tree:
    """Tree for evaluating the interpolant of the data sites xy_src at xy_tgt."""
    return Tree.for_evaluation(xy_src, c, xy_tgt, leaf=leaf, p=p, **kw)


def matvec(tree: Tree, u: torch.Tensor, prec: str = "fp64") -> torch.Tensor:
    return tree.matvec(u, prec)


def solve(tree: Tree, f: torch.Tensor, **kw):
    return tree.solve(f, **kw)


class IMQMatvec(torch.autograd.Function):
    """B = A(c, X) V with gradients for V, c and X through the adjoint kernels.

    xy: (N, 2) cuda tensor; c: a float or a 0-d tensor (a gradient for c is
    returned only when c is a tensor that requires it); v: (N,) or (nrhs, N).
    The tree is rebuilt from the saved (X, c) in backward, so no interaction
    list is kept alive between the passes.
    """

    @staticmethod
    def forward(ctx, xy, c, v, leaf: int = 64, p: int = 12, prec: str = "fp64"):
        cval = float(c)
        tree = Tree(xy.detach(), cval, leaf=leaf, p=p)
        b = tree.matvec(v.detach(), prec)
        tree.close()
        ctx.save_for_backward(xy, v)
        ctx.c = cval
        ctx.c_is_tensor = isinstance(c, torch.Tensor)
        ctx.c_dtype = c.dtype if ctx.c_is_tensor else None
        ctx.cfg = (leaf, p, prec)
        return b

    @staticmethod
    def backward(ctx, gb):
        xy, v = ctx.saved_tensors
        leaf, p, prec = ctx.cfg
        # the lists are rebuilt here (not kept from forward)
        tree = Tree(xy.detach(), ctx.c, leaf=leaf, p=p)
        dv, dc, dxy = tree.backward(v.detach(), gb.detach().to(v.dtype).contiguous(), prec)
        tree.close()
        gxy = dxy.to(xy.dtype) if ctx.needs_input_grad[0] else None
        gc = None
        if ctx.c_is_tensor and ctx.needs_input_grad[1]:
            gc = dc[0].to(ctx.c_dtype)
        gv = dv.to(v.dtype) if ctx.needs_input_grad[2] else None
        return gxy, gc, gv, None, None, None
