"""Autotuner for the fast product: translation orders per level, precision
and the launch shape of the translation batches.

The error of a configuration is measured, never modelled: the product is
compared on a sample of rows with exact FP64 direct sums computed on the GPU
(``Tree.rows_exact``).  The cost model of Sec. 2.3 is not used; the time of a
configuration is measured with events.

Search on one tree (``tune``, no rebuild):
  1. for each precision, the uniform order p is lowered from the tree's order
     while the sampled error stays within the target;
  2. per level, deepest first, the translation order is lowered while the
     error stays within the target (the lifted vertical offset c makes deep
     levels, whose boxes are small next to c, converge fastest); orders that
     fill the same 16-row matrix-core tiles cost the same, so each level is
     then raised to the top of its tile and levels are moved down by whole
     tiles, the most translation work first, while the error allows (on the
     1M mixture: 0.428 -> 0.421 ms per FP64 product, error 8.5e-7 -> 6.0e-7;
     kept only where it measures faster);
  3. the M2L kernel choice (register streaming or staged GEMM) and the staged
     GEMM's pipeline depth and row split are timed and the fastest kept;
  4. so is the number of near-field workgroups running beside the tree
     passes (their share of the CUs).
``tune_tree`` then rebuilds the tree at the highest tuned order (multipoles
need no more), and ``tune_leaf`` repeats all of it for several leaf
capacities, keeping the fastest tree: the level/leaf trade-off of the cost
model of Sec. 2.3 (eq. total_cost), measured instead of modelled.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np
import torch


@dataclass
class TuneResult:
    precision: str
    level_orders: List[int]
    m2l_kc: int
    m2l_split: int
    error: float
    ms: float
    m2l_mode: int = 0
    trials: List[dict] = field(default_factory=list)
    p2p_wg: int = 0


def _error(tree, u, rows, exact, prec):
    b = tree.matvec(u, prec)
    return float(torch.linalg.norm(b[..., rows] - exact) / torch.linalg.norm(exact))


def _time(tree, u, prec, reps=5, batches=2):
    """ms per product: the fastest of `batches` event-timed runs of `reps`
    back-to-back products, after two untimed ones (single runs differ by a
    few percent, enough to pick the wrong one of two close candidates)."""
    for _ in range(2):
        tree.matvec(u, prec)
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(batches):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            tree.matvec(u, prec)
        e1.record()
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1) / reps)
    return best


def _nrb(o: int) -> int:
    """16-row tiles of a translation of order o ((o+1)(o+2)/2 coefficients)."""
    return ((o + 1) * (o + 2) // 2 + 15) // 16


def _tile_top(o: int, pmax: int) -> int:
    """The largest order <= pmax whose translation fills the same tiles as o."""
    while o + 1 <= pmax and _nrb(o + 1) == _nrb(o):
        o += 1
    return o


def _tile_refine(tree, u, rows, exact, prec, orders, err, active, info, pmax, budget, trials):
    """Orders that fill the same 16-row tiles cost the same matrix-core work:
    raise every translated level to the top of its tile (less error, no
    matrix-core cost), then move levels down by whole tiles, those with the
    most translation work first, while the error stays within the budget.
    The shifts and L2P do grow with the orders, and levels of different tile
    counts run as separate launches, so the refined orders are kept only if
    the product is measured faster than with the greedy ones."""
    greedy, greedy_err = list(orders), err
    raised = [_tile_top(o, pmax) if l in active else o for l, o in enumerate(orders)]
    if raised != orders:
        tree.set_level_orders(raised)
        e = _error(tree, u, rows, exact, prec)
        trials.append({"prec": prec, "orders": list(raised), "err": e, "step": "tile top"})
        if e <= budget:
            orders, err = raised, e
    pairs = info["level_m2l_pairs"]
    for l in sorted(active, key=lambda l: -pairs[l] * _nrb(orders[l])):
        while _nrb(orders[l]) > 1:
            lower = orders[l]
            while lower > 1 and _nrb(lower) == _nrb(orders[l]):
                lower -= 1
            trial = list(orders)
            trial[l] = lower
            tree.set_level_orders(trial)
            e = _error(tree, u, rows, exact, prec)
            trials.append({"prec": prec, "orders": list(trial), "err": e, "step": "tile down"})
            if e > budget:
                break
            orders, err = trial, e
    if orders != greedy:
        tree.set_level_orders(greedy)
        t_greedy = _time(tree, u, prec, reps=10)
        tree.set_level_orders(orders)
        t_refined = _time(tree, u, prec, reps=10)
        trials.append({"prec": prec, "orders": list(orders), "ms": t_refined, "greedy_ms": t_greedy,
                       "step": "tile refine"})
        if t_refined >= t_greedy:
            orders, err = greedy, greedy_err
    tree.set_level_orders(orders)
    return orders, err


def tune(tree, u: torch.Tensor, target: float = 1e-6, precisions=("fp32", "fp64"),
         nrows: int = 1000, safety: float = 0.8, seed: int = 0,
         kcs=(16, 32, 64), splits=(1, 2), modes=(0, 1, 2, 3), p2p_wgs=(2048, 2560, 3072, 3584),
         tile_aware: bool = True) -> TuneResult:
    """Fastest configuration of ``tree`` whose sampled-row relative 2-norm
    error is at most ``safety * target``; the tree is left configured."""
    n = tree.n
    g = np.random.default_rng(seed)
    rows = torch.tensor(np.sort(g.choice(n, min(nrows, n), replace=False)), device=tree.device)
    exact = tree.rows_exact(u, rows)
    info = tree.info()
    nlev = info["nlevels"]
    pmax = info["order_p"]
    active = [l for l in range(nlev) if info["level_m2l_pairs"][l] > 0]
    budget = safety * target
    best: Optional[TuneResult] = None
    trials = []
    for prec in precisions:
        orders = [pmax] * nlev
        tree.set_level_orders(orders)
        tree.set_kernel_config()
        err = _error(tree, u, rows, exact, prec)      # default kernels while the orders are searched
        trials.append({"prec": prec, "orders": list(orders), "err": err})
        if err > budget:
            continue
        # 1. lower the uniform order
        while orders[0] > 2:
            trial = [o - 1 for o in orders]
            tree.set_level_orders(trial)
            e = _error(tree, u, rows, exact, prec)
            trials.append({"prec": prec, "orders": list(trial), "err": e})
            if e > budget:
                break
            orders, err = trial, e
        tree.set_level_orders(orders)
        # 2. lower the deep levels further
        for l in reversed(active):
            while orders[l] > 1:
                trial = list(orders)
                trial[l] -= 1
                tree.set_level_orders(trial)
                e = _error(tree, u, rows, exact, prec)
                trials.append({"prec": prec, "orders": list(trial), "err": e})
                if e > budget:
                    break
                orders, err = trial, e
        tree.set_level_orders(orders)
        if tile_aware:
            orders, err = _tile_refine(tree, u, rows, exact, prec, orders, err, active, info, pmax, budget,
                                       trials)
        # 3. translation kernels and the launch shape of the staged GEMM
        shape, ms = (0, 0, 0), float("inf")
        wide = max(orders) >= 12                   # translations above 80 coefficients
        for mode in modes:
            if prec == "fp64" and mode == 2:       # the BF16 form serves FP32 only
                continue
            if mode == 3 and not wide:             # the same kernels as mode 0
                continue
            for kc in (kcs if mode != 3 else kcs[:1]):   # mode 3 has no staged GEMM
                if prec == "fp64" and kc > 32:
                    continue
                for sp in (splits if mode != 3 else splits[:1]):
                    tree.set_kernel_config(m2l_kc=kc, m2l_split=sp, m2l_mode=mode)
                    t = _time(tree, u, prec)
                    trials.append({"prec": prec, "m2l_mode": mode, "m2l_kc": kc, "m2l_split": sp, "ms": t})
                    if t < ms:
                        shape, ms = (kc, sp, mode), t
        # 4. workgroups of the near field running beside the tree passes
        wg = 0
        for w in p2p_wgs:
            tree.set_kernel_config(m2l_kc=shape[0], m2l_split=shape[1], m2l_mode=shape[2], p2p_wg=w)
            t = _time(tree, u, prec)
            trials.append({"prec": prec, "p2p_wg": w, "ms": t})
            if t < ms:
                wg, ms = w, t
        res = TuneResult(prec, list(orders), shape[0], shape[1], err, ms, m2l_mode=shape[2], p2p_wg=wg)
        if best is None or res.ms < best.ms:
            best = res
    if best is None:
        raise RuntimeError(f"no precision reaches the target {target:g} at order {pmax}")
    tree.set_level_orders(best.level_orders)
    tree.set_kernel_config(m2l_kc=best.m2l_kc, m2l_split=best.m2l_split, m2l_mode=best.m2l_mode,
                           p2p_wg=best.p2p_wg)
    best.error = _error(tree, u, rows, exact, best.precision)
    best.trials = trials
    return best


def tune_tree(xy: torch.Tensor, c, u: torch.Tensor, leaf: int = 64, p: int = 12, target: float = 1e-6,
              precisions=("fp64",), seed: int = 1, **tree_kw):
    """Build a tree over ``xy``, tune it with :func:`tune`, and rebuild it at
    the highest tuned order when that is below ``p`` (P2M, M2M and the W-list
    evaluations then do less work).  Returns (tree, TuneResult)."""
    from . import build_tree
    tree = build_tree(xy, c, leaf=leaf, p=p, **tree_kw)
    res = tune(tree, u, target=target, precisions=precisions, seed=seed)
    pmax = max(res.level_orders)
    if pmax < p:
        tree.close()
        tree = build_tree(xy, c, leaf=leaf, p=pmax, **tree_kw)
        tree.set_level_orders(res.level_orders)
        tree.set_kernel_config(m2l_kc=res.m2l_kc, m2l_split=res.m2l_split, m2l_mode=res.m2l_mode,
                               p2p_wg=res.p2p_wg)
    return tree, res


def tune_leaf(xy: torch.Tensor, c, u: torch.Tensor, leaves=(32, 48, 64), p: int = 12, target: float = 1e-6,
              precisions=("fp64",), seed: int = 1, reps: int = 20, **tree_kw):
    """:func:`tune_tree` for every leaf capacity in ``leaves``; the fastest
    tuned tree is returned (the others are freed) with its TuneResult and a
    list of per-leaf records (leaf, precision, orders, error, ms)."""
    best, rec = None, []
    for leaf in leaves:
        tree, res = tune_tree(xy, c, u, leaf=leaf, p=p, target=target, precisions=precisions, seed=seed,
                              **tree_kw)
        ms = _time(tree, u, res.precision, reps, batches=3)
        rec.append({"leaf": leaf, "precision": res.precision, "level_orders": res.level_orders,
                    "error": res.error, "ms": ms})
        if best is None or ms < best[2]:
            if best is not None:
                best[0].close()
            best = (tree, res, ms, leaf)
        else:
            tree.close()
    tree, res, _, leaf = best
    res.leaf = leaf
    return tree, res, rec
