"""Training and evaluation of the learned solver aid.

Training pairs (g, phi) are produced by the library's own FP64 CG solver on
perturbed-atom FCC cells (training seeds 1000+i).  Each solved cell yields
many pairs through the exact symmetries of the periodic cubic problem: the
discrete Laplacian commutes with grid translations, axis permutations and
axis reflections, so applying one such map to g maps the solution phi the
same way.  All arithmetic of the network (forward, backward, Adam) runs in
the library's kernels; this module only schedules it.
"""
from __future__ import annotations

import math
import time
from typing import Dict, List

import numpy as np

from . import LEARNED, PLAIN_F64, Network, PoissonSolver, inputs


def _torch():
    import torch
    return torch


def solve_pairs(workloads, tol: float = 1e-10):
    """[(g, phi, h)] device tensors, phi from the plain FP64 solver to `tol`."""
    torch = _torch()
    out = []
    solvers = {}
    for w in workloads:
        g = torch.from_numpy(4.0 * math.pi * (w.rho + w.b)).cuda()
        g -= g.mean()
        key = (g.shape, w.cell.h)
        if key not in solvers:
            solvers[key] = PoissonSolver(g.shape, w.cell.h, 6, PLAIN_F64)
        phi = torch.zeros_like(g)
        solvers[key].solve(g, phi, tol)
        out.append((g, phi, w.cell.h))
    return out


def augment(g, phi, rng: np.random.Generator):
    """A random translation, axis permutation and reflection, applied to both."""
    perm = [int(v) for v in rng.permutation(3)]
    flips = [int(a) for a in range(3) if rng.random() < 0.5]
    shifts = [int(rng.integers(n)) for n in g.shape]

    def tf(t):
        t = t.permute(*perm)
        if flips:
            t = t.flip(flips)
        return t.roll(shifts, (0, 1, 2)).contiguous()

    return tf(g), tf(phi)


def train(net: Network, pairs, steps: int, lr: float = 1e-3, lr_final: float = 1e-4, seed: int = 0,
          log_every: int = 0) -> List[float]:
    """Adam on single augmented pairs; cosine decay from lr to lr_final.
    Pairs are visited grid size by grid size so the workspace is reused."""
    rng = np.random.default_rng(seed)
    by_shape: Dict[tuple, list] = {}
    for p in pairs:
        by_shape.setdefault(tuple(p[0].shape), []).append(p)
    groups = list(by_shape.values())
    losses = []
    per_group = max(1, steps // (4 * len(groups)))
    k = 0
    while k < steps:
        for grp in groups:
            for _ in range(per_group):
                if k >= steps:
                    break
                g, phi, h = grp[int(rng.integers(len(grp)))]
                ga, pa = augment(g, phi, rng)
                a = lr_final + 0.5 * (lr - lr_final) * (1.0 + math.cos(math.pi * k / max(1, steps)))
                losses.append(net.train_step(ga, pa, h, a))
                k += 1
                if log_every and k % log_every == 0:
                    print(f"[train] step {k} loss {np.mean(losses[-log_every:]):.4e}", flush=True)
    return losses


def evaluate(net: Network, w, tol: float = 1e-8) -> dict:
    """Plain FP64 CG vs the learned form on one cell, from a zero guess."""
    torch = _torch()
    g = torch.from_numpy(4.0 * math.pi * (w.rho + w.b)).cuda()
    res = {}
    plain = PoissonSolver(g.shape, w.cell.h, 6, PLAIN_F64)
    x = torch.zeros_like(g)
    plain.solve(g, x, tol)                         # warm-up of the code path
    x.zero_()
    st = plain.solve(g, x, tol)
    res["plain"] = {k: st[k] for k in ("iters", "seconds", "rel_res")}
    learned = PoissonSolver(g.shape, w.cell.h, 6, LEARNED)
    learned.set_network(net)
    y = torch.zeros_like(g)
    learned.solve(g, y, tol)
    y.zero_()
    st = learned.solve(g, y, tol)
    res["learned"] = {k: st[k] for k in ("iters", "seconds", "rel_res", "nn_applies", "fell_back")}
    res["max_abs_diff"] = float((x - y).abs().max().item())
    return res


def train_and_evaluate(n_cells: int = 96, augment_per_cell: int = 200, steps: int = 6000,
                       heldout=(0,), log_every: int = 500) -> dict:
    """End-to-end: generate and solve training cells, train, evaluate held-out cells."""
    t0 = time.perf_counter()
    cells = [inputs.training_workload(i) for i in range(n_cells)]
    t_gen = time.perf_counter() - t0
    t0 = time.perf_counter()
    pairs = solve_pairs(cells)
    t_solve = time.perf_counter() - t0
    net = Network(0)
    t0 = time.perf_counter()
    losses = train(net, pairs, steps, log_every=log_every)
    t_train = time.perf_counter() - t0
    report = {"cells": n_cells, "pairs_available": n_cells * augment_per_cell, "steps": steps,
              "t_generate_s": t_gen, "t_solve_s": t_solve, "t_train_s": t_train,
              "loss_first": float(np.mean(losses[:50])), "loss_last": float(np.mean(losses[-50:]))}
    for which in heldout:
        report[f"heldout_{which}"] = evaluate(net, inputs.heldout_workload(which))
    return report
