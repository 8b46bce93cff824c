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

from . import LEARNED, MULTIGRID, PLAIN_F64, Network, PoissonSolver, inputs


def _torch():
    import torch
    return torch


def _rhs(w, solver):
    """g = 4 pi (rho + b), zero mean, formed by the library (device tensor)."""
    torch = _torch()
    rho, b = torch.from_numpy(w.rho).cuda(), torch.from_numpy(w.b).cuda()
    g = torch.empty_like(rho)
    solver.rhs(rho, b, g)
    return g


def solve_pairs(workloads, tol: float = 1e-10, snapshots=(0,)):
    """[(rhs, solution, h)] device tensors from the plain FP64 solver.

    For each cell, g = 4 pi (rho + b) (zero mean) is solved to `tol` (phi).
    Every k > 0 in `snapshots` adds the pair (r_k, phi - x_k), where x_k is
    the iterate after k plain CG iterations from zero and r_k = g + L x_k its
    residual: the residuals a preconditioner meets inside a solve, with their
    exact corrections (A^-1 r_k = phi - x_k).  k = 0 adds (g, phi)."""
    torch = _torch()
    from . import fd_laplacian_apply
    out = []
    solvers = {}
    for w in workloads:
        key = (w.rho.shape, w.cell.h)
        if key not in solvers:
            solvers[key] = PoissonSolver(w.rho.shape, w.cell.h, 6, PLAIN_F64)
        g = _rhs(w, solvers[key])
        phi = torch.zeros_like(g)
        solvers[key].solve(g, phi, tol)
        for k in snapshots:
            if k == 0:
                out.append((g, phi, w.cell.h))
                continue
            x = torch.zeros_like(g)
            solvers[key].solve(g, x, 1e-30, max_iter=k, allow_not_converged=True)
            r = g.clone()
            fd_laplacian_apply(x, r, w.cell.h, 6, alpha=1.0, beta=1.0)
            out.append((r, phi - x, w.cell.h))
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


def correction_quality(net: Network, g, h) -> dict:
    """How the network's correction of a zero guess acts on the system with
    right-hand side g (zero mean): the step a = z.g / z.Az along z = N(g)
    (the solver's choice), and the energy-norm error and residual left,
    relative to the zero guess.  The exact solution comes from plain CG."""
    torch = _torch()
    from . import fd_laplacian_apply
    phi = torch.zeros_like(g)
    PoissonSolver(g.shape, h, 6, PLAIN_F64).solve(g, phi, 1e-11, allow_not_converged=True)
    h2 = float(np.cbrt(h[0] * h[1] * h[2])) ** 2
    z = torch.empty_like(g)
    net.forward(g, z, h, scale=h2)
    z -= z.mean()

    def A(v):                       # -L_h v
        out = torch.zeros_like(v)
        fd_laplacian_apply(v, out, h, 6, alpha=-1.0)
        return out

    Az = A(z)
    a = float((z * g).sum() / (z * Az).sum())
    e1 = phi - a * z
    return {"step": a,
            "energy_error_ratio": float(torch.sqrt((e1 * A(e1)).sum() / (phi * g).sum())),
            "residual_ratio": float((g - a * Az).norm() / g.norm())}


def evaluate(net: Network, w, tol: float = 1e-8, repeats: int = 3) -> dict:
    """Plain FP64 CG vs the learned forms on one cell, from a zero guess: best
    of `repeats` timed solves each (after one warm-up), iterations, network
    applications, fallback, the correction's quality, the solutions'
    difference and the time of one network application."""
    torch = _torch()
    g = _rhs(w, PoissonSolver(w.rho.shape, w.cell.h, 6, PLAIN_F64))
    return evaluate_rhs(net, g, w.cell.h, tol, repeats)


def evaluate_rhs(net: Network, g, h, tol: float = 1e-8, repeats: int = 3, multigrid: bool = False) -> dict:
    """evaluate() for a right-hand side g (zero mean) on a grid of spacing h;
    with multigrid, the multigrid-preconditioned CG is timed too."""
    torch = _torch()
    res = {}
    xs = {}
    forms = [("plain", PLAIN_F64, False)] + ([("multigrid", MULTIGRID, False)] if multigrid else []) + \
        [("learned", LEARNED, False), ("learned_fcg", LEARNED, True)]
    for name, mode, fcg in forms:
        s = PoissonSolver(g.shape, h, 6, mode)
        if mode == LEARNED:
            s.set_network(net)
            s.set_learned_mode(fcg)
        x = torch.zeros_like(g)
        s.solve(g, x, tol, allow_not_converged=True)
        best = None
        for _ in range(repeats):
            x.zero_()
            st = s.solve(g, x, tol, allow_not_converged=True)
            if best is None or st["seconds"] < best["seconds"]:
                best = st
        keys = ("iters", "seconds", "rel_res", "status") + (("nn_applies", "fell_back") if mode == LEARNED else ())
        best["seconds"] = float(best["seconds"])
        res[name] = {k: best[k] for k in keys}
        xs[name] = x
        s.close()
    res["max_abs_diff"] = float((xs["plain"] - xs["learned"]).abs().max().item())
    res["max_abs_diff_fcg"] = float((xs["plain"] - xs["learned_fcg"]).abs().max().item())
    res["correction"] = correction_quality(net, g, h)
    z = torch.empty_like(g)
    net.forward(g, z, h, scale=1.0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(5):
        net.forward(g, z, h, scale=1.0)
    torch.cuda.synchronize()
    res["nn_forward_s"] = (time.perf_counter() - t0) / 5
    return res


def train_and_evaluate(n_cells: int = 96, steps: int = 6000, snapshots=(0, 10, 40, 120),
                       loss_kind: int = Network.ENERGY, heldout=(0,), log_every: int = 500,
                       lr: float = 1e-3, seed: int = 0) -> dict:
    """End-to-end: generate and solve training cells, train, evaluate held-out cells."""
    t0 = time.perf_counter()
    cells = [inputs.training_workload(i) for i in range(n_cells)]
    t_gen = time.perf_counter() - t0
    t0 = time.perf_counter()
    pairs = solve_pairs(cells, snapshots=snapshots)
    t_solve = time.perf_counter() - t0
    net = Network(seed)
    net.set_loss(loss_kind)
    t0 = time.perf_counter()
    losses = train(net, pairs, steps, lr=lr, log_every=log_every, seed=seed)
    t_train = time.perf_counter() - t0
    report = {"cells": n_cells, "pairs": len(pairs), "snapshots": list(snapshots), "steps": steps,
              "loss_kind": loss_kind, "t_generate_s": t_gen, "t_solve_s": t_solve, "t_train_s": t_train,
              "loss_first": float(np.mean(losses[:50])), "loss_last": float(np.mean(losses[-50:]))}
    for which in heldout:
        report[f"heldout_{which}"] = evaluate(net, inputs.heldout_workload(which))
    return report, net


def cell_pairs(mg: PoissonSolver, plain: PoissonSolver, rho, b, h, snapshots, tol: float = 1e-10):
    """Solver-generated (right-hand side, solution) pairs of one cell, device
    tensors: g = 4 pi (rho + b) (zero mean, by the library) and phi from the
    multigrid-preconditioned solver to `tol`; for every k > 0 in `snapshots`
    (increasing) the plain FP64 CG iterate x after k iterations in total
    (continued from the previous snapshot's iterate) gives the pair
    (r, phi - x) with r = g + L_h x, the residual a preconditioner meets
    there and its exact correction."""
    torch = _torch()
    from . import fd_laplacian_apply
    g = torch.empty_like(rho)
    mg.rhs(rho, b, g)
    phi = torch.zeros_like(g)
    mg.solve(g, phi, tol)
    out = [(g, phi)] if 0 in snapshots else []
    x = torch.zeros_like(g)
    done = 0
    for k in sorted(k for k in snapshots if k > 0):
        plain.solve(g, x, 1e-30, max_iter=k - done, allow_not_converged=True)
        done = k
        r = g.clone()
        fd_laplacian_apply(x, r, h, 6, alpha=1.0, beta=1.0)
        out.append((r, phi - x))
    return out


def c5(n_pairs: int = 20000, ring: int = 512, snapshots=(0, 5, 10, 20, 40, 80, 120, 200),
       lr: float = 1e-3, lr_final: float = 1e-4, seed: int = 0, loss_kind: int = Network.ENERGY,
       log=None) -> tuple:
    """The learned aid as configured: n_pairs solver-generated pairs of
    perturbed 4^3-6^3 FCC cells on 64^3-112^3 grids (jitter 0.1, training
    seeds 1000 + i), produced on the fly into a device ring of `ring` pairs
    and consumed once each, in random order within the ring, as one training
    step of the network (Adam, cosine learning rate lr -> lr_final, a random
    exact symmetry of the periodic cube applied to each pair).  Returns
    (report, network)."""
    torch = _torch()
    dev = torch.device("cuda")
    rng = np.random.default_rng(seed)
    net = Network(seed)
    net.set_loss(loss_kind)
    solvers = {}
    losses, shapes = [], {}
    produced = cells = steps = 0
    t_gen = t_solve = t_train = 0.0
    while produced < n_pairs:
        slots = []
        while len(slots) < ring and produced < n_pairs:
            t0 = time.perf_counter()
            cell, b, rho = inputs.training_cell_torch(cells, dev)
            torch.cuda.synchronize()
            t_gen += time.perf_counter() - t0
            cells += 1
            key = (cell.shape, cell.h)
            if key not in solvers:
                solvers[key] = (PoissonSolver(cell.shape, cell.h, 6, MULTIGRID),
                                PoissonSolver(cell.shape, cell.h, 6, PLAIN_F64))
            t0 = time.perf_counter()
            for r, t in cell_pairs(*solvers[key], rho, b, cell.h, snapshots):
                if produced < n_pairs:
                    slots.append((r, t, cell.h))
                    produced += 1
            torch.cuda.synchronize()
            t_solve += time.perf_counter() - t0
            shapes[cell.shape[0]] = shapes.get(cell.shape[0], 0) + 1
        # consume the ring: every pair once, grid by grid (the network keeps
        # one workspace), random order within a grid
        t0 = time.perf_counter()
        order = sorted(rng.permutation(len(slots)), key=lambda i: slots[i][0].shape)
        for i in order:
            g, phi, h = slots[i]
            ga, pa = augment(g, phi, rng)
            a = lr_final + 0.5 * (lr - lr_final) * (1.0 + math.cos(math.pi * steps / max(1, n_pairs)))
            losses.append(net.train_step(ga, pa, h, a))
            steps += 1
        torch.cuda.synchronize()
        t_train += time.perf_counter() - t0
        del slots
        if log:
            log(f"c5: {produced} pairs from {cells} cells, loss {np.mean(losses[-200:]):.4f}")
    report = {"pairs": produced, "cells": cells, "cells_by_grid": shapes, "snapshots": list(snapshots),
              "ring": ring, "steps": steps, "loss_kind": loss_kind, "generate_s": t_gen, "solve_s": t_solve,
              "train_s": t_train, "loss_first": float(np.mean(losses[:200])),
              "loss_last": float(np.mean(losses[-200:]))}
    return report, net


def c5_heldout(net: Network, which: int, tol: float = 1e-8, repeats: int = 3) -> dict:
    """Held-out cell `which` (0: 5^3 cells on 96^3, 1: 10^3 on 192^3): plain
    FP64 CG, multigrid-preconditioned CG and the learned forms to `tol`."""
    torch = _torch()
    cell, b, rho = inputs.heldout_cell_torch(which, torch.device("cuda"))
    s = PoissonSolver(cell.shape, cell.h, 6, PLAIN_F64)
    g = torch.empty_like(rho)
    s.rhs(rho, b, g)
    s.close()
    out = evaluate_rhs(net, g, cell.h, tol, repeats, multigrid=True)
    out["grid"] = list(cell.shape)
    out["atoms"] = int(len(cell.atoms))
    return out
