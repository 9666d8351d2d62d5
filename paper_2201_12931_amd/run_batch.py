"""Command-line driver for the batched workload: one 192x96x96 grid with 8 point
load cases solved in lockstep, plus 16 independent cantilevers of uneven sizes
(32x16x16 .. 96x48x48), all advanced together by hexmg_batch_solve.

    python -m paper_2201_12931_amd.run_batch [--rtol 1e-6] [--reps 3]

Prints one JSON line with the batched time, the time of the same solves one
after another, iteration counts, residuals, and the kernel launches of the
batch against the launches the grids would have issued one by one.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from paper_2201_12931_amd import hexmg  # noqa: E402

UNEVEN_NX = [32, 32, 48, 48, 48, 48, 64, 64, 64, 64, 80, 80, 80, 80, 96, 96]


def levels_for(ny: int) -> int:
    """Coarsen while the dimensions stay even and the next ny is at least 3."""
    L = 1
    while ny % 2 == 0 and ny // 2 >= 3:
        ny //= 2
        L += 1
    return L


def build(precision):
    problems = []
    g = W.Grid(192, 96, 96)
    rho = W.random_field_density(g, seed=3, lo=0.01)
    f = W.point_loads(g, 8, seed=30)
    problems.append((g, 5, rho, f))
    for k, nx in enumerate(UNEVEN_NX):
        gk = W.Grid(nx, nx // 2, nx // 2)
        rk = W.random_field_density(gk, seed=300 + k, lo=0.01)
        problems.append((gk, levels_for(nx // 2), rk, W.cantilever_line_load(gk)[None, :]))
    grids, fs, us = [], [], []
    for g, L, rho, f in problems:
        grid = hexmg.Grid(g.nx, g.ny, g.nz, L, precision=precision, max_nrhs=f.shape[0])
        grid.set_density(torch.from_numpy(rho).cuda())
        grids.append(grid)
        fs.append(torch.from_numpy(np.ascontiguousarray(f)).cuda())
        us.append(torch.empty_like(fs[-1]))
    return problems, grids, fs, us


def pin_kernels(grids):
    """Give every grid, on each level it has, the kernel the first (largest) grid
    tuned for that level, so that each batched step is one launch for all grids
    (the streaming kernel with the first grid's tile shape and z-chunk; a level
    where it chose the node-gather kernel takes the streaming kernel's first
    shape)."""
    for dt in (hexmg.F32, hexmg.F64):
        for l in range(max(g.levels for g in grids)):
            lead = next(g for g in grids if g.levels > l)
            kind, zc, shape = lead.kernel_choice(l, dt)
            if kind != "stream":
                zc, shape = 4, 0
            for g in grids:
                if g.levels > l:
                    g.set_kernel_choice(l, dt, hexmg.KERNEL_STREAM, zc, shape)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--rtol", type=float, default=1e-6)
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--fp64", action="store_true")
    ap.add_argument("--no-pin", action="store_true",
                    help="keep each grid's own tuned kernels (steps whose grids chose differently then take "
                         "several launches)")
    args = ap.parse_args()
    prec = hexmg.FP64 if args.fp64 else hexmg.MIXED
    problems, grids, fs, us = build(prec)
    if not args.no_pin:
        pin_kernels(grids)
    hexmg.batch_solve(grids, fs, us, rtol=args.rtol)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.reps):
        code, infos = hexmg.batch_solve(grids, fs, us, rtol=args.rtol)
    torch.cuda.synchronize()
    t_batch = (time.perf_counter() - t0) / args.reps
    t0 = time.perf_counter()
    for _ in range(args.reps):
        for grid, f, u in zip(grids, fs, us):
            grid.solve(f, u, rtol=args.rtol)
    torch.cuda.synchronize()
    t_seq = (time.perf_counter() - t0) / args.reps
    dofs = sum(g.n_dof * f.shape[0] for (g, _, _, f) in problems)
    out = {
        "workload": "192x96x96 x 8 point loads + 16 uneven cantilevers (32x16x16 .. 96x48x48)",
        "precision": "fp64" if args.fp64 else "mixed",
        "rtol": args.rtol,
        "problems": [{"grid": [g.nx, g.ny, g.nz], "levels": L, "nrhs": int(f.shape[0]),
                      "iterations": [x["iterations"] for x in info],
                      "rel_res_true_max": max(x["rel_res_true"] for x in info)}
                     for (g, L, _, f), info in zip(problems, infos)],
        "status": code,
        "kernels": "pinned to the largest grid's per level" if not args.no_pin else "tuned per grid",
        "batch_launches": grids[0].batch_stats()[0],
        "batch_launches_if_one_by_one": grids[0].batch_stats()[1],
        "total_dofs_x_rhs": dofs,
        "batch_s": t_batch,
        "sequential_s": t_seq,
        "speedup": t_seq / t_batch,
        "gdofs_per_s": dofs / t_batch / 1e9,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
