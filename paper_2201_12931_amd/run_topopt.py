"""Command-line driver: optimality-criteria topology optimisation of the
cantilever on one GPU, with an optional finite-difference check of the adjoint
gradient.

    python -m paper_2201_12931_amd.run_topopt --nx 256 --ny 128 --nz 128 --levels 6 \\
        --iters 20 --volfrac 0.12 --fd 64
    python -m paper_2201_12931_amd.run_topopt --nx 64 --ny 32 --nz 32 --levels 4 \\
        --filter sensitivity --volfrac 0.3 --iters 300 --until 0.01

Prints one JSON line per OC iteration and a summary line.  The finite-difference
check compares dc/dx_e from the adjoint with the central difference
(c(x + h e_e) - c(x - h e_e)) / 2h.  At millions of elements a single element
changes c by ~1e-9 relative, so the difference is not formed from two
compliances: with u- = u(x - h e_e), the exact identity
    c(x+) - c(x-) = f^T d,   K(x+) d = (K(x-) - K(x+)) u-
is used, where the right-hand side is non-zero only around the filtered
perturbation (both products are computed by the same deterministic kernel, so
they cancel exactly elsewhere).  Both solves run in binary64 to rtol 1e-10.
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
from paper_2201_12931_amd.autograd import Compliance, DensityFilter  # noqa: E402
from paper_2201_12931_amd.topopt import TopOpt  # noqa: E402


def fd_check(opt: TopOpt, f, elems, h=1e-4, rtol=1e-10, levels=None):
    """Central differences at the current design for the given elements, against
    the adjoint gradient from a binary64 solve (and the solver's own gradient)."""
    nx, ny, nz = opt.shape
    grid = hexmg.Grid(nx, ny, nz, levels or opt.grid.levels, precision=hexmg.FP64)
    # the unfiltered derivative of c(x) (with the sensitivity filter the
    # optimiser uses a filtered one, which is not a derivative)
    xg = opt.x.detach().clone().requires_grad_(True)
    c_run, rho = opt.objective(xg)
    c_run.backward()
    grad_run = xg.grad.detach()
    rho = rho.detach()
    xr = opt.x.detach().clone().requires_grad_(True)
    phys = DensityFilter.apply(xr, opt.shape, opt.rmin) if opt.filter == "density" else xr
    c = Compliance.apply(phys, grid, f, rtol, 1000)
    c.backward()
    grad = xr.grad.detach()
    out = []
    u = torch.empty_like(f)
    d = torch.empty_like(f)
    ym = torch.empty_like(f)
    yp = torch.empty_like(f)
    dens = opt.filter == "density"
    for e in elems:
        xp, xm = opt.x.clone(), opt.x.clone()
        xp[e] += h
        xm[e] -= h
        rp = hexmg.density_filter(nx, ny, nz, opt.rmin, xp) if dens else xp
        rm = hexmg.density_filter(nx, ny, nz, opt.rmin, xm) if dens else xm
        grid.set_density(rm)
        grid.solve(f, u, rtol=rtol, maxit=1000)
        grid.apply_K(u, ym)
        grid.set_density(rp)
        grid.apply_K(u, yp)
        rhs = ym - yp
        grid.solve(rhs, d, rtol=rtol, maxit=1000)
        fd = float(torch.dot(f, d)) / (2 * h)
        g = float(grad[e])
        gr = float(grad_run[e])
        out.append({"element": int(e), "rho": float(rho[e]), "adjoint": g, "fd": fd,
                    "rel_err": abs(fd - g) / abs(g), "solver_adjoint": gr, "solver_rel_err": abs(gr - g) / abs(g)})
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--nx", type=int, default=256)
    ap.add_argument("--ny", type=int, default=128)
    ap.add_argument("--nz", type=int, default=128)
    ap.add_argument("--levels", type=int, default=6)
    ap.add_argument("--iters", type=int, default=20)
    ap.add_argument("--volfrac", type=float, default=0.12)
    ap.add_argument("--rmin", type=float, default=1.5)
    ap.add_argument("--rtol", type=float, default=1e-6)
    ap.add_argument("--fd", type=int, default=0, help="elements for the finite-difference check (0 = off)")
    ap.add_argument("--fd-seed", type=int, default=2)
    ap.add_argument("--fp64", action="store_true", help="binary64 V-cycle instead of the mixed-precision one")
    ap.add_argument("--coarse-avg", choices=["density", "modulus"], default="density")
    ap.add_argument("--filter", choices=["density", "sensitivity"], default="density")
    ap.add_argument("--coarse-op", choices=["rediscretize", "galerkin"], default="rediscretize")
    ap.add_argument("--omega", type=float, default=0.0,
                    help="Jacobi damping of the V-cycle smoother; 0 = the library's automatic choice "
                         "(0.6 re-discretized, 0.5 Galerkin: on black-and-white designs the Galerkin "
                         "hierarchy has lambda_max(D^-1 A) of 4-6, where 0.6 no longer smooths)")
    ap.add_argument("--until", type=float, default=0.0,
                    help="stop once the largest design change is below this (Alg. 4 uses 0.01); 0 = run --iters")
    args = ap.parse_args()

    g = W.Grid(args.nx, args.ny, args.nz)
    f = torch.from_numpy(W.cantilever_line_load(g)).cuda()
    opt = TopOpt(args.nx, args.ny, args.nz, args.levels, f, args.volfrac, rmin=args.rmin, rtol=args.rtol,
                 precision=hexmg.FP64 if args.fp64 else hexmg.MIXED,
                 coarse_avg=hexmg.AVG_DENSITY if args.coarse_avg == "density" else hexmg.AVG_MODULUS,
                 filter=args.filter,
                 coarse_op=hexmg.COARSE_GALERKIN if args.coarse_op == "galerkin" else hexmg.COARSE_REDISCRETIZE,
                 omega=args.omega)
    summary = {"grid": [args.nx, args.ny, args.nz], "elements": g.n_elem, "dofs": g.n_dof,
               "levels": args.levels, "volfrac": args.volfrac, "rmin": args.rmin, "rtol": args.rtol,
               "coarse_avg": args.coarse_avg, "precision": "fp64" if args.fp64 else "mixed",
               "filter": args.filter, "until": args.until, "coarse_op": args.coarse_op,
               "omega": args.omega}
    rng = np.random.Generator(np.random.PCG64(args.fd_seed))

    def fd_elements():
        # filtered density >= 0.05 (finite-difference truncation ~ (h / rho)^2) and
        # x +- h inside [0, 1]
        h = 1e-4
        with torch.no_grad():
            rho = (hexmg.density_filter(args.nx, args.ny, args.nz, args.rmin, opt.x) if args.filter == "density"
                   else opt.x).cpu().numpy()
        x = opt.x.cpu().numpy()
        cand = np.flatnonzero((rho >= 0.05) & (x >= h) & (x <= 1.0 - h))
        return rng.choice(cand, size=min(args.fd, cand.size), replace=False)

    if args.fd:
        t0 = time.perf_counter()
        res = fd_check(opt, f, fd_elements())
        summary["fd_iter0"] = {"max_rel_err": max(r["rel_err"] for r in res), "n": len(res),
                               "solver_max_rel_err": max(r["solver_rel_err"] for r in res),
                               "seconds": time.perf_counter() - t0}
        print(json.dumps({"fd_iteration": 0, "results": res}), flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hist = []
    for _ in range(args.iters):
        ts = time.perf_counter()
        r = opt.step()
        torch.cuda.synchronize()
        rec = dict(r.__dict__)
        rec["seconds"] = time.perf_counter() - ts
        hist.append(rec)
        print(json.dumps(rec), flush=True)
        if args.until > 0 and r.change < args.until:
            break
    summary["oc_seconds"] = time.perf_counter() - t0
    summary["oc_iterations"] = len(hist)
    summary["seconds_per_iteration"] = summary["oc_seconds"] / max(len(hist), 1)
    summary["final"] = hist[-1] if hist else None
    if args.fd and args.iters:
        t0 = time.perf_counter()
        res = fd_check(opt, f, fd_elements())
        summary["fd_final"] = {"max_rel_err": max(r["rel_err"] for r in res), "n": len(res),
                               "solver_max_rel_err": max(r["solver_rel_err"] for r in res),
                               "seconds": time.perf_counter() - t0}
        print(json.dumps({"fd_iteration": len(hist), "results": res}), flush=True)
    print(json.dumps({"summary": summary}), flush=True)


if __name__ == "__main__":
    main()
