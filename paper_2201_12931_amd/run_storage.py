"""Command-line driver of the reduced-precision storage study: the Galerkin
coarse operators (Eq. 23) of the binary32 V-cycle stored as binary32,
bfloat16 or binary16 stencils (HEXMG_STENCIL_*), against the binary64
Galerkin solve of the same problem.

    python -m paper_2201_12931_amd.run_storage [--workload cantilever_128x64x64_rf] [--rtol 1e-6] [--reps 3]

For each storage: workspace bytes, coarse-stencil bytes, set-up and solve
milliseconds (median of --reps solves after one untimed), CG iterations, the
binary64 true residual, and the relative differences of compliance and u from
the binary64 Galerkin solve.  Prints one JSON line.
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

STORES = {"f32": hexmg.STENCIL_F32, "bf16": hexmg.STENCIL_BF16, "f16": hexmg.STENCIL_F16}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="cantilever_128x64x64_rf")
    ap.add_argument("--rtol", type=float, default=1e-6)
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--maxit", type=int, default=1000)
    args = ap.parse_args()
    g, rho, f, mask, spec = W.workload(args.workload)
    levels = spec["levels"]
    rho_d = torch.from_numpy(rho).cuda()
    f_d = torch.from_numpy(np.ascontiguousarray(f)).cuda()
    del rho, f
    out = {"workload": args.workload, "grid": [g.nx, g.ny, g.nz], "dofs": g.n_dof, "levels": levels,
           "rtol": args.rtol, "coarse_op": "galerkin", "runs": {}}

    def run(name, precision, store):
        grid = hexmg.Grid(g.nx, g.ny, g.nz, levels, precision=precision, coarse_op=hexmg.COARSE_GALERKIN,
                          stencil_storage=store)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        grid.set_density(rho_d)
        torch.cuda.synchronize()
        setup_ms = (time.perf_counter() - t0) * 1e3
        u = torch.empty_like(f_d)
        grid.solve(f_d, u, rtol=args.rtol, maxit=args.maxit)  # untimed
        ms, info = [], None
        for _ in range(args.reps):
            code, inf = grid.solve(f_d, u, rtol=args.rtol, maxit=args.maxit)
            ms.append(inf[0]["ms_solve"])
            info = inf[0]
        nq = sum(243 * (g.nx // 2 ** l + 1) * (g.ny // 2 ** l + 1) * (g.nz // 2 ** l + 1) for l in range(1, levels))
        word = {hexmg.STENCIL_F32: 4, hexmg.STENCIL_BF16: 2, hexmg.STENCIL_F16: 2}[store]
        r = {"status": code, "iterations": info["iterations"], "rel_res_true": info["rel_res_true"],
             "compliance": info["compliance"], "solve_ms": sorted(ms)[len(ms) // 2], "setup_ms": setup_ms,
             "workspace_bytes": grid.workspace.numel(),
             "stencil_bytes_vcycle": nq * word if precision != hexmg.FP64 else nq * 8}
        grid.close()
        print(f"run_storage: {name}: {r}", file=sys.stderr, flush=True)
        return r, u

    ref, u64 = run("fp64", hexmg.FP64, hexmg.STENCIL_F32)
    out["runs"]["fp64"] = ref
    for name, st in STORES.items():
        r, u = run(name, hexmg.MIXED, st)
        r["compliance_rel_diff_vs_fp64"] = abs(r["compliance"] - ref["compliance"]) / abs(ref["compliance"])
        r["u_rel_diff_vs_fp64"] = float(torch.linalg.vector_norm(u - u64) / torch.linalg.vector_norm(u64))
        out["runs"][name] = r
        del u
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
