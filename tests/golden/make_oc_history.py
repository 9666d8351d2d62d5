"""Writes oc_sensitivity_32x16x16.json: the oracle's optimisation history of
the paper's loop (Alg. 4) with the sensitivity filter (Eq. 3) and the OC
update (Eqs. 8-9), run until the largest design change drops below 0.01.

Cantilever 32x16x16, face x = 0 fixed, unit line load on the free-end bottom
edge, volume fraction 0.12, r = 1.5, move 0.2, eta 1/2, gamma 1e-3, x0 = 0.12.
State solves by the oracle's MGPCG (3 levels) to a relative residual of 1e-12.
Calls only oracle/ (and the seeded input generators in workloads/).

    python tests/golden/make_oc_history.py
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle import fem, multigrid as mg, topopt as T  # noqa: E402

DIMS, LEVELS, VOLFRAC, RMIN, TOL, MAX_ITERS = (32, 16, 16), 3, 0.12, 1.5, 0.01, 200


def main():
    g = W.Grid(*DIMS)
    f = W.cantilever_line_load(g)
    mask = W.fixed_mask_face_x0(g)
    H, Hs = T.filter_matrix(*DIMS, RMIN)
    n = g.n_elem
    dv = np.full(n, 1.0 / n)
    x = np.full(n, VOLFRAC)
    hist = []
    for it in range(MAX_ITERS):
        u, its, rel, _ = mg.mgpcg(mg.Hierarchy(*DIMS, x, mask, LEVELS), f, rtol=1e-12, maxit=5000)
        c = fem.compliance(f, u)
        dc = T.sensitivity_filter(H, Hs, x, fem.sensitivity(*DIMS, x, u))
        x_new, lam, _ = T.oc_update(x, dc, dv, lambda z: z.mean(), VOLFRAC)
        change = float(np.abs(x_new - x).max())
        x = x_new
        hist.append({"iteration": it + 1, "compliance": c, "change": change, "volume": float(x.mean()),
                     "lambda": lam, "cg_iterations": its})
        print(f"it {it + 1} c {c:.10g} change {change:.4g} cg {its}", flush=True)
        if change < TOL:
            break
    out = {"dims": list(DIMS), "levels": LEVELS, "volfrac": VOLFRAC, "rmin": RMIN, "move": 0.2, "eta": 0.5,
           "gamma": 1e-3, "tol": TOL, "history": hist,
           "source": "oracle (Alg. 4 with Eq. 3 and Eqs. 8-9), tests/golden/make_oc_history.py"}
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "oc_sensitivity_32x16x16.json"), "w") as fh:
        json.dump(out, fh, indent=1)


if __name__ == "__main__":
    main()
