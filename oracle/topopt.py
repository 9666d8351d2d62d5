"""Density filter and optimality-criteria update -- test infrastructure only.

* Filter weights (Eq. 4): w(x_i, x_e) = r - ||x_i - x_e|| inside the radius,
  0 outside; neighbourhood (Eq. 5) = elements whose centres lie within r.  The
  paper applies these weights to sensitivities (Eq. 3); the density filter here
  applies them to the design, rho~ = (H x) / Hs with Hs = H 1, truncated at the
  domain boundary (only in-domain elements enter both sums).  Its adjoint is
  g_x = H^T (g / Hs) (H is symmetric).
* Sensitivity filter (Eq. 3), the paper's own regularisation: the filtered
  derivative of element e is sum_i w_ei x_i dc_i / (max(gamma, x_e) sum_i w_ei)
  with the same weights; the design is then the physical density itself.
* Optimality criteria (Eqs. 8-9): B_e = -dc/dx_e / (lambda dV/dx_e),
  x_new = clamp(x B^eta, max(0, x - m), min(1, x + m)), with the Lagrange
  multiplier found by bisection so that the volume constraint holds.  We read the
  garbled bounds of Eq. 8 as x -/+ m and take q = 1.  The volume is that of the
  filtered design, V = mean(rho~(x_new)) (Eq. 1 constrains V(rho)).
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp


def filter_matrix(nx: int, ny: int, nz: int, rmin: float) -> tuple[sp.csr_matrix, np.ndarray]:
    """(H, Hs): H_ei = max(0, rmin - dist(e, i)) over in-domain elements."""
    R = int(math.ceil(rmin)) - 1
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    i, j, k = i.reshape(-1), j.reshape(-1), k.reshape(-1)
    e = i + nx * (j + ny * k)
    rows, cols, vals = [], [], []
    for dk in range(-R, R + 1):
        for dj in range(-R, R + 1):
            for di in range(-R, R + 1):
                w = rmin - math.sqrt(di * di + dj * dj + dk * dk)
                if w <= 0.0:
                    continue
                ii, jj, kk = i + di, j + dj, k + dk
                ok = (ii >= 0) & (ii < nx) & (jj >= 0) & (jj < ny) & (kk >= 0) & (kk < nz)
                rows.append(e[ok])
                cols.append((ii + nx * (jj + ny * kk))[ok])
                vals.append(np.full(int(ok.sum()), w))
    n = nx * ny * nz
    H = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n, n)).tocsr()
    Hs = np.asarray(H.sum(axis=1)).reshape(-1)
    return H, Hs


def density_filter(H, Hs, x):
    """rho~ = H x / Hs."""
    return (H @ np.asarray(x, dtype=np.float64)) / Hs


def density_filter_adjoint(H, Hs, g):
    """g_x = H^T (g / Hs)."""
    return H.T @ (np.asarray(g, dtype=np.float64) / Hs)


def sensitivity_filter(H, Hs, x, dc, gamma=1e-3):
    """Eq. 3: dc~_e = (sum_i H_ei x_i dc_i) / (max(gamma, x_e) Hs_e)."""
    x = np.asarray(x, dtype=np.float64)
    return (H @ (x * np.asarray(dc, dtype=np.float64))) / (np.maximum(gamma, x) * Hs)


def oc_update(x, dc, dv, volume_of, volfrac, move=0.2, eta=0.5,
              lam_lo=1e-12, lam_hi=1e12, rel_tol=1e-12, max_steps=200):
    """One optimality-criteria update (Eqs. 8-9) with log-space bisection on lambda.

    ``dc`` and ``dv`` are the derivatives of the compliance and of the volume
    with respect to the design ``x``; ``volume_of(x_new)`` returns the volume of a
    candidate design.  The volume decreases as lambda grows; bisection keeps
    vol(lam_lo) > volfrac >= vol(lam_hi) and stops once lam_hi/lam_lo - 1 <=
    rel_tol.  Returns (x_new, lambda, bisection steps).
    """
    x = np.asarray(x, dtype=np.float64)
    lo, hi = float(lam_lo), float(lam_hi)
    xlo = np.maximum(0.0, x - move)
    xhi = np.minimum(1.0, x + move)

    def candidate(lam):
        B = -np.asarray(dc) / (lam * np.asarray(dv))
        return np.clip(x * np.power(np.maximum(B, 0.0), eta), xlo, xhi)

    steps = 0
    while hi / lo - 1.0 > rel_tol and steps < max_steps:
        mid = math.sqrt(lo * hi)
        if volume_of(candidate(mid)) > volfrac:
            lo = mid
        else:
            hi = mid
        steps += 1
    lam = math.sqrt(lo * hi)
    return candidate(lam), lam, steps
