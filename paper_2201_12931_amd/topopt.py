"""Optimality-criteria topology-optimisation loop (Alg. 4 of the paper) on the
hexmg C ABI, with either regularisation:

* filter="sensitivity" (the paper's, Eq. 3): c = Compliance(x) (MGPCG state
  solve) -> backward (adjoint sensitivity, Eq. 7) -> filtered sensitivity ->
  OC update (Eqs. 8-9) with V = mean(x);
* filter="density": rho~ = filter(x) -> c = Compliance(rho~) -> backward
  (adjoint sensitivity, then the filter adjoint) -> OC update with the
  filtered volume.

Passive regions (1 solid, 2 void per element; sensitivity filter) keep their
value and stay out of the volume constraint; ``gravity`` adds the self-weight
of the design to the single load case (its derivative included).  All
arithmetic runs in the HIP library; autograd only chains the hand-written
adjoints.  ``run(max_iters, tol)`` iterates until the largest design change
drops below tol (Alg. 4 stops at 0.01).
"""
from __future__ import annotations

import dataclasses

import torch

from . import hexmg
from .autograd import Compliance, DensityFilter, SelfWeightCompliance


@dataclasses.dataclass
class OCResult:
    iteration: int
    compliance: float
    volume: float
    change: float
    lam: float
    cg_iterations: int
    rel_res_true: float


class TopOpt:
    def __init__(self, nx, ny, nz, levels, f, volfrac, rmin=1.5, move=0.2, eta=0.5,
                 precision=hexmg.MIXED, rtol=1e-6, maxit=500, x0=None, device="cuda", filter="density",
                 gamma=1e-3, passive=None, gravity=0.0, **grid_kw):
        if filter not in ("density", "sensitivity"):
            raise ValueError("filter must be 'density' or 'sensitivity'")
        if passive is not None and filter != "sensitivity":
            raise ValueError("passive regions are supported with the sensitivity filter")
        if gravity and (f.dim() != 1):
            raise ValueError("self-weight loading takes one load case")
        self.passive, self.gravity = passive, float(gravity)
        self.shape = (nx, ny, nz)
        self.n = nx * ny * nz
        self.volfrac, self.rmin, self.move, self.eta = volfrac, rmin, move, eta
        self.rtol, self.maxit = rtol, maxit
        self.filter, self.gamma = filter, gamma
        self.grid = hexmg.Grid(nx, ny, nz, levels, precision=precision, device=device, **grid_kw)
        self.f = f
        self.x = (torch.full((self.n,), float(volfrac), dtype=torch.float64, device=device)
                  if x0 is None else x0.clone())
        if filter == "density":
            # dV/dx of V = mean(rho~): the filter adjoint of 1/Ne
            self.dv = hexmg.density_filter(nx, ny, nz, rmin, torch.full_like(self.x, 1.0 / self.n), adjoint=True)
        elif passive is None:
            self.dv = torch.full_like(self.x, 1.0 / self.n)
        else:
            # V = mean of x over the design (non-passive) elements; passive ones keep their value
            self.dv = self.grid.volume_weights(passive)
            hexmg.apply_passive(passive, self.x)
        self.it = 0

    def objective(self, x):
        """c(x) through the density filter (if any) and the state solve; returns
        (c_total, physical densities)."""
        rho = DensityFilter.apply(x, self.shape, self.rmin) if self.filter == "density" else x
        if self.gravity:
            c = SelfWeightCompliance.apply(rho, self.grid, self.f, self.gravity, self.rtol, self.maxit)
        else:
            c = Compliance.apply(rho, self.grid, self.f, self.rtol, self.maxit)
        return c.sum(), rho

    def gradient(self, x):
        """(c, dc/dx as used by the update, physical densities).  With the
        sensitivity filter the returned derivative is the filtered one (Eq. 3)."""
        xr = x.detach().clone().requires_grad_(True)
        c, rho = self.objective(xr)
        c.backward()
        g = xr.grad.detach()
        if self.filter == "sensitivity":
            g = hexmg.sensitivity_filter(*self.shape, self.rmin, x.detach(), g, gamma=self.gamma)
        return c.detach(), g, rho.detach()

    def step(self) -> OCResult:
        """One OC iteration; the result's volume is that of the new design (the
        constrained one: filtered with the density filter, of the design
        elements with passive regions)."""
        c, dc, rho = self.gradient(self.x)
        x_new, lam, change, vol = self.grid.oc_update(self.x, dc, self.dv, self.volfrac, self.move, self.eta,
                                                      stats=True)
        if self.passive is not None:
            hexmg.apply_passive(self.passive, x_new)
        self.x = x_new
        self.it += 1
        info = self.grid.last_info[0]
        return OCResult(self.it, float(c), vol, change, lam, info["iterations"], info["rel_res_true"])

    def run(self, max_iters, tol=0.01, callback=None):
        """OC iterations until max |x_new - x| < tol or max_iters; returns the
        list of OCResult."""
        hist = []
        for _ in range(max_iters):
            r = self.step()
            hist.append(r)
            if callback is not None:
                callback(r)
            if r.change < tol:
                break
        return hist
