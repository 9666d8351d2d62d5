"""Optimality-criteria topology-optimisation loop (Alg. 4 of the paper, with the
density filter in place of the sensitivity filter) on the hexmg C ABI.

Per iteration: rho~ = filter(x) -> c = Compliance(rho~) (MGPCG state solve) ->
backward (adjoint sensitivity, Eq. 7, then the filter adjoint) -> OC update
(Eqs. 8-9) with the filtered volume.  All arithmetic runs in the HIP library;
autograd only chains the two hand-written adjoints.
"""
from __future__ import annotations

import dataclasses

import torch

from . import hexmg
from .autograd import Compliance, DensityFilter


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
                 precision=hexmg.MIXED, rtol=1e-6, maxit=500, x0=None, device="cuda", **grid_kw):
        self.shape = (nx, ny, nz)
        self.n = nx * ny * nz
        self.volfrac, self.rmin, self.move, self.eta = volfrac, rmin, move, eta
        self.rtol, self.maxit = rtol, maxit
        self.grid = hexmg.Grid(nx, ny, nz, levels, precision=precision, device=device, **grid_kw)
        self.f = f
        self.x = (torch.full((self.n,), float(volfrac), dtype=torch.float64, device=device)
                  if x0 is None else x0.clone())
        # dV/dx of V = mean(rho~): the filter adjoint of 1/Ne
        self.dv = hexmg.density_filter(nx, ny, nz, rmin, torch.full_like(self.x, 1.0 / self.n), adjoint=True)
        self.it = 0

    def objective(self, x):
        """c(x) through the filter and the state solve; returns (c_total, rho~)."""
        rho = DensityFilter.apply(x, self.shape, self.rmin)
        c = Compliance.apply(rho, self.grid, self.f, self.rtol, self.maxit)
        return c.sum(), rho

    def gradient(self, x):
        xr = x.detach().clone().requires_grad_(True)
        c, rho = self.objective(xr)
        c.backward()
        return c.detach(), xr.grad.detach(), rho.detach()

    def step(self) -> OCResult:
        c, dc, rho = self.gradient(self.x)
        x_new, lam = self.grid.oc_update(self.x, dc, self.dv, self.volfrac, self.move, self.eta)
        change = float((x_new - self.x).abs().max())
        self.x = x_new
        self.it += 1
        info = self.grid.last_info[0]
        return OCResult(self.it, float(c), float(rho.mean()), change, lam, info["iterations"], info["rel_res_true"])
