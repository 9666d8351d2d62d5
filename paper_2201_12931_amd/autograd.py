"""torch.autograd.Function wrappers around the hexmg C ABI.

* ``DensityFilter``: rho~ = H x / Hs (Eqs. 4-5 weights); backward is the adjoint
  filter H (g / Hs).
* ``Compliance``: c_r = f_r^T u_r with K(rho~) u_r = f_r solved by MGPCG; backward
  is the hand-written adjoint sensitivity of Eq. 7 with u* = u (the compliance
  is self-adjoint, so no second solve), weighted by the incoming gradient per
  load case.
* ``SelfWeightCompliance``: as ``Compliance`` for one load case whose load
  includes the self-weight of the design, f = f_ext + f_g(rho); the derivative
  gains the load term 2 u^T df/drho.

All run entirely in the HIP library; tensors only carry device memory.  A
state solve that does not converge raises ``SolveNotConverged`` instead of
returning a compliance and gradient of an inexact state.
"""
from __future__ import annotations

import numpy as np
import torch

from . import hexmg


class SolveNotConverged(RuntimeError):
    """The state solve behind a compliance evaluation stopped at maxit (or broke
    down): its c and dc would not be the compliance and gradient of the design."""

    def __init__(self, code, info):
        worst = max(info, key=lambda r: r["rel_res_recursive"])
        super().__init__(f"state solve did not converge (status {code}): "
                         f"{worst['iterations']} iterations, recursive residual {worst['rel_res_recursive']:.3g}, "
                         f"true residual {worst['rel_res_true']:.3g}")
        self.code, self.info = code, info


def _solve(grid, f, rtol, maxit):
    u = torch.empty_like(f)
    code, info = grid.solve(f, u, rtol=rtol, maxit=maxit)
    grid.last_info = info
    if code != hexmg.OK:
        raise SolveNotConverged(code, info)
    return u, info


class DensityFilter(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, shape, rmin):
        nx, ny, nz = shape
        ctx.shape, ctx.rmin = shape, rmin
        return hexmg.density_filter(nx, ny, nz, rmin, x.detach().contiguous())

    @staticmethod
    def backward(ctx, g):
        nx, ny, nz = ctx.shape
        gx = hexmg.density_filter(nx, ny, nz, ctx.rmin, g.contiguous(), adjoint=True)
        return gx, None, None


class Compliance(torch.autograd.Function):
    """c = Compliance.apply(rho, grid, f, rtol, maxit): f is [nrhs, N] (or [N])."""

    @staticmethod
    def forward(ctx, rho, grid, f, rtol=1e-6, maxit=500):
        rho = rho.detach().contiguous()
        grid.set_density(rho)
        u, info = _solve(grid, f, rtol, maxit)
        c = grid.compliance_sensitivity(f, u)
        ctx.grid, ctx.version = grid, grid.density_version
        ctx.save_for_backward(rho, f, u)
        ctx.info = info
        return torch.as_tensor(c, dtype=torch.float64, device=rho.device).reshape(f.shape[:-1] if f.dim() > 1 else ())

    @staticmethod
    def backward(ctx, grad_c):
        rho, f, u = ctx.saved_tensors
        grid = ctx.grid
        if grid.density_version != ctx.version:
            grid.set_density(rho)
        w = np.atleast_1d(grad_c.detach().double().cpu().numpy()).reshape(-1)
        dc = torch.empty_like(rho)
        grid.compliance_sensitivity(f, u, dc=dc, weights=w)
        return dc, None, None, None, None


class SelfWeightCompliance(torch.autograd.Function):
    """c = SelfWeightCompliance.apply(rho, grid, f_ext, gz, rtol, maxit): one load
    case, f = f_ext + self-weight of rho (gravity gz along -z)."""

    @staticmethod
    def forward(ctx, rho, grid, f_ext, gz, rtol=1e-6, maxit=500):
        rho = rho.detach().contiguous()
        grid.set_density(rho)
        f = grid.gravity_load(gz, f_ext)
        u, info = _solve(grid, f, rtol, maxit)
        c = grid.compliance_sensitivity(f, u)
        ctx.grid, ctx.version, ctx.gz = grid, grid.density_version, gz
        ctx.save_for_backward(rho, f, u)
        return torch.as_tensor(c[0], dtype=torch.float64, device=rho.device)

    @staticmethod
    def backward(ctx, grad_c):
        rho, f, u = ctx.saved_tensors
        grid = ctx.grid
        if grid.density_version != ctx.version:
            grid.set_density(rho)
        w = float(grad_c.detach().double().cpu())
        dc = torch.empty_like(rho)
        grid.compliance_sensitivity(f, u, dc=dc, weights=np.array([w]))
        grid.gravity_sensitivity(u, ctx.gz, dc, weight=w)
        return dc, None, None, None, None, None
