"""Assembled geometric multigrid and MG-preconditioned CG -- test infrastructure only.

Written from Sec. 3 and Sec. 4.2.2 of the paper, with every operator assembled
as a sparse matrix so that it can be read against the text:

* level l = 0 is the given grid; level l+1 halves every dimension (the paper
  numbers the finest level 1; we start at 0);
* homogenization (Sec. 4.2.2, Sec. 6): the density of a coarse element is the
  mean of the densities of its eight children; the coarse modulus is then the
  SIMP modulus of that mean (``coarse_average="density"``).  The alternative
  reading -- mean of the children's moduli -- is ``coarse_average="modulus"``;
* the coarse element stiffness is re-computed "on the fly" for an element of
  side h = 2^l, i.e. 2^l * K0 (3-D elasticity scales linearly with h);
* a coarse DOF is fixed iff the coincident fine DOF is fixed;
* ``coarse_operator="galerkin"`` replaces the re-discretized coarse operators
  by the Galerkin products of Eq. 23, A_{l+1} = P~^T A_l P~ + (I - M_{l+1})
  with P~ = M_l P M_{l+1} (prolongation that leaves fixed DOFs untouched on both
  levels), so the coarse-grid correction is the A-orthogonal projection onto
  the range of P~;
* transfer: trilinear interpolation P (tensor product of 1-D linear
  interpolation) and restriction R = P^T (variational; the paper's 1/4 [1 2 1]
  stencil of Eq. 22 differs by a constant factor, which does not change the
  preconditioned iterates' solution);
* smoother: damped Jacobi u <- u + omega D^{-1} (f - A u) (Eq. 21), the same
  number of sweeps before and after the coarse correction;
* V-cycle (Alg. 3) with zero initial guess on every level; the coarsest level
  is solved directly (dense Cholesky) and not smoothed;
* PCG (Alg. 1) with x0 = 0, z0 = M^{-1} r0, p0 = z0, stopping on the relative
  recursive residual ||r_k||_2 <= rtol ||f||_2.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from .fem import assemble_stiffness, constrained_operator, free_dof_mask, simp_modulus


def homogenize(v: np.ndarray, nx: int, ny: int, nz: int) -> np.ndarray:
    """Mean of the 8 children of every coarse element (element order, x fastest)."""
    a = np.asarray(v, dtype=np.float64).reshape(nz, ny, nx)
    return a.reshape(nz // 2, 2, ny // 2, 2, nx // 2, 2).mean(axis=(1, 3, 5)).reshape(-1)


def inject_node_mask(mask: np.ndarray, nx: int, ny: int, nz: int) -> np.ndarray:
    """Coarse node mask = mask of the coincident fine node (2i, 2j, 2k)."""
    m = np.asarray(mask).reshape(nz + 1, ny + 1, nx + 1)
    return np.ascontiguousarray(m[::2, ::2, ::2]).reshape(-1)


def linear_interpolation_1d(nc: int) -> sp.csr_matrix:
    """(2 nc + 1) x (nc + 1) 1-D linear interpolation from coarse to fine nodes."""
    P = sp.lil_matrix((2 * nc + 1, nc + 1))
    for i in range(2 * nc + 1):
        if i % 2 == 0:
            P[i, i // 2] = 1.0
        else:
            P[i, i // 2] = 0.5
            P[i, i // 2 + 1] = 0.5
    return P.tocsr()


def prolongation(nxc: int, nyc: int, nzc: int) -> sp.csr_matrix:
    """DOF-level trilinear prolongation from the coarse grid (nxc, nyc, nzc elements)."""
    Px, Py, Pz = (linear_interpolation_1d(n) for n in (nxc, nyc, nzc))
    Pn = sp.kron(Pz, sp.kron(Py, Px))          # node index x fastest
    return sp.kron(Pn, sp.identity(3)).tocsr()  # DOF 3 n + c


class Hierarchy:
    """All levels of the assembled multigrid for one density field."""

    def __init__(self, nx, ny, nz, rho, node_mask, levels, E0=1.0, Emin=1e-9,
                 p=3.0, nu=0.3, omega=0.6, sweeps=2, coarse_average="density",
                 coarse_operator="rediscretize"):
        if coarse_operator not in ("rediscretize", "galerkin"):
            raise ValueError(coarse_operator)
        if levels < 1:
            raise ValueError("levels >= 1")
        for n in (nx, ny, nz):
            if n % (1 << (levels - 1)):
                raise ValueError("dimensions must be divisible by 2^(levels-1)")
        self.levels = levels
        self.omega = omega
        self.sweeps = sweeps
        self.dims, self.E, self.rho, self.A, self.D, self.free, self.P = [], [], [], [], [], [], []
        rho_l = np.asarray(rho, dtype=np.float64)
        E_unscaled = simp_modulus(rho_l, E0, Emin, p)
        mask_l = np.asarray(node_mask, dtype=np.uint8)
        for l in range(levels):
            d = (nx >> l, ny >> l, nz >> l)
            if l > 0:
                pd = self.dims[-1]
                rho_l = homogenize(rho_l, *pd)
                if coarse_average == "density":
                    E_unscaled = simp_modulus(rho_l, E0, Emin, p)
                elif coarse_average == "modulus":
                    E_unscaled = homogenize(E_unscaled, *pd)
                else:
                    raise ValueError(coarse_average)
                mask_l = inject_node_mask(mask_l, *pd)
            h = float(1 << l)
            E_l = E_unscaled
            K = assemble_stiffness(*d, E_l, nu=nu, h=h)
            free = free_dof_mask(mask_l)
            A = constrained_operator(K, free)
            self.dims.append(d)
            self.rho.append(rho_l)
            self.E.append(h * E_l)  # modulus times the element-size factor of level l
            self.A.append(A)
            self.D.append(A.diagonal().copy())
            self.free.append(free.astype(np.float64))
        for l in range(levels - 1):
            self.P.append(prolongation(*self.dims[l + 1]))
        if coarse_operator == "galerkin":
            for l in range(1, levels):
                Pt = sp.diags(self.free[l - 1]) @ self.P[l - 1] @ sp.diags(self.free[l])
                self.A[l] = (Pt.T @ self.A[l - 1] @ Pt + sp.diags(1.0 - self.free[l])).tocsr()
                self.D[l] = self.A[l].diagonal().copy()
        self._coarse = sla.cho_factor(self.A[-1].toarray(), lower=True)

    # -- pieces of Alg. 3 --------------------------------------------------
    def jacobi(self, l, u, f):
        """One damped-Jacobi sweep on level l (Eq. 21)."""
        return u + self.omega * (f - self.A[l] @ u) / self.D[l]

    def residual(self, l, u, f):
        """r = f - A u (Eq. 19)."""
        return f - self.A[l] @ u

    def restrict(self, l, r):
        """Coarse right-hand side M_{l+1} P^T r."""
        return self.free[l + 1] * (self.P[l].T @ r)

    def prolong(self, l, e):
        """Fine correction M_l P e."""
        return self.free[l] * (self.P[l] @ e)

    def coarse_solve(self, f):
        return sla.cho_solve(self._coarse, f)

    def vcycle(self, f, l=0):
        """u = V_l(f): Alg. 3 from a zero initial guess."""
        if l == self.levels - 1:
            return self.coarse_solve(f)
        u = np.zeros_like(f)
        for _ in range(self.sweeps):
            u = self.jacobi(l, u, f)
        e = self.vcycle(self.restrict(l, self.residual(l, u, f)), l + 1)
        u = u + self.prolong(l, e)
        for _ in range(self.sweeps):
            u = self.jacobi(l, u, f)
        return u

    def apply(self, u, l=0):
        return self.A[l] @ u


def pcg(apply_A, f, precond, rtol=1e-8, maxit=500, fixed_iters=None):
    """Preconditioned CG (Alg. 1) from x0 = 0.

    Returns (x, iterations, relative recursive residual, compliance history
    [f^T x_k for k = 1..]).  With ``fixed_iters`` the loop runs exactly that many
    iterations and ignores ``rtol``.
    """
    f = np.asarray(f, dtype=np.float64)
    x = np.zeros_like(f)
    r = f.copy()
    z = precond(r)
    p = z.copy()
    rz = float(r @ z)
    fnorm = float(np.linalg.norm(f))
    hist = []
    it = 0
    limit = fixed_iters if fixed_iters is not None else maxit
    if fnorm == 0.0:
        return x, 0, 0.0, hist
    while it < limit:
        q = apply_A(p)
        alpha = rz / float(p @ q)
        x = x + alpha * p
        r = r - alpha * q
        it += 1
        hist.append(float(f @ x))
        rnorm = float(np.linalg.norm(r))
        if fixed_iters is None and rnorm <= rtol * fnorm:
            break
        z = precond(r)
        rz_new = float(r @ z)
        beta = rz_new / rz
        p = z + beta * p
        rz = rz_new
    return x, it, float(np.linalg.norm(r)) / fnorm, hist


def mgpcg(h: Hierarchy, f, rtol=1e-8, maxit=500, fixed_iters=None):
    """PCG on the finest level of ``h`` preconditioned by one V-cycle."""
    return pcg(h.apply, f, h.vcycle, rtol=rtol, maxit=maxit, fixed_iters=fixed_iters)
