"""Assembled finite-element model of the SIMP state equation -- test infrastructure only.

Follows Sec. 2 of the paper:

* Eq. 2 (SIMP): K_e = K_min + rho_e^p (K_0 - K_min).  We read K_min as Emin*K0
  (the paper only calls it the stiffness of the least allowable density), so
  K_e = E(rho_e) K0 with E(rho) = Emin + rho^p (E0 - Emin).
* Eq. 1 / Eq. 10: K(rho) u = f with the global K assembled from the K_e.
* Eq. 6: compliance c = f^T u.
* Eq. 7: dc/drho_e = -u_e^T (p rho_e^(p-1) (K0 - K_min)) u_e, with u* = u because
  the compliance is self-adjoint; in our reading that is
  -p rho_e^(p-1) (E0 - Emin) u_e^T K0 u_e.
* Self-weight (the foot-bridge example's gravity loading): a load that depends
  on the design, f(rho), adds 2 u^T df/drho_e to the derivative.

Supports are imposed by elimination: fixed DOFs are removed from the system and
carry u = 0.  For operator-level comparisons the same supports are written as
A = M K M + (I - M) with M the diagonal 0/1 "free" mask (rows and columns of the
fixed DOFs replaced by identity), which has the same solution.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .element import hex8_stiffness


def simp_modulus(rho, E0=1.0, Emin=1e-9, p=3.0):
    """E(rho) = Emin + rho^p (E0 - Emin)  (Eq. 2 with K_min = Emin K0)."""
    rho = np.asarray(rho, dtype=np.float64)
    return Emin + rho ** p * (E0 - Emin)


def element_nodes(nx: int, ny: int, nz: int) -> np.ndarray:
    """(Ne, 8) global node numbers of each element's corners.

    Element e = i + nx (j + ny k); local corner a = ax + 2 ay + 4 az is the node
    (i+ax, j+ay, k+az) = (i+ax) + (nx+1) ((j+ay) + (ny+1) (k+az)).
    """
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    base = (i + (nx + 1) * (j + (ny + 1) * k)).reshape(-1)
    off = np.array([ax + (nx + 1) * (ay + (ny + 1) * az)
                    for az in (0, 1) for ay in (0, 1) for ax in (0, 1)])
    return base[:, None] + off[None, :]


def element_dofs(nx: int, ny: int, nz: int) -> np.ndarray:
    """(Ne, 24) global DOFs of each element, local DOF 3a + c -> 3 n_a + c."""
    en = element_nodes(nx, ny, nz)
    return (3 * en[:, :, None] + np.arange(3)[None, None, :]).reshape(en.shape[0], 24)


def assemble_stiffness(nx, ny, nz, E, nu=0.3, h=1.0, chunk=1 << 16) -> sp.csr_matrix:
    """Global K = sum_e E_e * K0(h) scattered by element DOFs (no supports)."""
    Ke = hex8_stiffness(nu, h=h)
    dofs = element_dofs(nx, ny, nz)
    E = np.asarray(E, dtype=np.float64)
    N = 3 * (nx + 1) * (ny + 1) * (nz + 1)
    K = sp.csr_matrix((N, N))
    for s in range(0, dofs.shape[0], chunk):
        d = dofs[s:s + chunk]
        rows = np.broadcast_to(d[:, :, None], (d.shape[0], 24, 24)).reshape(-1)
        cols = np.broadcast_to(d[:, None, :], (d.shape[0], 24, 24)).reshape(-1)
        vals = (E[s:s + chunk, None, None] * Ke[None, :, :]).reshape(-1)
        K = K + sp.coo_matrix((vals, (rows, cols)), shape=(N, N)).tocsr()
    return K.tocsr()


def free_dof_mask(node_mask: np.ndarray) -> np.ndarray:
    """Boolean per DOF: True where the DOF is free (mask bit c of its node unset)."""
    m = np.asarray(node_mask, dtype=np.uint8)
    bits = np.stack([(m >> c) & 1 for c in range(3)], axis=1).reshape(-1)
    return bits == 0


def constrained_operator(K: sp.spmatrix, free: np.ndarray) -> sp.csr_matrix:
    """A = M K M + (I - M): fixed rows/columns replaced by identity."""
    M = sp.diags(free.astype(np.float64))
    I_M = sp.diags((~free).astype(np.float64))
    return (M @ K @ M + I_M).tocsr()


def solve_direct(K: sp.spmatrix, f: np.ndarray, free: np.ndarray) -> np.ndarray:
    """u with u_free = K_ff^{-1} f_free (sparse LU) and u_fixed = 0."""
    idx = np.flatnonzero(free)
    Kff = K[idx][:, idx].tocsc()
    u = np.zeros(K.shape[0])
    u[idx] = spla.splu(Kff).solve(np.asarray(f, dtype=np.float64)[idx])
    return u


def compliance(f: np.ndarray, u: np.ndarray) -> float:
    """c = f^T u  (Eq. 6)."""
    return float(np.dot(f, u))


def element_energies(nx, ny, nz, u: np.ndarray, nu=0.3) -> np.ndarray:
    """u_e^T K0 u_e per element (unit modulus, h = 1)."""
    Ke = hex8_stiffness(nu)
    ue = np.asarray(u)[element_dofs(nx, ny, nz)]
    return np.einsum("ei,ij,ej->e", ue, Ke, ue)


def sensitivity(nx, ny, nz, rho, u, E0=1.0, Emin=1e-9, p=3.0, nu=0.3) -> np.ndarray:
    """dc/drho_e = -p rho_e^(p-1) (E0 - Emin) u_e^T K0 u_e   (Eq. 7, self-adjoint u* = u)."""
    rho = np.asarray(rho, dtype=np.float64)
    return -p * rho ** (p - 1.0) * (E0 - Emin) * element_energies(nx, ny, nz, u, nu)


def apply_constrained_at_nodes(nx, ny, nz, E, node_mask, u, nodes, nu=0.3, h=1.0):
    """(A u) at the given nodes, computed node by node from the <= 8 adjacent elements.

    A = M K M + (I - M).  Used to check large outputs at sampled nodes without
    assembling K.  Returns an array (len(nodes), 3).
    """
    Ke = hex8_stiffness(nu, h=h)
    E = np.asarray(E, dtype=np.float64)
    free = free_dof_mask(node_mask)
    uf = np.where(free, np.asarray(u, dtype=np.float64), 0.0)
    nxn, nyn = nx + 1, ny + 1
    out = np.zeros((len(nodes), 3))
    for t, n in enumerate(np.asarray(nodes, dtype=np.int64)):
        i, j, k = n % nxn, (n // nxn) % nyn, n // (nxn * nyn)
        acc = np.zeros(3)
        for az in (0, 1):
            for ay in (0, 1):
                for ax in (0, 1):
                    ei, ej, ek = i - ax, j - ay, k - az
                    if not (0 <= ei < nx and 0 <= ej < ny and 0 <= ek < nz):
                        continue
                    e = ei + nx * (ej + ny * ek)
                    a = ax + 2 * ay + 4 * az
                    ue = np.zeros(24)
                    for b in range(8):
                        bx, by, bz = b & 1, (b >> 1) & 1, (b >> 2) & 1
                        m = (ei + bx) + nxn * ((ej + by) + nyn * (ek + bz))
                        ue[3 * b:3 * b + 3] = uf[3 * m:3 * m + 3]
                    acc += E[e] * (Ke[3 * a:3 * a + 3, :] @ ue)
        for c in range(3):
            d = 3 * n + c
            out[t, c] = acc[c] if free[d] else u[d]
    return out


def gravity_load(nx, ny, nz, rho, g=1.0) -> np.ndarray:
    """Self-weight of the design (the gravity loading of the paper's foot-bridge
    example): element e of unit volume and unit mass density carries the body
    force -g rho_e along z.  For the trilinear element each shape function
    integrates to 1/8 of the element volume, so each of its eight nodes takes
    -g rho_e / 8."""
    rho = np.asarray(rho, dtype=np.float64)
    f = np.zeros(3 * (nx + 1) * (ny + 1) * (nz + 1))
    nodes = element_nodes(nx, ny, nz)
    np.add.at(f, 3 * nodes.reshape(-1) + 2, np.repeat(-g * rho / 8.0, 8))
    return f


def gravity_sensitivity(nx, ny, nz, u, g=1.0) -> np.ndarray:
    """Load part of dc/drho_e for c = f(rho)^T u with K u = f(rho):
    dc/drho_e = 2 u^T df/drho_e - u^T dK/drho_e u; this returns the first term,
    2 (-g / 8) (sum of u_z over the element's nodes)."""
    u = np.asarray(u, dtype=np.float64)
    uz = u[3 * element_nodes(nx, ny, nz) + 2]
    return 2.0 * (-g / 8.0) * uz.sum(axis=1)
