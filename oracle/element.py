"""Unit hex8 element stiffness -- test infrastructure only (see ``oracle/__init__``).

The paper uses the solid element stiffness K0 of an 8-node brick (Sec. 2,
Eq. 2; Algorithm 4 computes it once before the optimisation loop).  It is the
standard isoparametric trilinear element; we write the definition out:

    K0 = integral over the unit cube of B^T D B dV,

with B the 6x24 strain-displacement matrix (engineering shear strains) and D the
isotropic elasticity matrix of Young's modulus 1 and Poisson ratio nu.  The
integrand is a polynomial of degree 2 in each coordinate, so 2x2x2 Gauss
quadrature is exact.

Local node ``a = ax + 2*ay + 4*az`` sits at (ax, ay, az) in {0,1}^3; local DOF is
``3*a + c``.
"""
from __future__ import annotations

import numpy as np


def lame(E: float = 1.0, nu: float = 0.3):
    """Lame parameters (lambda, mu) of an isotropic material."""
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    mu = E / (2.0 * (1.0 + nu))
    return lam, mu


def elasticity_matrix(E: float = 1.0, nu: float = 0.3) -> np.ndarray:
    """6x6 isotropic D for strains (xx, yy, zz, xy, yz, zx), engineering shear."""
    lam, mu = lame(E, nu)
    D = np.zeros((6, 6))
    D[:3, :3] = lam
    for i in range(3):
        D[i, i] = lam + 2.0 * mu
        D[3 + i, 3 + i] = mu
    return D


def _shape_gradients(x: float, y: float, z: float) -> np.ndarray:
    """d N_a / d(x,y,z) for the 8 trilinear shape functions on the unit cube; (8, 3)."""
    g = np.zeros((8, 3))
    for a in range(8):
        ax, ay, az = a & 1, (a >> 1) & 1, (a >> 2) & 1
        fx = x if ax else 1.0 - x
        fy = y if ay else 1.0 - y
        fz = z if az else 1.0 - z
        sx = 1.0 if ax else -1.0
        sy = 1.0 if ay else -1.0
        sz = 1.0 if az else -1.0
        g[a] = (sx * fy * fz, fx * sy * fz, fx * fy * sz)
    return g


def strain_displacement(x: float, y: float, z: float) -> np.ndarray:
    """6x24 B at a point of the unit cube."""
    g = _shape_gradients(x, y, z)
    B = np.zeros((6, 24))
    for a in range(8):
        dx, dy, dz = g[a]
        B[0, 3 * a + 0] = dx
        B[1, 3 * a + 1] = dy
        B[2, 3 * a + 2] = dz
        B[3, 3 * a + 0] = dy
        B[3, 3 * a + 1] = dx
        B[4, 3 * a + 1] = dz
        B[4, 3 * a + 2] = dy
        B[5, 3 * a + 0] = dz
        B[5, 3 * a + 2] = dx
    return B


def hex8_stiffness(nu: float = 0.3, E: float = 1.0, h: float = 1.0) -> np.ndarray:
    """24x24 stiffness of a cube of side h: 2x2x2 Gauss rule on B^T D B.

    Scaling: B ~ 1/h and dV ~ h^3, so K(h) = h * K(1); we integrate on the unit
    cube and multiply by h.
    """
    D = elasticity_matrix(E, nu)
    q = [(1.0 - 1.0 / np.sqrt(3.0)) / 2.0, (1.0 + 1.0 / np.sqrt(3.0)) / 2.0]
    K = np.zeros((24, 24))
    for x in q:
        for y in q:
            for z in q:
                B = strain_displacement(x, y, z)
                K += B.T @ D @ B * (1.0 / 8.0)
    return K * h


def node_coords() -> np.ndarray:
    """(8, 3) local coordinates of the element nodes."""
    return np.array([[a & 1, (a >> 1) & 1, (a >> 2) & 1] for a in range(8)], dtype=float)
