"""Pins of the oracle's hex8 element stiffness against closed forms.

Every expected value below is derived by hand from linear elasticity on the unit
cube (Lame parameters lambda, mu), not from the oracle's own quadrature.
"""
import numpy as np
import pytest

from oracle.element import hex8_stiffness, lame, node_coords

NU = 0.3


@pytest.fixture(scope="module")
def Ke():
    return hex8_stiffness(NU)


def test_symmetric(Ke):
    assert np.abs(Ke - Ke.T).max() < 1e-15


def test_rigid_body_null_space(Ke):
    """Exactly 6 zero eigenvalues; the 3 translations and 3 infinitesimal rotations
    u = w x X are in the null space."""
    ev = np.linalg.eigvalsh(Ke)
    assert np.sum(np.abs(ev) < 1e-12) == 6
    assert ev[6] > 0.06
    X = node_coords() - 0.5
    modes = []
    for c in range(3):
        t = np.zeros((8, 3))
        t[:, c] = 1.0
        modes.append(t.reshape(-1))
    for w in np.eye(3):
        modes.append(np.cross(w, X).reshape(-1))
    R = np.stack(modes, axis=1)
    assert np.linalg.matrix_rank(R) == 6
    assert np.abs(Ke @ R).max() < 1e-14


def test_closed_form_entries(Ke):
    """K[x0,x0] = integral of (lambda+2mu)(dN/dx)^2 + mu((dN/dy)^2+(dN/dz)^2) with
    N = (1-x)(1-y)(1-z): each squared derivative integrates to 1/9, giving
    (lambda + 4 mu)/9.  K[x0,y0] = (lambda+mu) * integral dN/dx dN/dy = (lambda+mu)/12.
    Every diagonal entry equals K[x0,x0] by the cube's symmetry."""
    lam, mu = lame(1.0, NU)
    assert Ke[0, 0] == pytest.approx((lam + 4 * mu) / 9, rel=1e-14)
    assert Ke[0, 1] == pytest.approx((lam + mu) / 12, rel=1e-14)
    assert np.allclose(np.diag(Ke), (lam + 4 * mu) / 9, rtol=1e-14, atol=0)


def test_dilatation_eigenpair(Ke):
    """u = X - centre has strain I: energy 9 lambda + 6 mu over ||u||^2 = 6, and by
    symmetry it is an eigenvector: K u = (3 lambda + 2 mu)/2 u, the largest."""
    lam, mu = lame(1.0, NU)
    u = (node_coords() - 0.5).reshape(-1)
    assert np.allclose(Ke @ u, (3 * lam + 2 * mu) / 2 * u, rtol=0, atol=1e-14)
    assert np.linalg.eigvalsh(Ke)[-1] == pytest.approx((3 * lam + 2 * mu) / 2, rel=1e-13)


def test_twist_eigenpair(Ke):
    """u_z = (2x-1)(2y-1), u_y = -(2x-1)(2z-1): divergence-free with shear strains
    eps_xz = 2y-1, eps_xy = -(2z-1); energy 2 mu * 2 * (1/3 + 1/3) = 8 mu/3 over
    ||u||^2 = 16 gives the smallest non-zero eigenvalue mu/6."""
    lam, mu = lame(1.0, NU)
    X = node_coords()
    u = np.zeros((8, 3))
    u[:, 2] = (2 * X[:, 0] - 1) * (2 * X[:, 1] - 1)
    u[:, 1] = -(2 * X[:, 0] - 1) * (2 * X[:, 2] - 1)
    u = u.reshape(-1)
    assert np.allclose(Ke @ u, mu / 6 * u, rtol=0, atol=1e-14)
    assert np.linalg.eigvalsh(Ke)[6] == pytest.approx(mu / 6, rel=1e-12)


def test_size_scaling(Ke):
    """B ~ 1/h and dV ~ h^3, so K(h) = h K(1)."""
    assert np.abs(hex8_stiffness(NU, h=2.0) - 2.0 * Ke).max() < 1e-15
