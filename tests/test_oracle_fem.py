"""Pins of the oracle's assembly, supports, solve, compliance and sensitivity."""
import numpy as np
import pytest

import workloads as W
from oracle import fem
from oracle.element import hex8_stiffness, lame

NU = 0.3


def test_element_nodes_brute_force():
    nx, ny, nz = 3, 2, 2
    en = fem.element_nodes(nx, ny, nz)
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                e = i + nx * (j + ny * k)
                for a in range(8):
                    ax, ay, az = a & 1, (a >> 1) & 1, (a >> 2) & 1
                    n = (i + ax) + (nx + 1) * ((j + ay) + (ny + 1) * (k + az))
                    assert en[e, a] == n


def _dense_brute_force(nx, ny, nz, E, Ke):
    """Global K by explicit loops (independent of the oracle's vectorised assembly)."""
    N = 3 * (nx + 1) * (ny + 1) * (nz + 1)
    K = np.zeros((N, N))
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                e = i + nx * (j + ny * k)
                dofs = []
                for kk in (0, 1):
                    for jj in (0, 1):
                        for ii in (0, 1):
                            n = (i + ii) + (nx + 1) * ((j + jj) + (ny + 1) * (k + kk))
                            dofs += [3 * n, 3 * n + 1, 3 * n + 2]
                for r in range(24):
                    for c in range(24):
                        K[dofs[r], dofs[c]] += E[e] * Ke[r, c]
    return K


@pytest.mark.parametrize("dims", [(2, 1, 1), (3, 2, 2), (4, 2, 2)])
def test_assembly_and_solve_brute_force(dims):
    g = W.Grid(*dims)
    rho = W.iid_uniform_density(g, seed=7, lo=0.05)
    E = fem.simp_modulus(rho)
    Ke = hex8_stiffness(NU)
    Kd = _dense_brute_force(*dims, E, Ke)
    K = fem.assemble_stiffness(*dims, E)
    assert np.abs(K.toarray() - Kd).max() < 1e-15
    mask = W.fixed_mask_face_x0(g)
    f = W.cantilever_line_load(g)
    free = fem.free_dof_mask(mask)
    idx = np.flatnonzero(free)
    u_ref = np.zeros(g.n_dof)
    u_ref[idx] = np.linalg.solve(Kd[np.ix_(idx, idx)], f[idx])
    u = fem.solve_direct(K, f, free)
    assert np.linalg.norm(u - u_ref) <= 1e-10 * np.linalg.norm(u_ref)
    # energy identity c = f^T u = u^T K u
    c = fem.compliance(f, u)
    assert c == pytest.approx(float(u @ (Kd @ u)), rel=1e-10)
    assert c > 0


def test_patch_test_linear_field():
    """Uniform modulus, u = A X + b: constant stress, so interior nodal forces vanish."""
    nx, ny, nz = 4, 3, 3
    g = W.Grid(nx, ny, nz)
    K = fem.assemble_stiffness(nx, ny, nz, np.full(g.n_elem, 0.7))
    rng = np.random.default_rng(3)
    A, b = rng.standard_normal((3, 3)), rng.standard_normal(3)
    k, j, i = np.meshgrid(np.arange(nz + 1), np.arange(ny + 1), np.arange(nx + 1), indexing="ij")
    X = np.stack([i.ravel(), j.ravel(), k.ravel()], axis=1).astype(float)
    u = (X @ A.T + b).reshape(-1)
    y = (K @ u).reshape(-1, 3)
    interior = ((X[:, 0] > 0) & (X[:, 0] < nx) & (X[:, 1] > 0) & (X[:, 1] < ny)
                & (X[:, 2] > 0) & (X[:, 2] < nz))
    assert np.abs(y[interior]).max() < 1e-13 * np.abs(y).max() + 1e-14
    # rigid motions produce no force anywhere
    W_ = np.array([[0, -0.3, 0.2], [0.3, 0, -0.1], [-0.2, 0.1, 0]])
    ur = (X @ W_.T + b).reshape(-1)
    assert np.abs(K @ ur).max() < 1e-13


def test_uniaxial_bar_exact():
    """Block under uniaxial traction s on x = nx with roller supports on x=0, y=0,
    z=0.  The exact field u = (s x/E, -nu s y/E, -nu s z/E) is trilinear, so the
    discrete solution equals it to round-off, and c = s^2 V / E."""
    nx, ny, nz = 4, 3, 2
    g = W.Grid(nx, ny, nz)
    rho = 0.6
    E = float(fem.simp_modulus(rho))
    K = fem.assemble_stiffness(nx, ny, nz, np.full(g.n_elem, E))
    k, j, i = np.meshgrid(np.arange(nz + 1), np.arange(ny + 1), np.arange(nx + 1), indexing="ij")
    i, j, k = i.ravel(), j.ravel(), k.ravel()
    mask = ((i == 0) * 1 + (j == 0) * 2 + (k == 0) * 4).astype(np.uint8)
    s = 2.5
    f = np.zeros(g.n_dof)
    # consistent nodal forces of a uniform traction on unit bilinear faces: s/4 per face corner
    for kk in range(nz):
        for jj in range(ny):
            for dj in (0, 1):
                for dk in (0, 1):
                    f[3 * g.node(nx, jj + dj, kk + dk)] += s / 4
    u = fem.solve_direct(K, f, fem.free_dof_mask(mask))
    ue = np.stack([s * i / E, -NU * s * j / E, -NU * s * k / E], axis=1).reshape(-1)
    assert np.abs(u - ue).max() < 1e-11 * np.abs(ue).max()
    assert fem.compliance(f, u) == pytest.approx(s * s * nx * ny * nz / E, rel=1e-12)


def test_uniform_density_scaling():
    """K(rho = const) = E(const) K(rho = 1) / E(1), so c scales by E(1)/E(rho)."""
    g = W.Grid(6, 3, 3)
    f, mask = W.cantilever_line_load(g), W.fixed_mask_face_x0(g)
    free = fem.free_dof_mask(mask)
    c = {}
    for r in (0.3, 1.0):
        E = fem.simp_modulus(np.full(g.n_elem, r))
        c[r] = fem.compliance(f, fem.solve_direct(fem.assemble_stiffness(6, 3, 3, E), f, free))
    assert c[0.3] == pytest.approx(c[1.0] * fem.simp_modulus(1.0) / fem.simp_modulus(0.3), rel=1e-11)


def test_sensitivity_euler_identity_and_fd():
    """Sum_e rho_e dc_e = -p (c - Emin sum_e u_e^T K0 u_e) (homogeneity of E(rho) - Emin
    of degree p), and dc matches central finite differences of c."""
    nx, ny, nz = 4, 2, 2
    g = W.Grid(nx, ny, nz)
    rho = W.iid_uniform_density(g, seed=11, lo=0.2)
    f, mask = W.cantilever_line_load(g), W.fixed_mask_face_x0(g)
    free = fem.free_dof_mask(mask)
    Emin = 1e-3  # large enough that the Emin term is visible in the identity

    def comp(r):
        K = fem.assemble_stiffness(nx, ny, nz, fem.simp_modulus(r, Emin=Emin))
        u = fem.solve_direct(K, f, free)
        return fem.compliance(f, u), u

    c, u = comp(rho)
    dc = fem.sensitivity(nx, ny, nz, rho, u, Emin=Emin)
    assert np.all(dc <= 0)
    energy = fem.element_energies(nx, ny, nz, u)
    assert float(rho @ dc) == pytest.approx(-3.0 * (c - Emin * energy.sum()), rel=1e-12)
    h = 1e-5
    for e in (0, 5, 9, 15):
        rp, rm = rho.copy(), rho.copy()
        rp[e] += h
        rm[e] -= h
        fd = (comp(rp)[0] - comp(rm)[0]) / (2 * h)
        assert fd == pytest.approx(dc[e], rel=1e-6)


def test_apply_at_nodes_matches_assembled():
    g = W.Grid(5, 3, 4)
    rho = W.iid_uniform_density(g, seed=2, lo=0.01)
    E = fem.simp_modulus(rho)
    mask = W.fixed_mask_face_x0(g)
    A = fem.constrained_operator(fem.assemble_stiffness(5, 3, 4, E), fem.free_dof_mask(mask))
    u = W.random_vector(g.n_dof, seed=5)
    nodes = np.arange(g.n_node)
    y = fem.apply_constrained_at_nodes(5, 3, 4, E, mask, u, nodes)
    assert np.abs(y.reshape(-1) - A @ u).max() < 1e-14 * np.abs(A @ u).max()


def test_line_load_total():
    g = W.Grid(32, 16, 16)
    f = W.cantilever_line_load(g)
    assert f.sum() == pytest.approx(-1.0, rel=1e-15)
    assert np.count_nonzero(f) == 17


def test_gravity_consistent_load_is_an_eighth_per_node():
    """The consistent nodal load of a constant body force on the trilinear
    element is the integral of each shape function: 2x2x2 Gauss quadrature of
    N_a = prod(1 - t or t) over the unit cube gives 1/8 for every corner."""
    gp = [0.5 - 0.5 / np.sqrt(3.0), 0.5 + 0.5 / np.sqrt(3.0)]
    for a in range(8):
        ax, ay, az = a & 1, (a >> 1) & 1, a >> 2
        s = 0.0
        for x in gp:
            for y in gp:
                for z in gp:
                    s += 0.125 * (x if ax else 1 - x) * (y if ay else 1 - y) * (z if az else 1 - z)
        assert s == pytest.approx(0.125, rel=1e-14)
    g = W.Grid(5, 3, 4)
    rho = W.iid_uniform_density(g, seed=2, lo=0.0)
    f = fem.gravity_load(5, 3, 4, rho, g=9.81)
    assert f[2::3].sum() == pytest.approx(-9.81 * rho.sum(), rel=1e-13)
    assert np.all(f[0::3] == 0) and np.all(f[1::3] == 0)
    fu = fem.gravity_load(5, 3, 4, np.full(g.n_elem, 0.5), g=2.0)
    interior = 2 + 6 * (1 + 4 * 2)  # node (2, 1, 2): eight adjacent elements
    assert fu[3 * interior + 2] == pytest.approx(-2.0 * 0.5, rel=1e-15)


def test_self_weight_compliance_gradient_finite_differences():
    """c(rho) = f(rho)^T u(rho) with a design-dependent load: the adjoint
    derivative (stiffness part + 2 u^T df/drho) against central differences of
    direct solves."""
    nx, ny, nz = 4, 2, 2
    g = W.Grid(nx, ny, nz)
    rho = W.iid_uniform_density(g, seed=3, lo=0.3)
    free = fem.free_dof_mask(W.fixed_mask_face_x0(g))
    f_ext = W.cantilever_line_load(g)

    def comp(r):
        f = f_ext + fem.gravity_load(nx, ny, nz, r, g=0.7)
        u = fem.solve_direct(fem.assemble_stiffness(nx, ny, nz, fem.simp_modulus(r)), f, free)
        return fem.compliance(f * free, u), u

    c0, u = comp(rho)
    dc = fem.sensitivity(nx, ny, nz, rho, u) + fem.gravity_sensitivity(nx, ny, nz, u, g=0.7)
    h = 1e-6
    for e in range(g.n_elem):
        rp, rm = rho.copy(), rho.copy()
        rp[e] += h
        rm[e] -= h
        fd = (comp(rp)[0] - comp(rm)[0]) / (2 * h)
        assert fd == pytest.approx(dc[e], rel=1e-6, abs=1e-9 * abs(dc).max()), e
