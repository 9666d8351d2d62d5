"""Pins of the oracle's multigrid hierarchy, V-cycle and MG-preconditioned CG."""
import numpy as np
import pytest

import workloads as W
from oracle import fem, multigrid as mg


def test_interpolation_reproduces_linear_fields():
    """Trilinear P maps the nodal values of any affine field on the coarse grid to
    the nodal values of the same field on the fine grid."""
    nxc, nyc, nzc = 3, 2, 2
    P = mg.prolongation(nxc, nyc, nzc)
    rng = np.random.default_rng(0)
    A, b = rng.standard_normal((3, 3)), rng.standard_normal(3)

    def field(nx, ny, nz, h):
        k, j, i = np.meshgrid(np.arange(nz + 1), np.arange(ny + 1), np.arange(nx + 1), indexing="ij")
        X = h * np.stack([i.ravel(), j.ravel(), k.ravel()], axis=1)
        return (X @ A.T + b).reshape(-1)

    uc = field(nxc, nyc, nzc, 2.0)
    uf = field(2 * nxc, 2 * nyc, 2 * nzc, 1.0)
    assert np.abs(P @ uc - uf).max() < 1e-13
    # rows are partitions of unity
    assert np.allclose(np.asarray(P.sum(axis=1)).ravel(), 1.0)


def test_galerkin_identity_uniform_density():
    """For a uniform modulus the re-discretised coarse operator (element side 2,
    i.e. 2 K0 per element) equals P^T K_fine P: this pins P's weights, R = P^T and
    the size scaling used for the coarse levels."""
    nxc, nyc, nzc = 2, 2, 1
    Ef = np.full(8 * nxc * nyc * nzc, 0.37)
    Kf = fem.assemble_stiffness(2 * nxc, 2 * nyc, 2 * nzc, Ef)
    Kc = fem.assemble_stiffness(nxc, nyc, nzc, np.full(nxc * nyc * nzc, 0.37), h=2.0)
    P = mg.prolongation(nxc, nyc, nzc)
    G = (P.T @ Kf @ P).toarray()
    assert np.abs(G - Kc.toarray()).max() < 1e-14 * np.abs(G).max()


def test_homogenize_and_injection():
    g = W.Grid(4, 2, 6)
    rho = W.iid_uniform_density(g, seed=1, lo=0.0)
    c = mg.homogenize(rho, 4, 2, 6)
    assert c.shape == (2 * 1 * 3,)
    a = rho.reshape(6, 2, 4)
    assert c[0] == pytest.approx(a[0:2, 0:2, 0:2].mean(), rel=1e-15)
    assert c[-1] == pytest.approx(a[4:6, 0:2, 2:4].mean(), rel=1e-15)
    assert mg.homogenize(np.full(48, 0.3), 4, 2, 6) == pytest.approx(np.full(6, 0.3))
    m = W.fixed_mask_face_x0(g)
    mc = mg.inject_node_mask(m, 4, 2, 6)
    assert np.array_equal(mc, W.fixed_mask_face_x0(W.Grid(2, 1, 3)))


def _hier(dims, levels, seed=4, **kw):
    g = W.Grid(*dims)
    rho = W.random_field_density(g, seed=seed, length_scale=4.0, lo=0.01)
    return g, rho, mg.Hierarchy(*dims, rho, W.fixed_mask_face_x0(g), levels, **kw)


@pytest.mark.parametrize("avg", ["density", "modulus"])
def test_vcycle_symmetric_positive_definite(avg):
    g, rho, h = _hier((8, 4, 4), 3, coarse_average=avg)
    rng = np.random.default_rng(9)
    a, b = rng.standard_normal(g.n_dof), rng.standard_normal(g.n_dof)
    Va, Vb = h.vcycle(a), h.vcycle(b)
    assert float(b @ Va) == pytest.approx(float(a @ Vb), rel=1e-12)
    for _ in range(3):
        x = rng.standard_normal(g.n_dof)
        assert float(x @ h.vcycle(x)) > 0


def test_one_level_is_exact_solve():
    """With a single level the V-cycle is the direct solve, so PCG stops after one
    iteration at the exact solution."""
    g = W.Grid(4, 2, 2)
    rho = W.iid_uniform_density(g, seed=4, lo=0.5)
    h = mg.Hierarchy(4, 2, 2, rho, W.fixed_mask_face_x0(g), 1)
    f = W.cantilever_line_load(g)
    u_ref = fem.solve_direct(fem.assemble_stiffness(4, 2, 2, fem.simp_modulus(rho)), f,
                             fem.free_dof_mask(W.fixed_mask_face_x0(g)))
    u, its, rel, _ = mg.mgpcg(h, f, rtol=1e-9)
    assert its == 1
    assert np.linalg.norm(u - u_ref) <= 1e-10 * np.linalg.norm(u_ref)


def test_mgpcg_matches_direct_and_compliance_from_below():
    """MGPCG converges to the direct solution; with x0 = 0 the compliance f^T x_k
    rises monotonically to c* (c* - c_k = ||e_k||_K^2)."""
    dims = (16, 8, 8)
    g, rho, h = _hier(dims, 3)
    f = W.cantilever_line_load(g)
    K = fem.assemble_stiffness(*dims, fem.simp_modulus(rho))
    u_ref = fem.solve_direct(K, f, fem.free_dof_mask(W.fixed_mask_face_x0(g)))
    c_ref = fem.compliance(f, u_ref)
    u, its, rel, hist = mg.mgpcg(h, f, rtol=1e-12, maxit=300)
    assert rel <= 1e-12
    assert np.linalg.norm(u - u_ref) <= 1e-7 * np.linalg.norm(u_ref)
    assert fem.compliance(f, u) == pytest.approx(c_ref, rel=1e-12)
    hist = np.array(hist)
    assert np.all(np.diff(hist) >= -1e-12 * c_ref)
    assert np.all(hist <= c_ref * (1 + 1e-12))


def test_jacobi_smoother_reduces_energy_error():
    """omega = 0.6 damped Jacobi is a convergent smoother: the A-norm of the error
    decreases on every sweep."""
    g, rho, h = _hier((8, 4, 4), 2)
    f = W.cantilever_line_load(g)
    u_ref = np.linalg.solve(h.A[0].toarray(), f)
    u = np.zeros_like(f)
    prev = np.inf
    for _ in range(5):
        u = h.jacobi(0, u, f)
        e = u - u_ref
        en = float(e @ (h.A[0] @ e))
        assert en < prev
        prev = en


def test_galerkin_hierarchy_equals_rediscretized_for_uniform_density():
    """Eq. 23 products with the supports: for a uniform density every Galerkin
    coarse operator equals the re-discretized one (the face x = 0 is fixed, so the
    masked prolongation is exercised)."""
    g = W.Grid(8, 4, 4)
    rho = np.full(g.n_elem, 0.45)
    mask = W.fixed_mask_face_x0(g)
    hr = mg.Hierarchy(8, 4, 4, rho, mask, 3)
    hg = mg.Hierarchy(8, 4, 4, rho, mask, 3, coarse_operator="galerkin")
    for l in range(3):
        d = (hr.A[l] - hg.A[l]).toarray()
        assert np.abs(d).max() < 1e-13 * abs(hr.A[l]).max(), l


def test_galerkin_coarse_correction_is_a_projection():
    """With Galerkin operators the two-grid coarse correction
    C = I - P~ A_c^-1 P~^T A is an A-orthogonal projection on the free DOFs
    (C^2 = C and A C symmetric); the re-discretized operator on a random field
    is not, which shows the check can fail."""
    g = W.Grid(8, 4, 4)
    rho = W.random_field_density(g, seed=4, length_scale=2.0, lo=0.05)
    mask = W.fixed_mask_face_x0(g)
    rng = np.random.default_rng(9)
    errs = {}
    for op in ("galerkin", "rediscretize"):
        h = mg.Hierarchy(8, 4, 4, rho, mask, 2, coarse_operator=op)
        A, Ac = h.A[0].toarray(), h.A[1].toarray()
        Pt = np.diag(h.free[0]) @ h.P[0].toarray() @ np.diag(h.free[1])
        C = np.eye(A.shape[0]) - Pt @ np.linalg.solve(Ac, Pt.T @ A)
        Mf = np.diag(h.free[0])
        x = h.free[0] * rng.standard_normal(A.shape[0])
        errs[op] = np.linalg.norm(Mf @ C @ (Mf @ C @ x) - Mf @ C @ x) / np.linalg.norm(x)
        if op == "galerkin":
            AC = Mf @ A @ C @ Mf
            assert np.abs(AC - AC.T).max() < 1e-10 * np.abs(AC).max()
    assert errs["galerkin"] < 1e-10
    assert errs["rediscretize"] > 1e-3


def test_galerkin_mgpcg_matches_direct():
    g = W.Grid(16, 8, 8)
    rho = W.random_field_density(g, seed=2, length_scale=3.0, lo=0.01)
    mask = W.fixed_mask_face_x0(g)
    f = W.cantilever_line_load(g)
    free = fem.free_dof_mask(mask)
    u_ref = fem.solve_direct(fem.assemble_stiffness(16, 8, 8, fem.simp_modulus(rho)), f, free)
    h = mg.Hierarchy(16, 8, 8, rho, mask, 3, coarse_operator="galerkin")
    u, its, rel, _ = mg.mgpcg(h, f, rtol=1e-10)
    assert np.linalg.norm(u - u_ref) / np.linalg.norm(u_ref) < 1e-8
