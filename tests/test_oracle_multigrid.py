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


# ---- homogenization on non-uniform densities (Sec. 4.2.2, Sec. 6) ---------
def _mean_of_children(v, nx, ny, nz):
    """Coarse value of every coarse element as the mean over its eight children,
    written out with loops (x fastest, as the element numbering)."""
    out = []
    for kc in range(nz // 2):
        for jc in range(ny // 2):
            for ic in range(nx // 2):
                s = 0.0
                for dk in (0, 1):
                    for dj in (0, 1):
                        for di in (0, 1):
                            s += v[(2 * ic + di) + nx * ((2 * jc + dj) + ny * (2 * kc + dk))]
                out.append(s / 8.0)
    return np.array(out)


def _simp_scalar(r, E0=1.0, Emin=1e-9):
    # SIMP modulus with p = 3 for one density, as a plain product
    return Emin + r * r * r * (E0 - Emin)


def _coarse_moduli_loops(rho, dims, levels, avg):
    """Per level, the modulus the re-discretized coarse element carries, by loops:
    'density' averages the densities over the children and then applies SIMP;
    'modulus' applies SIMP on the finest level and averages the moduli.  Level l
    also carries the element-size factor 2^l."""
    nx, ny, nz = dims
    r = list(rho)
    e = [_simp_scalar(v) for v in rho]
    out = [np.array(e)]
    for l in range(1, levels):
        r = list(_mean_of_children(r, nx, ny, nz))
        e = list(_mean_of_children(e, nx, ny, nz))
        nx, ny, nz = nx // 2, ny // 2, nz // 2
        mod = [_simp_scalar(v) for v in r] if avg == "density" else e
        out.append((1 << l) * np.array(mod))
    return out


def _dense_loops(nx, ny, nz, E, Ke):
    N = 3 * (nx + 1) * (ny + 1) * (nz + 1)
    K = np.zeros((N, N))
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                dofs = []
                for kk in (0, 1):
                    for jj in (0, 1):
                        for ii in (0, 1):
                            n = (i + ii) + (nx + 1) * ((j + jj) + (ny + 1) * (k + kk))
                            dofs += [3 * n, 3 * n + 1, 3 * n + 2]
                K[np.ix_(dofs, dofs)] += E[i + nx * (j + ny * k)] * Ke
    return K


@pytest.mark.parametrize("avg", ["density", "modulus"])
def test_homogenized_moduli_on_nonuniform_density(avg):
    """On i.i.d. densities the hierarchy's coarse moduli equal the loop-written
    rule of its reading (average, then SIMP; or SIMP, then average; times 2^l),
    and its assembled coarse operator equals the loop-assembled one with the
    unit element stiffness, these moduli and the injected supports."""
    from oracle.element import hex8_stiffness

    dims, levels = (8, 8, 8), 3
    g = W.Grid(*dims)
    rho = W.iid_uniform_density(g, seed=21, lo=0.01)
    mask = W.fixed_mask_face_x0(g)
    h = mg.Hierarchy(*dims, rho, mask, levels, coarse_average=avg)
    ref = _coarse_moduli_loops(rho, dims, levels, avg)
    for l in range(levels):
        assert np.abs(h.E[l] - ref[l]).max() <= 1e-15 * np.abs(ref[l]).max(), l
    # level 1 operator, 4x4x4 elements, by loops
    K1 = _dense_loops(4, 4, 4, ref[1], hex8_stiffness(0.3))
    m1 = W.fixed_mask_face_x0(W.Grid(4, 4, 4))
    free = np.repeat(m1 == 0, 3).astype(np.float64)
    A1 = np.diag(free) @ K1 @ np.diag(free) + np.diag(1.0 - free)
    assert np.abs(h.A[1].toarray() - A1).max() <= 1e-14 * np.abs(A1).max()


def test_the_two_averaging_readings_differ():
    """The two readings give coarse moduli that differ far beyond rounding on a
    non-uniform density (so the test above would catch a swap), while on a
    uniform density they coincide."""
    dims = (8, 8, 8)
    g = W.Grid(*dims)
    mask = W.fixed_mask_face_x0(g)
    rho = W.iid_uniform_density(g, seed=21, lo=0.01)
    hd = mg.Hierarchy(*dims, rho, mask, 3, coarse_average="density")
    hm = mg.Hierarchy(*dims, rho, mask, 3, coarse_average="modulus")
    for l in (1, 2):
        rel = np.abs(hd.E[l] - hm.E[l]).max() / np.abs(hm.E[l]).max()
        assert rel > 1e-2, (l, rel)
        # Jensen: the mean of x^3 is at least the cube of the mean
        assert np.all(hm.E[l] >= hd.E[l] * (1 - 1e-15))
    u = np.full(g.n_elem, 0.4)
    hd = mg.Hierarchy(*dims, u, mask, 3, coarse_average="density")
    hm = mg.Hierarchy(*dims, u, mask, 3, coarse_average="modulus")
    for l in (1, 2):
        assert np.abs(hd.E[l] - hm.E[l]).max() <= 1e-15 * hm.E[l].max()


# ---- PCG iterates: Krylov minimisers (Alg. 1) -------------------------------
def _krylov_minimiser(A, B, f, k):
    """argmin of x^T A x / 2 - f^T x over span{B f, (B A) B f, ..., (B A)^(k-1) B f},
    by a dense projection onto an orthonormal basis (Gram-Schmidt applied twice)."""
    Q = []
    v = B @ f
    for _ in range(k):
        w = v.copy()
        for _rep in range(2):
            for q in Q:
                w -= (q @ w) * q
        nrm = np.linalg.norm(w)
        Q.append(w / nrm)
        v = B @ (A @ v)
    Q = np.column_stack(Q)
    return Q @ np.linalg.solve(Q.T @ A @ Q, Q.T @ f)


def test_pcg_iterates_are_krylov_minimisers_jacobi():
    """With a fixed SPD preconditioner B, the k-th PCG iterate from x0 = 0 is the
    A-energy minimiser over the k-dimensional Krylov space of B A and B f; here B
    is the inverse diagonal, which converges slowly enough for ten steps."""
    g, rho, h = _hier((6, 2, 2), 1)
    A = h.A[0].toarray()
    B = np.diag(1.0 / np.diag(A))
    f = W.cantilever_line_load(g)
    for k in range(1, 11):
        x, its, _, _ = mg.pcg(lambda v: A @ v, f, lambda r: B @ r, fixed_iters=k)
        xs = _krylov_minimiser(A, B, f, k)
        e = x - xs
        assert its == k
        assert float(e @ A @ e) <= 1e-18 * float(xs @ A @ xs), k


def test_mgpcg_iterates_are_krylov_minimisers():
    """The same property for MGPCG with the V-cycle as B (a fixed linear SPD
    operator, formed column by column on a small grid), which pins the recurrence
    behind the fixed-iteration GPU parity cases."""
    g = W.Grid(8, 4, 4)
    rho = W.iid_uniform_density(g, seed=5, lo=0.05)
    h = mg.Hierarchy(8, 4, 4, rho, W.fixed_mask_face_x0(g), 2)
    n = g.n_dof
    B = np.column_stack([h.vcycle(np.eye(n)[:, j]) for j in range(n)])
    A = h.A[0].toarray()
    f = W.cantilever_line_load(g)
    for k in range(1, 6):
        x, its, _, _ = mg.mgpcg(h, f, fixed_iters=k)
        xs = _krylov_minimiser(A, B, f, k)
        e = x - xs
        assert float(e @ A @ e) <= 1e-16 * float(xs @ A @ xs), k
