"""GPU-vs-oracle parity of the HIP path, through the C ABI.

Tolerances (relative, norm-wise unless stated):
* binary64 K u, element quantities: 1e-13 -- same products, different summation order;
* binary64 V-cycle and fixed-iteration MGPCG: 1e-10 -- the coarsest solve differs
  (Gauss-Jordan inverse here, Cholesky in the oracle), each within ~kappa*eps;
* binary32 K u: 1e-5 (a few ulp of float32 per accumulated product);
* mixed-precision solve: compliance within 1e-5 of the binary64 result.
"""
import numpy as np
import pytest

import workloads as W
from oracle import fem, multigrid as mg

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _require_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def rel(a, b):
    a, b = np.asarray(a, dtype=np.float64).ravel(), np.asarray(b, dtype=np.float64).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def make_case(dims, levels, density="field", seed=1, **kw):
    from paper_2201_12931_amd import hexmg

    _require_gpu()
    g = W.Grid(*dims)
    if density == "field":
        rho = W.random_field_density(g, seed=seed, length_scale=4.0, lo=0.01)
    elif density == "uniform":
        rho = W.uniform_density(g, 0.3)
    else:
        rho = W.iid_uniform_density(g, seed=seed, lo=0.3)
    mask = W.fixed_mask_face_x0(g)
    kw.setdefault("vcycle_both", 1)  # the cases run V-cycles in both precisions
    grid = hexmg.Grid(*dims, levels, **kw)
    grid.set_density(torch.from_numpy(rho).cuda())
    torch.cuda.synchronize()
    return g, rho, mask, grid


def gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


DIMS = [((4, 2, 2), 1), ((20, 12, 10), 2), ((32, 16, 16), 3), ((24, 8, 16), 4)]


@pytest.mark.parametrize("dims,levels", DIMS)
def test_apply_K_fp64_every_level(dims, levels):
    print(f"case apply_K fp64 dims={dims} levels={levels}", flush=True)
    g, rho, mask, grid = make_case(dims, levels)
    h = mg.Hierarchy(*dims, rho, mask, levels)
    for l in range(levels):
        n = grid.level_dofs(l)
        u = W.random_vector(n, seed=10 + l)
        y = torch.empty(n, dtype=torch.float64, device="cuda")
        grid.apply_K(gpu(u), y, level=l)
        ref = h.A[l] @ u
        got = y.cpu().numpy()
        assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max(), (l, rel(got, ref))


@pytest.mark.parametrize("dims,levels", DIMS[1:3])
def test_apply_K_fp32(dims, levels):
    print(f"case apply_K fp32 dims={dims}", flush=True)
    g, rho, mask, grid = make_case(dims, levels)
    h = mg.Hierarchy(*dims, rho, mask, levels)
    u = W.random_vector(g.n_dof, seed=3).astype(np.float32)
    y = torch.empty(g.n_dof, dtype=torch.float32, device="cuda")
    grid.apply_K(gpu(u), y)
    ref = h.A[0] @ u.astype(np.float64)
    assert rel(y.cpu().numpy(), ref) < 1e-5


def test_apply_K_multi_rhs_and_fixed_dofs():
    """nrhs vectors in one call; fixed DOFs return u itself and ignore their value
    as input of the neighbours' rows."""
    dims = (16, 8, 8)
    g, rho, mask, grid = make_case(dims, 3)
    A = fem.constrained_operator(fem.assemble_stiffness(*dims, fem.simp_modulus(rho)), fem.free_dof_mask(mask))
    U = W.random_vector(g.n_dof, seed=4, nrhs=3)
    Y = torch.empty(3, g.n_dof, dtype=torch.float64, device="cuda")
    grid.apply_K(gpu(U), Y)
    for r in range(3):
        ref = A @ U[r]
        assert np.abs(Y[r].cpu().numpy() - ref).max() <= 1e-13 * np.abs(ref).max()


@pytest.mark.parametrize("avg", ["density", "modulus"])
@pytest.mark.parametrize("sweeps,omega", [(1, 0.6), (2, 0.6), (3, 0.8)])
def test_vcycle_fp64_parity(avg, sweeps, omega):
    print(f"case vcycle fp64 avg={avg} sweeps={sweeps}", flush=True)
    from paper_2201_12931_amd import hexmg

    dims, levels = (32, 16, 16), 3
    g, rho, mask, grid = make_case(dims, levels, smooth_sweeps=sweeps, omega=omega,
                                   coarse_avg=hexmg.AVG_DENSITY if avg == "density" else hexmg.AVG_MODULUS)
    h = mg.Hierarchy(*dims, rho, mask, levels, omega=omega, sweeps=sweeps, coarse_average=avg)
    r = W.random_vector(g.n_dof, seed=21) * h.free[0]
    z = torch.empty(g.n_dof, dtype=torch.float64, device="cuda")
    grid.vcycle(gpu(r), z)
    assert rel(z.cpu().numpy(), h.vcycle(r)) < 1e-10


def test_vcycle_fp32_close_to_fp64():
    dims, levels = (32, 16, 16), 3
    g, rho, mask, grid = make_case(dims, levels)
    h = mg.Hierarchy(*dims, rho, mask, levels)
    r = W.random_vector(g.n_dof, seed=22) * h.free[0]
    z = torch.empty(g.n_dof, dtype=torch.float32, device="cuda")
    grid.vcycle(gpu(r.astype(np.float32)), z)
    assert rel(z.cpu().numpy(), h.vcycle(r)) < 1e-4


def test_vcycle_symmetric_positive():
    dims, levels = (32, 16, 16), 3
    g, rho, mask, grid = make_case(dims, levels)
    free = fem.free_dof_mask(mask)
    a = W.random_vector(g.n_dof, seed=1) * free
    b = W.random_vector(g.n_dof, seed=2) * free
    za = torch.empty(g.n_dof, dtype=torch.float64, device="cuda")
    zb = torch.empty_like(za)
    grid.vcycle(gpu(a), za)
    grid.vcycle(gpu(b), zb)
    ba, ab = float(b @ za.cpu().numpy()), float(a @ zb.cpu().numpy())
    assert abs(ba - ab) <= 1e-11 * abs(ab)
    assert float(a @ za.cpu().numpy()) > 0


@pytest.mark.parametrize("dims,levels,iters", [((32, 16, 16), 3, 6), ((24, 8, 16), 4, 5)])
def test_mgpcg_fixed_iterations_parity(dims, levels, iters):
    """rtol <= 0 runs exactly `iters` PCG iterations; the iterate must equal the
    oracle's PCG iterate after the same number of steps."""
    print(f"case mgpcg fixed dims={dims} iters={iters}", flush=True)
    g, rho, mask, grid = make_case(dims, levels)
    h = mg.Hierarchy(*dims, rho, mask, levels)
    f = W.cantilever_line_load(g)
    u = torch.empty(g.n_dof, dtype=torch.float64, device="cuda")
    code, info = grid.solve(gpu(f), u, rtol=0.0, maxit=iters)
    assert info[0]["iterations"] == iters
    x, its, _, _ = mg.mgpcg(h, f, fixed_iters=iters)
    assert rel(u.cpu().numpy(), x) < 1e-10


def test_cantilever_32x16x16_fp64_against_direct():
    """The 32x16x16 cantilever (uniform density 0.3, 3 levels, rtol 1e-8): u,
    compliance and sensitivity against the sparse direct solve."""
    print("case cantilever 32x16x16 fp64", flush=True)
    dims = (32, 16, 16)
    g, rho, mask, grid = make_case(dims, 3, density="uniform")
    f = W.cantilever_line_load(g)
    K = fem.assemble_stiffness(*dims, fem.simp_modulus(rho))
    u_ref = fem.solve_direct(K, f, fem.free_dof_mask(mask))
    c_ref = fem.compliance(f, u_ref)
    u = torch.empty(g.n_dof, dtype=torch.float64, device="cuda")
    code, info = grid.solve(gpu(f), u, rtol=1e-8, maxit=200)
    assert code == 0 and info[0]["status"] == 0
    assert info[0]["rel_res_true"] < 2e-8
    assert info[0]["compliance"] == pytest.approx(c_ref, rel=1e-10)
    un = u.cpu().numpy()
    assert rel(un, u_ref) < 1e-6
    dc = torch.empty(g.n_elem, dtype=torch.float64, device="cuda")
    c = grid.compliance_sensitivity(gpu(f), u, dc)
    assert c[0] == pytest.approx(info[0]["compliance"], rel=1e-14)
    # element parity of the sensitivity kernel for the same u
    ref_dc = fem.sensitivity(*dims, rho, un)
    assert np.abs(dc.cpu().numpy() - ref_dc).max() <= 1e-12 * np.abs(ref_dc).max()
    # parity mode: tighter solve, u against the direct solve
    code, info = grid.solve(gpu(f), u, rtol=1e-12, maxit=400)
    assert rel(u.cpu().numpy(), u_ref) < 1e-9
    # c* - c_k = ||e_k||_K^2 > 0: a loosely converged iterate's compliance lies
    # below c* (at rtol 1e-8 the gap is below the direct solve's own rounding)
    code, info = grid.solve(gpu(f), u, rtol=1e-3, maxit=400)
    assert info[0]["compliance"] < c_ref
    assert info[0]["compliance"] > c_ref * (1 - 1e-4)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_single_level_solve_against_direct(precision):
    """One level: the preconditioner is the exact coarse inverse itself (no
    sweep to fuse the residual update or r . z into), so PCG stops after one
    or two iterations at the direct solution."""
    from paper_2201_12931_amd import hexmg

    print(f"case single-level solve {precision}", flush=True)
    dims = (6, 4, 4)
    prec = hexmg.FP64 if precision == "fp64" else hexmg.MIXED
    g, rho, mask, grid = make_case(dims, 1, density="uniform", precision=prec)
    f = W.cantilever_line_load(g)
    K = fem.assemble_stiffness(*dims, fem.simp_modulus(rho))
    u_ref = fem.solve_direct(K, f, fem.free_dof_mask(mask))
    u = torch.empty(g.n_dof, dtype=torch.float64, device="cuda")
    code, info = grid.solve(gpu(f), u, rtol=1e-10, maxit=20)
    assert code == 0 and info[0]["status"] == 0
    assert info[0]["iterations"] <= (1 if precision == "fp64" else 4)
    assert rel(u.cpu().numpy(), u_ref) < (1e-9 if precision == "fp64" else 1e-6)
    assert info[0]["compliance"] == pytest.approx(fem.compliance(f, u_ref), rel=1e-8)


def test_sensitivity_multi_rhs_weights():
    dims = (16, 8, 8)
    g, rho, mask, grid = make_case(dims, 3)
    U = W.random_vector(g.n_dof, seed=8, nrhs=2) * fem.free_dof_mask(mask)
    F = W.random_vector(g.n_dof, seed=9, nrhs=2)
    w = np.array([0.25, 2.0])
    dc = torch.empty(g.n_elem, dtype=torch.float64, device="cuda")
    c = grid.compliance_sensitivity(gpu(F), gpu(U), dc, weights=w)
    ref = w[0] * fem.sensitivity(*dims, rho, U[0]) + w[1] * fem.sensitivity(*dims, rho, U[1])
    assert np.abs(dc.cpu().numpy() - ref).max() <= 1e-12 * np.abs(ref).max()
    assert c == pytest.approx([F[0] @ U[0], F[1] @ U[1]], rel=1e-13)


def test_mixed_precision_solve():
    """FP32 V-cycle inside FP64 CG: same compliance as the FP64 path to 1e-5 and a
    true binary64 residual at the requested tolerance."""
    from paper_2201_12931_amd import hexmg

    dims, levels = (64, 32, 32), 4
    _require_gpu()
    g = W.Grid(*dims)
    rho = W.random_field_density(g, seed=1, lo=0.01)
    f = W.cantilever_line_load(g)
    res = {}
    for prec in (hexmg.FP64, hexmg.MIXED):
        grid = hexmg.Grid(*dims, levels, precision=prec)
        grid.set_density(gpu(rho))
        u = torch.empty(g.n_dof, dtype=torch.float64, device="cuda")
        code, info = grid.solve(gpu(f), u, rtol=1e-6, maxit=300)
        assert code == 0
        assert info[0]["rel_res_true"] < 1.5e-6
        res[prec] = (info[0], u.cpu().numpy())
    c64, c32 = res[hexmg.FP64][0]["compliance"], res[hexmg.MIXED][0]["compliance"]
    assert c32 == pytest.approx(c64, rel=1e-5)


@pytest.mark.parametrize("rr_every", [0, 3, 8])
def test_mixed32_solve_against_direct(rr_every):
    """Binary32 outer K p with binary64 CG vectors: the residual is replaced by
    the binary64 M f - A x every rr_every iterations, and CG restarts from its
    iterate while the binary64 residual misses rtol, so the solve reaches a
    binary64 residual of 1e-10 and the direct solution."""
    from paper_2201_12931_amd import hexmg

    print(f"case mixed32 solve rr_every={rr_every}", flush=True)
    dims, levels = (32, 16, 16), 3
    g, rho, mask, grid = make_case(dims, levels, precision=hexmg.MIXED32, rr_every=rr_every, vcycle_both=0)
    f = W.cantilever_line_load(g)
    K = fem.assemble_stiffness(*dims, fem.simp_modulus(rho))
    u_ref = fem.solve_direct(K, f, fem.free_dof_mask(mask))
    c_ref = fem.compliance(f, u_ref)
    u = torch.empty(g.n_dof, dtype=torch.float64, device="cuda")
    code, info = grid.solve(gpu(f), u, rtol=1e-10, maxit=300)
    assert code == 0 and info[0]["status"] == 0, info
    assert info[0]["rel_res_true"] <= 1e-10
    assert info[0]["compliance"] == pytest.approx(c_ref, rel=1e-9)
    assert rel(u.cpu().numpy(), u_ref) < 1e-7


def test_mixed32_matches_mixed_and_fp64_compliance():
    """The three precisions at rtol 1e-6 on a random field: binary64 residuals at
    the tolerance and compliances within 1e-5 of each other."""
    from paper_2201_12931_amd import hexmg

    print("case mixed32 vs mixed vs fp64", flush=True)
    dims, levels = (64, 32, 32), 4
    _require_gpu()
    g = W.Grid(*dims)
    rho = W.random_field_density(g, seed=1, lo=0.01)
    f = W.cantilever_line_load(g)
    res = {}
    for prec in (hexmg.FP64, hexmg.MIXED, hexmg.MIXED32):
        grid = hexmg.Grid(*dims, levels, precision=prec)
        grid.set_density(gpu(rho))
        u = torch.empty(g.n_dof, dtype=torch.float64, device="cuda")
        code, info = grid.solve(gpu(f), u, rtol=1e-6, maxit=300)
        assert code == 0, prec
        assert info[0]["rel_res_true"] <= 1e-6, (prec, info)
        res[prec] = info[0]["compliance"]
    assert res[hexmg.MIXED32] == pytest.approx(res[hexmg.FP64], rel=1e-5)
    assert res[hexmg.MIXED] == pytest.approx(res[hexmg.FP64], rel=1e-5)


def test_mixed32_multi_rhs_equals_single():
    """Lockstep right-hand sides with binary32 K p and residual replacement equal
    single solves bit for bit (same kernels, same order of every sum)."""
    from paper_2201_12931_amd import hexmg

    print("case mixed32 multi-rhs", flush=True)
    dims, levels = (32, 16, 16), 3
    _require_gpu()
    g = W.Grid(*dims)
    rho = gpu(W.random_field_density(g, seed=3, lo=0.01))
    F = gpu(W.point_loads(g, 3, seed=30))
    multi = hexmg.Grid(*dims, levels, precision=hexmg.MIXED32, max_nrhs=3, rr_every=4)
    single = hexmg.Grid(*dims, levels, precision=hexmg.MIXED32, max_nrhs=1, rr_every=4)
    for grid in (multi, single):
        grid.set_density(rho)
        for l in range(levels):
            for dt in (hexmg.F32, hexmg.F64):
                grid.set_kernel_choice(l, dt, hexmg.KERNEL_STREAM, 4, 0)
        grid.set_coarse_cycle(hexmg.F32, 0)
    U = torch.empty_like(F)
    code, info = multi.solve(F, U, rtol=1e-9, maxit=200)
    assert code == 0
    for r in range(3):
        u1 = torch.empty_like(F[r])
        c1, i1 = single.solve(F[r].contiguous(), u1, rtol=1e-9, maxit=200)
        assert i1[0]["iterations"] == info[r]["iterations"], r
        assert torch.equal(u1, U[r]), r
        assert info[r]["rel_res_true"] <= 1e-9


def test_mixed32_single_level():
    """One level (no sweep to fuse into): the restart path alone."""
    from paper_2201_12931_amd import hexmg

    print("case mixed32 single level", flush=True)
    dims = (6, 4, 4)
    g, rho, mask, grid = make_case(dims, 1, density="uniform", precision=hexmg.MIXED32, vcycle_both=0)
    f = W.cantilever_line_load(g)
    u_ref = fem.solve_direct(fem.assemble_stiffness(*dims, fem.simp_modulus(rho)), f, fem.free_dof_mask(mask))
    u = torch.empty(g.n_dof, dtype=torch.float64, device="cuda")
    code, info = grid.solve(gpu(f), u, rtol=1e-10, maxit=40)
    assert code == 0 and info[0]["rel_res_true"] <= 1e-10
    assert rel(u.cpu().numpy(), u_ref) < 1e-8


def test_vcycle_dtype_not_held_is_rejected():
    from paper_2201_12931_amd import hexmg

    g, rho, mask, grid = make_case((16, 8, 8), 3, vcycle_both=0)  # binary64 grid
    r = torch.zeros(g.n_dof, dtype=torch.float32, device="cuda")
    with pytest.raises(hexmg.HexmgError) as e:
        grid.vcycle(r, torch.empty_like(r))
    assert e.value.code == hexmg.ERR_INVALID


def test_uniaxial_bar_custom_supports():
    """Roller supports on x=0, y=0, z=0 given as a mask; uniaxial traction on x=nx.
    The exact trilinear solution u = (s x/E, -nu s y/E, -nu s z/E) is recovered."""
    from paper_2201_12931_amd import hexmg

    _require_gpu()
    nx, ny, nz = 16, 8, 8
    g = W.Grid(nx, ny, nz)
    k, j, i = np.meshgrid(np.arange(nz + 1), np.arange(ny + 1), np.arange(nx + 1), indexing="ij")
    i, j, k = i.ravel(), j.ravel(), k.ravel()
    mask = ((i == 0) * 1 + (j == 0) * 2 + (k == 0) * 4).astype(np.uint8)
    mask_t = gpu(mask)
    grid = hexmg.Grid(nx, ny, nz, 3, fixed_mask=mask_t)
    rho = 0.8
    grid.set_density(gpu(np.full(g.n_elem, rho)))
    E = float(fem.simp_modulus(rho))
    s = 1.5
    f = np.zeros(g.n_dof)
    for kk in range(nz):
        for jj in range(ny):
            for dj in (0, 1):
                for dk in (0, 1):
                    f[3 * g.node(nx, jj + dj, kk + dk)] += s / 4
    u = torch.empty(g.n_dof, dtype=torch.float64, device="cuda")
    code, info = grid.solve(gpu(f), u, rtol=1e-12, maxit=200)
    ue = np.stack([s * i / E, -0.3 * s * j / E, -0.3 * s * k / E], axis=1).ravel()
    assert np.abs(u.cpu().numpy() - ue).max() < 1e-9 * np.abs(ue).max()
    assert info[0]["compliance"] == pytest.approx(s * s * nx * ny * nz / E, rel=1e-10)


def test_set_density_rejects_bad_input():
    from paper_2201_12931_amd import hexmg

    g, rho, mask, grid = make_case((8, 4, 4), 2)
    bad = rho.copy()
    bad[3] = np.nan
    with pytest.raises(hexmg.HexmgError) as e:
        grid.set_density(gpu(bad))
    assert e.value.code == hexmg.ERR_NONFINITE
    bad[3] = 1.5
    with pytest.raises(hexmg.HexmgError):
        grid.set_density(gpu(bad))
    # a valid density restores the grid
    grid.set_density(gpu(rho))
    u = torch.zeros(g.n_dof, dtype=torch.float64, device="cuda")
    y = torch.empty_like(u)
    grid.apply_K(u, y)
    assert float(y.abs().max()) == 0.0


def test_zero_load_and_not_converged():
    g, rho, mask, grid = make_case((16, 8, 8), 3)
    u = torch.empty(g.n_dof, dtype=torch.float64, device="cuda")
    code, info = grid.solve(torch.zeros(g.n_dof, dtype=torch.float64, device="cuda"), u, rtol=1e-8)
    assert code == 0 and info[0]["iterations"] == 0 and float(u.abs().max()) == 0.0
    code, info = grid.solve(gpu(W.cantilever_line_load(g)), u, rtol=1e-14, maxit=2)
    assert code == 1 and info[0]["iterations"] == 2 and info[0]["status"] == 1


STREAM_SHAPES = [((1, 1, 1), 1), ((3, 5, 7), 1), ((61, 2, 3), 1), ((124, 16, 4), 3), ((128, 8, 64), 4),
                 ((64, 40, 24), 4)]


@pytest.mark.parametrize("dims,levels", STREAM_SHAPES)
def test_stream_kernel_shapes(dims, levels):
    """The z-streaming kernel against the assembled operator on grids that cut
    its tiles raggedly in x (62 columns per tile), y (rows per workgroup) and z
    (planes per chunk), in both precisions and on every level."""
    print(f"case stream dims={dims} levels={levels}", flush=True)
    g, rho, mask, grid = make_case(dims, levels)
    h = mg.Hierarchy(*dims, rho, mask, levels)
    for l in range(levels):
        n = grid.level_dofs(l)
        u = W.random_vector(n, seed=30 + l)
        ref = h.A[l] @ u
        y = torch.empty(n, dtype=torch.float64, device="cuda")
        grid.apply_K(gpu(u), y, level=l)
        got = y.cpu().numpy()
        assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max(), (l, rel(got, ref))
        y32 = torch.empty(n, dtype=torch.float32, device="cuda")
        grid.apply_K(gpu(u.astype(np.float32)), y32, level=l)
        assert rel(y32.cpu().numpy(), ref) < 1e-5, l


def test_stream_and_gather_kernels_agree():
    """The two K u kernels give the same V-cycle and the same MGPCG iterate."""
    from paper_2201_12931_amd import hexmg

    dims, levels = (64, 32, 32), 4
    _require_gpu()
    g = W.Grid(*dims)
    rho = W.random_field_density(g, seed=2, lo=0.01)
    f = gpu(W.cantilever_line_load(g))
    r = gpu(W.random_vector(g.n_dof, seed=3) * fem.free_dof_mask(W.fixed_mask_face_x0(g)))
    out = {}
    for kern in (hexmg.KERNEL_STREAM, hexmg.KERNEL_GATHER):
        grid = hexmg.Grid(*dims, levels, kernel=kern)
        grid.set_density(gpu(rho))
        z = torch.empty_like(r)
        grid.vcycle(r, z)
        u = torch.empty_like(f)
        grid.solve(f, u, rtol=0.0, maxit=8)
        out[kern] = (z.cpu().numpy(), u.cpu().numpy())
    assert rel(out[0][0], out[1][0]) < 1e-12
    assert rel(out[0][1], out[1][1]) < 1e-10


@pytest.mark.parametrize("dtype_name,shape", [("f32", 0), ("f32", 1), ("f32", 2), ("f32", 3), ("f32", 4),
                                              ("f32", 5), ("f32", 6), ("f64", 0), ("f64", 1), ("f64", 2)])
@pytest.mark.parametrize("zchunk", [1, 2, 3, 8])
def test_every_stream_shape(dtype_name, shape, zchunk):
    """Each streaming tile shape and several z-chunk lengths, forced through
    hexmg_set_kernel_choice, on a grid that cuts the tiles raggedly (129 node
    columns, 25 node rows, 17 node planes), in all three modes (K u through
    apply_K; Jacobi and residual through a one-level-deep V-cycle)."""
    from paper_2201_12931_amd import hexmg

    print(f"case stream shape {dtype_name} {shape} zchunk={zchunk}", flush=True)
    dims, levels = (128, 24, 16), 4
    g, rho, mask, grid = make_case(dims, levels)
    dt = hexmg.F32 if dtype_name == "f32" else hexmg.F64
    npdt = np.float32 if dtype_name == "f32" else np.float64
    tol = 1e-5 if dtype_name == "f32" else 1e-13
    grid.set_kernel_choice(0, dt, hexmg.KERNEL_STREAM, zchunk, shape)
    assert grid.kernel_choice(0, dt) == ("stream", zchunk, shape)
    h = mg.Hierarchy(*dims, rho, mask, levels)
    u = W.random_vector(g.n_dof, seed=40)
    y = torch.empty(g.n_dof, dtype=torch.float32 if dt == hexmg.F32 else torch.float64, device="cuda")
    grid.apply_K(gpu(u.astype(npdt)), y)
    ref = h.A[0] @ u.astype(npdt).astype(np.float64)
    assert rel(y.cpu().numpy(), ref) < tol
    # smoothing and residual modes run inside the V-cycle
    r = W.random_vector(g.n_dof, seed=41) * h.free[0]
    z = torch.empty_like(y)
    grid.vcycle(gpu(r.astype(npdt)), z)
    assert rel(z.cpu().numpy(), h.vcycle(r)) < (1e-4 if dt == hexmg.F32 else 1e-10)


@pytest.mark.parametrize("precision,dtype_name,shape,zchunk", [
    ("mixed", "f32", 0, 4), ("mixed", "f32", 5, 3), ("mixed", "f32", 6, 1), ("fp64", "f64", 0, 4),
    ("fp64", "f64", 2, 1), ("mixed32", "f32", 0, 8)])
def test_first_sweep_formed_on_load_bitwise(precision, dtype_name, shape, zchunk):
    """The level-0 pre-smoothing whose second sweep forms the first sweep from
    zero, (omega/D) r, as it loads its input (fuse_first = 1) gives the same
    iterates, bit for bit, as the residual update writing that first sweep
    (fuse_first = 0), for each tile shape that has the form, with ragged tiles
    and z-chunks (including the preloaded one-plane form)."""
    from paper_2201_12931_amd import hexmg

    print(f"case first sweep {precision} shape {shape} zchunk={zchunk}", flush=True)
    _require_gpu()
    dims, levels = (124, 24, 20), 3
    g = W.Grid(*dims)
    rho = W.random_field_density(g, seed=5, length_scale=4.0, lo=0.01)
    f = gpu(W.cantilever_line_load(g))
    prec = {"mixed": hexmg.MIXED, "fp64": hexmg.FP64, "mixed32": hexmg.MIXED32}[precision]
    dt = hexmg.F32 if dtype_name == "f32" else hexmg.F64
    out = []
    for fuse in (1, 0):
        grid = hexmg.Grid(*dims, levels, precision=prec, fuse_first=fuse)
        grid.set_density(gpu(rho))
        for l in range(levels):  # the same kernels on both grids (timed choices can differ)
            for d in (hexmg.F32, hexmg.F64):
                if l == 0 and d == dt:
                    grid.set_kernel_choice(l, d, hexmg.KERNEL_STREAM, zchunk, shape)
                else:
                    grid.set_kernel_choice(l, d, hexmg.KERNEL_STREAM, 4, 0)
        for d in (hexmg.F32, hexmg.F64):
            grid.set_coarse_cycle(d, 0)
        u = torch.zeros_like(f)
        code, info = grid.solve(f, u, rtol=1e-7, maxit=60)
        out.append((u.cpu().numpy(), info[0]["iterations"], info[0]["compliance"], code))
    assert out[0][1] == out[1][1] and out[0][3] == out[1][3]
    assert np.array_equal(out[0][0], out[1][0])
    assert out[0][2] == out[1][2]


@pytest.mark.parametrize("shape,zchunk", [(0, 4), (1, 3), (2, 8), (2, 1)])
def test_binary64_product_on_binary32_direction_every_shape(shape, zchunk):
    """The mixed form's binary64 K p reads the binary32 search direction with
    its own kernels (one per tile shape): with the level-0 binary64 choice
    forced to each streaming shape and z-chunk, a fixed number of CG
    iterations gives the iterate of the node-gather kernel, which reads the
    same binary32 direction (binary64 sums in another order; the tolerance
    leaves room for a residual entry that then rounds to the other binary32
    neighbour on its way into the V-cycle)."""
    from paper_2201_12931_amd import hexmg

    print(f"case binary64 K p on binary32 direction shape {shape} zchunk={zchunk}", flush=True)
    _require_gpu()
    dims, levels = (124, 24, 20), 3
    g = W.Grid(*dims)
    rho = W.random_field_density(g, seed=6, length_scale=4.0, lo=0.01)
    f = gpu(W.cantilever_line_load(g))
    out = []
    for kern in (hexmg.KERNEL_STREAM, hexmg.KERNEL_GATHER):
        grid = hexmg.Grid(*dims, levels, precision=hexmg.MIXED)
        grid.set_density(gpu(rho))
        for l in range(levels):
            grid.set_kernel_choice(l, hexmg.F32, hexmg.KERNEL_STREAM, 4, 0)
        if kern == hexmg.KERNEL_STREAM:
            grid.set_kernel_choice(0, hexmg.F64, kern, zchunk, shape)
        else:
            grid.set_kernel_choice(0, hexmg.F64, kern)
        grid.set_coarse_cycle(hexmg.F32, 0)
        u = torch.zeros_like(f)
        grid.solve(f, u, rtol=0.0, maxit=8)
        out.append(u.cpu().numpy())
    assert rel(out[0], out[1]) < 1e-9


@pytest.mark.parametrize("iters", [1, 2, 3, 4, 7])
def test_mixed_deferred_x_updates(iters):
    """The mixed form brings x up to date after every even iteration only (two
    binary32 directions, alternating buffers) and applies what is pending
    when the solve stops: after any number of iterations, odd or even, the
    binary64 residual of the returned x equals the recursive residual that
    the iteration tracked (a direction applied twice or not at all would
    leave them apart by the size of that step), on two right-hand sides in
    lockstep."""
    from paper_2201_12931_amd import hexmg

    print(f"case mixed deferred x iters={iters}", flush=True)
    _require_gpu()
    dims, levels = (64, 16, 16), 3
    g = W.Grid(*dims)
    rho = W.random_field_density(g, seed=7, lo=0.01)
    f1 = W.cantilever_line_load(g)
    f2 = W.random_vector(g.n_dof, seed=8) * fem.free_dof_mask(W.fixed_mask_face_x0(g))
    grid = hexmg.Grid(*dims, levels, precision=hexmg.MIXED, max_nrhs=2)
    grid.set_density(gpu(rho))
    f = torch.stack([gpu(f1), gpu(f2)])
    u = torch.zeros_like(f)
    code, info = grid.solve(f, u, rtol=0.0, maxit=iters)
    for k in range(2):
        assert info[k]["iterations"] == iters
        rec, true = info[k]["rel_res_recursive"], info[k]["rel_res_true"]
        assert abs(true - rec) <= 1e-8 * rec, (k, rec, true)


def test_mixed_multi_rhs_equals_single():
    """Lockstep right-hand sides of the mixed form, which stop at their own
    iterations (odd or even, with one or two directions then pending), equal
    single solves bit for bit."""
    from paper_2201_12931_amd import hexmg

    print("case mixed multi-rhs", flush=True)
    dims, levels = (32, 16, 16), 3
    _require_gpu()
    g = W.Grid(*dims)
    rho = gpu(W.random_field_density(g, seed=3, lo=0.01))
    F = gpu(W.point_loads(g, 4, seed=31))
    multi = hexmg.Grid(*dims, levels, precision=hexmg.MIXED, max_nrhs=4)
    single = hexmg.Grid(*dims, levels, precision=hexmg.MIXED, max_nrhs=1)
    for grid in (multi, single):
        grid.set_density(rho)
        for l in range(levels):
            for dt in (hexmg.F32, hexmg.F64):
                grid.set_kernel_choice(l, dt, hexmg.KERNEL_STREAM, 4, 0)
        grid.set_coarse_cycle(hexmg.F32, 0)
    U = torch.empty_like(F)
    code, info = multi.solve(F, U, rtol=1e-9, maxit=200)
    assert code == 0
    for r in range(4):
        u1 = torch.empty_like(F[r])
        c1, i1 = single.solve(F[r].contiguous(), u1, rtol=1e-9, maxit=200)
        assert i1[0]["iterations"] == info[r]["iterations"], r
        assert torch.equal(u1, U[r]), r
        assert info[r]["rel_res_true"] <= 1e-9
    print("iterations", [info[r]["iterations"] for r in range(4)], flush=True)
