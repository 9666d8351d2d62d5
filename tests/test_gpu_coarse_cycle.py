"""The coarse part of the V-cycle as one cooperative launch must be the same
cycle as the one launched step by step (Alg. 3): bit for bit when both use the
node-gather arithmetic, and within the V-cycle tolerance of the oracle."""
import numpy as np
import pytest

import workloads as W
from oracle import multigrid as mg

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def rel(a, b):
    a, b = np.asarray(a, dtype=np.float64).ravel(), np.asarray(b, dtype=np.float64).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _grid(dims, levels, **kw):
    from paper_2201_12931_amd import hexmg

    _gpu()
    g = W.Grid(*dims)
    rho = W.random_field_density(g, seed=5, length_scale=4.0, lo=0.01)
    kw.setdefault("vcycle_both", 1)  # V-cycles in both precisions
    grid = hexmg.Grid(*dims, levels, **kw)
    grid.set_density(gpu(rho))
    return g, rho, grid


@pytest.mark.parametrize("dims,levels", [((32, 16, 16), 4), ((48, 24, 24), 4), ((40, 24, 16), 4)])
@pytest.mark.parametrize("dtype_name", ["f64", "f32"])
def test_coarse_cycle_bitwise_equal_to_step_launches(dims, levels, dtype_name):
    from paper_2201_12931_amd import hexmg

    print(f"case coarse cycle bitwise {dims} levels={levels} {dtype_name}", flush=True)
    g, rho, grid = _grid(dims, levels, max_nrhs=2)
    dt = hexmg.F64 if dtype_name == "f64" else hexmg.F32
    tdt = torch.float64 if dt == hexmg.F64 else torch.float32
    for l in range(1, levels):  # same arithmetic on both paths
        grid.set_kernel_choice(l, dt, hexmg.KERNEL_GATHER)
    r = torch.from_numpy(np.stack([W.random_vector(g.n_dof, seed=s) for s in (31, 32)])).to("cuda", tdt)
    grid.set_coarse_cycle(dt, 0)
    ref = torch.empty_like(r)
    grid.vcycle(r, ref)
    for ls in range(1, levels - 1):
        for blocks in (3, 64, 0):
            grid.set_coarse_cycle(dt, ls, blocks)
            assert grid.coarse_cycle_choice(dt)[0] == ls
            z = torch.full_like(r, float("nan"))
            grid.vcycle(r, z)
            assert torch.equal(z, ref), (ls, blocks)


def test_coarse_cycle_vcycle_oracle_parity():
    from paper_2201_12931_amd import hexmg

    print("case coarse cycle vs oracle", flush=True)
    dims, levels = (32, 16, 16), 4
    g, rho, grid = _grid(dims, levels)
    h = mg.Hierarchy(*dims, rho, W.fixed_mask_face_x0(g), levels)
    r = W.random_vector(g.n_dof, seed=23) * h.free[0]
    ref = h.vcycle(r)
    for ls in (1, 2):
        grid.set_coarse_cycle(hexmg.F64, ls)
        z = torch.empty(g.n_dof, dtype=torch.float64, device="cuda")
        grid.vcycle(gpu(r), z)
        assert rel(z.cpu().numpy(), ref) < 1e-10, ls
        grid.set_coarse_cycle(hexmg.F32, ls)
        z32 = torch.empty(g.n_dof, dtype=torch.float32, device="cuda")
        grid.vcycle(gpu(r.astype(np.float32)), z32)
        assert rel(z32.cpu().numpy(), ref) < 1e-4, ls


def test_coarse_cycle_multi_rhs_solve_equals_single():
    """Right-hand sides that converge early are skipped inside the cooperative
    launch exactly as in the step-by-step kernels."""
    from paper_2201_12931_amd import hexmg

    print("case coarse cycle multi-rhs solve", flush=True)
    dims, levels = (48, 24, 24), 4
    g = W.Grid(*dims)
    rho = gpu(W.random_field_density(g, seed=3, lo=0.01))
    F = gpu(W.point_loads(g, 3, seed=30))
    multi = hexmg.Grid(*dims, levels, precision=hexmg.MIXED, max_nrhs=3)
    single = hexmg.Grid(*dims, levels, precision=hexmg.MIXED, max_nrhs=1)
    for grid in (multi, single):
        grid.set_density(rho)
        for l in range(levels):
            for dt in (hexmg.F32, hexmg.F64):
                grid.set_kernel_choice(l, dt, hexmg.KERNEL_STREAM, 4, 0)
        for dt in (hexmg.F32, hexmg.F64):
            grid.set_coarse_cycle(dt, 1, 64)
    U = torch.empty_like(F)
    code, info = multi.solve(F, U, rtol=1e-8)
    assert code == 0
    for r in range(3):
        u1 = torch.empty_like(F[r])
        c1, i1 = single.solve(F[r].contiguous(), u1, rtol=1e-8)
        assert i1[0]["iterations"] == info[r]["iterations"]
        assert torch.equal(u1, U[r]), r


def test_coarse_cycle_choice_validation():
    from paper_2201_12931_amd import hexmg

    _, _, grid = _grid((16, 8, 8), 3)
    with pytest.raises(hexmg.HexmgError):
        grid.set_coarse_cycle(hexmg.F32, 2)  # levels - 2 = 1 is the deepest start
    with pytest.raises(hexmg.HexmgError):
        grid.set_coarse_cycle(hexmg.F32, 1, -1)
    grid.set_coarse_cycle(hexmg.F32, 0)
    assert grid.coarse_cycle_choice(hexmg.F32) == (0, 0)
