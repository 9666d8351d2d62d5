"""The density filter entry point that allocates nothing against hexmg_filter.

Both share the filter kernels; the no-allocation variant takes the adjoint's
intermediate from the library's static device scratch.  Two calls in a row, the
second on a smaller grid, each compared with hexmg_filter on the same input
(bit for bit: same kernels, same order of summation)."""
import numpy as np
import pytest
import torch

import workloads as W
from paper_2201_12931_amd import hexmg

pytestmark = pytest.mark.gpu


def _pair(dims, rmin, adjoint, seed):
    nx, ny, nz = dims
    n = nx * ny * nz
    x = torch.from_numpy(np.random.default_rng(seed).uniform(-1.0, 1.0, n)).cuda()
    ref = hexmg.density_filter(nx, ny, nz, rmin, x, adjoint=adjoint)
    out = torch.full_like(x, float("nan"))
    hexmg.density_filter_noalloc(nx, ny, nz, rmin, x, out, adjoint=adjoint)
    torch.cuda.synchronize()
    return ref.cpu().numpy(), out.cpu().numpy()


@pytest.mark.parametrize("adjoint", [True, False])
def test_noalloc_filter_matches_filter_twice(adjoint):
    # first a large grid, then a smaller one: the second call must not see the
    # first one's scratch contents
    for k, (dims, rmin) in enumerate([((96, 48, 40), 2.6), ((17, 9, 5), 1.5)]):
        ref, out = _pair(dims, rmin, adjoint, seed=700 + k)
        assert np.array_equal(ref, out), (dims, np.abs(ref - out).max())


def test_noalloc_filter_against_oracle():
    from oracle import topopt as otop

    dims = (20, 12, 10)
    n = int(np.prod(dims))
    x = np.random.default_rng(5).uniform(0.0, 1.0, n)
    H, Hs = otop.filter_matrix(*dims, 1.5)
    out = torch.empty(n, dtype=torch.float64, device="cuda")
    hexmg.density_filter_noalloc(*dims, 1.5, torch.from_numpy(x).cuda(), out, adjoint=True)
    ref = H @ (x / Hs)
    assert np.abs(out.cpu().numpy() - ref).max() <= 1e-14 * np.abs(ref).max()


def test_noalloc_filter_rejects_oversize_adjoint():
    nx, ny, nz = 256, 128, 129  # 2^22 + 2^15 elements
    n = nx * ny * nz
    x = torch.zeros(n, dtype=torch.float64, device="cuda")
    out = torch.empty_like(x)
    with pytest.raises(hexmg.HexmgError) as e:
        hexmg.density_filter_noalloc(nx, ny, nz, 1.5, x, out, adjoint=True)
    assert e.value.code == hexmg.ERR_INVALID
