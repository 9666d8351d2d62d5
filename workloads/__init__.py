"""Seeded synthetic inputs for structured hex8 cantilever problems.

This module is the only code shared by the CPU oracle, the GPU tests and the
benchmark.  It builds inputs only -- grids, supports, loads and density fields --
and holds none of the method's arithmetic (no stiffness, no solver, no filter).

Numbering used by every input produced here:

* element ``e = i + nx*(j + ny*k)`` for ``0 <= i < nx`` etc. (x fastest);
* node ``n = i + (nx+1)*(j + (ny+1)*k)``;
* degree of freedom ``3*n + c`` with ``c`` = 0, 1, 2 for x, y, z;
* per-node support mask: bit ``c`` set means DOF ``3*n + c`` is fixed.

The workloads follow the cantilever set-up of Sec. 5.1 (fixed face, line load at
the free end) with the sizes and density recipes listed for each named workload
below.  Nothing here reads any file.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = [
    "Grid",
    "fixed_mask_face_x0",
    "cantilever_line_load",
    "point_loads",
    "uniform_density",
    "iid_uniform_density",
    "random_field_density",
    "random_vector",
    "WORKLOADS",
    "workload",
]


@dataclasses.dataclass(frozen=True)
class Grid:
    nx: int
    ny: int
    nz: int

    @property
    def n_elem(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def n_node(self) -> int:
        return (self.nx + 1) * (self.ny + 1) * (self.nz + 1)

    @property
    def n_dof(self) -> int:
        return 3 * self.n_node

    def node(self, i, j, k):
        return i + (self.nx + 1) * (j + (self.ny + 1) * k)


def fixed_mask_face_x0(g: Grid) -> np.ndarray:
    """uint8 mask per node: all three DOFs fixed on the face x = 0."""
    m = np.zeros((g.nz + 1, g.ny + 1, g.nx + 1), dtype=np.uint8)
    m[:, :, 0] = 7
    return m.reshape(-1)


def cantilever_line_load(g: Grid, total: float = 1.0, consistent: bool = True) -> np.ndarray:
    """Load vector (length 3*n_node, float64): a -z line load of the given total
    on the free-end bottom edge (x = nx, z = 0).

    ``consistent=True`` gives the nodal forces of a uniform line load on linear
    edges (interior nodes total/ny, the two end nodes total/(2 ny));
    ``consistent=False`` spreads the total equally over the ny+1 edge nodes.
    """
    f = np.zeros(g.n_dof, dtype=np.float64)
    j = np.arange(g.ny + 1)
    nodes = g.node(g.nx, j, 0)
    if consistent:
        w = np.full(g.ny + 1, total / g.ny)
        w[0] = w[-1] = total / (2 * g.ny)
    else:
        w = np.full(g.ny + 1, total / (g.ny + 1))
    f[3 * nodes + 2] = -w
    return f


def point_loads(g: Grid, nrhs: int, seed: int) -> np.ndarray:
    """``nrhs`` load cases (shape [nrhs, 3*n_node]); each is a unit point load at a
    node drawn from the free-end face x = nx, pointing along +y, -y, +z or -z."""
    rng = np.random.Generator(np.random.PCG64(seed))
    f = np.zeros((nrhs, g.n_dof), dtype=np.float64)
    js = rng.integers(0, g.ny + 1, size=nrhs)
    ks = rng.integers(0, g.nz + 1, size=nrhs)
    dirs = rng.integers(0, 4, size=nrhs)
    for r in range(nrhs):
        n = g.node(g.nx, int(js[r]), int(ks[r]))
        comp = 1 if dirs[r] < 2 else 2
        sign = 1.0 if dirs[r] % 2 == 0 else -1.0
        f[r, 3 * n + comp] = sign
    return f


def uniform_density(g: Grid, value: float) -> np.ndarray:
    return np.full(g.n_elem, float(value), dtype=np.float64)


def iid_uniform_density(g: Grid, seed: int, lo: float, hi: float = 1.0) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(lo, hi, size=g.n_elem).astype(np.float64)


def random_field_density(g: Grid, seed: int, length_scale: float = 8.0,
                         lo: float = 0.01, hi: float = 1.0) -> np.ndarray:
    """Smooth random density field in [lo, hi] (element order, float64).

    White N(0,1) noise on the element lattice (array [nz][ny][nx], PCG64(seed)) is
    smoothed with a Gaussian of sigma = length_scale/sqrt(2) elements (which gives
    a squared-exponential covariance of length ``length_scale``; reflecting
    boundaries, kernel truncated at 4 sigma) and mapped affinely so that its
    minimum is ``lo`` and its maximum ``hi``.
    """
    from scipy.ndimage import gaussian_filter

    rng = np.random.Generator(np.random.PCG64(seed))
    w = rng.standard_normal((g.nz, g.ny, g.nx))
    s = gaussian_filter(w, sigma=length_scale / math.sqrt(2.0), mode="reflect", truncate=4.0)
    smin, smax = float(s.min()), float(s.max())
    if smax == smin:  # a single element: no spread to map
        return np.full(g.n_elem, hi, dtype=np.float64)
    s = (s - smin) / (smax - smin)
    return (lo + (hi - lo) * s).reshape(-1).astype(np.float64)


def random_vector(n: int, seed: int, nrhs: int | None = None) -> np.ndarray:
    """Standard normal test vector(s) (float64) for operator-level checks."""
    rng = np.random.Generator(np.random.PCG64(seed))
    shape = (n,) if nrhs is None else (nrhs, n)
    return rng.standard_normal(shape)


# Named workloads.  Material: E0 = 1, Emin = 1e-9, nu = 0.3, SIMP penalty 3;
# all DOFs fixed on the face x = 0.
WORKLOADS = {
    # 32x16x16, uniform density 0.3, line load, 3 levels, FP64, rtol 1e-8.
    "cantilever_32x16x16": dict(grid=Grid(32, 16, 16), levels=3, rtol=1e-8,
                                density=("uniform", 0.3)),
    # 128x64x64, random field (length 8, seed 1) in [0.01, 1], 5 levels, rtol 1e-6.
    "cantilever_128x64x64_rf": dict(grid=Grid(128, 64, 64), levels=5, rtol=1e-6,
                                    density=("field", 1, 0.01)),
    # 256x128x128, 20 optimality-criteria iterations from uniform 0.12.
    "topopt_256x128x128": dict(grid=Grid(256, 128, 128), levels=6, rtol=1e-6,
                               density=("uniform", 0.12)),
    # 256x128x128, random field (length 8, seed 2) in [0.01, 1], 6 levels (size study).
    "cantilever_256x128x128_rf": dict(grid=Grid(256, 128, 128), levels=6, rtol=1e-6,
                                      density=("field", 2, 0.01)),
    # 192x96x96, random field (seed 3) in [0.01,1], 8 point-load cases.
    "batched_192x96x96_8rhs": dict(grid=Grid(192, 96, 96), levels=5, rtol=1e-6,
                                   density=("field", 3, 0.01)),
    # 768x384x384 (113M elements), random field (seed 4) in [0.001,1], 7 levels.
    "cantilever_768x384x384_rf": dict(grid=Grid(768, 384, 384), levels=7, rtol=1e-6,
                                      density=("field", 4, 0.001)),
}


def workload(name: str):
    """Return (grid, density, load, fixed_mask, spec) for a named workload."""
    spec = WORKLOADS[name]
    g = spec["grid"]
    d = spec["density"]
    if d[0] == "uniform":
        rho = uniform_density(g, d[1])
    else:
        rho = random_field_density(g, seed=d[1], lo=d[2])
    if name.startswith("batched"):
        f = point_loads(g, 8, seed=30)
    else:
        f = cantilever_line_load(g)
    return g, rho, f, fixed_mask_face_x0(g), spec
