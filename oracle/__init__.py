"""FP64 CPU oracle for the hex8 SIMP state solve -- TEST INFRASTRUCTURE ONLY.

Plain, slow, obviously-correct NumPy/SciPy code written from the paper's
equations and algorithms.  It exists to check the HIP library; only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may import
it.  It shares no code with the HIP path (the seeded input generators in
``workloads`` are the one common module and hold none of the method's arithmetic).

Modules:

* ``element``   -- unit hex8 element stiffness (Gauss quadrature of B^T D B);
* ``fem``       -- assembly, SIMP modulus (Eq. 2), supports, direct solve,
                   compliance (Eq. 6), adjoint sensitivity (Eq. 7);
* ``multigrid`` -- assembled level hierarchy with homogenized coarse densities
                   (Sec. 4.2.2), damped Jacobi (Eq. 21), the V-cycle (Alg. 3) and
                   preconditioned CG (Alg. 1);
* ``topopt``    -- density filter with the weights of Eqs. 4-5 and the
                   optimality-criteria update with bisection (Eqs. 8-9).

Every function is pinned by ``tests/test_oracle_*.py`` against closed forms,
invariants, brute force or textbook routines; see each function's docstring.
"""
from . import element, fem, multigrid, topopt  # noqa: F401
