"""MI355X-native (gfx950 HIP) matrix-free multigrid-preconditioned CG for the
SIMP hex8 state equation, with compliance and adjoint sensitivity.

The compute path is the C-ABI library ``libhexmg.so`` (include/hexmg.h); the
Python module ``hexmg`` is its thin ctypes binding.
"""
from . import hexmg  # noqa: F401
