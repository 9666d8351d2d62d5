"""Host-side checks of the C ABI: the library loads, exports every declared
symbol, validates descriptors and computes its element matrix -- no GPU needed."""
import ctypes

import numpy as np
import pytest

from oracle.element import hex8_stiffness
from paper_2201_12931_amd import hexmg


def test_library_exports_every_declared_function():
    L = hexmg.lib()
    names = hexmg.header_functions()
    assert len(names) >= 12
    for n in names:
        assert hasattr(L, n), n


@pytest.mark.parametrize("nu", [0.3, 0.0, 0.45, -0.2])
def test_element_matrix_matches_oracle(nu):
    """The library derives K0 from the modal energy of trilinear fields; the oracle
    integrates B^T D B by Gauss quadrature.  They must agree to round-off."""
    Ke = hexmg.element_matrix(nu)
    ref = hex8_stiffness(nu)
    assert np.abs(Ke - ref).max() < 1e-15 * np.abs(ref).max() * 10


def test_descriptor_validation():
    d = hexmg.default_desc(32, 16, 16, 3)
    assert d.E0 == 1.0 and d.Emin == 1e-9 and d.nu == 0.3 and d.penal == 3.0
    assert d.fuse_first == 1 and d.rr_every == 8 and d.smooth_sweeps == 2
    assert hexmg.workspace_size(d) > 0
    bad = [
        dict(nx=33),          # not divisible by 2^(levels-1)
        dict(levels=0),
        dict(Emin=0.0),
        dict(nu=0.5),
        dict(omega=1.5),
        dict(smooth_sweeps=0),
        dict(precision=7),
        dict(coarse_avg=3),
        dict(fuse_first=2),
    ]
    for kw in bad:
        d = hexmg.default_desc(32, 16, 16, 3)
        for k, v in kw.items():
            setattr(d, k, v)
        with pytest.raises(hexmg.HexmgError) as e:
            hexmg.workspace_size(d)
        assert e.value.code == hexmg.ERR_INVALID
        assert hexmg.last_error()
    # coarsest level too large for the dense direct solve
    with pytest.raises(hexmg.HexmgError):
        hexmg.workspace_size(hexmg.default_desc(64, 32, 32, 1))
    # node planes beyond the launch grid's y/z limits
    for shape in ((2, 65536, 2), (2, 2, 65536)):
        with pytest.raises(hexmg.HexmgError) as e:
            hexmg.workspace_size(hexmg.default_desc(*shape, 1))
        assert "65535" in hexmg.last_error()


def test_workspace_scales_with_grid():
    # same coarsest grid (8x4x4), 8x the fine-level DOFs
    s0 = hexmg.workspace_size(hexmg.default_desc(64, 32, 32, 4))
    s1 = hexmg.workspace_size(hexmg.default_desc(128, 64, 64, 5))
    assert 5 < s1 / s0 < 9


def test_null_arguments_rejected():
    L = hexmg.lib()
    assert L.hexmg_workspace_size(None, None) == hexmg.ERR_INVALID
    assert L.hexmg_set_density(None, None, None) == hexmg.ERR_INVALID
    assert L.hexmg_element_matrix(ctypes.c_double(0.3), None) == hexmg.ERR_INVALID
