"""Thin ctypes binding of the hexmg C ABI (include/hexmg.h).

Argument marshalling only: torch tensors supply device pointers and the current
HIP stream; every step of the computation runs in the HIP library.  The library
must be built (``python -m paper_2201_12931_amd._build`` or
``__graft_entry__.build()``); importing this module on a machine without it
raises immediately -- there is no fallback implementation.
"""
from __future__ import annotations

import atexit
import ctypes
import os
import re
import weakref

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
LIB_PATH = os.path.join(PKG, "libhexmg.so")
HEADER = os.path.join(ROOT, "include", "hexmg.h")

OK, NOT_CONVERGED = 0, 1
ERR_INVALID, ERR_WORKSPACE, ERR_DEVICE, ERR_NONFINITE, ERR_BREAKDOWN = -1, -2, -3, -4, -5
FP64, MIXED, MIXED32 = 0, 1, 2
F64, F32 = 0, 1
AVG_DENSITY, AVG_MODULUS = 0, 1
STENCIL_F32, STENCIL_BF16, STENCIL_F16 = 0, 1, 2
KERNEL_STREAM, KERNEL_GATHER, KERNEL_AUTO = 0, 1, 2
COARSE_REDISCRETIZE, COARSE_GALERKIN = 0, 1


class HexmgError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"hexmg error {code}: {msg}")
        self.code = code


class GridDesc(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
        ("levels", ctypes.c_int),
        ("E0", ctypes.c_double), ("Emin", ctypes.c_double), ("nu", ctypes.c_double),
        ("penal", ctypes.c_double),
        ("precision", ctypes.c_int), ("smooth_sweeps", ctypes.c_int),
        ("omega", ctypes.c_double), ("coarse_avg", ctypes.c_int), ("max_nrhs", ctypes.c_int),
        ("kernel", ctypes.c_int), ("fixed_mask", ctypes.c_void_p), ("coarse_op", ctypes.c_int),
        ("vcycle_both", ctypes.c_int), ("rr_every", ctypes.c_int), ("stencil_storage", ctypes.c_int),
        ("fuse_first", ctypes.c_int),
    ]


class SolveInfo(ctypes.Structure):
    _fields_ = [
        ("iterations", ctypes.c_int), ("status", ctypes.c_int),
        ("rel_res_recursive", ctypes.c_double), ("rel_res_true", ctypes.c_double),
        ("compliance", ctypes.c_double), ("ms_solve", ctypes.c_float),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def lib() -> ctypes.CDLL:
    """Load libhexmg.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2201_12931_amd._build.build()")
        L = ctypes.CDLL(LIB_PATH)
        vp, i, d, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t
        sig = {
            "hexmg_default_desc": (i, [i, i, i, i, ctypes.POINTER(GridDesc)]),
            "hexmg_workspace_size": (i, [ctypes.POINTER(GridDesc), ctypes.POINTER(sz)]),
            "hexmg_grid_create": (i, [ctypes.POINTER(GridDesc), vp, sz, vp, ctypes.POINTER(vp)]),
            "hexmg_grid_destroy": (i, [vp]),
            "hexmg_set_density": (i, [vp, vp, vp]),
            "hexmg_apply_K": (i, [vp, i, i, vp, vp, i, vp]),
            "hexmg_vcycle": (i, [vp, i, vp, vp, i, vp]),
            "hexmg_solve": (i, [vp, vp, vp, i, d, i, ctypes.POINTER(SolveInfo), vp]),
            "hexmg_compliance_sensitivity": (i, [vp, vp, vp, i, vp, vp, vp, vp]),
            "hexmg_batch_solve": (i, [ctypes.POINTER(vp), i, ctypes.POINTER(vp), ctypes.POINTER(vp),
                                      ctypes.POINTER(i), d, i, ctypes.POINTER(SolveInfo), vp]),
            "hexmg_batch_stats": (i, [vp, ctypes.POINTER(sz), ctypes.POINTER(sz)]),
            "hexmg_element_matrix": (i, [d, vp]),
            "hexmg_filter": (i, [i, i, i, d, i, vp, vp, vp, vp]),
            "hexmg_filter_noalloc": (i, [i, i, i, d, i, vp, vp, vp]),
            "hexmg_sensitivity_filter": (i, [i, i, i, d, d, vp, vp, vp, vp]),
            "hexmg_gravity_load": (i, [vp, d, vp, vp, vp]),
            "hexmg_gravity_sensitivity": (i, [vp, vp, d, d, vp, vp]),
            "hexmg_apply_passive": (i, [ctypes.c_longlong, vp, vp, vp]),
            "hexmg_oc_update": (i, [vp, vp, vp, vp, d, d, d, vp, ctypes.POINTER(d), ctypes.POINTER(d),
                                    ctypes.POINTER(d), vp]),
            "hexmg_volume_weights": (i, [vp, vp, vp, vp]),
            "hexmg_kernel_choice": (i, [vp, i, i, i, ctypes.POINTER(i), ctypes.POINTER(i), ctypes.POINTER(i)]),
            "hexmg_set_kernel_choice": (i, [vp, i, i, i, i, i]),
            "hexmg_coarse_cycle_choice": (i, [vp, i, ctypes.POINTER(i), ctypes.POINTER(i)]),
            "hexmg_set_coarse_cycle": (i, [vp, i, i, i]),
            "hexmg_profile_enable": (i, [vp, i]),
            "hexmg_profile_query": (i, [vp, ctypes.c_char_p, ctypes.POINTER(i), ctypes.POINTER(d)]),
            "hexmg_last_error": (ctypes.c_char_p, []),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def header_functions() -> list[str]:
    """Names of the functions declared in include/hexmg.h."""
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(hexmg_\w+)\s*\(", txt, re.M)))


def last_error() -> str:
    return lib().hexmg_last_error().decode()


def _check(code: int, ok=(OK,)) -> int:
    if code not in ok:
        raise HexmgError(code, last_error())
    return code


# ---- host-only entry points ------------------------------------------------
def default_desc(nx, ny, nz, levels, **kw) -> GridDesc:
    d = GridDesc()
    _check(lib().hexmg_default_desc(nx, ny, nz, levels, ctypes.byref(d)))
    for k, v in kw.items():
        if k == "fixed_mask":
            v = None if v is None else v.data_ptr()
        setattr(d, k, v)
    return d


def workspace_size(desc: GridDesc) -> int:
    n = ctypes.c_size_t()
    _check(lib().hexmg_workspace_size(ctypes.byref(desc), ctypes.byref(n)))
    return n.value


def element_matrix(nu: float = 0.3):
    import numpy as np

    Ke = np.zeros((24, 24), dtype=np.float64)
    _check(lib().hexmg_element_matrix(nu, Ke.ctypes.data_as(ctypes.c_void_p)))
    return Ke


# ---- device entry points (torch tensors) -----------------------------------
def _stream(stream=None):
    import torch

    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dev(t, dtype=None, numel=None, name="tensor"):
    import torch

    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must have dtype {dtype}, got {t.dtype}")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} must have {numel} elements, got {t.numel()}")
    return ctypes.c_void_p(t.data_ptr())


def density_filter(nx, ny, nz, rmin, x, out=None, adjoint=False, tmp=None, stream=None):
    """S13: rho~ = H x / Hs (adjoint: H (x / Hs)) on the GPU; returns out."""
    import torch

    n = nx * ny * nz
    if out is None:
        out = torch.empty_like(x)
    if adjoint and tmp is None:
        tmp = torch.empty_like(x)
    _check(lib().hexmg_filter(nx, ny, nz, float(rmin), 1 if adjoint else 0, _dev(x, torch.float64, n, "x"),
                              _dev(out, torch.float64, n, "out"),
                              _dev(tmp, torch.float64, n, "tmp") if adjoint else None, _stream(stream)))
    return out


def density_filter_noalloc(nx, ny, nz, rmin, x, out, adjoint=False, stream=None):
    """S13 through the entry point that allocates nothing (the adjoint's
    intermediate lives in the library's static device scratch); out must be
    given."""
    import torch

    n = nx * ny * nz
    _check(lib().hexmg_filter_noalloc(nx, ny, nz, float(rmin), 1 if adjoint else 0, _dev(x, torch.float64, n, "x"),
                                      _dev(out, torch.float64, n, "out"), _stream(stream)))
    return out


def sensitivity_filter(nx, ny, nz, rmin, x, dc, out=None, gamma=1e-3, stream=None):
    """Eq. 3: dc~ = H (x dc) / (max(gamma, x) Hs) on the GPU; returns out."""
    import torch

    n = nx * ny * nz
    if out is None:
        out = torch.empty_like(dc)
    _check(lib().hexmg_sensitivity_filter(nx, ny, nz, float(rmin), float(gamma), _dev(x, torch.float64, n, "x"),
                                          _dev(dc, torch.float64, n, "dc"), _dev(out, torch.float64, n, "out"),
                                          _stream(stream)))
    return out


def apply_passive(passive, x, stream=None):
    """x_e = 1 where passive_e == 1 (solid), 0 where passive_e == 2 (void); in place."""
    import torch

    if passive.dtype != torch.uint8 or passive.numel() != x.numel() or not passive.is_contiguous():
        raise ValueError("passive must be a contiguous uint8 tensor with one entry per element")
    _check(lib().hexmg_apply_passive(x.numel(), ctypes.c_void_p(passive.data_ptr()),
                                     _dev(x, torch.float64, name="x"), _stream(stream)))
    return x


def batch_solve(grids, fs, us, rtol=1e-6, maxit=500, stream=None, check=True):
    """S15: solve grids[i] with right-hand sides fs[i] ([nrhs_i, N_i] or [N_i]) into us[i]
    together.  Returns (status, list of per-grid info lists)."""
    import torch

    n = len(grids)
    nr = [f.numel() // g.n_dof for g, f in zip(grids, fs)]
    for g, f, u in zip(grids, fs, us):
        if f.numel() % g.n_dof or u.shape != f.shape:
            raise ValueError("f, u must be [nrhs, N] for their grid")
    H = (ctypes.c_void_p * n)(*[g.handle.value for g in grids])
    F = (ctypes.c_void_p * n)(*[_dev(f, torch.float64, name="f").value for f in fs])
    U = (ctypes.c_void_p * n)(*[_dev(u, torch.float64, name="u").value for u in us])
    R = (ctypes.c_int * n)(*nr)
    infos = (SolveInfo * sum(nr))()
    code = lib().hexmg_batch_solve(H, n, F, U, R, float(rtol), int(maxit), infos, _stream(stream))
    if check:
        _check(code, ok=(OK, NOT_CONVERGED))
    out, k = [], 0
    for m in nr:
        out.append([infos[k + j].as_dict() for j in range(m)])
        k += m
    return code, out


_live_grids: "weakref.WeakSet[Grid]" = weakref.WeakSet()


@atexit.register
def _close_live_grids():
    """Destroy the grids still open at interpreter exit while the HIP runtime is
    still up (their streams and pinned buffers), before module teardown."""
    for g in list(_live_grids):
        try:
            g.close()
        except Exception:
            pass


class Grid:
    """Owns the workspace tensor and the opaque grid handle of one hexmg grid."""

    def __init__(self, nx, ny, nz, levels, device="cuda", stream=None, **kw):
        import torch

        self.desc = default_desc(nx, ny, nz, levels, **kw)
        self.nx, self.ny, self.nz, self.levels = nx, ny, nz, levels
        self.n_elem = nx * ny * nz
        self.n_dof = 3 * (nx + 1) * (ny + 1) * (nz + 1)
        self.workspace = torch.empty(workspace_size(self.desc), dtype=torch.uint8, device=device)
        h = ctypes.c_void_p()
        _check(lib().hexmg_grid_create(ctypes.byref(self.desc), ctypes.c_void_p(self.workspace.data_ptr()),
                                       self.workspace.numel(), _stream(stream), ctypes.byref(h)))
        self.handle = h
        self.density_version = 0
        self.last_info = None
        _live_grids.add(self)

    def close(self):
        """Destroy the grid (waits for the library's own streams), then drop the workspace."""
        if getattr(self, "handle", None) is not None and self.handle.value:
            lib().hexmg_grid_destroy(self.handle)
            self.handle = None
        self.workspace = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def level_dofs(self, level):
        q = 1 << level
        return 3 * (self.nx // q + 1) * (self.ny // q + 1) * (self.nz // q + 1)

    def set_density(self, rho, stream=None):
        import torch

        _check(lib().hexmg_set_density(self.handle, _dev(rho, torch.float64, self.n_elem, "rho"), _stream(stream)))
        self.density_version += 1

    def apply_K(self, u, y, level=0, stream=None):
        import torch

        dt = F64 if u.dtype == torch.float64 else F32
        n = self.level_dofs(level)
        if u.numel() % n or y.shape != u.shape or y.dtype != u.dtype:
            raise ValueError("u, y must be [nrhs, N_level] of one dtype")
        _check(lib().hexmg_apply_K(self.handle, level, dt, _dev(u, name="u"), _dev(y, name="y"),
                                   u.numel() // n, _stream(stream)))
        return y

    def vcycle(self, r, z, stream=None):
        import torch

        dt = F64 if r.dtype == torch.float64 else F32
        if r.numel() % self.n_dof or z.shape != r.shape or z.dtype != r.dtype:
            raise ValueError("r, z must be [nrhs, N] of one dtype")
        _check(lib().hexmg_vcycle(self.handle, dt, _dev(r, name="r"), _dev(z, name="z"),
                                  r.numel() // self.n_dof, _stream(stream)))
        return z

    def solve(self, f, u, rtol=1e-6, maxit=500, stream=None, check=True):
        import torch

        if f.numel() % self.n_dof or u.shape != f.shape:
            raise ValueError("f, u must be [nrhs, N]")
        nrhs = f.numel() // self.n_dof
        infos = (SolveInfo * nrhs)()
        code = lib().hexmg_solve(self.handle, _dev(f, torch.float64, name="f"), _dev(u, torch.float64, name="u"),
                                 nrhs, float(rtol), int(maxit), infos, _stream(stream))
        if check:
            _check(code, ok=(OK, NOT_CONVERGED))
        return code, [x.as_dict() for x in infos]

    def compliance_sensitivity(self, f, u, dc=None, weights=None, stream=None, compliance=True):
        """Compliances f . u (returned; None with compliance=False, which skips
        the dot products and their host read) and, with dc, the sensitivity."""
        import numpy as np
        import torch

        nrhs = f.numel() // self.n_dof
        c = np.zeros(nrhs, dtype=np.float64) if compliance else None
        w = None if weights is None else np.ascontiguousarray(weights, dtype=np.float64)
        _check(lib().hexmg_compliance_sensitivity(
            self.handle, _dev(f, torch.float64, name="f"), _dev(u, torch.float64, name="u"), nrhs,
            None if w is None else w.ctypes.data_as(ctypes.c_void_p),
            None if c is None else c.ctypes.data_as(ctypes.c_void_p),
            None if dc is None else _dev(dc, torch.float64, self.n_elem, "dc"), _stream(stream)))
        return c

    def oc_update(self, x, dc, dv, volfrac, move=0.2, eta=0.5, x_new=None, stream=None, stats=False):
        """S14: returns (x_new, lambda), with stats also the largest change and
        the volume dv . x_new: (x_new, lambda, change, volume)."""
        import torch

        if x_new is None:
            x_new = torch.empty_like(x)
        lam, ch, vol = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        n = self.n_elem
        _check(lib().hexmg_oc_update(self.handle, _dev(x, torch.float64, n, "x"), _dev(dc, torch.float64, n, "dc"),
                                     _dev(dv, torch.float64, n, "dv"), float(volfrac), float(move), float(eta),
                                     _dev(x_new, torch.float64, n, "x_new"), ctypes.byref(lam),
                                     ctypes.byref(ch) if stats else None, ctypes.byref(vol) if stats else None,
                                     _stream(stream)))
        if stats:
            return x_new, lam.value, ch.value, vol.value
        return x_new, lam.value

    def volume_weights(self, passive, dv=None, stream=None):
        """dv_e = [passive_e == 0] / (number of design elements)."""
        import torch

        if dv is None:
            dv = torch.empty(self.n_elem, dtype=torch.float64, device=passive.device)
        _check(lib().hexmg_volume_weights(self.handle, _dev(passive, torch.uint8, self.n_elem, "passive"),
                                          _dev(dv, torch.float64, self.n_elem, "dv"), _stream(stream)))
        return dv

    def kernel_choice(self, level, dtype=F32, mode=1):
        """(kind, z-chunk, shape) of the element-product kernel of a level and
        precision in mode 0 (K u), 1 (sweep, default) or 2 (residual)."""
        k, z, sh = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _check(lib().hexmg_kernel_choice(self.handle, level, dtype, mode, ctypes.byref(k), ctypes.byref(z),
                                         ctypes.byref(sh)))
        return ("stream" if k.value == KERNEL_STREAM else "gather"), z.value, sh.value

    def set_kernel_choice(self, level, dtype, kernel, zchunk=4, shape=0):
        _check(lib().hexmg_set_kernel_choice(self.handle, level, dtype, kernel, zchunk, shape))

    def batch_stats(self):
        """(launches issued, launches recorded) of the last batch solve this grid was in."""
        a, b = ctypes.c_size_t(), ctypes.c_size_t()
        _check(lib().hexmg_batch_stats(self.handle, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def gravity_load(self, gz, f_ext=None, f=None, stream=None):
        """f = f_ext + self-weight of the last set density (-gz rho_e / 8 per node along z)."""
        import torch

        if f is None:
            f = torch.empty(self.n_dof, dtype=torch.float64, device=self.workspace.device)
        _check(lib().hexmg_gravity_load(self.handle, float(gz),
                                        None if f_ext is None else _dev(f_ext, torch.float64, self.n_dof, "f_ext"),
                                        _dev(f, torch.float64, self.n_dof, "f"), _stream(stream)))
        return f

    def gravity_sensitivity(self, u, gz, dc, weight=1.0, stream=None):
        """dc += weight * 2 u^T df/drho (the load part of the compliance derivative)."""
        import torch

        _check(lib().hexmg_gravity_sensitivity(self.handle, _dev(u, torch.float64, self.n_dof, "u"), float(gz),
                                               float(weight), _dev(dc, torch.float64, self.n_elem, "dc"),
                                               _stream(stream)))
        return dc

    def coarse_cycle_choice(self, dtype=F32):
        """(first level of the cooperative coarse-cycle launch or 0, workgroups)."""
        lv, b = ctypes.c_int(), ctypes.c_int()
        _check(lib().hexmg_coarse_cycle_choice(self.handle, dtype, ctypes.byref(lv), ctypes.byref(b)))
        return lv.value, b.value

    def set_coarse_cycle(self, dtype, level, blocks=0):
        _check(lib().hexmg_set_coarse_cycle(self.handle, dtype, level, blocks))

    def profile_enable(self, on=True):
        _check(lib().hexmg_profile_enable(self.handle, 1 if on else 0))

    def profile_query(self, family):
        n, ms = ctypes.c_int(), ctypes.c_double()
        _check(lib().hexmg_profile_query(self.handle, family.encode(), ctypes.byref(n), ctypes.byref(ms)))
        return n.value, ms.value
