"""Pins of the oracle's density filter (Eqs. 4-5), sensitivity filter (Eq. 3)
and OC update (Eqs. 8-9)."""
import math

import numpy as np
import pytest

from oracle import topopt as T


def test_filter_brute_force():
    """H from an O(Ne^2) loop over all element pairs and their centre distances."""
    nx, ny, nz, r = 4, 3, 2, 1.5
    H, Hs = T.filter_matrix(nx, ny, nz, r)
    n = nx * ny * nz
    Hb = np.zeros((n, n))
    for e in range(n):
        ce = (e % nx, (e // nx) % ny, e // (nx * ny))
        for i in range(n):
            ci = (i % nx, (i // nx) % ny, i // (nx * ny))
            d = math.dist(ce, ci)
            if d <= r:
                Hb[e, i] = r - d
    assert np.abs(H.toarray() - Hb).max() < 1e-15
    assert np.allclose(Hs, Hb.sum(axis=1))


def test_filter_weight_sums_closed_form():
    """r = 1.5: self 1.5, 6 face neighbours 0.5, 12 edge neighbours 1.5 - sqrt 2,
    corners (sqrt 3 > 1.5) excluded."""
    H, Hs = T.filter_matrix(5, 5, 5, 1.5)
    interior = 2 + 5 * (2 + 5 * 2)
    assert Hs[interior] == pytest.approx(1.5 + 6 * 0.5 + 12 * (1.5 - math.sqrt(2)), rel=1e-15)
    assert Hs[0] == pytest.approx(1.5 + 3 * 0.5 + 3 * (1.5 - math.sqrt(2)), rel=1e-15)
    assert H[interior].nnz == 19  # self + 6 faces + 12 edges
    assert np.abs(H - H.T).max() == 0


def test_filter_constant_and_adjoint():
    nx, ny, nz = 6, 4, 5
    H, Hs = T.filter_matrix(nx, ny, nz, 1.5)
    n = nx * ny * nz
    assert np.allclose(T.density_filter(H, Hs, np.full(n, 0.12)), 0.12, rtol=1e-15)
    rng = np.random.default_rng(1)
    x, y = rng.standard_normal(n), rng.standard_normal(n)
    lhs = float(y @ T.density_filter(H, Hs, x))
    rhs = float(x @ T.density_filter_adjoint(H, Hs, y))
    assert lhs == pytest.approx(rhs, rel=1e-13)


def test_oc_uniform_closed_form():
    """Uniform design and sensitivities: every element moves to the same value, so
    the volume constraint gives x_new = volfrac when within the move limit."""
    n = 50
    x = np.full(n, 0.3)
    dc, dv = np.full(n, -2.0), np.full(n, 1.0 / n)
    xn, lam, steps = T.oc_update(x, dc, dv, lambda z: z.mean(), volfrac=0.25)
    assert np.allclose(xn, 0.25, rtol=1e-10)
    # x B^eta = volfrac  ->  lambda = -dc / dv (x/volfrac)^2
    assert lam == pytest.approx(2.0 * n * (0.3 / 0.25) ** 2, rel=1e-10)
    xn, _, _ = T.oc_update(x, dc, dv, lambda z: z.mean(), volfrac=0.01)
    assert np.allclose(xn, 0.1)  # move limit 0.2


def test_oc_volume_and_bounds():
    nx, ny, nz = 6, 4, 4
    H, Hs = T.filter_matrix(nx, ny, nz, 1.5)
    n = nx * ny * nz
    rng = np.random.default_rng(5)
    x = rng.uniform(0.05, 0.6, n)
    dc = -rng.uniform(0.1, 3.0, n)
    dcx = T.density_filter_adjoint(H, Hs, dc)
    dvx = T.density_filter_adjoint(H, Hs, np.full(n, 1.0 / n))
    vol = lambda z: T.density_filter(H, Hs, z).mean()  # noqa: E731
    xn, lam, steps = T.oc_update(x, dcx, dvx, vol, volfrac=0.3)
    assert abs(vol(xn) - 0.3) < 1e-9
    assert np.all(xn >= np.maximum(0, x - 0.2) - 1e-15)
    assert np.all(xn <= np.minimum(1, x + 0.2) + 1e-15)
    # the filtered volume is linear in x: mean(rho~(z)) = dv_x . z
    assert vol(xn) == pytest.approx(float(dvx @ xn), rel=1e-13)


def test_sensitivity_filter_brute_force():
    """Eq. 3 by explicit loops over element centres, independent of the CSR matrix."""
    nx, ny, nz, r, gamma = 3, 4, 2, 1.5, 1e-3
    H, Hs = T.filter_matrix(nx, ny, nz, r)
    n = nx * ny * nz
    rng = np.random.default_rng(11)
    x = rng.uniform(0.0, 1.0, n)
    x[3] = 0.0  # below gamma: the denominator uses gamma
    dc = -rng.uniform(0.1, 2.0, n)
    out = T.sensitivity_filter(H, Hs, x, dc, gamma)
    for e in range(n):
        ce = (e % nx, (e // nx) % ny, e // (nx * ny))
        num = den = 0.0
        for i in range(n):
            d = math.dist(ce, (i % nx, (i // nx) % ny, i // (nx * ny)))
            if d <= r:
                num += (r - d) * x[i] * dc[i]
                den += r - d
        assert out[e] == pytest.approx(num / (max(gamma, x[e]) * den), rel=1e-13)


def test_sensitivity_filter_special_cases():
    nx, ny, nz = 5, 4, 3
    n = nx * ny * nz
    H, Hs = T.filter_matrix(nx, ny, nz, 1.5)
    # uniform design and sensitivity: the weighted mean of a constant
    assert np.allclose(T.sensitivity_filter(H, Hs, np.full(n, 0.4), np.full(n, -3.0)), -3.0, rtol=1e-14)
    # radius below one element: only the self weight, so dc~ = x dc / max(gamma, x)
    H1, Hs1 = T.filter_matrix(nx, ny, nz, 0.9)
    rng = np.random.default_rng(12)
    x, dc = rng.uniform(0.01, 1.0, n), rng.standard_normal(n)
    assert np.allclose(T.sensitivity_filter(H1, Hs1, x, dc), dc, rtol=1e-14)
    # linear in dc
    d2 = rng.standard_normal(n)
    a = T.sensitivity_filter(H, Hs, x, dc + 2.0 * d2)
    b = T.sensitivity_filter(H, Hs, x, dc) + 2.0 * T.sensitivity_filter(H, Hs, x, d2)
    assert np.allclose(a, b, rtol=1e-12, atol=1e-14)


def test_stored_oc_history_matches_oracle():
    """The stored optimisation history (tests/golden/oc_sensitivity_32x16x16.json,
    written by tests/golden/make_oc_history.py) is the oracle's: its first three
    iterations recomputed, and its stop rule holds exactly at its last entry."""
    import json
    import os

    import workloads as W
    from oracle import fem, multigrid as mg

    ref = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "oc_sensitivity_32x16x16.json")))
    hist = ref["history"]
    assert hist[-1]["change"] < ref["tol"] <= min(h["change"] for h in hist[:-1])
    dims = tuple(ref["dims"])
    g = W.Grid(*dims)
    f = W.cantilever_line_load(g)
    mask = W.fixed_mask_face_x0(g)
    H, Hs = T.filter_matrix(*dims, ref["rmin"])
    n = g.n_elem
    dv = np.full(n, 1.0 / n)
    x = np.full(n, ref["volfrac"])
    for h in hist[:3]:
        u, _, _, _ = mg.mgpcg(mg.Hierarchy(*dims, x, mask, ref["levels"]), f, rtol=1e-12, maxit=5000)
        c = fem.compliance(f, u)
        dc = T.sensitivity_filter(H, Hs, x, fem.sensitivity(*dims, x, u))
        x_new, _, _ = T.oc_update(x, dc, dv, lambda z: z.mean(), ref["volfrac"])
        assert c == pytest.approx(h["compliance"], rel=1e-10)
        assert abs(float(np.abs(x_new - x).max()) - h["change"]) < 1e-12
        x = x_new
