"""Pins of the oracle's stencils, transfers, sources and residual fields.

The stencils are checked against mathematics (polynomial exactness, Fourier
symbols derived from exp(i theta j)), not against a retyped formula; the
numpy judge (a second implementation) cross-checks the C residual fields.
"""
import numpy as np
import pytest
import sympy as sp

import oracle
from oracle import judge

RNG = np.random.default_rng(1234)


def robin_params(n, length=3.0):
    # Robin grid: no wrap, so interior cells see only true neighbours
    return oracle.params(n, bc=oracle.BC_ROBIN, length=length, origin=(-1.3, -0.7, -1.1),
                         puncture_pos=(5.0, 5.0, 5.0))


def cell_coords(p):
    h = p.length / p.n
    c = [p.origin[a] + (np.arange(p.n) + 0.5) * h for a in range(3)]
    return np.meshgrid(*c, indexing="ij")


INTERIOR = (slice(2, -2),) * 3


def test_first_derivative_exact_to_degree_4():
    p = robin_params(12)
    X, Y, Z = cell_coords(p)
    f = X ** 4 - 2.0 * X ** 3 * Y + Y ** 2 * Z ** 2 + 3.0 * Z ** 3 - X * Y * Z + 0.5
    exact = [4 * X ** 3 - 6 * X ** 2 * Y - Y * Z,
             -2 * X ** 3 + 2 * Y * Z ** 2 - X * Z,
             2 * Y ** 2 * Z + 9 * Z ** 2 - X * Y]
    for a in range(3):
        got = oracle.apply_d1(p, np.ascontiguousarray(f), a)
        np.testing.assert_allclose(got[INTERIOR], exact[a][INTERIOR], rtol=0, atol=1e-10)


def test_first_derivative_not_exact_at_degree_5():
    # the 4th-order stencil leaves a 5th-derivative error term: the pin is sharp
    p = robin_params(12)
    X, _, _ = cell_coords(p)
    got = oracle.apply_d1(p, np.ascontiguousarray(X ** 5), 0)
    err = np.abs(got - 5 * X ** 4)[INTERIOR]
    assert err.max() > 1e-6


def test_laplacian_exact_to_degree_5():
    p = robin_params(12)
    X, Y, Z = cell_coords(p)
    f = X ** 5 + X ** 2 * Y ** 3 - 4 * Y ** 4 * Z + Z ** 5 - 2 * X * Y * Z ** 2 + 7.0
    exact = (20 * X ** 3 + 2 * Y ** 3) + (6 * X ** 2 * Y - 48 * Y ** 2 * Z) + (20 * Z ** 3 - 4 * X * Y)
    got = oracle.apply_lap(p, np.ascontiguousarray(f))
    np.testing.assert_allclose(got[INTERIOR], exact[INTERIOR], rtol=0, atol=1e-8)


@pytest.mark.parametrize("n", [8, 13])
def test_fourier_symbols_periodic(n):
    p = oracle.params(n, length=1.0)
    h = 1.0 / n
    X, Y, Z = cell_coords(p)
    k = (1, 3, 2)
    arg = 2 * np.pi * (k[0] * X + k[1] * Y + k[2] * Z)
    th = [2 * np.pi * kk / n for kk in k]
    lam = sum((-2 * np.cos(2 * t) + 32 * np.cos(t) - 30) / (12 * h * h) for t in th)
    got = oracle.apply_lap(p, np.ascontiguousarray(np.cos(arg)))
    np.testing.assert_allclose(got, lam * np.cos(arg), rtol=0, atol=1e-9 * abs(lam))
    # D_y of cos -> -(8 sin t - sin 2t)/(6h) * sin
    s = (8 * np.sin(th[1]) - np.sin(2 * th[1])) / (6 * h)
    got = oracle.apply_d1(p, np.ascontiguousarray(np.cos(arg)), 1)
    np.testing.assert_allclose(got, -s * np.sin(arg), rtol=0, atol=1e-10 * abs(s))


def test_deltaL_continuum_limit_and_symbol():
    # plane wave W = e cos(k.x): Delta_L W = -|k|^2 W - (1/3) k (k.e) cos, up to O(h^4)
    n = 32
    p = oracle.params(n, length=1.0)
    X, Y, Z = cell_coords(p)
    k = np.array([1.0, 2.0, 0.0]) * 2 * np.pi
    e = np.array([0.3, -0.2, 0.5])
    cosv = np.cos(k[0] * X + k[1] * Y + k[2] * Z)
    W = np.ascontiguousarray(np.stack([e[a] * cosv for a in range(3)]))
    got = oracle.apply_deltaL(p, W)
    exact = np.stack([(-(k @ k) * e[a] - (k[a] * (k @ e)) / 3.0) * cosv for a in range(3)])
    assert np.abs(got - exact).max() < 2e-3 * np.abs(exact).max()
    # and it equals the judge's independent implementation to rounding
    np.testing.assert_allclose(got, judge.deltaL(judge.Grid(n), W), rtol=0, atol=1e-9)


def test_restrict_preserves_sum():
    f = RNG.standard_normal((8, 8, 8))
    c = oracle.restrict(np.ascontiguousarray(f))
    assert abs(c.sum() * 8 - f.sum()) < 1e-12
    np.testing.assert_allclose(c[1, 2, 3], f[2:4, 4:6, 6:8].mean(), rtol=1e-14)


def test_prolong_exact_on_linear_functions():
    nc = 8
    p = robin_params(nc)
    X, Y, Z = cell_coords(p)
    lin = lambda x, y, z: 0.5 + 2 * x - 3 * y + 0.25 * z
    pf = robin_params(2 * nc)
    Xf, Yf, Zf = cell_coords(pf)
    fine = oracle.prolong_add(p, np.ascontiguousarray(lin(X, Y, Z)), np.zeros((2 * nc,) * 3))
    sl = (slice(2, -2),) * 3
    np.testing.assert_allclose(fine[sl], lin(Xf, Yf, Zf)[sl], rtol=0, atol=1e-12)
    # periodic: constants are reproduced everywhere (weights sum to one)
    pp = oracle.params(nc)
    fine = oracle.prolong_add(pp, np.full((nc,) * 3, 1.7), np.zeros((2 * nc,) * 3))
    np.testing.assert_allclose(fine, 1.7, rtol=0, atol=1e-14)


def test_cubic_interp_exact_on_cubics():
    nc = 10
    p = robin_params(nc)
    X, Y, Z = cell_coords(p)
    cub = lambda x, y, z: x ** 3 - 2 * x * y * z + y ** 2 * z + z ** 3 - 0.5 * y + 1.0
    pf = robin_params(2 * nc)
    Xf, Yf, Zf = cell_coords(pf)
    fine = oracle.interp_cubic(p, np.ascontiguousarray(cub(X, Y, Z)))
    sl = (slice(4, -4),) * 3
    np.testing.assert_allclose(fine[sl], cub(Xf, Yf, Zf)[sl], rtol=0, atol=1e-11)


def test_cubic_prolongation_of_corrections():
    check_cubic_prolongation_of_corrections()


def test_cubic_prolongation_planted_mistake_is_caught():
    # the flag ignored: corrections prolonged trilinearly, not exact on cubics
    with oracle.planted([("    if (p->flags & OFLAG_CUBIC_PROLONG) {", "    if (0) {")]):
        with pytest.raises(AssertionError):
            check_cubic_prolongation_of_corrections()
    check_cubic_prolongation_of_corrections()


def check_cubic_prolongation_of_corrections():
    """With the cubic flag the V-cycles' prolongation adds the 4-point cubic
    interpolation: exact on cubics in the interior (the trilinear one is not even
    exact on quadratics), constants reproduced on a periodic grid, and an added
    field, not a replaced one."""
    nc = 10
    pc = oracle.params(nc, bc=oracle.BC_ROBIN, length=3.0, origin=(-1.3, -0.7, -1.1),
                       puncture_pos=(5.0, 5.0, 5.0), cubic_prolong=True)
    X, Y, Z = cell_coords(pc)
    cub = lambda x, y, z: x ** 3 - 2 * x * y * z + y ** 2 * z + z ** 3 - 0.5 * y + 1.0
    pf = robin_params(2 * nc)
    Xf, Yf, Zf = cell_coords(pf)
    base = RNG.standard_normal((2 * nc,) * 3)
    fine = oracle.prolong_add(pc, np.ascontiguousarray(cub(X, Y, Z)), base.copy())
    sl = (slice(4, -4),) * 3
    np.testing.assert_allclose((fine - base)[sl], cub(Xf, Yf, Zf)[sl], rtol=0, atol=1e-11)
    quad = lambda x, y, z: x * x + y * z
    lin = oracle.prolong_add(robin_params(nc), np.ascontiguousarray(quad(X, Y, Z)), np.zeros((2 * nc,) * 3))
    assert np.abs(lin[sl] - quad(Xf, Yf, Zf)[sl]).max() > 1e-3
    pp = oracle.params(nc, cubic_prolong=True)
    fine = oracle.prolong_add(pp, np.full((nc,) * 3, 1.7), np.zeros((2 * nc,) * 3))
    np.testing.assert_allclose(fine, 1.7, rtol=0, atol=1e-13)


def _dense(op, shape):
    m = int(np.prod(shape))
    A = np.zeros((m, m))
    e = np.zeros(m)
    for j in range(m):
        e[:] = 0.0
        e[j] = 1.0
        A[:, j] = op(e.reshape(shape)).ravel()
    return A


def test_coarse_solve_psi_matches_dense_solve_robin_and_periodic():
    for bc in (oracle.BC_PERIODIC, oracle.BC_ROBIN):
        n = 4
        p = oracle.params(n, bc=bc, length=2.0, origin=(-1.0, -1.0, -1.0))
        g = judge.Grid(n, 2.0, bc, (-1.0, -1.0, -1.0))
        c = -1.0 - RNG.uniform(0, 2, (n, n, n))
        A = _dense(lambda e: judge.lap(g, e) + c * e, (n, n, n))
        r = RNG.standard_normal((n, n, n))
        x = oracle.coarse_solve_psi(p, np.ascontiguousarray(c), r)
        np.testing.assert_allclose(x.ravel(), np.linalg.solve(A, r.ravel()), rtol=1e-11, atol=1e-13)


def test_coarse_solve_W_is_the_mean_free_solution():
    n = 4
    p = oracle.params(n)
    g = judge.Grid(n)
    r = RNG.standard_normal((3, n, n, n))
    x = oracle.coarse_solve_W(p, np.ascontiguousarray(r))
    rp = r - r.mean(axis=(1, 2, 3), keepdims=True)
    np.testing.assert_allclose(judge.deltaL(g, x), rp, rtol=0, atol=1e-11)
    np.testing.assert_allclose(x.mean(axis=(1, 2, 3)), 0.0, atol=1e-13)


def test_residual_fields_match_judge_periodic():
    n = 12
    K = 3.1
    p = oracle.params(n, K=K)
    u = 0.05 * RNG.standard_normal((n, n, n))
    W = 0.02 * RNG.standard_normal((3, n, n, n))
    rho5 = RNG.uniform(0, 1, (n, n, n))
    rho1 = RNG.uniform(0, 1, (n, n, n))
    S = RNG.standard_normal((3, n, n, n))
    f = RNG.standard_normal((n, n, n))
    H, M, c = oracle.residuals(p, u, W, rho5, rho1, S, f)
    Hj, Mj, cj = judge.residuals(judge.Grid(n), u, W, rho5, rho1, S, K, f=f)
    np.testing.assert_allclose(H, Hj, rtol=1e-12, atol=1e-9)
    np.testing.assert_allclose(M, Mj, rtol=1e-12, atol=1e-9)
    np.testing.assert_allclose(c, cj, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(M.mean(axis=(1, 2, 3)), 0.0, atol=1e-9)


def test_residual_fields_match_judge_robin_puncture():
    n = 10
    p = oracle.params(n, bc=oracle.BC_ROBIN, length=8.0, origin=(-4, -4, -4), puncture_mass=1.0)
    g = judge.Grid(n, 8.0, judge.BC_ROBIN, (-4, -4, -4))
    u = 0.05 * RNG.standard_normal((n, n, n))
    W = np.zeros((3, n, n, n))
    rho5 = RNG.uniform(0, 0.1, (n, n, n))
    rho1 = RNG.uniform(0, 0.1, (n, n, n))
    S = np.zeros((3, n, n, n))
    H, _, c = oracle.residuals(p, u, W, rho5, rho1, S)
    Hj, _, cj = judge.residuals(g, u, W, rho5, rho1, S, 0.0, puncture_mass=1.0)
    np.testing.assert_allclose(H, Hj, rtol=1e-12, atol=1e-11)
    np.testing.assert_allclose(c, cj, rtol=1e-12, atol=1e-12)


def test_norms_definition():
    H = np.array([3.0, -4.0, 0.0, 0.0]).reshape(1, 1, 4)
    H = np.broadcast_to(H, (4, 4, 4)).copy()
    M = np.zeros((3, 4, 4, 4))
    M[0, 0, 0, 0], M[1, 0, 0, 0] = 3.0, 4.0
    out = oracle.norms(H, M)
    np.testing.assert_allclose(out, [np.sqrt(25 / 4), np.sqrt(25 / 64), 4.0, 5.0], rtol=1e-15)


# ---- sources -----------------------------------------------------------------------

def test_scalar_sources_mean_closed_forms():
    # distinct, non-opposite wavevectors: cross terms average to zero on the grid
    n = 16
    p = oracle.params(n)
    phi = np.array([[1, 0, 0, 0.3, 0.4], [0, 2, 1, 0.2, 1.1], [1, 1, -1, 0.1, 2.0]])
    pim = np.array([[1, 0, 0, 0.5, 1.3], [2, 0, 0, 0.25, 0.2]])
    rho5, rho1, S = oracle.scalar_sources(p, phi, pim, mass=1.5)
    k2 = np.sum(phi[:, :3] ** 2, axis=1)
    # <|grad phi|^2>/2 = sum A^2 (2 pi |k|)^2 / 4
    np.testing.assert_allclose(rho1.mean(), np.sum(phi[:, 3] ** 2 * (2 * np.pi) ** 2 * k2) / 4, rtol=1e-12)
    # <Pi^2/2 + m^2 phi^2/2> = sum B^2/4 + m^2 sum A^2/4
    np.testing.assert_allclose(rho5.mean(), np.sum(pim[:, 3] ** 2) / 4 + 1.5 ** 2 * np.sum(phi[:, 3] ** 2) / 4,
                               rtol=1e-12)
    # <S_a> = <-Pi d_a phi>: only the shared k=(1,0,0) pair contributes,
    # A B pi k_a sin(theta - chi)
    expect = 0.3 * 0.5 * np.pi * np.array([1, 0, 0]) * np.sin(0.4 - 1.3)
    np.testing.assert_allclose(S.mean(axis=(1, 2, 3)), expect, atol=1e-13)


def test_shell_sources_match_symbolic_gradient():
    n = 12
    p = oracle.params(n, bc=oracle.BC_ROBIN, length=24.0, origin=(-12, -12, -12))
    rho5, rho1, S = oracle.shell_sources(p, 0.1, 5.0, 4.0, mass=1.0)
    x, y, z = sp.symbols("x y z", real=True)
    r = sp.sqrt(x * x + y * y + z * z)
    phi = sp.Rational(1, 10) * sp.exp(-(r - 5) ** 2 / 4) * sp.sqrt(3 / (4 * sp.pi)) * x / r
    grad2 = sum(sp.diff(phi, v) ** 2 for v in (x, y, z))
    f_rho1 = sp.lambdify((x, y, z), grad2 / 2, "numpy")
    f_phi = sp.lambdify((x, y, z), phi, "numpy")
    X, Y, Z = cell_coords(p)
    np.testing.assert_allclose(rho1, f_rho1(X, Y, Z), rtol=1e-12, atol=1e-18)
    np.testing.assert_allclose(rho5, f_phi(X, Y, Z) ** 2 / 2, rtol=1e-12, atol=1e-20)
    assert np.all(S == 0.0)


@pytest.mark.parametrize("bc", [judge.BC_PERIODIC, judge.BC_ROBIN])
def test_judge_sampled_hamiltonian_matches_full(bc):
    n = 12
    g = judge.Grid(n, 6.0, bc, (-3, -3, -3))
    u = 0.05 * RNG.standard_normal((n, n, n))
    W = 0.02 * RNG.standard_normal((3, n, n, n))
    rho5 = RNG.uniform(0, 1, (n, n, n))
    rho1 = RNG.uniform(0, 1, (n, n, n))
    S = np.zeros((3, n, n, n))
    cells = RNG.integers(0, n, size=(200, 3))
    cells[:6] = [[0, 0, 0], [n - 1, n - 1, n - 1], [0, 5, n - 1], [1, 1, 1], [n - 2, 0, 3], [6, 6, 6]]
    for conf in (False, True):
        H, _, _ = judge.residuals(g, u, W, rho5, rho1, S, 1.7, 0.5 if bc else 0.0, conformal_matter=conf)
        Hs = judge.hamiltonian_at(g, u, W, rho5, rho1, 1.7, cells, 0.5 if bc else 0.0, conformal_matter=conf)
        np.testing.assert_allclose(Hs, H[cells[:, 0], cells[:, 1], cells[:, 2]], rtol=1e-12, atol=1e-12)
