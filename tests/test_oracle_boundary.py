"""Pins of the reflective and extrapolating boundary rules (Key features,
"Boundary conditions": extrapolating, reflective and periodic boundaries).

Reflective: the mirror image across each boundary face.  A field on n^3 with
this rule is the restriction of its even extension, periodic on (2n)^3, so
* every stencil equals the periodic stencil on the mirrored (2n)^3 grid;
* the cell-centred cosines cos(pi k (i + 1/2)/n) are eigenvectors of D_aa with
  the symbol (-2 cos 2t + 32 cos t - 30)/(12 h^2), t = pi k / n;
* (L_h + c0) u = f is solved exactly by a type-II discrete cosine transform.
Extrapolating (zeroth order): every ghost layer takes the value of the cell
next to the face, so
* a field constant along the normal over the two cells next to every face is
  continued exactly (L_h then agrees with the mirror rule, and vanishes on
  constants), while a field with a slope at the face is not;
* a small system is checked against a dense solve of the judge's operator.
Each pin fails on an oracle with a planted mistake in the rule.
"""
import numpy as np
import pytest
import scipy.fft

import oracle
from oracle import judge

RNG = np.random.default_rng(96)


def params(n, bc, levels=1, length=1.0):
    return oracle.params(n, levels=levels, bc=bc, length=length)


def mirrored(u):
    """Even extension of an n^3 field to a (2n)^3 periodic field."""
    for ax in range(3):
        u = np.concatenate([u, np.flip(u, axis=ax)], axis=ax)
    return np.ascontiguousarray(u)


def symbol(t, h):
    return (-2 * np.cos(2 * t) + 32 * np.cos(t) - 30) / (12 * h * h)


# ---- pins (run on whichever oracle library is loaded) -----------------------------------

def check_reflect_mirror(n=6):
    u = RNG.standard_normal((n, n, n))
    got = oracle.apply_lap(params(n, oracle.BC_REFLECT), u)
    ext = oracle.apply_lap(params(2 * n, oracle.BC_PERIODIC, length=2.0), mirrored(u))[:n, :n, :n]
    assert np.abs(got - ext).max() <= 1e-12 * np.abs(ext).max()
    for axis in range(3):
        d = oracle.apply_d1(params(n, oracle.BC_REFLECT), u, axis)
        de = oracle.apply_d1(params(2 * n, oracle.BC_PERIODIC, length=2.0), mirrored(u), axis)[:n, :n, :n]
        assert np.abs(d - de).max() <= 1e-12 * np.abs(de).max()


def check_reflect_cosines(n=8):
    h = 1.0 / n
    i = np.arange(n)
    for k in range(n):
        for axis in range(3):
            v = np.cos(np.pi * k * (i + 0.5) / n)
            shape = [1, 1, 1]
            shape[axis] = n
            u = np.ascontiguousarray(np.broadcast_to(v.reshape(shape), (n, n, n)))
            got = oracle.apply_lap(params(n, oracle.BC_REFLECT), u)
            assert np.abs(got - symbol(np.pi * k / n, h) * u).max() <= 1e-10 / h ** 2


def check_extrap_constant_layers(n=10):
    # a field that is constant along the face normal over the two cells next to every
    # face is continued exactly, so L_h agrees with the mirrored (reflective) operator
    # there and vanishes on constants; a field with a slope at the face is not.
    x = (np.arange(n) + 0.5) / n
    prof = np.where(np.arange(n) < 2, 0.0, np.where(np.arange(n) >= n - 2, 0.0, np.sin(np.pi * x) ** 2))
    bump = prof[:, None, None] * prof[None, :, None] * prof[None, None, :]
    u = np.ascontiguousarray(1.3 + bump)
    pe, pr = params(n, oracle.BC_EXTRAP), params(n, oracle.BC_REFLECT)
    le = oracle.apply_lap(pe, u)
    assert np.abs(le - oracle.apply_lap(pr, u)).max() <= 1e-12 * np.abs(le).max()
    assert np.abs(oracle.apply_lap(pe, np.full((n, n, n), 2.5))).max() <= 1e-12
    X = np.ascontiguousarray(np.broadcast_to(x[:, None, None], (n, n, n)))
    lx = oracle.apply_lap(pe, X)
    assert np.abs(lx[2:-2]).max() <= 1e-9 and np.abs(lx[0]).min() > 1.0


def dense_operator(g, c):
    n = g.n
    m = n ** 3
    A = np.zeros((m, m))
    e = np.zeros(m)
    for col in range(m):
        e[:] = 0.0
        e[col] = 1.0
        E = e.reshape(n, n, n)
        A[:, col] = (judge.lap(g, E) + c * E).ravel()
    return A


def check_extrap_dense(n=6):
    g = judge.Grid(n, 1.0, judge.BC_EXTRAP)
    c = -5.0 - RNG.uniform(0, 10, (n, n, n))
    r = RNG.standard_normal((n, n, n))
    ref = np.linalg.solve(dense_operator(g, c), r.ravel()).reshape(n, n, n)
    got = oracle.coarse_solve_psi(params(n, oracle.BC_EXTRAP), c, r)
    assert np.abs(got - ref).max() <= 1e-10 * np.abs(ref).max()


# ---- tests ---------------------------------------------------------------------------------

def test_reflective_equals_periodic_on_the_mirrored_grid():
    check_reflect_mirror()


def test_reflective_cosines_are_eigenvectors():
    check_reflect_cosines()


@pytest.mark.parametrize("bc", [oracle.BC_REFLECT, oracle.BC_EXTRAP])
def test_oracle_operator_matches_judge(bc):
    n = 7
    u = RNG.standard_normal((n, n, n))
    got = oracle.apply_lap(params(n, bc), u)
    ref = judge.lap(judge.Grid(n, 1.0, bc), u)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


def test_reflective_multigrid_reaches_the_cosine_transform_solution():
    n, levels = 32, 4
    c0 = -7.5
    f = RNG.standard_normal((n, n, n))
    h = 1.0 / n
    t = np.pi * np.arange(n) / n
    lam = symbol(t, h)
    denom = lam[:, None, None] + lam[None, :, None] + lam[None, None, :] + c0
    exact = scipy.fft.idctn(scipy.fft.dctn(f, type=2) / denom, type=2)
    p = oracle.params(n, levels=levels, bc=oracle.BC_REFLECT, length=1.0)
    c = np.full((n, n, n), c0)
    g = judge.Grid(n, 1.0, judge.BC_REFLECT)
    d = np.zeros((n, n, n))
    for _ in range(30):
        r = np.ascontiguousarray(f - (judge.lap(g, d) + c0 * d))
        d = d + oracle.vcycle_psi(p, c, r)
    assert np.abs(d - exact).max() <= 1e-11 * np.abs(exact).max()


def test_extrapolation_continues_constant_layers():
    check_extrap_constant_layers()


def test_extrapolating_coarse_solve_matches_dense_judge_operator():
    check_extrap_dense()


@pytest.mark.parametrize("bc", [oracle.BC_REFLECT, oracle.BC_EXTRAP])
def test_nonlinear_solve_with_the_rule(bc):
    """The Hamiltonian constraint with smooth sources and constant K on a 16^3 box
    under the rule, solved to 1e-11 by the oracle, checked by the judge."""
    n = 16
    x = (np.arange(n) + 0.5) / n
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
    rho5 = np.ascontiguousarray(0.05 * (1.0 + np.cos(np.pi * X) * np.cos(2 * np.pi * Y) * np.cos(np.pi * Z)))
    rho1 = np.ascontiguousarray(0.02 * (1.0 + 0.5 * np.sin(np.pi * X * Y)))
    K = np.sqrt(24 * np.pi * np.mean(rho5 + rho1))
    p = oracle.params(n, levels=3, bc=bc, K=K)
    u = np.zeros((n, n, n))
    W = np.zeros((3, n, n, n))
    S = np.zeros((3, n, n, n))
    res = oracle.solve(p, u, W, rho5, rho1, S, tol=1e-11, max_outer=60)
    assert res.status == 0, res
    H, _, _ = judge.residuals(judge.Grid(n, 1.0, bc), u, None, rho5, rho1, None, K)
    assert judge.norms(H)[0] <= 1e-11


# ---- planted mistakes -----------------------------------------------------------------------

MIRROR_OFF_BY_ONE = ("        idx[0] = i < 0 ? -1 - i : 2 * n - 1 - i;",
                     "        idx[0] = i < 0 ? -i : 2 * n - 2 - i;")
EXTRAP_FROM_SECOND = ("        idx[0] = i < 0 ? 0 : n - 1;\n    }\n    w[0] = 1.0;",
                      "        idx[0] = i < 0 ? 1 : n - 2;\n    }\n    w[0] = 1.0;")
EXTRAP_DAMPED = ("        idx[0] = i < 0 ? 0 : n - 1;\n    }\n    w[0] = 1.0;",
                 "        idx[0] = i < 0 ? 0 : n - 1;\n        w[0] = 0.9;\n        return 1;\n    }\n    w[0] = 1.0;")
EXTRAP_AS_MIRROR = ("        idx[0] = i < 0 ? 0 : n - 1;\n    }\n    w[0] = 1.0;",
                    "        idx[0] = i < 0 ? -1 - i : 2 * n - 1 - i;\n    }\n    w[0] = 1.0;")


@pytest.mark.parametrize("plant,check", [
    (MIRROR_OFF_BY_ONE, check_reflect_mirror),
    (MIRROR_OFF_BY_ONE, check_reflect_cosines),
    (EXTRAP_DAMPED, check_extrap_constant_layers),
    (EXTRAP_FROM_SECOND, check_extrap_dense),
    (EXTRAP_AS_MIRROR, check_extrap_dense),
], ids=["mirror-mirror", "mirror-cosines", "extrap-damped", "extrap-second-cell", "extrap-as-mirror"])
def test_planted_mistake_is_caught(plant, check):
    with oracle.planted([plant]):
        with pytest.raises(AssertionError):
            check()
    check()
