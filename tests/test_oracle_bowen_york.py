"""Pins of the Bowen-York puncture data (Key features, "Flexibility": binary
black holes with boosted and/or spinning punctures), which solve the momentum
constraint (Summary, eq. Mom with K = 0 and no matter) analytically and leave
the Hamiltonian constraint for u = psi - psi0, psi0 = 1 + sum m / (2 r).

* closed forms of Abar_ij Abar_ij for one puncture: boost
  (9 P^2 / (2 r^4)) (1 + 2 cos^2 theta), spin 18 S^2 sin^2 theta / r^6;
* tracelessness, and zero divergence d_j Abar_ij (the momentum constraint) at
  points off the punctures, by sixth-order finite differences;
* the ADM momentum (1/8pi) surface integral of Abar_ij n_j over a sphere around a
  binary is P1 + P2, and the ADM angular momentum (1/8pi) eps_ijk surface
  integral of x_j Abar_kl n_l is S1 + S2 + C1 x P1 + C2 x P2;
* without momenta and spins psi = psi0 (Brill-Lindquist) is the exact solution;
* each pin fails on an oracle with a planted mistake in the formula.
"""
import numpy as np
import pytest

import oracle
from oracle import judge

RNG = np.random.default_rng(2501)
BINARY = np.array([
    [0.5, 3.0, 0.0, 0.0, 0.0, 0.1, 0.02, 0.0, 0.05, 0.2],
    [0.4, -3.0, 0.0, 0.0, 0.0, -0.1, 0.01, 0.1, 0.0, -0.15],
])


def full(t6):
    xx, xy, xz, yy, yz, zz = t6
    return np.array([[xx, xy, xz], [xy, yy, yz], [xz, yz, zz]])


def sphere_rule(nt=48, nph=96):
    mu, wmu = np.polynomial.legendre.leggauss(nt)
    ph = 2 * np.pi * np.arange(nph) / nph
    MU, PH = np.meshgrid(mu, ph, indexing="ij")
    st = np.sqrt(1 - MU ** 2)
    nvec = np.stack([st * np.cos(PH), st * np.sin(PH), MU], axis=-1).reshape(-1, 3)
    w = (wmu[:, None] * np.full(nph, 2 * np.pi / nph)[None, :]).reshape(-1)
    return nvec, w


def check_closed_forms():
    P, S = np.array([0.3, -0.2, 0.5]), np.array([-0.1, 0.4, 0.25])
    boost = np.array([[1.0, 0, 0, 0, *P, 0, 0, 0]])
    spin = np.array([[1.0, 0, 0, 0, 0, 0, 0, *S]])
    for _ in range(40):
        x = RNG.uniform(-4, 4, 3)
        r = np.linalg.norm(x)
        nv = x / r
        a = full(oracle.bowen_york_tensor(boost, x))
        cos_t = nv @ P / np.linalg.norm(P)
        assert abs(np.sum(a * a) - 9 * (P @ P) / (2 * r ** 4) * (1 + 2 * cos_t ** 2)) <= 1e-12 * np.sum(a * a)
        b = full(oracle.bowen_york_tensor(spin, x))
        sin2 = 1 - (nv @ S) ** 2 / (S @ S)
        assert abs(np.sum(b * b) - 18 * (S @ S) * sin2 / r ** 6) <= 1e-12 * np.sum(b * b) + 1e-300


def check_traceless_divergence_free():
    d = 2e-3
    c6 = np.array([-1, 9, -45, 0, 45, -9, 1]) / 60.0  # sixth-order first derivative
    for _ in range(20):
        x = RNG.uniform(-6, 6, 3)
        if min(np.linalg.norm(x - BINARY[q, 1:4]) for q in range(2)) < 1.0:
            continue
        a = full(oracle.bowen_york_tensor(BINARY, x))
        assert abs(np.trace(a)) <= 1e-14 * np.abs(a).max()
        div = np.zeros(3)
        for j in range(3):
            for s, cw in zip(range(-3, 4), c6):
                if cw == 0.0:
                    continue
                y = x.copy()
                y[j] += s * d
                div += cw * full(oracle.bowen_york_tensor(BINARY, y))[:, j] / d
        assert np.abs(div).max() <= 1e-8 * np.abs(a).max(), div


def check_adm_momenta(R=10.0):
    nvec, w = sphere_rule()
    P = np.zeros(3)
    J = np.zeros(3)
    for nv, wt in zip(nvec, w):
        x = R * nv
        a = full(oracle.bowen_york_tensor(BINARY, x))
        flux = a @ nv
        P += wt * R * R * flux
        J += wt * R * R * np.cross(x, flux)
    P /= 8 * np.pi
    J /= 8 * np.pi
    Pw = BINARY[:, 4:7].sum(axis=0)
    Jw = BINARY[:, 7:10].sum(axis=0) + sum(np.cross(BINARY[q, 1:4], BINARY[q, 4:7]) for q in range(2))
    assert np.abs(P - Pw).max() <= 1e-10, (P, Pw)
    assert np.abs(J - Jw).max() <= 1e-10, (J, Jw)


def test_closed_forms_of_one_puncture():
    check_closed_forms()


def test_traceless_and_divergence_free():
    check_traceless_divergence_free()


def test_adm_momentum_and_angular_momentum():
    check_adm_momenta()


def test_grid_fields():
    n = 16
    p = oracle.params(n, bc=oracle.BC_ROBIN, length=16.0, origin=(-8.0, -8.0, -8.0))
    psi0, A2 = oracle.bowen_york(p, BINARY)
    x = -8.0 + (np.arange(n) + 0.5)
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
    ref = 1.0 + sum(BINARY[q, 0] / (2 * np.sqrt((X - BINARY[q, 1]) ** 2 + (Y - BINARY[q, 2]) ** 2 +
                                               (Z - BINARY[q, 3]) ** 2)) for q in range(2))
    assert np.abs(psi0 - ref).max() <= 1e-14
    for (i, j, k) in RNG.integers(0, n, size=(30, 3)):
        a = full(oracle.bowen_york_tensor(BINARY, np.array([x[i], x[j], x[k]])))
        assert abs(A2[i, j, k] - np.sum(a * a)) <= 1e-14 * np.sum(a * a)


def binary_problem(n=32, L=32.0, table=BINARY):
    p0 = oracle.params(n, bc=oracle.BC_ROBIN, length=L, origin=(-L / 2,) * 3)
    psi0, A2 = oracle.bowen_york(p0, table)
    p = oracle.params(n, levels=4, bc=oracle.BC_ROBIN, length=L, origin=(-L / 2,) * 3,
                      bg_psi0=psi0, bg_A2=A2)
    return p, psi0, A2


def test_brill_lindquist_limit_is_exact():
    table = BINARY.copy()
    table[:, 4:] = 0.0
    p, psi0, A2 = binary_problem(table=table)
    assert not A2.any()
    n = p.n
    z = np.zeros((n, n, n))
    u = np.zeros((n, n, n))
    res = oracle.solve(p, u, np.zeros((3, n, n, n)), z, z, np.zeros((3, n, n, n)), tol=1e-12, max_outer=5)
    assert res.status == 0 and res.iters == 0 and not u.any()


def test_binary_solve_converges_and_the_judge_agrees():
    p, psi0, A2 = binary_problem()
    n = p.n
    z = np.zeros((n, n, n))
    u = np.zeros((n, n, n))
    res = oracle.solve(p, u, np.zeros((3, n, n, n)), z, z, np.zeros((3, n, n, n)), tol=1e-11, max_outer=60)
    assert res.status == 0, res
    g = judge.Grid(n, p.length, judge.BC_ROBIN, tuple(p.origin))
    H, _, _ = judge.residuals(g, u, None, z, z, None, 0.0, psi0_field=psi0, A2_bg=A2)
    assert judge.norms(H)[0] <= 1e-11
    # the momenta raise the energy: u > 0 everywhere
    assert u.min() > 0.0


SPIN_SIGN = ("double spin = sxn[a] * nv[b] + sxn[b] * nv[a];", "double spin = -(sxn[a] * nv[b] + sxn[b] * nv[a]);")
NO_TRACE_TERM = ("((a == b ? 1.0 : 0.0) - nv[a] * nv[b]) * pn;", "(0.0 - nv[a] * nv[b]) * pn;")
BOOST_FACTOR = ("A[a][b] += 1.5 / (r * r) * boost", "A[a][b] += 3.0 / (r * r) * boost")


@pytest.mark.parametrize("plant,check", [
    (SPIN_SIGN, check_adm_momenta),
    (NO_TRACE_TERM, check_traceless_divergence_free),
    (BOOST_FACTOR, check_adm_momenta),
    (BOOST_FACTOR, check_closed_forms),
], ids=["spin-sign", "trace-term", "boost-factor-adm", "boost-factor-closed"])
def test_planted_mistake_is_caught(plant, check):
    with oracle.planted([plant]):
        with pytest.raises(AssertionError):
            check()
    check()
