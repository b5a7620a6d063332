"""Pins of the oracle's multigrid solver against closed forms, FFT-exact
discrete solutions, brute-force dense solves and manufactured solutions."""
import numpy as np
import pytest
import sympy as sp
from scipy.special import erf

import oracle
import synth
from oracle import judge

RNG = np.random.default_rng(99)


def centres(n, length=1.0, origin=(0.0, 0.0, 0.0)):
    h = length / n
    c = [origin[a] + (np.arange(n) + 0.5) * h for a in range(3)]
    return np.meshgrid(*c, indexing="ij")


def smooth_field(n, seed, amp=1.0):
    X, Y, Z = centres(n)
    tab = synth.random_smooth_field(seed, n, count=4, amplitude=amp)
    f = np.zeros((n, n, n))
    for kx, ky, kz, a, ph in tab:
        f += a * np.cos(2 * np.pi * (kx * X + ky * Y + kz * Z) + ph)
    return f


def test_fft_exact_linear_psi():
    # rho1 = -q (constant) makes H_h linear: (L_h - 2 pi q) u = 2 pi q - f
    n, q = 32, 0.2
    p = oracle.params(n, levels=4)
    f = smooth_field(n, 3) + RNG.standard_normal((n, n, n)) * 0.1
    rho5 = np.zeros((n, n, n))
    rho1 = np.full((n, n, n), -q)
    S = np.zeros((3, n, n, n))
    u = np.zeros((n, n, n))
    W = np.zeros((3, n, n, n))
    res = oracle.solve(p, u, W, rho5, rho1, S, f=f, tol=1e-11, max_outer=40)
    assert res.status == 0, res
    exact = judge.fft_solve_psi(2 * np.pi * q - f, -2 * np.pi * q, 1.0 / n)
    assert np.abs(u - exact).max() < 1e-12 * max(1.0, np.abs(exact).max()) * 10


def test_fft_exact_linear_W():
    # psi frozen at 1: Delta_L,h W = 8 pi S - mean(8 pi S)
    n = 16
    p = oracle.params(n, levels=3, solve_momentum=True)
    S = RNG.standard_normal((3, n, n, n))
    u = np.zeros((n, n, n))
    W = np.zeros((3, n, n, n))
    z = np.zeros((n, n, n))
    for _ in range(25):
        oracle.step(p, 2, u, W, z, z, S)
    rhs = 8 * np.pi * S
    rhs -= rhs.mean(axis=(1, 2, 3), keepdims=True)
    exact = judge.fft_solve_W(rhs, 1.0 / n)
    Wm = W - W.mean(axis=(1, 2, 3), keepdims=True)
    assert np.abs(Wm - exact).max() < 1e-12 * np.abs(exact).max() * 10


def test_uniform_density_gives_psi_one():
    n = 16
    rho5v = 0.37
    K = np.sqrt(24 * np.pi * rho5v)
    p = oracle.params(n, levels=3, K=K)
    rho5 = np.full((n, n, n), rho5v)
    z = np.zeros((n, n, n))
    S = np.zeros((3, n, n, n))
    u = np.zeros((n, n, n))
    W = np.zeros((3, n, n, n))
    H, _, _ = oracle.residuals(p, u, W, rho5, z, S)
    assert np.abs(H).max() <= 1e-15 * 2 * np.pi * rho5v * 10
    res = oracle.solve(p, u, W, rho5, z, S, tol=1e-12)
    assert res.status == 0 and res.iters == 0
    assert np.all(u == 0.0)


def test_vacuum_puncture_returns_to_zero():
    n = 16
    p = oracle.params(n, levels=3, bc=oracle.BC_ROBIN, length=16.0, origin=(-8, -8, -8),
                      puncture_mass=1.0)
    z = np.zeros((n, n, n))
    S = np.zeros((3, n, n, n))
    W = np.zeros((3, n, n, n))
    H, _, _ = oracle.residuals(p, z, W, z, z, S)
    assert np.all(H == 0.0)  # u = 0 is exact
    u = 0.05 * smooth_field(n, 5)
    res = oracle.solve(p, u, W, z, z, S, tol=1e-12, max_outer=60)
    assert res.status == 0, res
    assert np.abs(u).max() < 1e-11


def gaussian_case(n, half=8.0, s=1.0, Q=1.0):
    X, Y, Z = centres(n, 2 * half, (-half,) * 3)
    r = np.sqrt(X * X + Y * Y + Z * Z)
    sigma = Q * np.exp(-r * r / (2 * s * s)) / (2 * np.pi * s * s) ** 1.5
    exact = Q * erf(r / (np.sqrt(2) * s)) / r
    return sigma, exact


def test_gaussian_source_robin_fourth_order():
    errs = []
    for n in (16, 32, 64):
        sigma, exact = gaussian_case(n)
        levels = {16: 3, 32: 4, 64: 5}[n]
        p = oracle.params(n, levels=levels, bc=oracle.BC_ROBIN, length=16.0, origin=(-8, -8, -8))
        z = np.zeros((n, n, n))
        S = np.zeros((3, n, n, n))
        u = np.zeros((n, n, n))
        W = np.zeros((3, n, n, n))
        res = oracle.solve(p, u, W, z, z, S, f=4 * np.pi * sigma, tol=1e-11, max_outer=60)
        assert res.status == 0, res
        errs.append(np.abs(u - exact).max())
    ratios = [errs[i] / errs[i + 1] for i in range(2)]
    assert ratios[-1] > 13.0, (errs, ratios)


def test_variable_coefficient_matches_brute_force():
    for bc in (oracle.BC_PERIODIC, oracle.BC_ROBIN):
        n = 8
        L = 2.0
        org = (-1.0, -1.0, -1.0)
        p = oracle.params(n, levels=2, bc=bc, length=L, origin=org)
        g = judge.Grid(n, L, bc, org)
        q = 0.5 + RNG.uniform(0, 1, (n, n, n))  # rho1 = -q -> c = -2 pi q
        f = RNG.standard_normal((n, n, n))
        z = np.zeros((n, n, n))
        S = np.zeros((3, n, n, n))
        u = np.zeros((n, n, n))
        W = np.zeros((3, n, n, n))
        res = oracle.solve(p, u, W, z, -q, S, f=f, tol=1e-12, max_outer=80)
        assert res.status == 0, res
        m = n ** 3
        A = np.zeros((m, m))
        e = np.zeros(m)
        c = -2 * np.pi * q
        for j in range(m):
            e[:] = 0.0
            e[j] = 1.0
            E = e.reshape(n, n, n)
            A[:, j] = (judge.lap(g, E) + c * E).ravel()
        exact = np.linalg.solve(A, (2 * np.pi * q - f).ravel()).reshape(n, n, n)
        assert np.abs(u - exact).max() < 1e-11


def test_vcycle_contracts_error():
    # one V(2,2) cycle reduces the error of the variable-coefficient problem
    n = 32
    p = oracle.params(n, levels=4)
    c = -1.0 - RNG.uniform(0, 3, (n, n, n))
    r = smooth_field(n, 8) + 0.3 * RNG.standard_normal((n, n, n))
    g = judge.Grid(n)
    d = np.zeros((n, n, n))
    norms = []
    for _ in range(5):
        defect = r - (judge.lap(g, d) + c * d)
        norms.append(np.sqrt(np.mean(defect ** 2)))
        d = d + oracle.vcycle_psi(p, c, np.ascontiguousarray(defect))
    rates = [norms[i + 1] / norms[i] for i in range(4)]
    assert max(rates) < 0.25, rates


# ---- manufactured solution: coupled system, 4th-order convergence --------------------

def mms_fields():
    x, y, z = sp.symbols("x y z", real=True)
    tp = 2 * sp.pi
    psi = 1 + sp.Rational(1, 10) * sp.sin(tp * x) * sp.sin(tp * y) * sp.sin(tp * z)
    # not divergence-free, so the (1/3) d_a d_b W_b coupling and the trace part
    # of Abar are exercised
    W = [sp.Rational(1, 100) * sp.sin(tp * x) * sp.cos(tp * y),
         sp.Rational(1, 100) * sp.sin(tp * y) * sp.cos(tp * z),
         sp.Rational(1, 100) * sp.sin(tp * z) * sp.cos(tp * x)]
    X = (x, y, z)
    K2 = 150
    div = sum(sp.diff(W[a], X[a]) for a in range(3))
    A2 = 0
    for a in range(3):
        for b in range(3):
            Ab = sp.diff(W[b], X[a]) + sp.diff(W[a], X[b]) - (sp.Rational(2, 3) * div if a == b else 0)
            A2 += Ab * Ab
    lap = lambda f: sum(sp.diff(f, v, 2) for v in X)
    rho1 = (-lap(psi) + sp.Rational(K2, 12) * psi ** 5 - A2 * psi ** -7 / 8) / (2 * sp.pi * psi)
    S = [(lap(W[a]) + sp.diff(div, X[a]) / 3) / (8 * sp.pi * psi ** 6) for a in range(3)]
    fn = lambda e: sp.lambdify((x, y, z), e, "numpy")
    return dict(psi=fn(psi), W=[fn(w) for w in W], rho1=fn(rho1), S=[fn(s) for s in S], K=np.sqrt(K2))


@pytest.mark.slow
def test_mms_coupled_fourth_order():
    F = mms_fields()
    errs_psi, errs_W = [], []
    for n in (16, 32, 64):
        X, Y, Z = centres(n)
        levels = synth.coarsest_levels(n)
        p = oracle.params(n, levels=levels, K=F["K"], solve_momentum=True)
        rho1 = F["rho1"](X, Y, Z)
        S = np.ascontiguousarray(np.stack([F["S"][a](X, Y, Z) for a in range(3)]))
        rho5 = np.zeros((n, n, n))
        u = np.zeros((n, n, n))
        W = np.zeros((3, n, n, n))
        res = oracle.solve(p, u, W, rho5, rho1, S, tol=1e-11, max_outer=60)
        assert res.status == 0, res
        We = np.stack([F["W"][a](X, Y, Z) * np.ones_like(X) for a in range(3)])
        errs_psi.append(np.abs(1.0 + u - F["psi"](X, Y, Z)).max())
        Wm = W - W.mean(axis=(1, 2, 3), keepdims=True)
        errs_W.append(np.abs(Wm - (We - We.mean(axis=(1, 2, 3), keepdims=True))).max())
    rp = [errs_psi[i] / errs_psi[i + 1] for i in range(2)]
    rw = [errs_W[i] / errs_W[i + 1] for i in range(2)]
    assert rp[-1] > 14.0 and rw[-1] > 14.0, (errs_psi, errs_W, rp, rw)


def test_mms_planted_mistake_is_caught():
    # a dropped 1/3 in the momentum operator destroys convergence to the
    # manufactured W: the residual of the exact fields stays O(1) under refinement
    F = mms_fields()
    out = []
    for n in (16, 32):
        X, Y, Z = centres(n)
        p = oracle.params(n, K=F["K"])
        We = np.ascontiguousarray(np.stack([F["W"][a](X, Y, Z) * np.ones_like(X) for a in range(3)]))
        psi = F["psi"](X, Y, Z)
        S = np.stack([F["S"][a](X, Y, Z) for a in range(3)])
        _, M, _ = oracle.residuals(p, np.ascontiguousarray(psi - 1.0), We, np.zeros_like(X),
                                   np.ascontiguousarray(F["rho1"](X, Y, Z)), np.ascontiguousarray(S))
        g = judge.Grid(n)
        Wp = [g.pad(We[a]) for a in range(3)]
        wrong = np.stack([judge.d2(g, Wp[a], 0) + judge.d2(g, Wp[a], 1) + judge.d2(g, Wp[a], 2)
                          for a in range(3)]) - 8 * np.pi * psi ** 6 * S
        out.append((np.abs(M).max(), np.abs(wrong).max()))
    (m16, w16), (m32, w32) = out
    assert m16 / m32 > 12.0        # true operator: truncation error shrinks as h^4
    assert w32 > 0.5 * w16         # planted mistake: no convergence


def test_hamiltonian_32_converges_below_1e11():
    w = synth.hamiltonian_32(seed=0)
    rho5, rho1, S, K = oracle.sources_for(w)
    p = oracle.params_from_workload(w, K)
    n = w.n
    u = np.zeros((n, n, n))
    W = np.zeros((3, n, n, n))
    res = oracle.solve(p, u, W, rho5, rho1, S, tol=1e-11, max_outer=40)
    assert res.status == 0, res
    H, _, _ = judge.residuals(judge.Grid(n), u, W, rho5, rho1, S, K)
    assert judge.norms(H)[0] <= 1e-11
    # psi stays on the positive branch near 1
    assert np.all(np.abs(u) < 0.1)


def test_mms_conformal_matter_fourth_order():
    # rho_bar := (-lap psi + (K^2/12) psi^5 - A2 psi^-7/8) psi^3 / (2 pi) and
    # S_bar := Delta_L W / (8 pi) make (psi_e, W_e) a solution of the rescaled system
    x, y, z = sp.symbols("x y z", real=True)
    tp = 2 * sp.pi
    psi = 1 + sp.Rational(1, 10) * sp.sin(tp * x) * sp.sin(tp * y) * sp.sin(tp * z)
    W = [sp.Rational(1, 100) * sp.sin(tp * x) * sp.cos(tp * y),
         sp.Rational(1, 100) * sp.sin(tp * y) * sp.cos(tp * z),
         sp.Rational(1, 100) * sp.sin(tp * z) * sp.cos(tp * x)]
    X = (x, y, z)
    K2 = 150
    div = sum(sp.diff(W[a], X[a]) for a in range(3))
    A2 = sum((sp.diff(W[b], X[a]) + sp.diff(W[a], X[b]) - (sp.Rational(2, 3) * div if a == b else 0)) ** 2
             for a in range(3) for b in range(3))
    lap = lambda f: sum(sp.diff(f, v, 2) for v in X)
    rbar = (-lap(psi) + sp.Rational(K2, 12) * psi ** 5 - A2 * psi ** -7 / 8) * psi ** 3 / (2 * sp.pi)
    Sb = [(lap(W[a]) + sp.diff(div, X[a]) / 3) / (8 * sp.pi) for a in range(3)]
    fn = lambda e: sp.lambdify((x, y, z), e, "numpy")
    f_psi, f_r, f_S = fn(psi), fn(rbar), [fn(s) for s in Sb]
    errs = []
    for n in (16, 32):
        Xc, Yc, Zc = centres(n)
        p = oracle.params(n, levels=synth.coarsest_levels(n), K=np.sqrt(K2), solve_momentum=True,
                          conformal_matter=True)
        S = np.ascontiguousarray(np.stack([f_S[a](Xc, Yc, Zc) * np.ones_like(Xc) for a in range(3)]))
        # rho_bar split arbitrarily between the two arrays: only the sum enters
        r = f_r(Xc, Yc, Zc)
        u = np.zeros((n, n, n))
        Wd = np.zeros((3, n, n, n))
        res = oracle.solve(p, u, Wd, np.ascontiguousarray(0.25 * r), np.ascontiguousarray(0.75 * r), S,
                           tol=1e-11, max_outer=60)
        assert res.status == 0, res
        errs.append(np.abs(1.0 + u - f_psi(Xc, Yc, Zc)).max())
    assert errs[0] / errs[1] > 13.0, errs


def check_same_state_step():
    """With the same-state coupling an outer step of both equations equals the W step
    and the psi step each taken alone from the step's starting state; without it the
    psi step reads the W step's result.  Bitwise: the same arithmetic either way."""
    n = 16
    w = synth.coupled(n, seed=3, precision=synth.PREC_FP64)
    rho5, rho1, S, K = oracle.sources_for(w)
    u0 = 0.01 * smooth_field(n, 5)
    W0 = np.ascontiguousarray(np.stack([0.002 * smooth_field(n, 6 + a) for a in range(3)]))
    out = {}
    for same in (True, False):
        w.same_state = same
        p = oracle.params_from_workload(w, K)
        u, W = u0.copy(), W0.copy()
        oracle.step(p, 3, u, W, rho5, rho1, S)
        uw, Ww = u0.copy(), W0.copy()
        oracle.step(p, 2, uw, Ww, rho5, rho1, S)  # the W step alone
        up, Wp = u0.copy(), (W0 if same else Ww).copy()
        oracle.step(p, 1, up, Wp, rho5, rho1, S)  # the psi step alone, from the W it reads
        assert np.array_equal(W, Ww) and np.array_equal(u, up), same
        out[same] = u
    # the two couplings differ: A2 of the W the psi step reads enters H_h and c
    assert np.abs(out[True] - out[False]).max() > 1e-9


def check_same_state_solve_iterates_the_step():
    """The solve loop with the same-state coupling takes the pinned outer step: its state
    after k iterations equals k steps from the same start."""
    n = 16
    w = synth.coupled(n, seed=3, precision=synth.PREC_FP64)
    w.same_state = True
    rho5, rho1, S, K = oracle.sources_for(w)
    p = oracle.params_from_workload(w, K)
    u, W = np.zeros((n, n, n)), np.zeros((3, n, n, n))
    res = oracle.solve(p, u, W, rho5, rho1, S, tol=1e-30, max_outer=3)
    assert res.iters == 3
    us, Ws = np.zeros((n, n, n)), np.zeros((3, n, n, n))
    for _ in range(3):
        oracle.step(p, 3, us, Ws, rho5, rho1, S)
    np.testing.assert_allclose(u, us, rtol=0, atol=1e-14)
    np.testing.assert_allclose(W, Ws, rtol=0, atol=1e-14)


def test_same_state_step_takes_both_steps_from_the_starting_state():
    check_same_state_step()


def test_same_state_solve_iterates_the_pinned_step():
    check_same_state_solve_iterates_the_step()


# psi step of the same-state outer step reading the W step's result, in the step and in the
# solve loop
SAME_STATE_STEP = ("rc = step_psi(&HP, p, u, W_start ? W_start : W, &s);", "rc = step_psi(&HP, p, u, W, &s);")
SAME_STATE_SOLVE = ("if (!rc) rc = step_psi(&HP, p, u, M, &s);", "if (!rc) rc = step_psi(&HP, p, u, W, &s);")


@pytest.mark.parametrize("plant,check", [
    (SAME_STATE_STEP, check_same_state_step),
    (SAME_STATE_SOLVE, check_same_state_solve_iterates_the_step),
], ids=["step", "solve-loop"])
def test_same_state_planted_mistake_is_caught(plant, check):
    with oracle.planted([plant]):
        with pytest.raises(AssertionError):
            check()
    check()  # and the real oracle passes again


def test_same_state_solve_reaches_the_same_discrete_solution():
    """Both couplings have the discrete solution as their fixed point: each solve meets
    the tolerance by the judge's own residuals, and the two solutions agree."""
    n = 32
    w = synth.coupled(n, seed=4, precision=synth.PREC_FP64)
    rho5, rho1, S, K = oracle.sources_for(w)
    sols = {}
    for same in (False, True):
        w.same_state = same
        p = oracle.params_from_workload(w, K)
        u = np.zeros((n, n, n))
        W = np.zeros((3, n, n, n))
        res = oracle.solve(p, u, W, rho5, rho1, S, tol=1e-11, max_outer=40)
        assert res.status == 0, res
        H, M, _ = judge.residuals(judge.Grid(n, w.length), u, W, rho5, rho1, S, K)
        nr = judge.norms(H, M)
        assert nr[0] <= 1.01e-11 and nr[1] <= 1.01e-11, (same, nr)
        sols[same] = (u, W - W.mean(axis=(1, 2, 3), keepdims=True), res.iters)
    (u0, W0, i0), (u1, W1, i1) = sols[False], sols[True]
    assert np.abs(u1 - u0).max() < 1e-9 and np.abs(W1 - W0).max() < 1e-9 * np.abs(W0).max()
    assert abs(i1 - i0) <= 2
