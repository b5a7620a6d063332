"""Pins of the oracle's CTTK and CTTK-Hybrid methods (Summary; Key features,
"Methods": the two CTT variants with a spatially varying trace K).

The oracle folds the new terms of eqs. Ham and Mom into shifted CTT sources; the
numpy judge evaluates the equations as written instead, with K(x)^2 in eq. Ham
and -(2/3) psi^6 D_a K in eq. Mom, from the original sources.  So:

* uniform density, no momentum: both methods give the Friedmann trace
  K^2 = 24 pi rho everywhere (eq. Ham of a homogeneous slice with psi = 1), with
  W = 0 and, for the hybrid, psi = 1;
* the K of the CTTK update solves eq. Ham exactly at any (u, W): the judge's H
  with that K vanishes to rounding;
* converged solves of both methods satisfy the judge's eqs. Ham and Mom to 1e-10,
  and CTTK leaves the free data psi untouched, also for a chosen psi != 1;
* each pin fails on an oracle with a planted mistake in the method.
"""
import numpy as np
import pytest

import oracle
import synth
from oracle import judge

N = 16


def workload(n=N, seed=3):
    w = synth.coupled(n, seed=seed)
    rho5, rho1, S, _ = oracle.sources_for(w)
    return w, rho5, rho1, S


def grid(w):
    return judge.Grid(w.n, w.length, judge.BC_PERIODIC, tuple(w.origin))


def check_friedmann(a=0.37, b=0.81):
    n = 8
    rho5, rho1 = np.full((n,) * 3, a), np.full((n,) * 3, b)
    S = np.zeros((3, n, n, n))
    want = np.sqrt(24.0 * np.pi * (a + b))
    p = oracle.params(n, levels=2, solve_momentum=True)
    r5h, Sh, K, K0 = oracle.cttk_hybrid_sources(p, rho5, rho1, S)
    assert np.abs(K - want).max() <= 1e-13 * want
    assert abs(K0 - np.sqrt(24.0 * np.pi * b)) <= 1e-13 * K0
    assert not r5h.any() and np.abs(Sh).max() <= 1e-12
    ph = oracle.params(n, levels=2, solve_momentum=True, K=K0)
    u, W = np.zeros((n,) * 3), np.zeros((3, n, n, n))
    res = oracle.solve(ph, u, W, r5h, rho1, Sh, tol=1e-12, max_outer=5)
    assert res.status == 0 and res.iters == 0
    u, W = np.zeros((n,) * 3), np.zeros((3, n, n, n))
    res, Kc = oracle.cttk_solve(p, u, W, rho5, rho1, S, tol=1e-12, max_outer=5)
    assert res.status == 0 and res.iters == 0 and not W.any()
    assert np.abs(Kc - want).max() <= 1e-13 * want


def check_update_solves_ham():
    w, rho5, rho1, S = workload()
    n = w.n
    x = (np.arange(n) + 0.5) / n
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
    # |D_aa u| stays below 2 pi rho everywhere, so K^2 > 0
    u = 0.1 + 2e-4 * np.sin(2 * np.pi * X) * np.cos(2 * np.pi * Z)
    W = 0.02 * np.stack([np.cos(2 * np.pi * (Y + Z)), np.sin(2 * np.pi * X), np.cos(4 * np.pi * Y)])
    p = oracle.params_from_workload(w)
    r5e, Se, K = oracle.cttk_update(p, u, W, rho5, rho1, S)
    assert K.min() > 0.0
    H, M, _ = judge.residuals(grid(w), u, W, rho5, rho1, S, K)
    scale = np.abs(2 * np.pi * rho1 * (1 + u)).max()
    assert np.abs(H).max() <= 1e-12 * scale, np.abs(H).max()
    # the shifted sources give the same momentum residual as the judge's direct terms
    _, Mo, _ = judge.residuals(grid(w), u, W, r5e, rho1, Se, 0.0)
    assert np.abs(M - Mo).max() <= 1e-10 * np.abs(M).max()


def check_hybrid_solve(tol=1e-11):
    w, rho5, rho1, S = workload()
    n = w.n
    r5h, Sh, K, K0 = oracle.cttk_hybrid_sources(oracle.params_from_workload(w), rho5, rho1, S)
    p = oracle.params_from_workload(w, K=K0)
    u, W = np.zeros((n,) * 3), np.zeros((3, n, n, n))
    res = oracle.solve(p, u, W, r5h, rho1, Sh, tol=tol, max_outer=60)
    assert res.status == 0, res
    H, M, _ = judge.residuals(grid(w), u, W, rho5, rho1, S, K)
    hr, mr, _, _ = judge.norms(H, M)
    assert hr <= 1e-10 and mr <= 1e-10, (hr, mr)
    return u, W, K


def check_cttk_solve(u0=None, tol=1e-11):
    w, rho5, rho1, S = workload()
    n = w.n
    u = np.zeros((n,) * 3) if u0 is None else u0.copy()
    W = np.zeros((3, n, n, n))
    res, K = oracle.cttk_solve(oracle.params_from_workload(w), u, W, rho5, rho1, S, tol=tol, max_outer=80)
    assert res.status == 0, res
    assert np.array_equal(u, np.zeros((n,) * 3) if u0 is None else u0)  # psi is free data
    assert K.min() > 0.0
    H, M, _ = judge.residuals(grid(w), u, W, rho5, rho1, S, K)
    hr, mr, _, _ = judge.norms(H, M)
    assert hr <= 1e-10 and mr <= 1e-10, (hr, mr)
    return W, K


def test_uniform_density_gives_the_friedmann_trace():
    check_friedmann()


def test_cttk_trace_solves_the_hamiltonian_constraint():
    check_update_solves_ham()


def test_hybrid_solution_satisfies_the_constraints():
    u, W, K = check_hybrid_solve()
    # the hybrid K is psi-independent and only mildly varying on this workload
    assert K.max() / K.min() < 1.1 and np.abs(W).max() > 1e-3


def test_cttk_solution_satisfies_the_constraints():
    W, K = check_cttk_solve()
    assert np.abs(W).max() > 1e-2


def test_cttk_with_a_chosen_conformal_factor():
    n = N
    x = (np.arange(n) + 0.5) / n
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
    # psi = 1.1 plus a ripple whose Laplacian stays below 2 pi rho (K^2 > 0 everywhere)
    u0 = 0.1 + 2e-4 * np.cos(2 * np.pi * X) * np.sin(2 * np.pi * Y)
    check_cttk_solve(u0)


def test_cttk_reports_a_conformal_factor_without_real_trace():
    """A psi whose Laplacian outweighs the energy density leaves K^2 < 0 somewhere:
    K is NaN there and the solve stops with a non-finite norm (status 5)."""
    w, rho5, rho1, S = workload()
    n = w.n
    x = (np.arange(n) + 0.5) / n
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
    u = 0.05 * np.cos(2 * np.pi * X)
    W = np.zeros((3, n, n, n))
    res, K = oracle.cttk_solve(oracle.params_from_workload(w), u, W, rho5, rho1, S, tol=1e-11, max_outer=5)
    assert res.status == 5 and np.isnan(K).any()


def test_methods_differ_from_ctt_where_the_density_varies():
    """CTTK puts the whole energy into K: its trace varies where rho does, while
    CTT keeps K constant and moves psi instead."""
    w, rho5, rho1, S = workload()
    W, K = check_cttk_solve()
    rho = rho5 + rho1
    corr = np.corrcoef(K.ravel() ** 2, rho.ravel())[0, 1]
    assert corr > 0.9, corr


# ---- planted mistakes ------------------------------------------------------------------

HYB_DK = ("S[a * m + q] += D1(&g, K, i, j, k, a) / (12.0 * M_PI);",
          "S[a * m + q] += D1(&g, K, i, j, k, a) / (8.0 * M_PI);")
HYB_K2 = ("K[q] = sqrt(24.0 * M_PI * (rho5[q] + mean1));", "K[q] = sqrt(12.0 * M_PI * (rho5[q] + mean1));")
CTTK_K2 = ("double K2 = 12.0 * K[q] / pow(psi, 5);", "double K2 = 8.0 * K[q] / pow(psi, 5);")
CTTK_DK = ("(S ? S[a * m + q] : 0.0) + D1(&g, K, i, j, k, a) / (12.0 * M_PI);",
           "(S ? S[a * m + q] : 0.0) - D1(&g, K, i, j, k, a) / (12.0 * M_PI);")
CTTK_RHO = ("rho5_eff[q] = rho5[q] - K2 / (24.0 * M_PI);", "rho5_eff[q] = rho5[q] - K2 / (12.0 * M_PI);")


@pytest.mark.parametrize("plant,check", [
    (HYB_DK, check_hybrid_solve),
    (HYB_K2, check_hybrid_solve),
    (HYB_K2, check_friedmann),
    (CTTK_K2, check_update_solves_ham),
    (CTTK_K2, check_friedmann),
    (CTTK_DK, check_update_solves_ham),
    (CTTK_DK, check_cttk_solve),
    (CTTK_RHO, check_cttk_solve),
], ids=["hybrid-dK", "hybrid-K2", "hybrid-K2-friedmann", "cttk-K2", "cttk-K2-friedmann", "cttk-dK-sign",
        "cttk-dK-solve", "cttk-rho5"])
def test_planted_mistake_is_caught(plant, check):
    with oracle.planted([plant]):
        with pytest.raises(AssertionError):
            check()
    check()


# ---- Anderson mixing over several steps ----------------------------------------------------

def anderson_reference(w, rho5, rho1, S, depth, iters):
    """The CTTK iteration written out over the oracle's own single steps (the trace and
    shifted sources of the state, one W step at K = 0), mixed in numpy: gamma minimises
    |f - sum_j gamma_j dF_j| over the newest `depth` difference pairs (the secant quotient
    for one pair; a ridge of 1e-12 of the largest Gram diagonal entry for more), and
    W -> W + f - sum_j gamma_j (dW_j + dF_j)."""
    n = w.n
    p0 = oracle.params_from_workload(w)
    p0.K = 0.0
    u = np.zeros((n,) * 3)
    W = np.zeros((3, n, n, n))
    dWs, dFs = [], []
    Wp = fp = None
    for it in range(iters):
        r5e, Se, _ = oracle.cttk_update(p0, u, W, rho5, rho1, S)
        Wk = W.copy()
        oracle.step(p0, 2, u, W, r5e, rho1, Se)
        f = W - Wk
        if it > 0:
            dFs.append(f - fp)
            dWs.append(Wk - Wp)
            dFs, dWs = dFs[-depth:], dWs[-depth:]
        gam = np.zeros(len(dFs))
        if dFs:
            F = np.stack([d.ravel() for d in dFs])
            A, b = F @ F.T, F @ f.ravel()
            if len(dFs) == 1:
                gam[0] = b[0] / A[0, 0] if A[0, 0] > 0 else 0.0
            else:
                A = A + 1e-12 * A.diagonal().max() * np.eye(len(dFs))
                gam = np.linalg.solve(A, b)
        W = Wk + f - sum(g * (dw + df) for g, dw, df in zip(gam, dWs, dFs))
        Wp, fp = Wk, f
    return W


@pytest.mark.parametrize("depth", [1, 3, 5])
def test_mixing_over_several_steps_matches_its_definition(depth):
    w, rho5, rho1, S = workload()
    w.mix_depth = depth
    n = w.n
    u = np.zeros((n,) * 3)
    W = np.zeros((3, n, n, n))
    res, _ = oracle.cttk_solve(oracle.params_from_workload(w), u, W, rho5, rho1, S, tol=1e-30, max_outer=7)
    assert res.iters == 7
    ref = anderson_reference(w, rho5, rho1, S, depth, 7)
    assert np.abs(W - ref).max() <= 1e-9 * np.abs(ref).max()


def test_deeper_mixing_needs_fewer_iterations():
    w, rho5, rho1, S = workload(32)
    its = {}
    for depth in (1, 5):
        w.mix_depth = depth
        u = np.zeros((32,) * 3)
        W = np.zeros((3, 32, 32, 32))
        res, K = oracle.cttk_solve(oracle.params_from_workload(w), u, W, rho5, rho1, S, tol=1e-10, max_outer=200)
        assert res.status == 0, res
        H, M, _ = judge.residuals(grid(w), u, W, rho5, rho1, S, K)
        assert max(judge.norms(H, M)[:2]) <= 1.01e-10
        its[depth] = res.iters
    print(f"CTTK 32^3 iterations: one-step mixing {its[1]}, five steps {its[5]}")
    assert its[5] < its[1]


def test_mixing_planted_mistake_is_caught():
    # the newest difference pair stored with the wrong sign of dW
    with oracle.planted([("dWn[q] = Wk[q] - Wp[q];", "dWn[q] = Wp[q] - Wk[q];")]):
        with pytest.raises(AssertionError):
            test_mixing_over_several_steps_matches_its_definition(3)
    test_mixing_over_several_steps_matches_its_definition(3)
