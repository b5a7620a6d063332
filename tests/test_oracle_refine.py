"""Pins of the oracle's two-level static mesh refinement (Key features, "Adaptive
Mesh Refinement" and "Fast"; the composite grid is stated in oracle/refine.py)
and of the zero ghost rule its refined box uses.

* zero rule: the operator equals the periodic operator of a larger grid on the
  field extended by zeros (no wrap reaches the field);
* the composite solution of a linear problem equals a brute-force dense solve of
  the composite equations, written here independently: ghosts by Lagrange
  polynomials in the cell coordinates, residuals by the numpy judge;
* refinement buys the fine grid's accuracy where it refines: around the
  puncture the composite solution is within a few 1e-5 of the solution on a
  uniform grid of the box's spacing (the base grid alone: ~1e-3), and closer on
  a finer pair of grids;
* each pin fails on an oracle with a planted mistake.
"""
import numpy as np
import pytest

import oracle
import synth
from oracle import judge, refine

RNG = np.random.default_rng(13046)


# ---- the zero ghost rule ---------------------------------------------------------------

def check_zero_rule(n=6):
    u = RNG.standard_normal((n, n, n))
    got = oracle.apply_lap(oracle.params(n, bc=oracle.BC_ZERO), u)
    big = np.zeros((n + 8,) * 3)
    big[4:-4, 4:-4, 4:-4] = u
    ref = oracle.apply_lap(oracle.params(n + 8, bc=oracle.BC_PERIODIC, length=(n + 8) / n), big)[4:-4, 4:-4, 4:-4]
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


def test_zero_rule_is_the_embedded_periodic_operator():
    check_zero_rule()


def test_zero_rule_coarse_solve_matches_the_judge_operator():
    n = 5
    g = judge.Grid(n, 1.0, judge.BC_ZERO)
    c = -2.0 - RNG.uniform(0, 3, (n, n, n))
    r = RNG.standard_normal((n, n, n))
    m = n ** 3
    A = np.zeros((m, m))
    e = np.zeros(m)
    for col in range(m):
        e[:] = 0.0
        e[col] = 1.0
        E = e.reshape(n, n, n)
        A[:, col] = (judge.lap(g, E) + c * E).ravel()
    ref = np.linalg.solve(A, r.ravel()).reshape(n, n, n)
    got = oracle.coarse_solve_psi(oracle.params(n, bc=oracle.BC_ZERO), c, r)
    assert np.abs(got - ref).max() <= 1e-10 * np.abs(ref).max()


# ---- composite grid: brute force -------------------------------------------------------

# base 12^3 on [-12, 12]^3 (Robin rule about the puncture at the centre), box of 4^3 base
# cells at offset 4 (fine 8^3 on [-4, 4]^3); puncture of mass 1 and a scalar shell,
# conformal matter, K = 0
NC, M, B0, L = 12, 4, 4, 24.0
SHELL = dict(amplitude=0.2, r0=4.0, width2=4.0)


def small_problem():
    h = L / NC
    org = (-L / 2,) * 3
    pc = oracle.params(NC, levels=2, bc=oracle.BC_ROBIN, length=L, origin=org, nu_pre=2, nu_post=2,
                       puncture_mass=1.0, conformal_matter=True)
    pf = oracle.params(2 * M, levels=2, bc=oracle.BC_ZERO, length=M * h, origin=(-L / 2 + B0 * h,) * 3,
                       nu_pre=2, nu_post=2, puncture_mass=1.0, conformal_matter=True)
    rc5, rc1, _ = oracle.shell_sources(pc, SHELL["amplitude"], SHELL["r0"], SHELL["width2"])
    rf5, rf1, _ = oracle.shell_sources(pf, SHELL["amplitude"], SHELL["r0"], SHELL["width2"])
    return refine.Problem(pc, pf, B0, rc5, rc1, rf5, rf1)


def lagrange_rows(h):
    """Rows: fine cells -2 .. 2M+1 of the box along one axis (spacing h/2); columns: base
    cells; the cubic through the four base centres around each fine centre."""
    W = np.zeros((2 * M + 4, NC))
    for F in range(-2, 2 * M + 2):
        x = (2 * B0 + F + 0.5) * h / 2
        I = (2 * B0 + F) // 2
        nodes = [I - 2, I - 1, I, I + 1] if (2 * B0 + F) % 2 == 0 else [I - 1, I, I + 1, I + 2]
        xs = [(q + 0.5) * h for q in nodes]
        for a, q in enumerate(nodes):
            W[F + 2, q] = np.prod([(x - xs[b]) / (xs[a] - xs[b]) for b in range(4) if b != a])
    return W


def composite_residual(x, prob, mask, W):
    """The composite equations written out: base cells under the box hold the average
    of their children, box ghosts the Lagrange cubic of the base values, eq. Ham (the
    judge's H_h) on the box and on the uncovered base cells."""
    h = L / NC
    nu = int(mask.sum())
    uc = np.zeros((NC,) * 3)
    uc[mask] = x[:nu]
    uf = x[nu:].reshape((2 * M,) * 3)
    uc[prob.cov] = uf.reshape(M, 2, M, 2, M, 2).mean(axis=(1, 3, 5))
    P = np.einsum("ai,bj,ck,ijk->abc", W, W, W, uc)
    P[2:-2, 2:-2, 2:-2] = uf
    gf = judge.Grid(2 * M, M * h, judge.BC_ZERO, (-L / 2 + B0 * h,) * 3)
    # eq. Ham on the box: the judge's H_h with zero ghosts, plus the ghost taps of P
    Hf, _, _ = judge.residuals(gf, uf, None, prob.rf5, prob.rf1, None, 0.0, 1.0, conformal_matter=True)
    G = P.copy()
    G[2:-2, 2:-2, 2:-2] = 0.0
    Hf = Hf + sum(judge.d2(gf, G, a) for a in range(3))
    gc = judge.Grid(NC, L, judge.BC_ROBIN, (-L / 2,) * 3)
    Hc, _, _ = judge.residuals(gc, uc, None, prob.rc5, prob.rc1, None, 0.0, 1.0, conformal_matter=True)
    return np.concatenate([Hc[mask], Hf.ravel()])


def dense_composite_solution(prob):
    mask = np.ones((NC,) * 3, dtype=bool)
    mask[prob.cov] = False
    W = lagrange_rows(L / NC)
    nu, nf = int(mask.sum()), (2 * M) ** 3
    x = np.zeros(nu + nf)
    F0 = composite_residual(x, prob, mask, W)
    J = np.zeros((nu + nf, nu + nf))
    eps = 1e-7
    for j in range(nu + nf):
        e = np.zeros(nu + nf)
        e[j] = eps
        J[:, j] = (composite_residual(x + e, prob, mask, W) - F0) / eps
    import scipy.linalg
    lu = scipy.linalg.lu_factor(J)
    for _ in range(40):  # chord iteration with the Jacobian at the start
        F = composite_residual(x, prob, mask, W)
        if np.abs(F).max() <= 1e-13:
            break
        x = x - scipy.linalg.lu_solve(lu, F)
    assert np.abs(composite_residual(x, prob, mask, W)).max() <= 1e-12
    return x[:nu], x[nu:].reshape((2 * M,) * 3), mask


_DENSE = {}


def check_brute_force():
    prob = small_problem()
    if "sol" not in _DENSE:
        _DENSE["sol"] = dense_composite_solution(prob)
    xc, xf, mask = _DENSE["sol"]
    uc, uf = np.zeros((NC,) * 3), np.zeros((2 * M,) * 3)
    it, hist, st = refine.solve(prob, uc, uf, tol=1e-12, max_outer=80)
    assert st == 0, (it, hist[-3:])
    scale = max(np.abs(xc).max(), np.abs(xf).max())
    assert np.abs(uc[mask] - xc).max() <= 1e-9 * scale
    assert np.abs(uf - xf).max() <= 1e-9 * scale


def test_composite_solution_matches_a_dense_solve():
    check_brute_force()


# ---- composite grid: accuracy where refined -------------------------------------------

def puncture_pair(nc, m, levels_c, levels_f):
    w = synth.puncture_shell(nc, levels=levels_c)
    pc = oracle.params_from_workload(w)
    b0 = (nc - m) // 2
    h = w.length / nc
    pf = oracle.params(2 * m, levels=levels_f, bc=oracle.BC_ZERO, length=m * h,
                       origin=tuple(w.origin[a] + b0 * h for a in range(3)), nu_pre=w.nu_pre,
                       nu_post=w.nu_post, puncture_mass=w.puncture_mass, puncture_pos=w.puncture_pos,
                       conformal_matter=True)
    sh = w.shell
    rc5, rc1, _ = oracle.shell_sources(pc, sh["amplitude"], sh["r0"], sh["width2"], w.scalar_mass)
    rf5, rf1, _ = oracle.shell_sources(pf, sh["amplitude"], sh["r0"], sh["width2"], w.scalar_mass)
    return w, refine.Problem(pc, pf, b0, rc5, rc1, rf5, rf1)


def refined_errors(nc, m, lc, lf, luni):
    w, prob = puncture_pair(nc, m, lc, lf)
    uc, uf = np.zeros((nc,) * 3), np.zeros((2 * m,) * 3)
    it, hist, st = refine.solve(prob, uc, uf, tol=1e-10, max_outer=40)
    assert st == 0, hist[-3:]
    wu = synth.puncture_shell(2 * nc, levels=luni)
    r5, r1, S, _ = oracle.sources_for(wu)
    u2 = np.zeros((2 * nc,) * 3)
    assert oracle.solve(oracle.params_from_workload(wu), u2, None, r5, r1, S, tol=1e-10, max_outer=60).status == 0
    b = 2 * prob.b0
    box = u2[b:b + 2 * m, b:b + 2 * m, b:b + 2 * m]
    u1 = np.zeros((nc,) * 3)
    r5c, r1c, Sc, _ = oracle.sources_for(w)
    assert oracle.solve(prob.pc, u1, None, r5c, r1c, Sc, tol=1e-10, max_outer=60).status == 0
    return np.abs(uf - box).max(), np.abs(u1[prob.cov] - oracle.restrict(box)).max()


def check_accuracy():
    e32, base32 = refined_errors(32, 16, 4, 4, 5)
    assert e32 <= 5e-5 and base32 >= 20 * e32, (e32, base32)
    return e32


def test_refinement_reaches_the_fine_grid_accuracy_where_it_refines():
    e32 = check_accuracy()
    e48, base48 = refined_errors(48, 24, 4, 3, 5)
    print(f"box vs uniform fine grid: {e32:.2e} (base 32^3), {e48:.2e} (base 48^3); base grid alone {base48:.2e}")
    assert e48 <= e32 / 2.0


# ---- planted mistakes (in the oracle's Python, on the CPU) ----------------------------

def test_planted_ghost_parity_is_caught(monkeypatch):
    monkeypatch.setattr(refine, "_W0", refine._W1.copy())
    with pytest.raises(AssertionError):
        check_brute_force()


def test_planted_tau_sign_is_caught(monkeypatch):
    real = refine.oracle.restrict

    def solve_flipped(prob, uc, uf, tol=1e-10, max_outer=60, nu_f=1, nu_c=1):
        # the base forcing with the opposite sign
        hist, status = [], 4
        for it in range(max_outer + 1):
            Hf, Hc, _ = prob.residuals(uc, uf)
            nr = prob.norm(Hf, Hc)
            hist.append(nr)
            if not np.isfinite(nr[0]):
                return it, hist, 5
            if nr[0] <= tol:
                return it, hist, 0
            if it == max_outer:
                return it, hist, 4
            for _ in range(nu_f):
                uc[prob.cov] = real(uf)
                oracle.step(prob.pf, 1, uf, None, prob.rf5, prob.rf1, None,
                            refine.ghost_forcing(uc, uf, prob.b0, prob.h_f))
            Hf, Hc, _ = prob.residuals(uc, uf)
            fc = np.zeros_like(uc)
            fc[prob.cov] = Hc[prob.cov] - real(Hf)
            before = uc.copy()
            oracle.step(prob.pc, 1, uc, None, prob.rc5, prob.rc1, None, fc)
            uf += refine.cubic_children(uc - before, prob.b0, prob.m)
        return it, hist, status

    monkeypatch.setattr(refine, "solve", solve_flipped)
    with pytest.raises(AssertionError):
        check_brute_force()


def test_planted_injection_is_caught(monkeypatch):
    # the base value under the box taken from one child instead of the average of eight
    monkeypatch.setattr(refine.oracle, "restrict", lambda fine: np.ascontiguousarray(fine[::2, ::2, ::2]))
    with pytest.raises(AssertionError):
        check_brute_force()


ZERO_AS_EXTRAP = ("    if (g->bc == OBC_ZERO) return 0.0; /* homogeneous ghosts (the interface of a refined box) */",
                  "    if (g->bc == OBC_ZERO) return a[idx3(n, clampi(i, n), clampi(j, n), clampi(k, n))];")


def test_planted_zero_rule_is_caught():
    with oracle.planted([ZERO_AS_EXTRAP]):
        with pytest.raises(AssertionError):
            check_zero_rule()
    check_zero_rule()


# ---- nested boxes ---------------------------------------------------------------------

def nested_problem(nc, boxes, levels, L=None, shell=None, length=None):
    """Base grid on [-L/2, L/2]^3 (Robin rule, puncture of mass 1 at the centre, a scalar
    shell, conformal matter) and boxes (m, b): box k over m cells of level k-1 from its
    cell b, refined by 2."""
    length = 64.0 if length is None else length
    sh = SHELL if shell is None else shell
    h = length / nc
    org = np.full(3, -length / 2)
    ps = [oracle.params(nc, levels=levels[0], bc=oracle.BC_ROBIN, length=length, origin=tuple(org), nu_pre=2,
                        nu_post=2, puncture_mass=1.0, conformal_matter=True)]
    bs = [0]
    for (m, b), lv in zip(boxes, levels[1:]):
        org = org + b * h
        h = h / 2
        ps.append(oracle.params(2 * m, levels=lv, bc=oracle.BC_ZERO, length=2 * m * h, origin=tuple(org), nu_pre=2,
                                nu_post=2, puncture_mass=1.0, conformal_matter=True))
        bs.append(b)
    src = [oracle.shell_sources(p, sh["amplitude"], sh["r0"], sh["width2"]) for p in ps]
    return refine.Nested(ps, bs, [q[0] for q in src], [q[1] for q in src])


def lagrange_rows_pair(nc_parent, b0, m, h):
    """Cubic rows of the children -2 .. 2m+1 (along one axis) of box (b0, m) from its parent."""
    W = np.zeros((2 * m + 4, nc_parent))
    for F in range(-2, 2 * m + 2):
        x = (2 * b0 + F + 0.5) * h / 2
        I = (2 * b0 + F) // 2
        nodes = [I - 2, I - 1, I, I + 1] if (2 * b0 + F) % 2 == 0 else [I - 1, I, I + 1, I + 2]
        xs = [(q + 0.5) * h for q in nodes]
        for a, q in enumerate(nodes):
            W[F + 2, q] = np.prod([(x - xs[b]) / (xs[a] - xs[b]) for b in range(4) if b != a])
    return W


def nested_residual(x, prob, masks, rows):
    """The nested composite equations written out (as composite_residual, level by level)."""
    L = prob.L
    u, off = [], 0
    for k in range(L):
        n = prob.p[k].n
        uk = np.zeros((n,) * 3)
        cnt = int(masks[k].sum())
        uk[masks[k]] = x[off:off + cnt]
        off += cnt
        u.append(uk)
    for k in range(L - 1, 0, -1):
        m, b = prob.p[k].n // 2, prob.b[k]
        u[k - 1][b:b + m, b:b + m, b:b + m] = u[k].reshape(m, 2, m, 2, m, 2).mean(axis=(1, 3, 5))
    out = []
    for k in range(L):
        p = prob.p[k]
        if k == 0:
            g0 = judge.Grid(p.n, p.length, judge.BC_ROBIN, tuple(p.origin))
            Hk, _, _ = judge.residuals(g0, u[0], None, prob.r5[0], prob.r1[0], None, 0.0, 1.0, conformal_matter=True)
        else:
            gk = judge.Grid(p.n, p.length, judge.BC_ZERO, tuple(p.origin))
            Hk, _, _ = judge.residuals(gk, u[k], None, prob.r5[k], prob.r1[k], None, 0.0, 1.0, conformal_matter=True)
            Wr = rows[k]
            G = np.einsum("ai,bj,ck,ijk->abc", Wr, Wr, Wr, u[k - 1])
            G[2:-2, 2:-2, 2:-2] = 0.0
            Hk = Hk + sum(judge.d2(gk, G, a) for a in range(3))
        out.append(Hk[masks[k]])
    return np.concatenate(out)


def check_nested_brute_force():
    # base 12^3 on [-12, 12]^3, box 1: 4^3 base cells at 4 (8^3, [-4, 4]), box 2: 2^3 cells of
    # box 1 at 3 (4^3, [-1, 1]) around the puncture
    prob = nested_problem(NC, [(4, 4), (2, 3)], [2, 2, 1], length=L)
    masks = []
    for k in range(prob.L):
        mk = np.ones((prob.p[k].n,) * 3, dtype=bool)
        if k + 1 < prob.L:
            mk[prob.covered(k)] = False
        masks.append(mk)
    rows = [None] + [lagrange_rows_pair(prob.p[k - 1].n, prob.b[k], prob.p[k].n // 2, prob.h[k - 1])
                     for k in range(1, prob.L)]
    nx = sum(int(mk.sum()) for mk in masks)
    if "nested" in _DENSE:
        x = _DENSE["nested"]
    else:
        x = dense_nested_solution(prob, masks, rows, nx)
        _DENSE["nested"] = x
    u = [np.zeros((p.n,) * 3) for p in prob.p]
    it, hist, st = refine.solve_nested(prob, u, tol=1e-12, max_outer=80)
    assert st == 0, hist[-3:]
    got = np.concatenate([u[k][masks[k]] for k in range(prob.L)])
    assert np.abs(got - x).max() <= 1e-9 * np.abs(x).max(), np.abs(got - x).max()


def dense_nested_solution(prob, masks, rows, nx):
    x = np.zeros(nx)
    F0 = nested_residual(x, prob, masks, rows)
    J = np.zeros((nx, nx))
    eps = 1e-7
    for j in range(nx):
        e = np.zeros(nx)
        e[j] = eps
        J[:, j] = (nested_residual(x + e, prob, masks, rows) - F0) / eps
    import scipy.linalg
    lu = scipy.linalg.lu_factor(J)
    for _ in range(40):
        F = nested_residual(x, prob, masks, rows)
        if np.abs(F).max() <= 1e-13:
            break
        x = x - scipy.linalg.lu_solve(lu, F)
    assert np.abs(nested_residual(x, prob, masks, rows)).max() <= 1e-12
    return x


def test_nested_composite_solution_matches_a_dense_solve():
    check_nested_brute_force()


def test_nested_boxes_agree_with_one_box_of_the_same_spacing():
    """Base 32^3 with two nested boxes (h = 2, 1, 0.5 around the puncture) against base 64^3
    with one box (h = 1, 0.5): the innermost boxes cover the same cells at the same spacing
    and differ only through the base grids far away."""
    shell = dict(amplitude=0.1, r0=10.0, width2=4.0)
    p3 = nested_problem(32, [(16, 8), (16, 8)], [4, 4, 4], shell=shell)
    u3 = [np.zeros((p.n,) * 3) for p in p3.p]
    assert refine.solve_nested(p3, u3, tol=1e-10, max_outer=40)[2] == 0
    p2 = nested_problem(64, [(16, 24)], [5, 4], shell=shell)
    u2 = [np.zeros((p.n,) * 3) for p in p2.p]
    assert refine.solve_nested(p2, u2, tol=1e-10, max_outer=40)[2] == 0
    d = np.abs(u3[2] - u2[1]).max()
    print(f"innermost boxes differ by {d:.2e} (|u| up to {np.abs(u2[1]).max():.3f})")
    assert d <= 2e-5


def test_planted_nested_tau_without_the_inner_forcing_is_caught(monkeypatch):
    # the FAS forcing of a parent built from the level's residual without its own tau
    real_H = refine.Nested.H

    def H_no_tau(self, u, k, f):
        if f is not None and k > 0 and k + 1 < self.L:
            f = self.ghosts(u, k)  # drops the tau a middle level received
        return real_H(self, u, k, f)

    monkeypatch.setattr(refine.Nested, "H", H_no_tau)
    with pytest.raises(AssertionError):
        check_nested_brute_force()
