"""Pins of the oracle's relaxation and V-cycles (Key features, "Fast": the
multigrid smoother and the cycle over the hierarchy of discretisations).

A colour pass of double-buffered red-black Gauss-Seidel on A d = r sets every
active cell to d + (r - A d)/a_qq, where a_qq is the diagonal entry of A.  The
diagonal is therefore pinned by the operator itself, taken from the numpy
judge (an independent evaluation of the same stencils and boundary rule):

* impulse: for d = e_q (unit value at one cell of the active colour) and
  r = 0 the pass returns 1 - a_qq/diag at q, which vanishes only if the pass's
  diagonal equals a_qq; for r = a_qq e_q it returns exactly 1;
* fixed point: the exact solution of A x = r is left unchanged;
* colour: colour 0 changes exactly the cells with (i + j + k) even.

Each pin is shown to fail on an oracle built with a planted mistake (a dropped
term of the diagonal, a dropped ghost weight, a flipped colour, a flipped
correction sign, a black-first sweep).
"""
import numpy as np
import pytest

import oracle
from oracle import judge

RNG = np.random.default_rng(20250123)

PERIODIC = dict(bc=oracle.BC_PERIODIC, length=2.0, origin=(-1.0, -1.0, -1.0))
ROBIN = dict(bc=oracle.BC_ROBIN, length=2.0, origin=(-1.0, -1.0, -1.0))


def grid(n, cfg):
    return judge.Grid(n, cfg["length"], cfg["bc"], cfg["origin"])


def impulse_cells(n):
    # corner, edge, face and interior cells of both colours
    cells = {(0, 0, 0), (0, 0, 1), (n - 1, 0, n // 2), (1, n - 1, n - 2), (n // 2, n // 2, n // 2),
             (n // 2, n // 2 - 1, n // 2), (n - 1, n - 1, n - 1)}
    return sorted(cells)


def unit(n, q, comps=None, comp=0):
    e = np.zeros((n, n, n) if comps is None else (comps, n, n, n))
    if comps is None:
        e[q] = 1.0
    else:
        e[(comp,) + q] = 1.0
    return e


def colour_of(q):
    return (q[0] + q[1] + q[2]) % 2


# ---- the pins themselves (run on whichever oracle library is loaded) --------------------

def check_psi_impulse(n, cfg):
    p = oracle.params(n, **cfg)
    g = grid(n, cfg)
    c = -3.0 - RNG.uniform(0, 4, (n, n, n))
    for q in impulse_cells(n):
        e = unit(n, q)
        a_qq = (judge.lap(g, e) + c * e)[q]          # diagonal entry, from the judge
        out0 = oracle.pass_psi(p, e, np.zeros_like(e), c, colour_of(q))
        out1 = oracle.pass_psi(p, e, a_qq * e, c, colour_of(q))
        assert abs(out0[q]) <= 1e-13, (q, out0[q])
        assert abs(out1[q] - 1.0) <= 1e-13, (q, out1[q])


def check_W_impulse(n):
    cfg = PERIODIC
    p = oracle.params(n, **cfg)
    g = grid(n, cfg)
    for q in impulse_cells(n):
        for a in range(3):
            e = unit(n, q, 3, a)
            Ae = judge.deltaL(g, e)
            a_qq = Ae[(a,) + q]
            out0 = oracle.pass_W(p, e, np.zeros_like(e), colour_of(q))
            out1 = oracle.pass_W(p, e, np.ascontiguousarray(a_qq * e), colour_of(q))
            assert abs(out0[(a,) + q]) <= 1e-13, (q, a, out0[(a,) + q])
            assert abs(out1[(a,) + q] - 1.0) <= 1e-13, (q, a, out1[(a,) + q])
            for b in range(3):  # the other components at q have no self-coupling to W_a
                if b != a:
                    assert Ae[(b,) + q] == 0.0 and out0[(b,) + q] == 0.0


def check_fixed_point(n, cfg):
    p = oracle.params(n, **cfg)
    g = grid(n, cfg)
    x = RNG.standard_normal((n, n, n))
    c = -2.0 - RNG.uniform(0, 3, (n, n, n))
    r = np.ascontiguousarray(judge.lap(g, x) + c * x)
    for colour in (0, 1):
        out = oracle.pass_psi(p, x, r, c, colour)
        assert np.abs(out - x).max() <= 1e-11 * np.abs(x).max()
    if cfg["bc"] == oracle.BC_PERIODIC:
        X = RNG.standard_normal((3, n, n, n))
        R = np.ascontiguousarray(judge.deltaL(g, X))
        for colour in (0, 1):
            out = oracle.pass_W(p, X, R, colour)
            assert np.abs(out - X).max() <= 1e-11 * np.abs(X).max()


def check_colour(n):
    p = oracle.params(n, **PERIODIC)
    i, j, k = np.meshgrid(*(np.arange(n),) * 3, indexing="ij")
    even = (i + j + k) % 2 == 0
    d = RNG.standard_normal((n, n, n))
    r = RNG.standard_normal((n, n, n))
    c = -1.0 - RNG.uniform(0, 1, (n, n, n))
    for colour, active in ((0, even), (1, ~even)):
        out = oracle.pass_psi(p, d, r, c, colour)
        assert np.array_equal(out != d, active)
        W = RNG.standard_normal((3, n, n, n))
        R = RNG.standard_normal((3, n, n, n))
        outW = oracle.pass_W(p, W, R, colour)
        for a in range(3):
            assert np.array_equal(outW[a] != W[a], active)


def two_level_psi(p, c, r):
    """The V-cycle on two levels spelled out: nu_pre sweeps of colour 0 then
    colour 1 from zero, defect, 8-child restriction of defect and coefficient,
    exact coarse solve, trilinear prolongation, nu_post sweeps."""
    d = np.zeros_like(r)
    for _ in range(p.nu_pre):
        for colour in (0, 1):
            d = oracle.pass_psi(p, d, r, c, colour)
    g = judge.Grid(p.n, p.length, p.bc, tuple(p.origin))
    defect = r - (judge.lap(g, d) + c * d)
    pc = oracle.params(p.n // 2, bc=p.bc, length=p.length, origin=tuple(p.origin))
    dc = oracle.coarse_solve_psi(pc, oracle.restrict(c), oracle.restrict(defect))
    if p.flags & oracle.FLAG_CUBIC_PROLONG:  # the cubic of the FMG start, added
        d = d + oracle.interp_cubic(pc, dc)
    else:
        d = oracle.prolong_add(p, dc, d)
    for _ in range(p.nu_post):
        for colour in (0, 1):
            d = oracle.pass_psi(p, d, r, c, colour)
    return d


def check_cycle_order(n, cubic=False):
    p = oracle.params(n, levels=2, nu_pre=1, nu_post=2, cubic_prolong=cubic, **PERIODIC)
    c = -2.0 - RNG.uniform(0, 3, (n, n, n))
    r = RNG.standard_normal((n, n, n))
    got = oracle.vcycle_psi(p, c, r)
    want = two_level_psi(p, c, r)
    assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()


def W_contraction(n=32, levels=4, cycles=6):
    p = oracle.params(n, levels=levels, **PERIODIC)
    g = grid(n, PERIODIC)
    r = RNG.standard_normal((3, n, n, n))
    r -= r.mean(axis=(1, 2, 3), keepdims=True)
    d = np.zeros_like(r)
    norms = []
    for _ in range(cycles):
        defect = r - judge.deltaL(g, d)
        defect -= defect.mean(axis=(1, 2, 3), keepdims=True)
        norms.append(np.sqrt(np.mean(defect ** 2)))
        d = d + oracle.vcycle_W(p, np.ascontiguousarray(defect))
    return [norms[i + 1] / norms[i] for i in range(cycles - 1)]


# ---- tests on the oracle ------------------------------------------------------------------

@pytest.mark.parametrize("n", [4, 8])
def test_psi_pass_diagonal_periodic(n):
    check_psi_impulse(n, PERIODIC)


@pytest.mark.parametrize("n", [4, 8])
def test_psi_pass_diagonal_robin(n):
    check_psi_impulse(n, ROBIN)


@pytest.mark.parametrize("n", [4, 8])
def test_W_pass_diagonal(n):
    check_W_impulse(n)


@pytest.mark.parametrize("cfg", [PERIODIC, ROBIN], ids=["periodic", "robin"])
def test_passes_fix_the_exact_solution(cfg):
    check_fixed_point(8, cfg)


def test_colour_zero_is_even_parity():
    check_colour(6)


def test_vcycle_runs_red_then_black_around_an_exact_coarse_solve():
    check_cycle_order(8)


def test_vcycle_with_cubic_prolongation_of_the_correction():
    check_cycle_order(8, cubic=True)


def test_W_vcycle_contracts():
    # V(2,2) on Delta_L,h, 32^3 on 4 levels: measured 0.04 for the first cycle, rising to
    # 0.176 after 12 cycles (the asymptotic rate); the same bound as the psi cycle's
    rates = W_contraction()
    assert max(rates) < 0.25, rates


# ---- the same pins fail on an oracle with a planted mistake --------------------------------

DIAG_W = ("    /* the mixed taps D_ab W_b act on other components: no diagonal part */\n    return s + t / 3.0;",
          "    /* the mixed taps D_ab W_b act on other components: no diagonal part */\n    return s;")
GHOST = ("            s += W2[d + 2] * self_weight(g, i, j, k, o[0], o[1], o[2]);\n        }\n    return s / (12.0 * g->h * g->h);\n}\n\n/* Diagonal entry of component a",
         "            s += d == 0 ? W2[d + 2] : 0.0;\n        }\n    return s / (12.0 * g->h * g->h);\n}\n\n/* Diagonal entry of component a")
C_DIAG = ("double diag = lap_diag(&g, i, j, k) + c[q];", "double diag = lap_diag(&g, i, j, k);")
COLOUR = ("                if (((i + j + k) & 1) != colour) {\n                    out[q] = in[q];",
          "                if (((i + j + k) & 1) == colour) {\n                    out[q] = in[q];")
SIGN_W = ("out[a * m + q] = in[a * m + q] + (r[a * m + q] - Ad) / diag;",
          "out[a * m + q] = in[a * m + q] + (Ad - r[a * m + q]) / diag;")
BLACK_FIRST = ("    memset(H->d[l], 0, m * sizeof(double));\n    for (int s = 0; s < p->nu_pre; s++)\n        for (int col = 0; col < 2; col++) {\n            orc_pass_psi(p, n, H->d[l], H->t[l], H->r[l], H->c[l], col);",
               "    memset(H->d[l], 0, m * sizeof(double));\n    for (int s = 0; s < p->nu_pre; s++)\n        for (int col = 0; col < 2; col++) {\n            orc_pass_psi(p, n, H->d[l], H->t[l], H->r[l], H->c[l], 1 - col);")


@pytest.mark.parametrize("plant,check", [
    (DIAG_W, lambda: check_W_impulse(8)),                 # (1/3) D_aa dropped from the W diagonal
    (GHOST, lambda: check_psi_impulse(8, ROBIN)),         # Robin ghost weight dropped
    (C_DIAG, lambda: check_psi_impulse(8, PERIODIC)),     # Newton coefficient dropped from the diagonal
    (COLOUR, lambda: check_colour(6)),                    # colours swapped
    (SIGN_W, lambda: check_W_impulse(8)),                 # correction with the wrong sign
    (BLACK_FIRST, lambda: check_cycle_order(8)),          # pre-smoothing black before red
], ids=["W-diagonal", "ghost-weight", "c-in-diagonal", "colour", "W-sign", "black-first"])
def test_planted_mistake_is_caught(plant, check):
    with oracle.planted([plant]):
        with pytest.raises(AssertionError):
            check()
    check()  # and the real oracle passes again


def test_planted_W_sign_breaks_contraction():
    with oracle.planted([SIGN_W]):
        rates = W_contraction(16, 3, 4)
    assert max(rates) > 0.25, rates
