"""Two-level static mesh refinement of the Hamiltonian constraint (test
infrastructure only, like the rest of ``oracle/``).

Key features, "Adaptive Mesh Refinement" (a block-structured hierarchy of
refined boxes, tagged where the sources are) and "Fast" (multigrid over the
hierarchy of discretisations).  This is the static form of that hierarchy: a
base grid of n_c^3 cells (spacing h) and one box of m^3 base cells, offset b0
cells from the base grid's corner on every axis, refined by 2 (n_f = 2m cells of
spacing h/2).  The paper gives no composite-grid discretisation; the reading:

* unknowns: u on the fine box, and u on the base cells the box does not cover;
  the base value of a covered cell is the average of its 8 children;
* fine equations: H_h of the box with two ghost layers taken from the base grid
  by the cubic interpolation of the FMG start (the ghosts are the children of the
  base cells in the layer around the box), so the 4th-order stencil of every
  fine cell is complete;
* base equations: H_h of the uncovered cells (their stencils reach into covered
  cells, which hold the averages);
* composite norm: volume-weighted RMS of H over fine cells and uncovered base
  cells, sqrt((sum_f H^2 h_f^3 + sum_c H^2 h^3) / L^3).

The fine box is solved as a grid of its own with homogeneous ghosts (the zero
boundary rule) plus a forcing that carries the interpolated ghosts:
f = sum over the stencil taps outside the box of w g / (12 (h/2)^2), w the tap
weight (16 or -1) and g the interpolated ghost value.  Its V-cycles then see the
true Jacobian of the box problem (the ghosts do not depend on the box's own
values); an extrapolating rule in their place makes the box operator Neumann-like
and the iteration diverges on its near-constant mode.

Iteration (Brandt's multi-level adaptive technique, a two-level FAS cycle):
  1. base cells under the box take the average of their children;
  2. nu_f Newton-multigrid steps on the box (the ghost forcing formed before each);
  3. base forcing on covered cells tau = R H_f - H_c(R u_f) (zero elsewhere), so that
     the base problem H_c(u_c) + tau = 0 has the restricted fine residual there;
  4. nu_c Newton-multigrid steps on the base grid with that forcing;
  5. the fine box adds the cubic interpolation of the base grid's change.
The box needs a margin of at least 3 base cells on every side (the cubic stencils
of the ghost layer stay inside the base grid).
"""
from __future__ import annotations

import numpy as np

import oracle

_W0 = np.array([-5.0, 35.0, 105.0, -7.0]) / 128.0   # child nearer the lower coarse neighbour
_W1 = np.array([-7.0, 105.0, 35.0, -5.0]) / 128.0


def _cubic_axis(a, axis):
    """Children along one axis of the interior of a (two extra coarse cells on each
    side along that axis): length L + 4 -> 2 L."""
    L = a.shape[axis] - 4
    take = lambda lo: np.take(a, np.arange(lo, lo + L), axis=axis)
    even = sum(_W0[e] * take(e) for e in range(4))        # nodes I-2 .. I+1
    odd = sum(_W1[e] * take(e + 1) for e in range(4))     # nodes I-1 .. I+2
    shape = list(even.shape)
    shape[axis] = 2 * L
    out = np.empty(shape)
    sl_e = [slice(None)] * 3
    sl_o = [slice(None)] * 3
    sl_e[axis] = slice(0, None, 2)
    sl_o[axis] = slice(1, None, 2)
    out[tuple(sl_e)] = even
    out[tuple(sl_o)] = odd
    return out


def cubic_children(uc, lo, count):
    """Children (at spacing h/2) of the base cells lo .. lo + count - 1 on every axis,
    by the 4-point cubic: an array of (2 count)^3."""
    a = uc[lo - 2:lo + count + 2, lo - 2:lo + count + 2, lo - 2:lo + count + 2]
    for axis in range(3):
        a = _cubic_axis(a, axis)
    return a


def _d2(ap, axis, n, h):
    w = {-2: -1.0, -1: 16.0, 0: -30.0, 1: 16.0, 2: -1.0}
    out = 0.0
    for off, c in w.items():
        s = [slice(2, 2 + n)] * 3
        s[axis] = slice(2 + off, 2 + off + n)
        out = out + c * ap[tuple(s)]
    return out / (12.0 * h * h)


def padded_fine(uc, uf, b0):
    """The box with two ghost layers: interior uf, ghosts interpolated from uc."""
    m = uf.shape[0] // 2
    P = cubic_children(uc, b0 - 1, m + 2)
    P[2:-2, 2:-2, 2:-2] = uf
    return P


def ghost_forcing(uc, uf, b0, h_f):
    """Forcing of the box solved under the zero rule that restores the interpolated
    ghosts: sum_a D_aa G with G the padded box holding the ghosts only."""
    n = uf.shape[0]
    G = padded_fine(uc, uf, b0)
    G[2:-2, 2:-2, 2:-2] = 0.0
    return sum(_d2(G, a, n, h_f) for a in range(3))


class Problem:
    """Base and box parameters (oracle params) and sources of a two-level composite grid."""

    def __init__(self, pc, pf, b0, rho5c, rho1c, rho5f, rho1f):
        m = pf.n // 2
        assert pf.bc == oracle.BC_ZERO and pc.n >= b0 + m + 3 and b0 >= 3
        assert abs(pf.length - pc.length * m / pc.n) <= 1e-12 * pc.length
        self.pc, self.pf, self.b0, self.m = pc, pf, b0, m
        self.rc5, self.rc1, self.rf5, self.rf1 = rho5c, rho1c, rho5f, rho1f
        self.cov = (slice(b0, b0 + m),) * 3
        self.h_c = pc.length / pc.n
        self.h_f = pf.length / pf.n

    def residuals(self, uc, uf, fc=None):
        """(H_f with the interpolated ghosts, H_c) after the base cells under the box
        took their children's average (uc is updated in place)."""
        uc[self.cov] = oracle.restrict(uf)
        ff = ghost_forcing(uc, uf, self.b0, self.h_f)
        Hf = oracle.residuals(self.pf, uf, None, self.rf5, self.rf1, None, ff)[0]
        Hc = oracle.residuals(self.pc, uc, None, self.rc5, self.rc1, None, fc)[0]
        return Hf, Hc, ff

    def norm(self, Hf, Hc):
        mask = np.ones(Hc.shape, dtype=bool)
        mask[self.cov] = False
        s = np.sum(Hf * Hf) * self.h_f ** 3 + np.sum(Hc[mask] ** 2) * self.h_c ** 3
        return float(np.sqrt(s / self.pc.length ** 3)), float(max(np.abs(Hf).max(), np.abs(Hc[mask]).max()))


def solve(prob: Problem, uc, uf, tol=1e-10, max_outer=60, nu_f=1, nu_c=1):
    """Two-level FAS iteration in place on (uc, uf); returns (iterations, history of
    (rms, max) composite norms, status 0 / 4 / 5 as the single-grid oracle)."""
    hist = []
    it = 0
    status = 4
    for it in range(max_outer + 1):
        Hf, Hc, _ = prob.residuals(uc, uf)
        nr = prob.norm(Hf, Hc)
        hist.append(nr)
        if not np.isfinite(nr[0]):
            status = 5
            break
        if nr[0] <= tol:
            status = 0
            break
        if it == max_outer:
            break
        for _ in range(nu_f):
            uc[prob.cov] = oracle.restrict(uf)
            ff = ghost_forcing(uc, uf, prob.b0, prob.h_f)
            oracle.step(prob.pf, 1, uf, None, prob.rf5, prob.rf1, None, ff)
        Hf, Hc, _ = prob.residuals(uc, uf)
        fc = np.zeros_like(uc)
        fc[prob.cov] = oracle.restrict(Hf) - Hc[prob.cov]
        before = uc.copy()
        for _ in range(nu_c):
            oracle.step(prob.pc, 1, uc, None, prob.rc5, prob.rc1, None, fc)
        uf += cubic_children(uc - before, prob.b0, prob.m)
    return it, hist, status
