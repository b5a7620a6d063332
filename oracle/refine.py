"""Static mesh refinement of the Hamiltonian constraint by nested boxes (test
infrastructure only, like the rest of ``oracle/``).

Key features, "Adaptive Mesh Refinement" (a block-structured hierarchy of
refined boxes, tagged where the sources are) and "Fast" (multigrid over the
hierarchy of discretisations).  This is the static form of that hierarchy:
level 0 is a base grid; level k >= 1 is a box of m_k^3 cells of level k-1,
offset b_k cells from that level's corner on every axis, refined by 2 (n_k = 2 m_k
cells of half the spacing).  Every box lies inside its parent with a margin of at
least 3 parent cells.  The paper gives no composite-grid discretisation; the
reading:

* unknowns: u on every level's cells that no finer box covers; a covered cell's
  value is the average of its 8 children;
* box equations: H_h of the box with two ghost layers taken from its parent by
  the cubic interpolation of the FMG start (the ghosts are the children of the
  parent cells in the layer around the box), so every 4th-order stencil is
  complete;
* equations of the uncovered cells of every level: H_h of that level (stencils
  reaching into covered cells see the averages);
* composite norm: volume-weighted RMS of H over the uncovered cells of all
  levels, sqrt(sum_k sum_uncovered H^2 h_k^3 / L^3).

A box is solved as a grid of its own with homogeneous ghosts (the zero boundary
rule) plus a forcing that carries the interpolated ghosts:
f = sum over the stencil taps outside the box of w g / (12 h_k^2), w the tap
weight (16 or -1) and g the interpolated ghost value.  Its V-cycles then see the
true Jacobian of the box problem (the ghosts do not depend on the box's own
values); an extrapolating rule in their place makes the box operator Neumann-like
and the iteration diverges on its near-constant mode.

Iteration (Brandt's multi-level adaptive technique, FAS over the levels): every
covered cell takes the average of its children; then from the finest level down
to level 1: nu_f Newton-multigrid steps of the level (its ghost forcing formed
before each, plus the fixed FAS forcing tau from the level above it), then the
FAS forcing of its parent on the covered cells, tau = R H_k - H_{k-1}(R u_k), where
H_{k-1} carries the parent's own ghost forcing; nu_c steps of the base grid with
its tau; then from level 1 up, every box adds the cubic interpolation of its
parent's change.  With two levels this is the two-level FAS cycle.
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
    """Children (at half the spacing) of the parent cells lo .. lo + count - 1 on every
    axis, by the 4-point cubic: an array of (2 count)^3."""
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
    """The box with two ghost layers: interior uf, ghosts interpolated from its parent uc."""
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


class Nested:
    """Levels 0 .. L-1: oracle params (level 0 any rule, boxes the zero rule), the
    offsets b[k] of box k in level k-1 (b[0] unused), and the sources of every level."""

    def __init__(self, params, offsets, rho5, rho1):
        self.p, self.b, self.r5, self.r1 = list(params), list(offsets), list(rho5), list(rho1)
        self.L = len(self.p)
        self.h = [p.length / p.n for p in self.p]
        for k in range(1, self.L):
            pc, pf, b0 = self.p[k - 1], self.p[k], self.b[k]
            m = pf.n // 2
            assert pf.bc == oracle.BC_ZERO and pf.n % 2 == 0 and b0 >= 3 and pc.n >= b0 + m + 3
            assert abs(pf.length - pc.length * m / pc.n) <= 1e-12 * self.p[0].length
        self.vol = self.p[0].length ** 3

    def covered(self, k):
        """Cells of level k covered by box k + 1."""
        b0, m = self.b[k + 1], self.p[k + 1].n // 2
        return (slice(b0, b0 + m),) * 3

    def sync(self, u):
        for k in range(self.L - 1, 0, -1):
            u[k - 1][self.covered(k - 1)] = oracle.restrict(u[k])

    def ghosts(self, u, k):
        return ghost_forcing(u[k - 1], u[k], self.b[k], self.h[k]) if k > 0 else np.zeros_like(u[0])

    def H(self, u, k, f):
        return oracle.residuals(self.p[k], u[k], None, self.r5[k], self.r1[k], None, f)[0]

    def residuals(self, u):
        """H of every level (ghost forcing included, no FAS forcing) at the
        synchronised state (u is updated in place)."""
        self.sync(u)
        return [self.H(u, k, self.ghosts(u, k) if k else None) for k in range(self.L)]

    def norm(self, Hs):
        s, mx = 0.0, 0.0
        for k, Hk in enumerate(Hs):
            mask = np.ones(Hk.shape, dtype=bool)
            if k + 1 < self.L:
                mask[self.covered(k)] = False
            s += np.sum(Hk[mask] ** 2) * self.h[k] ** 3
            mx = max(mx, float(np.abs(Hk[mask]).max()))
        return float(np.sqrt(s / self.vol)), mx


def solve_nested(prob: Nested, u, tol=1e-10, max_outer=60, nu_f=1, nu_c=1):
    """FAS iteration over the nested levels, in place on the list u (one array per
    level); returns (iterations, history of (rms, max) composite norms, status 0 / 4 / 5
    as the single-grid oracle)."""
    L = prob.L
    hist = []
    it = 0
    status = 4

    def to_parent(k):  # the parent's cells under box k take their children's average
        u[k - 1][prob.covered(k - 1)] = oracle.restrict(u[k])

    def forcing(k, tau):
        f = prob.ghosts(u, k)
        return f + tau[k] if tau[k] is not None else f

    for it in range(max_outer + 1):
        nr = Nested.norm(prob, Nested.residuals(prob, u))  # the per-level forms (Problem names its own)
        hist.append(nr)
        if not np.isfinite(nr[0]):
            status = 5
            break
        if nr[0] <= tol:
            status = 0
            break
        if it == max_outer:
            break
        tau = [None] * L
        before = [None] * L
        for k in range(L - 1, 0, -1):
            for _ in range(nu_f):
                to_parent(k)
                oracle.step(prob.p[k], 1, u[k], None, prob.r5[k], prob.r1[k], None, forcing(k, tau))
            to_parent(k)
            # FAS forcing of the parent on the cells under box k: the restricted residual
            # of the box's own (FAS) equation minus the parent's operator at the average
            Hk = prob.H(u, k, forcing(k, tau))
            Hp = prob.H(u, k - 1, prob.ghosts(u, k - 1) if k > 1 else None)
            t = np.zeros_like(u[k - 1])
            cov = prob.covered(k - 1)
            t[cov] = oracle.restrict(Hk) - Hp[cov]
            tau[k - 1] = t
            before[k - 1] = u[k - 1].copy()
            if k > 1:  # the intermediate level's own steps follow with this tau
                continue
        for _ in range(nu_c):
            oracle.step(prob.p[0], 1, u[0], None, prob.r5[0], prob.r1[0], None, tau[0])
        for k in range(1, L):
            u[k] += cubic_children(u[k - 1] - before[k - 1], prob.b[k], prob.p[k].n // 2)
    return it, hist, status


class Problem(Nested):
    """Two levels: a base grid and one box (the names of the two-level tests)."""

    def __init__(self, pc, pf, b0, rho5c, rho1c, rho5f, rho1f):
        super().__init__([pc, pf], [0, b0], [rho5c, rho5f], [rho1c, rho1f])
        self.pc, self.pf, self.b0, self.m = pc, pf, b0, pf.n // 2
        self.rc5, self.rc1, self.rf5, self.rf1 = rho5c, rho1c, rho5f, rho1f
        self.h_c, self.h_f = self.h[0], self.h[1]

    @property
    def cov(self):
        """Base cells under the box."""
        return self.covered(0)

    def residuals(self, uc, uf, fc=None):
        """(H_f with the interpolated ghosts, H_c, ghost forcing) after the base cells
        under the box took their children's average (uc is updated in place)."""
        uc[self.covered(0)] = oracle.restrict(uf)
        ff = ghost_forcing(uc, uf, self.b0, self.h_f)
        Hf = oracle.residuals(self.pf, uf, None, self.rf5, self.rf1, None, ff)[0]
        Hc = oracle.residuals(self.pc, uc, None, self.rc5, self.rc1, None, fc)[0]
        return Hf, Hc, ff

    def norm(self, Hf, Hc=None):
        if Hc is None:  # the nested form: a list of per-level residuals
            return super().norm(Hf)
        return super().norm([Hc, Hf])


def solve(prob: Problem, uc, uf, tol=1e-10, max_outer=60, nu_f=1, nu_c=1):
    """Two-level FAS iteration in place on (uc, uf)."""
    u = [uc, uf]
    return solve_nested(prob, u, tol, max_outer, nu_f, nu_c)
