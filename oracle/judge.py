"""Independent numpy FP64 evaluator of the discrete constraint residuals, and
FFT exact solvers of constant-coefficient periodic problems.

Test infrastructure only (see ``oracle/__init__.py``).  Written separately
from ``mg_oracle.c`` (whole-array numpy instead of per-cell loops) so that the
two check each other; the residual norms it returns are the authority for the
1e-10 constraint target (paper, Key features, "Diagnostics": the norm of the
Hamiltonian and momentum constraint errors over the grid).

Fourier symbols (derived from the stencils acting on exp(i theta j)):
  D_a  -> i (8 sin t - sin 2t) / (6 h)
  D_aa -> (-2 cos 2t + 32 cos t - 30) / (12 h^2)
"""
from __future__ import annotations

import numpy as np

BC_PERIODIC = 0
BC_ROBIN = 1
BC_REFLECT = 2
BC_EXTRAP = 3
BC_ZERO = 4


class Grid:
    def __init__(self, n, length=1.0, bc=BC_PERIODIC, origin=(0.0, 0.0, 0.0),
                 centre=(0.0, 0.0, 0.0)):
        self.n, self.length, self.bc = n, length, bc
        self.h = length / n
        self.origin = np.asarray(origin, dtype=np.float64)
        self.centre = np.asarray(centre, dtype=np.float64)

    def coords(self, lo=0, hi=None):
        """Cell-centre coordinates relative to ``centre`` for indices lo..hi-1."""
        hi = self.n if hi is None else hi
        idx = np.arange(lo, hi, dtype=np.float64)
        return [self.origin[a] + (idx + 0.5) * self.h - self.centre[a] for a in range(3)]

    def radius(self, lo=0, hi=None):
        x, y, z = self.coords(lo, hi)
        return np.sqrt(x[:, None, None] ** 2 + y[None, :, None] ** 2 + z[None, None, :] ** 2)

    def pad(self, a):
        """Array of shape (n+4)^3 holding a and two ghost layers by the boundary rule."""
        n = self.n
        if self.bc == BC_PERIODIC:
            return np.pad(a, 2, mode="wrap")
        if self.bc == BC_REFLECT:   # mirror across each face, edge cell repeated
            return np.pad(a, 2, mode="symmetric")
        if self.bc == BC_ZERO:      # homogeneous ghosts
            return np.pad(a, 2, mode="constant")
        if self.bc == BC_EXTRAP:    # the cell next to each face continued outwards
            return np.pad(a, 2, mode="edge")
        ii = np.arange(-2, n + 2)
        cl = np.clip(ii, 0, n - 1)
        inner = a[np.ix_(cl, cl, cl)]
        rg = self.radius(-2, n + 2)
        xb = [self.origin[d] + (cl + 0.5) * self.h - self.centre[d] for d in range(3)]
        rb = np.sqrt(xb[0][:, None, None] ** 2 + xb[1][None, :, None] ** 2 + xb[2][None, None, :] ** 2)
        return inner * rb / rg


def _sl(off, n):
    return slice(2 + off, 2 + off + n)


def d1(g: Grid, ap, axis):
    n = g.n
    w = {-2: 1.0, -1: -8.0, 1: 8.0, 2: -1.0}
    out = 0.0
    for off, c in w.items():
        s = [_sl(0, n)] * 3
        s[axis] = _sl(off, n)
        out = out + c * ap[tuple(s)]
    return out / (12.0 * g.h)


def d2(g: Grid, ap, axis):
    n = g.n
    w = {-2: -1.0, -1: 16.0, 0: -30.0, 1: 16.0, 2: -1.0}
    out = 0.0
    for off, c in w.items():
        s = [_sl(0, n)] * 3
        s[axis] = _sl(off, n)
        out = out + c * ap[tuple(s)]
    return out / (12.0 * g.h ** 2)


def dmix(g: Grid, ap, p, q):
    n = g.n
    w = {-2: 1.0, -1: -8.0, 1: 8.0, 2: -1.0}
    out = 0.0
    for o1, c1 in w.items():
        for o2, c2 in w.items():
            s = [_sl(0, n)] * 3
            s[p] = _sl(o1, n)
            s[q] = _sl(o2, n)
            out = out + c1 * c2 * ap[tuple(s)]
    return out / (144.0 * g.h ** 2)


def lap(g: Grid, a):
    ap = g.pad(a)
    return d2(g, ap, 0) + d2(g, ap, 1) + d2(g, ap, 2)


def deltaL(g: Grid, W):
    Wp = [g.pad(W[a]) for a in range(3)]
    out = np.zeros_like(W)
    for a in range(3):
        s = d2(g, Wp[a], 0) + d2(g, Wp[a], 1) + d2(g, Wp[a], 2)
        t = d2(g, Wp[a], a)
        for b in range(3):
            if b != a:
                t = t + dmix(g, Wp[b], a, b)
        out[a] = s + t / 3.0
    return out


def A2(g: Grid, W):
    Wp = [g.pad(W[a]) for a in range(3)]
    dW = [[d1(g, Wp[b], a) for b in range(3)] for a in range(3)]  # dW[a][b] = D_a W_b
    div = dW[0][0] + dW[1][1] + dW[2][2]
    s = 0.0
    for a in range(3):
        for b in range(3):
            Ab = dW[a][b] + dW[b][a] - (2.0 / 3.0 * div if a == b else 0.0)
            s = s + Ab * Ab
    return s


def psi0(g: Grid, puncture_mass):
    if puncture_mass > 0.0:
        return 1.0 + puncture_mass / (2.0 * g.radius())
    return np.ones((g.n,) * 3)


def residuals(g: Grid, u, W, rho5, rho1, S, K, puncture_mass=0.0, f=None,
              conformal_matter=False, psi0_field=None, A2_bg=None):
    """H_h, mean-free M_h (periodic) and c = dH_h/dpsi, as whole arrays.
    conformal_matter: sources are rho_bar = psi^8 rho (= rho5 + rho1) and
    S_bar = psi^6 S, entering as 2 pi rho_bar psi^-3 and 8 pi S_bar.
    psi0_field replaces 1 + M/(2r) (several punctures); A2_bg is added to the
    A2 of W (an analytic extrinsic curvature such as Bowen-York's).
    K may be a field (the CTTK methods): eq. Ham then takes K(x)^2 per cell and
    eq. Mom the term -(2/3) psi^6 D_a K beside the matter source (both inside the
    mean removal of periodic grids)."""
    psi = (psi0(g, puncture_mass) if psi0_field is None else psi0_field) + u
    a2 = A2(g, W) if W is not None else 0.0
    if A2_bg is not None:
        a2 = a2 + A2_bg
    K2 = K * K
    if conformal_matter:
        rbar = rho5 + rho1
        matter = 2 * np.pi * rbar * psi ** -3
        dmatter = -6 * np.pi * rbar * psi ** -4
    else:
        matter = 2 * np.pi * rho5 * psi ** 5 + 2 * np.pi * rho1 * psi
        dmatter = 10 * np.pi * rho5 * psi ** 4 + 2 * np.pi * rho1
    H = lap(g, u) + matter - K2 / 12.0 * psi ** 5 + a2 * psi ** -7 / 8.0
    if f is not None:
        H = H + f
    c = dmatter - 5 * K2 / 12.0 * psi ** 4 - 7.0 / 8.0 * a2 * psi ** -8
    M = None
    if W is not None:
        w6 = 1.0 if conformal_matter else psi[None] ** 6
        src = 8 * np.pi * w6 * S
        if np.ndim(K) == 3:
            Kp = g.pad(K)
            src = src + 2.0 / 3.0 * w6 * np.stack([d1(g, Kp, a) for a in range(3)])
        if g.bc == BC_PERIODIC:
            src = src - src.mean(axis=(1, 2, 3), keepdims=True)
        M = deltaL(g, W) - src
    return H, M, c


def norms(H, M=None):
    """(rms H, rms |M|, max |H|, max |M|)."""
    hr = float(np.sqrt(np.mean(H * H)))
    hm = float(np.max(np.abs(H)))
    if M is None:
        return np.array([hr, 0.0, hm, 0.0])
    m2 = np.sum(M * M, axis=0)
    return np.array([hr, float(np.sqrt(np.mean(m2))), hm, float(np.sqrt(np.max(m2)))])


# ---- FFT exact solves (periodic, constant coefficients) ---------------------------

def _thetas(n):
    return 2.0 * np.pi * np.fft.fftfreq(n)


def sym_d1(theta, h):
    return 1j * (8.0 * np.sin(theta) - np.sin(2.0 * theta)) / (6.0 * h)


def sym_d2(theta, h):
    return (-2.0 * np.cos(2.0 * theta) + 32.0 * np.cos(theta) - 30.0) / (12.0 * h * h)


def fft_solve_psi(f, c0, h):
    """Exact discrete solution of (L_h + c0) u = f on a periodic grid."""
    n = f.shape[0]
    t = _thetas(n)
    lam = sym_d2(t, h)
    sym = lam[:, None, None] + lam[None, :, None] + lam[None, None, :] + c0
    return np.real(np.fft.ifftn(np.fft.fftn(f) / sym))


def fft_solve_W(f, h):
    """Exact mean-free discrete solution of Delta_L,h W = f (f mean-free)."""
    n = f.shape[1]
    t = _thetas(n)
    grids = np.meshgrid(t, t, t, indexing="ij")
    lam = [sym_d2(g_, h) for g_ in grids]
    sd = [sym_d1(g_, h) for g_ in grids]
    lsum = lam[0] + lam[1] + lam[2]
    Fh = np.stack([np.fft.fftn(f[a]) for a in range(3)])
    Mx = np.zeros((n, n, n, 3, 3), dtype=np.complex128)
    for a in range(3):
        for b in range(3):
            if a == b:
                Mx[..., a, b] = lsum + lam[a] / 3.0
            else:
                Mx[..., a, b] = sd[a] * sd[b] / 3.0
    Mx[0, 0, 0] = np.eye(3)
    rhs = np.moveaxis(Fh, 0, -1)[..., None]
    rhs[0, 0, 0] = 0.0
    sol = np.linalg.solve(Mx, rhs)[..., 0]
    return np.stack([np.real(np.fft.ifftn(sol[..., a])) for a in range(3)])


# ---- residuals at selected cells (full-size checks without whole-grid arrays) ------

def _at(g: Grid, a, i, j, k):
    """Boundary-ruled values of a at integer cells (arrays i, j, k, possibly outside)."""
    n = g.n
    if g.bc == BC_PERIODIC:
        return a[i % n, j % n, k % n]
    if g.bc in (BC_REFLECT, BC_EXTRAP, BC_ZERO):
        return g.pad(a)[i + 2, j + 2, k + 2]
    ci, cj, ck = np.clip(i, 0, n - 1), np.clip(j, 0, n - 1), np.clip(k, 0, n - 1)

    def rad(x, y, z):
        return np.sqrt((g.origin[0] + (x + 0.5) * g.h - g.centre[0]) ** 2 +
                       (g.origin[1] + (y + 0.5) * g.h - g.centre[1]) ** 2 +
                       (g.origin[2] + (z + 0.5) * g.h - g.centre[2]) ** 2)
    return a[ci, cj, ck] * rad(ci, cj, ck) / rad(i, j, k)


def hamiltonian_at(g: Grid, u, W, rho5, rho1, K, cells, puncture_mass=0.0,
                   conformal_matter=False):
    """H_h at the given cells (array of shape (m, 3)); same definition as residuals()."""
    i, j, k = cells[:, 0], cells[:, 1], cells[:, 2]
    w2 = {-2: -1.0, -1: 16.0, 0: -30.0, 1: 16.0, 2: -1.0}
    w1 = {-2: 1.0, -1: -8.0, 1: 8.0, 2: -1.0}
    lapu = 0.0
    for ax in range(3):
        for d, c in w2.items():
            o = [0, 0, 0]
            o[ax] = d
            lapu = lapu + c * _at(g, u, i + o[0], j + o[1], k + o[2])
    lapu = lapu / (12.0 * g.h ** 2)
    a2 = 0.0
    if W is not None:
        dW = [[0.0] * 3 for _ in range(3)]
        for a in range(3):
            for b in range(3):
                s = 0.0
                for d, c in w1.items():
                    o = [0, 0, 0]
                    o[a] = d
                    s = s + c * _at(g, W[b], i + o[0], j + o[1], k + o[2])
                dW[a][b] = s / (12.0 * g.h)
        div = dW[0][0] + dW[1][1] + dW[2][2]
        for a in range(3):
            for b in range(3):
                Ab = dW[a][b] + dW[b][a] - (2.0 / 3.0 * div if a == b else 0.0)
                a2 = a2 + Ab * Ab
    x = [g.origin[ax] + (cells[:, ax] + 0.5) * g.h - g.centre[ax] for ax in range(3)]
    r = np.sqrt(x[0] ** 2 + x[1] ** 2 + x[2] ** 2)
    psi = (1.0 + puncture_mass / (2.0 * r) if puncture_mass > 0.0 else 1.0) + u[i, j, k]
    r5, r1 = rho5[i, j, k], rho1[i, j, k]
    if conformal_matter:
        matter = 2 * np.pi * (r5 + r1) * psi ** -3
    else:
        matter = 2 * np.pi * r5 * psi ** 5 + 2 * np.pi * r1 * psi
    return lapu + matter - K * K / 12.0 * psi ** 5 + a2 * psi ** -7 / 8.0
