"""CPU FP64 oracle for the constraint multigrid (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It wraps ``liboracle.so`` built from
``mg_oracle.c`` (plain C, FP64) and shares no code with the GPU library.

The discrete system, the boundary rule and the multigrid algorithm it follows
are stated at the top of ``mg_oracle.c``; the problem is the paper's
Hamiltonian and momentum constraints (Summary, eqs. Ham and Mom) in CTT form,
solved by multigrid (Key features, "Fast"), with per-iteration constraint
norms (Key features, "Diagnostics").

Pins (tests marked ``not gpu``): polynomial exactness and Fourier symbols of
the stencils, FFT-exact linear solves, uniform density (psi = 1), vacuum
puncture (u = 0), the Gaussian-source closed form under the Robin rule,
brute-force dense solves, 4th-order convergence to manufactured solutions,
the smoothers' diagonals against the operator's impulse response (periodic
and Robin, psi with its Newton coefficient, all three W components), the
exact solution as a fixed point of every colour pass, the colour convention,
the cycle order and contraction of both V-cycles; the CTTK and CTTK-Hybrid
methods against the Friedmann trace and the judge's direct evaluation of eqs.
Ham and Mom with a varying K; the two-level mesh refinement (``refine.py``)
against a dense solve of independently written composite equations and the
accuracy of a uniform grid of the box's spacing, with the zero ghost rule
against the embedded periodic operator; each such pin is shown to fail on a
copy of the oracle with a planted mistake (``planted``, or a patched function
of ``refine.py``).  No
oracle function is left "parity unpinned".
"""
from __future__ import annotations

import contextlib
import ctypes as C
import os
import subprocess
import tempfile

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
SRC_PATH = os.path.join(_HERE, "mg_oracle.c")

BC_PERIODIC = 0
BC_ROBIN = 1
BC_REFLECT = 2
BC_EXTRAP = 3
BC_ZERO = 4
FLAG_CONFORMAL_MATTER = 1
FLAG_CUBIC_PROLONG = 2  # corrections prolonged by the 4-point cubic (reading A10')
FLAG_SAME_STATE = 4  # both steps of an outer iteration linearise at its starting state


def build(verbose: bool = False) -> str:
    """Compile liboracle.so with gcc (FP64, no fast-math, no FMA contraction)."""
    cmd = _cc(SRC_PATH, LIB_PATH + ".tmp")
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


class OrcParams(C.Structure):
    _fields_ = [("n", C.c_int32), ("levels", C.c_int32), ("bc", C.c_int32),
                ("nu_pre", C.c_int32), ("nu_post", C.c_int32),
                ("solve_momentum", C.c_int32), ("flags", C.c_int32), ("mix_depth", C.c_int32),
                ("length", C.c_double), ("origin", C.c_double * 3), ("K", C.c_double),
                ("puncture_mass", C.c_double), ("puncture_pos", C.c_double * 3),
                ("bg_psi0", C.c_void_p), ("bg_A2", C.c_void_p)]


_lib = None


def _cc(src, out):
    return ["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fopenmp", "-ffp-contract=off",
            "-fPIC", "-shared", "-Wall", "-o", out, src, "-lm"]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        _lib = _bind(C.CDLL(LIB_PATH))
    return _lib


@contextlib.contextmanager
def planted(substitutions):
    """Test support: for the duration of the block, every function of this
    module runs on a copy of mg_oracle.c with a deliberate mistake planted by
    the given (old, new) text substitutions (each old text must occur exactly
    once), built on the CPU into a temporary directory.  Used to show that a
    pin fails when the oracle is wrong."""
    global _lib
    with open(SRC_PATH) as fh:
        src = fh.read()
    for old, new in substitutions:
        if src.count(old) != 1:
            raise ValueError(f"planted substitution must match once: {old!r}")
        src = src.replace(old, new)
    with tempfile.TemporaryDirectory() as d:
        c_path, so_path = os.path.join(d, "planted.c"), os.path.join(d, "libplanted.so")
        with open(c_path, "w") as fh:
            fh.write(src)
        subprocess.check_call(_cc(c_path, so_path))
        saved = _lib
        _lib = _bind(C.CDLL(so_path))
        try:
            yield
        finally:
            _lib = saved


def _bind(L):
    dp = C.POINTER(C.c_double)
    pp = C.POINTER(OrcParams)
    ip = C.c_int
    sig = {
        "orc_residuals": [pp, dp, dp, dp, dp, dp, dp, dp, dp, dp],
        "orc_norms": [ip, dp, dp, dp],
        "orc_apply_lap": [pp, ip, dp, dp],
        "orc_apply_d1": [pp, ip, dp, ip, dp],
        "orc_apply_deltaL": [pp, ip, dp, dp],
        "orc_pass_psi": [pp, ip, dp, dp, dp, dp, ip],
        "orc_pass_W": [pp, ip, dp, dp, dp, ip],
        "orc_restrict": [ip, dp, dp],
        "orc_prolong_add": [pp, ip, dp, dp],
        "orc_interp_cubic": [pp, ip, dp, dp],
        "orc_coarse_solve_psi": [pp, ip, dp, dp, dp],
        "orc_coarse_solve_W": [pp, ip, dp, dp],
        "orc_vcycle_psi": [pp, dp, dp, dp],
        "orc_vcycle_W": [pp, dp, dp],
        "orc_step": [pp, ip, dp, dp, dp, dp, dp, dp],
        "orc_solve": [pp, dp, dp, dp, dp, dp, dp, C.c_double, ip, dp, ip,
                      C.POINTER(C.c_int), dp],
        "orc_scalar_sources": [pp, ip, dp, ip, dp, C.c_double, dp, dp, dp],
        "orc_shell_sources": [pp, C.c_double, C.c_double, C.c_double, C.c_double,
                              dp, dp, dp],
        "orc_num_threads": [],
        "orc_bowen_york_tensor": [ip, dp, dp, dp],
        "orc_bowen_york": [pp, ip, dp, dp, dp],
        "orc_cttk_hybrid_sources": [pp, dp, dp, dp, dp, dp],
        "orc_cttk_update": [pp, dp, dp, dp, dp, dp, dp, dp, dp, dp],
        "orc_cttk_solve": [pp, dp, dp, dp, dp, dp, dp, dp, C.c_double, ip, dp, ip,
                           C.POINTER(C.c_int), dp],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = C.c_int if name in ("orc_coarse_solve_psi", "orc_coarse_solve_W",
                                        "orc_vcycle_psi", "orc_vcycle_W", "orc_step",
                                        "orc_solve", "orc_cttk_solve", "orc_num_threads") else None
    return L


def _ptr(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous, "float64 C-contiguous array expected"
    return a.ctypes.data_as(C.POINTER(C.c_double))


class _Params(OrcParams):
    """OrcParams that keeps the optional background arrays alive."""
    _keep = None


def params(n, levels=1, bc=BC_PERIODIC, length=1.0, origin=(0.0, 0.0, 0.0), K=0.0,
           nu_pre=2, nu_post=2, solve_momentum=False, puncture_mass=0.0,
           puncture_pos=(0.0, 0.0, 0.0), conformal_matter=False, bg_psi0=None,
           bg_A2=None, cubic_prolong=False, same_state=False, mix_depth=0) -> OrcParams:
    """bg_psi0, bg_A2: optional n^3 fields (several punctures: psi0 in place of
    1 + M/(2r); Bowen-York: A2 of the analytic extrinsic curvature).  cubic_prolong:
    the V-cycles prolong corrections with the 4-point cubic of interp_cubic.
    same_state: the psi step of an outer iteration reads the W the iteration
    started from, not the W step's result.  mix_depth: steps the CTTK solve's
    Anderson mixing combines (0 or 1: the one-step secant form; at most 6)."""
    p = _Params()
    keep = []
    for name, arr in (("bg_psi0", bg_psi0), ("bg_A2", bg_A2)):
        if arr is not None:
            arr = np.ascontiguousarray(arr, dtype=np.float64)
            assert arr.shape == (n, n, n)
            keep.append(arr)
            setattr(p, name, arr.ctypes.data)
    p._keep = keep
    p.flags = ((FLAG_CONFORMAL_MATTER if conformal_matter else 0) | (FLAG_CUBIC_PROLONG if cubic_prolong else 0)
               | (FLAG_SAME_STATE if same_state else 0))
    p.n, p.levels, p.bc = n, levels, bc
    p.nu_pre, p.nu_post = nu_pre, nu_post
    assert 0 <= mix_depth <= 6
    p.mix_depth = mix_depth
    p.solve_momentum = 1 if solve_momentum else 0
    p.length = length
    for a in range(3):
        p.origin[a] = origin[a]
        p.puncture_pos[a] = puncture_pos[a]
    p.K = K
    p.puncture_mass = puncture_mass
    return p


def params_from_workload(w, K=0.0) -> OrcParams:
    return params(w.n, w.levels, w.bc, w.length, w.origin, K, w.nu_pre, w.nu_post,
                  w.solve_momentum, w.puncture_mass, w.puncture_pos, w.conformal_matter,
                  cubic_prolong=w.cubic_prolong, same_state=w.same_state, mix_depth=w.mix_depth)


def _z(n, comps=1):
    return np.zeros((comps, n, n, n) if comps > 1 else (n, n, n), dtype=np.float64)


# ---- sources (matter projections) ------------------------------------------------

def scalar_sources(p: OrcParams, phi_modes, pi_modes, mass=1.0):
    n = p.n
    rho5, rho1, S = _z(n), _z(n), _z(n, 3)
    phi_modes = np.ascontiguousarray(phi_modes, dtype=np.float64)
    pi_modes = np.ascontiguousarray(pi_modes, dtype=np.float64)
    lib().orc_scalar_sources(C.byref(p), len(phi_modes), _ptr(phi_modes) if len(phi_modes) else None,
                             len(pi_modes), _ptr(pi_modes) if len(pi_modes) else None, mass,
                             _ptr(rho5), _ptr(rho1), _ptr(S))
    return rho5, rho1, S


def shell_sources(p: OrcParams, amplitude, r0, width2, mass=1.0):
    n = p.n
    rho5, rho1, S = _z(n), _z(n), _z(n, 3)
    lib().orc_shell_sources(C.byref(p), amplitude, r0, width2, mass, _ptr(rho5), _ptr(rho1), _ptr(S))
    return rho5, rho1, S


def K_from_mean_density(rho5, rho1):
    """K^2 = 24 pi <rho> at psi = 1 (periodic workloads)."""
    return float(np.sqrt(24.0 * np.pi * np.mean(rho5 + rho1)))


def sources_for(w):
    """Sources and K for a synthetic workload (periodic: K from the mean density;
    puncture: K = 0)."""
    p = params_from_workload(w)
    if w.shell is not None:
        rho5, rho1, S = shell_sources(p, w.shell["amplitude"], w.shell["r0"], w.shell["width2"],
                                      w.scalar_mass)
        K = 0.0
    else:
        rho5, rho1, S = scalar_sources(p, w.phi_modes, w.pi_modes, w.scalar_mass)
        K = K_from_mean_density(rho5, rho1)
    return rho5, rho1, S, K


# ---- residuals and norms ---------------------------------------------------------

def residuals(p, u, W, rho5, rho1, S, f=None):
    n = p.n
    H, M, c = _z(n), _z(n, 3), _z(n)
    lib().orc_residuals(C.byref(p), _ptr(u), _ptr(W), _ptr(rho5), _ptr(rho1), _ptr(S), _ptr(f),
                        _ptr(H), _ptr(M), _ptr(c))
    return H, M, c


def norms(H, M=None):
    out = np.zeros(4)
    lib().orc_norms(H.shape[0], _ptr(np.ascontiguousarray(H)),
                    _ptr(np.ascontiguousarray(M)) if M is not None else None, _ptr(out))
    return out


# ---- operators -------------------------------------------------------------------

def apply_lap(p, a):
    out = np.zeros_like(a)
    lib().orc_apply_lap(C.byref(p), a.shape[-1], _ptr(a), _ptr(out))
    return out


def apply_d1(p, a, axis):
    out = np.zeros_like(a)
    lib().orc_apply_d1(C.byref(p), a.shape[-1], _ptr(a), axis, _ptr(out))
    return out


def apply_deltaL(p, W):
    out = np.zeros_like(W)
    lib().orc_apply_deltaL(C.byref(p), W.shape[-1], _ptr(W), _ptr(out))
    return out


def pass_psi(p, d, r, c, colour):
    out = np.zeros_like(d)
    lib().orc_pass_psi(C.byref(p), d.shape[-1], _ptr(d), _ptr(out), _ptr(r), _ptr(c), colour)
    return out


def pass_W(p, d, r, colour):
    out = np.zeros_like(d)
    lib().orc_pass_W(C.byref(p), d.shape[-1], _ptr(d), _ptr(out), _ptr(r), colour)
    return out


def restrict(fine):
    nf = fine.shape[-1]
    coarse = np.zeros((nf // 2,) * 3)
    lib().orc_restrict(nf, _ptr(np.ascontiguousarray(fine)), _ptr(coarse))
    return coarse


def prolong_add(p, coarse, fine):
    fine = fine.copy()
    lib().orc_prolong_add(C.byref(p), coarse.shape[-1], _ptr(np.ascontiguousarray(coarse)), _ptr(fine))
    return fine


def interp_cubic(p, coarse):
    nc = coarse.shape[-1]
    fine = np.zeros((2 * nc,) * 3)
    lib().orc_interp_cubic(C.byref(p), nc, _ptr(np.ascontiguousarray(coarse)), _ptr(fine))
    return fine


def coarse_solve_psi(p, c, r):
    x = np.zeros_like(r)
    rc = lib().orc_coarse_solve_psi(C.byref(p), r.shape[-1], _ptr(c), _ptr(r), _ptr(x))
    if rc:
        raise ArithmeticError("singular coarse matrix")
    return x


def coarse_solve_W(p, r):
    x = np.zeros_like(r)
    rc = lib().orc_coarse_solve_W(C.byref(p), r.shape[-1], _ptr(r), _ptr(x))
    if rc:
        raise ArithmeticError("singular coarse matrix")
    return x


def vcycle_psi(p, c, r):
    d = np.zeros_like(r)
    rc = lib().orc_vcycle_psi(C.byref(p), _ptr(c), _ptr(r), _ptr(d))
    if rc:
        raise ArithmeticError("singular coarse matrix")
    return d


def vcycle_W(p, r):
    d = np.zeros_like(r)
    rc = lib().orc_vcycle_W(C.byref(p), _ptr(r), _ptr(d))
    if rc:
        raise ArithmeticError("singular coarse matrix")
    return d


def step(p, eq, u, W, rho5, rho1, S, f=None):
    """One outer update (eq 1: psi, 2: W, 3: W then psi), in place on u and W."""
    rc = lib().orc_step(C.byref(p), eq, _ptr(u), _ptr(W), _ptr(rho5), _ptr(rho1), _ptr(S), _ptr(f))
    if rc:
        raise ArithmeticError("singular coarse matrix")


class SolveResult:
    def __init__(self, status, iters, history, norms):
        self.status, self.iters, self.history, self.norms = status, iters, history, norms

    def __repr__(self):
        return f"SolveResult(status={self.status}, iters={self.iters}, norms={self.norms})"


def solve(p, u, W, rho5, rho1, S, f=None, tol=1e-10, max_outer=60):
    """Newton-multigrid solve in place on (u, W); returns a SolveResult."""
    hist = np.zeros((max_outer + 1, 4))
    it = C.c_int(0)
    nr = np.zeros(4)
    st = lib().orc_solve(C.byref(p), _ptr(u), _ptr(W), _ptr(rho5), _ptr(rho1), _ptr(S), _ptr(f),
                         tol, max_outer, _ptr(hist), max_outer + 1, C.byref(it), _ptr(nr))
    return SolveResult(st, it.value, hist[: min(it.value + 1, max_outer + 1)], nr)


# ---- CTTK and CTTK-Hybrid (spatially varying K; readings stated in mg_oracle.c) ---------

def cttk_hybrid_sources(p, rho5, rho1, S):
    """CTTK-Hybrid sources: returns (rho5_h, S_h, K, K0) with rho5_h = 0,
    S_h = S + D K / (12 pi), K^2 = 24 pi (rho5 + <rho1>), K0^2 = 24 pi <rho1>."""
    r5 = np.array(rho5, dtype=np.float64, order="C")
    Sh = np.array(S, dtype=np.float64, order="C")
    K = _z(p.n)
    K0 = np.zeros(1)
    lib().orc_cttk_hybrid_sources(C.byref(p), _ptr(r5), _ptr(np.ascontiguousarray(rho1)), _ptr(Sh), _ptr(K),
                                  _ptr(K0))
    return r5, Sh, K, float(K0[0])


def cttk_update(p, u, W, rho5, rho1, S, f=None):
    """CTTK: (rho5_eff, S_eff, K) at (u, W), K^2 = 12 H_h(K=0) / psi^5."""
    n = p.n
    r5, Se, K = _z(n), _z(n, 3), _z(n)
    lib().orc_cttk_update(C.byref(p), _ptr(u), _ptr(W), _ptr(rho5), _ptr(rho1), _ptr(S), _ptr(f), _ptr(r5),
                          _ptr(Se), _ptr(K))
    return r5, Se, K


def cttk_solve(p, u, W, rho5, rho1, S, f=None, tol=1e-10, max_outer=60):
    """CTTK solve in place on W (u is data); returns (SolveResult, K)."""
    hist = np.zeros((max_outer + 1, 4))
    it = C.c_int(0)
    nr = np.zeros(4)
    K = _z(p.n)
    st = lib().orc_cttk_solve(C.byref(p), _ptr(u), _ptr(W), _ptr(rho5), _ptr(rho1), _ptr(S), _ptr(f), _ptr(K),
                              tol, max_outer, _ptr(hist), max_outer + 1, C.byref(it), _ptr(nr))
    return SolveResult(st, it.value, hist[: min(it.value + 1, max_outer + 1)], nr), K


# ---- Bowen-York punctures -----------------------------------------------------------

def bowen_york_tensor(table, x):
    """Abar_ij (xx, xy, xz, yy, yz, zz) at point x; table rows (m, C[3], P[3], S[3])."""
    tab = np.ascontiguousarray(table, dtype=np.float64).reshape(-1, 10)
    out = np.zeros(6)
    xx = np.ascontiguousarray(x, dtype=np.float64)
    lib().orc_bowen_york_tensor(len(tab), _ptr(tab), _ptr(xx), _ptr(out))
    return out


def bowen_york(p, table):
    """psi0 = 1 + sum m/(2r) and A2 = Abar_ij Abar_ij at the cell centres of p's grid."""
    tab = np.ascontiguousarray(table, dtype=np.float64).reshape(-1, 10)
    psi0, A2 = _z(p.n), _z(p.n)
    lib().orc_bowen_york(C.byref(p), len(tab), _ptr(tab), _ptr(psi0), _ptr(A2))
    return psi0, A2


def num_threads() -> int:
    return lib().orc_num_threads()
