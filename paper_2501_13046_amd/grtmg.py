"""ctypes binding of libgrtmg.so (the C ABI declared in include/grtmg.h).

Argument marshalling only: PyTorch supplies device memory and the current
HIP stream; every step of the solve runs in the library's HIP kernels.  There
is no fallback: if the library is missing, importing it raises.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np
import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libgrtmg.so")

MG_OK, MG_ERR_INVALID, MG_ERR_WORKSPACE, MG_ERR_HIP = 0, 1, 2, 3
MG_ERR_NOT_CONVERGED, MG_ERR_DIVERGED, MG_ERR_SINGULAR = 4, 5, 6
BC_PERIODIC, BC_ROBIN, BC_REFLECT, BC_EXTRAP, BC_ZERO = 0, 1, 2, 3, 4
PREC_FP64, PREC_FP32_IR = 0, 1
EQ_PSI, EQ_W, EQ_BOTH = 1, 2, 3
FLAG_CONFORMAL_MATTER = 1
FLAG_EAGER = 2
FLAG_CTTK = 4
FLAG_CUBIC_PROLONG = 8
FLAG_SAME_STATE = 16  # both steps of an outer iteration from one state (MG_FLAG_SAME_STATE)
OP_PASS_PSI, OP_PASS_W, OP_DEFECT_RESTRICT_PSI, OP_DEFECT_RESTRICT_W = 1, 2, 3, 4
OP_PROLONG_ADD, OP_COARSE_PSI, OP_COARSE_W, OP_FOURIER_W = 5, 6, 7, 8
PROBE_NONE, PROBE_PASS_PSI, PROBE_PASS_W, PROBE_RESIDUAL = 0, 1, 2, 3
PROBE_DEFECT_RESTRICT_PSI, PROBE_DEFECT_RESTRICT_W, PROBE_PROLONG = 4, 5, 6
PROBE_COARSE, PROBE_UPDATE = 7, 8
SOURCES_SCRATCH_BYTES = 32768


class MgParams(C.Structure):
    _fields_ = [("n", C.c_int32), ("levels", C.c_int32), ("bc", C.c_int32),
                ("precision", C.c_int32), ("nu_pre", C.c_int32), ("nu_post", C.c_int32),
                ("solve_momentum", C.c_int32), ("flags", C.c_int32),
                ("length", C.c_double), ("origin", C.c_double * 3), ("K", C.c_double),
                ("puncture_mass", C.c_double), ("puncture_pos", C.c_double * 3),
                ("nu_pre_W", C.c_int32), ("nu_post_W", C.c_int32), ("mix_depth", C.c_int32)]


class MgReport(C.Structure):
    _fields_ = [("outer_iters", C.c_int32), ("vcycles_psi", C.c_int32),
                ("vcycles_W", C.c_int32), ("status", C.c_int32),
                ("h_rms", C.c_double), ("m_rms", C.c_double), ("h_max", C.c_double),
                ("m_max", C.c_double), ("seconds", C.c_double),
                ("history", C.POINTER(C.c_double)), ("history_cap", C.c_int32),
                ("history_len", C.c_int32)]


TUNE_PASS_PSI, TUNE_PASS_W, TUNE_RESIDUAL, TUNE_TAIL_PSI, TUNE_TAIL_W, TUNE_FOURIER_W = 1, 2, 3, 4, 5, 6


def fourier_level(p) -> int:
    """Level of the W V-cycle solved exactly by discrete Fourier modes (the first level
    below the finest with 16, 32 or 64 cells per axis, in an FP32 periodic context that
    solves the momentum constraint), or -1."""
    if p.precision != PREC_FP32_IR or p.bc != BC_PERIODIC or not p.solve_momentum:
        return -1
    return next((l for l in range(1, p.levels) if p.n >> l in (16, 32, 64)), -1)


class MgTune(C.Structure):
    _fields_ = [("family", C.c_int32), ("level", C.c_int32), ("chosen", C.c_int32), ("ncand", C.c_int32),
                ("cand", C.c_int32 * 4), ("us", C.c_double * 4)]


class MGError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {status_str(status)} (status {status})")


_lib = None


def lib() -> C.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run __graft_entry__.build() first")
        L = C.CDLL(LIB_PATH)
        vp, dp, pp = C.c_void_p, C.POINTER(C.c_double), C.POINTER(MgParams)
        i32, st = C.c_int32, C.c_int
        L.mg_workspace_size.argtypes = [pp, C.POINTER(C.c_size_t)]
        L.mg_setup.argtypes = [pp, vp, C.c_size_t, vp, vp, vp, vp, vp, C.POINTER(vp)]
        L.mg_vcycle.argtypes = [vp, i32, vp, vp]
        L.mg_solve_constraints.argtypes = [vp, vp, vp, C.c_double, i32, C.POINTER(MgReport)]
        L.mg_solve_constraints_continue.argtypes = [vp, vp, vp, C.c_double, i32, C.POINTER(MgReport)]
        L.mg_residual_norm.argtypes = [vp, vp, vp, dp]
        L.mg_residual_fields.argtypes = [vp, vp, vp, vp, vp, vp]
        L.mg_destroy.argtypes = [vp]
        L.mg_destroy.restype = None
        L.mg_status_str.argtypes = [st]
        L.mg_status_str.restype = C.c_char_p
        L.mg_scalar_field_sources.argtypes = [pp, i32, dp, i32, dp, C.c_double, vp, vp, vp, vp,
                                              C.c_size_t, dp, dp, vp]
        L.mg_scalar_field_sources_static.argtypes = [pp, i32, dp, i32, dp, C.c_double, vp, vp, vp, dp, dp, vp]
        L.mg_shell_field_sources.argtypes = [pp, C.c_double, C.c_double, C.c_double, C.c_double,
                                             vp, vp, vp, vp]
        L.mg_interp_cubic.argtypes = [pp, vp, vp, vp]
        L.mg_set_background.argtypes = [vp, vp, vp]
        L.mg_bowen_york_sources.argtypes = [pp, i32, dp, vp, vp, vp]
        L.mg_cttk_trace.argtypes = [vp, vp, vp, vp]
        L.mg_refine_workspace_size.argtypes = [pp, pp, i32, C.POINTER(C.c_size_t)]
        L.mg_refine_solve.argtypes = [vp, vp, i32, vp, vp, vp, C.c_size_t, C.c_double, i32, i32, i32,
                                      C.POINTER(MgReport)]
        L.mg_refine_nested_workspace_size.argtypes = [i32, C.POINTER(pp), C.POINTER(i32), C.POINTER(C.c_size_t)]
        L.mg_refine_solve_nested.argtypes = [i32, C.POINTER(vp), C.POINTER(i32), C.POINTER(vp), vp, C.c_size_t,
                                             C.c_double, i32, i32, i32, C.POINTER(MgReport)]
        L.mg_cttk_hybrid_sources.argtypes = [pp, vp, vp, vp, vp, vp, C.c_size_t, dp, vp]
        L.mg_kernel_op.argtypes = [vp, i32, i32, i32, vp, vp, vp, vp]
        L.mg_batch_workspace_size.argtypes = [pp, i32, C.POINTER(C.c_size_t)]
        L.mg_setup_batch.argtypes = [pp, i32, vp, C.c_size_t, vp, C.POINTER(vp), C.POINTER(vp),
                                     C.POINTER(vp), C.POINTER(vp)]
        L.mg_solve_batch.argtypes = [vp, C.POINTER(vp), C.POINTER(vp), C.c_double, i32,
                                     C.POINTER(MgReport)]
        L.mg_destroy_batch.argtypes = [vp]
        L.mg_destroy_batch.restype = None
        L.mg_autotune.argtypes = [vp, vp, vp, i32, C.POINTER(MgTune), i32, C.POINTER(i32)]
        L.mg_set_tile.argtypes = [vp, i32, i32, i32]
        L.mg_batch_launch_mode.argtypes = [vp, i32, C.POINTER(i32), dp]
        L.mg_batch_groups.argtypes = [vp, C.POINTER(i32), C.POINTER(i32)]
        L.mg_fmg_start.argtypes = [vp, vp, vp, vp, C.c_double, i32, vp, vp, C.POINTER(MgReport)]
        L.mg_probe.argtypes = [vp, i32, i32]
        L.mg_probe_result.argtypes = [vp, C.POINTER(i32), C.POINTER(C.c_double)]
        for f in ("mg_workspace_size", "mg_setup", "mg_vcycle", "mg_solve_constraints", "mg_solve_constraints_continue",
                  "mg_residual_norm", "mg_residual_fields", "mg_scalar_field_sources",
                  "mg_scalar_field_sources_static", "mg_set_background", "mg_bowen_york_sources",
                  "mg_shell_field_sources", "mg_interp_cubic", "mg_kernel_op", "mg_probe",
                  "mg_probe_result", "mg_batch_workspace_size", "mg_setup_batch", "mg_solve_batch",
                  "mg_fmg_start", "mg_batch_launch_mode", "mg_batch_groups", "mg_autotune", "mg_set_tile",
                  "mg_cttk_trace", "mg_cttk_hybrid_sources", "mg_refine_workspace_size", "mg_refine_solve",
                  "mg_refine_nested_workspace_size", "mg_refine_solve_nested"):
            getattr(L, f).restype = st
        _lib = L
    return _lib


def status_str(s: int) -> str:
    return lib().mg_status_str(s).decode()


def _check(st: int, where: str, ok=(MG_OK,)):
    if st not in ok:
        raise MGError(st, where)
    return st


def params(n: int, levels: int = 1, bc: int = BC_PERIODIC, precision: int = PREC_FP64,
           length: float = 1.0, origin=(0.0, 0.0, 0.0), K: float = 0.0, nu_pre: int = 2,
           nu_post: int = 2, solve_momentum: bool = False, puncture_mass: float = 0.0,
           puncture_pos=(0.0, 0.0, 0.0), conformal_matter: bool = False,
           eager: bool = False, cttk: bool = False, nu_pre_W: int = 0, nu_post_W: int = 0,
           cubic_prolong: bool = False, same_state: bool = False, mix_depth: int = 0) -> MgParams:
    """nu_pre_W / nu_post_W: sweeps of the W V-cycle while its bottom is exact (see
    fourier_level; 0: nu_pre / nu_post).  cubic_prolong: corrections prolonged by the
    4-point cubic (MG_FLAG_CUBIC_PROLONG).  same_state: both steps of an outer
    iteration from one state (MG_FLAG_SAME_STATE).  mix_depth: steps the CTTK
    solve's Anderson mixing combines (0 or 1: one step)."""
    p = MgParams()
    p.n, p.levels, p.bc, p.precision = n, levels, bc, precision
    p.nu_pre, p.nu_post = nu_pre, nu_post
    p.nu_pre_W, p.nu_post_W = nu_pre_W, nu_post_W
    p.mix_depth = mix_depth
    p.solve_momentum = 1 if solve_momentum else 0
    p.flags = ((FLAG_CONFORMAL_MATTER if conformal_matter else 0) | (FLAG_EAGER if eager else 0)
               | (FLAG_CTTK if cttk else 0) | (FLAG_CUBIC_PROLONG if cubic_prolong else 0)
               | (FLAG_SAME_STATE if same_state else 0))
    p.length = length
    for a in range(3):
        p.origin[a] = origin[a]
        p.puncture_pos[a] = puncture_pos[a]
    p.K = K
    p.puncture_mass = puncture_mass
    return p


def workspace_size(p: MgParams) -> int:
    b = C.c_size_t(0)
    _check(lib().mg_workspace_size(C.byref(p), C.byref(b)), "mg_workspace_size")
    return b.value


def _dptr(t: Optional[torch.Tensor], dtype=torch.float64, numel: Optional[int] = None):
    if t is None:
        return None
    if not (t.is_cuda and t.dtype == dtype and t.is_contiguous()):
        raise ValueError(f"expected a contiguous CUDA tensor of {dtype}, got {t.dtype} on {t.device}")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"expected {numel} elements, got {t.numel()}")
    return C.c_void_p(t.data_ptr())


def _stream(device) -> C.c_void_p:
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


class Solver:
    """One mg_ctx: borrowed sources, a torch-allocated workspace, the current stream."""

    def __init__(self, p: MgParams, rho5: torch.Tensor, rho1: torch.Tensor,
                 S: Optional[torch.Tensor] = None, f: Optional[torch.Tensor] = None):
        self.p = p
        n = p.n
        self.cells = n ** 3
        self.device = rho5.device
        self.vtype = torch.float32 if p.precision == PREC_FP32_IR else torch.float64
        self._keep = (rho5, rho1, S, f)
        nbytes = workspace_size(p)
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = _stream(self.device)
        ctx = C.c_void_p(None)
        _check(lib().mg_setup(C.byref(p), C.c_void_p(self.ws.data_ptr()), nbytes, self.stream,
                              _dptr(rho5, numel=self.cells), _dptr(rho1, numel=self.cells),
                              _dptr(S, numel=3 * self.cells), _dptr(f, numel=self.cells),
                              C.byref(ctx)), "mg_setup")
        self.ctx = ctx

    def set_background(self, psi0: Optional[torch.Tensor] = None, A2: Optional[torch.Tensor] = None):
        """Background psi0 (several punctures) and A2 (Bowen-York) fields, borrowed."""
        self._bg = (psi0, A2)
        _check(lib().mg_set_background(self.ctx, _dptr(psi0, numel=self.cells), _dptr(A2, numel=self.cells)),
               "mg_set_background")

    def close(self):
        if getattr(self, "ctx", None) is not None and self.ctx.value:
            lib().mg_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _W(self, W):
        return _dptr(W, numel=3 * self.cells) if W is not None else None

    def autotune(self, u: torch.Tensor, W: Optional[torch.Tensor] = None, reps: int = 20) -> list:
        """Time the brick-depth candidates of the tiled kernels on this state; keep the fastest."""
        cap = 16
        out = (MgTune * cap)()
        cnt = C.c_int32(0)
        _check(lib().mg_autotune(self.ctx, _dptr(u, numel=self.cells), self._W(W), reps, out, cap, C.byref(cnt)),
               "mg_autotune")
        return [dict(family=e.family, level=e.level, chosen=e.chosen,
                     candidates={e.cand[q]: e.us[q] for q in range(e.ncand)}) for e in out[:cnt.value]]

    def set_tile(self, family: int, level: int, tx: int):
        _check(lib().mg_set_tile(self.ctx, family, level, tx), "mg_set_tile")

    def vcycle(self, eq: int, u: torch.Tensor, W: Optional[torch.Tensor] = None):
        _check(lib().mg_vcycle(self.ctx, eq, _dptr(u, numel=self.cells), self._W(W)), "mg_vcycle")

    def solve(self, u: torch.Tensor, W: Optional[torch.Tensor] = None, tol: float = 1e-10,
              max_outer: int = 100, raise_on_failure: bool = True, resume: bool = False) -> dict:
        """resume: continue from the state the last solve (or a kept warm start) left
        in these same arrays (mg_solve_constraints_continue)."""
        hist = np.zeros((max_outer + 2, 4))
        rep = MgReport()
        rep.history = hist.ctypes.data_as(C.POINTER(C.c_double))
        rep.history_cap = max_outer + 2
        fn = lib().mg_solve_constraints_continue if resume else lib().mg_solve_constraints
        st = fn(self.ctx, _dptr(u, numel=self.cells), self._W(W), tol, max_outer, C.byref(rep))
        out = dict(status=st, outer_iters=rep.outer_iters, vcycles_psi=rep.vcycles_psi,
                   vcycles_W=rep.vcycles_W, h_rms=rep.h_rms, m_rms=rep.m_rms, h_max=rep.h_max,
                   m_max=rep.m_max, seconds=rep.seconds, history=hist[: rep.history_len].copy())
        if raise_on_failure:
            _check(st, "mg_solve_constraints")
        return out

    def residual_norm(self, u: torch.Tensor, W: Optional[torch.Tensor] = None) -> np.ndarray:
        out = np.zeros(4)
        _check(lib().mg_residual_norm(self.ctx, _dptr(u, numel=self.cells), self._W(W),
                                      out.ctypes.data_as(C.POINTER(C.c_double))), "mg_residual_norm")
        return out

    def residual_fields(self, u: torch.Tensor, W: Optional[torch.Tensor] = None, want_M=True):
        n = self.p.n
        H = torch.empty((n, n, n), dtype=torch.float64, device=self.device)
        c = torch.empty_like(H)
        M = torch.empty((3, n, n, n), dtype=torch.float64, device=self.device) if want_M else None
        _check(lib().mg_residual_fields(self.ctx, _dptr(u, numel=self.cells), self._W(W),
                                        _dptr(H), _dptr(M), _dptr(c)), "mg_residual_fields")
        return H, M, c

    def cttk_trace(self, u: torch.Tensor, W: torch.Tensor) -> torch.Tensor:
        """K of the state (u, W) of a CTTK context (K^2 = 12 H0 / psi^5)."""
        K = torch.empty((self.p.n,) * 3, dtype=torch.float64, device=self.device)
        _check(lib().mg_cttk_trace(self.ctx, _dptr(u, numel=self.cells), _dptr(W, numel=3 * self.cells), _dptr(K)),
               "mg_cttk_trace")
        return K

    def probe(self, kernel: int, level: int = 0):
        _check(lib().mg_probe(self.ctx, kernel, level), "mg_probe")

    def probe_result(self):
        n = C.c_int32(0)
        ms = C.c_double(0.0)
        _check(lib().mg_probe_result(self.ctx, C.byref(n), C.byref(ms)), "mg_probe_result")
        return n.value, ms.value

    def kernel_op(self, op: int, level: int, arg: int, inp, out, r=None, c=None):
        vt = self.vtype
        _check(lib().mg_kernel_op(self.ctx, op, level, arg, _dptr(inp, vt), _dptr(out, vt),
                                  _dptr(r, vt), _dptr(c, vt)), "mg_kernel_op")


def _ptr_array(ts, dtype=torch.float64):
    arr = (C.c_void_p * len(ts))()
    for i, t in enumerate(ts):
        arr[i] = None if t is None else _dptr(t, dtype).value
    return arr


BATCH_AUTO, BATCH_GRAPH, BATCH_LANES, BATCH_GROUPS = 0, 1, 2, 3


class Batch:
    """A batch of independent instances solved together (one graph launch per
    outer iteration for the whole batch)."""

    def __init__(self, plist, rho5s, rho1s, Ss=None):
        self.count = len(plist)
        self.params = (MgParams * self.count)(*plist)
        self.device = rho5s[0].device
        self._keep = (list(rho5s), list(rho1s), list(Ss) if Ss is not None else None)
        nb = C.c_size_t(0)
        _check(lib().mg_batch_workspace_size(self.params, self.count, C.byref(nb)),
               "mg_batch_workspace_size")
        self.ws = torch.empty(nb.value, dtype=torch.uint8, device=self.device)
        self._r5, self._r1 = _ptr_array(rho5s), _ptr_array(rho1s)
        self._S = _ptr_array(Ss) if Ss is not None else None
        b = C.c_void_p(None)
        _check(lib().mg_setup_batch(self.params, self.count, C.c_void_p(self.ws.data_ptr()), nb.value,
                                    _stream(self.device), self._r5, self._r1, self._S, C.byref(b)),
               "mg_setup_batch")
        self.b = b

    def close(self):
        if getattr(self, "b", None) is not None and self.b.value:
            lib().mg_destroy_batch(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def launch_mode(self, request: int = -1):
        """Set (request >= 0) and/or query the launch mode: (mode in use, [ms graph, ms lanes, ms groups])."""
        chosen = C.c_int32(0)
        ms = (C.c_double * 3)()
        _check(lib().mg_batch_launch_mode(self.b, request, C.byref(chosen), ms), "mg_batch_launch_mode")
        return chosen.value, [ms[0], ms[1], ms[2]]

    def groups(self):
        """(number of groups, group of every member)."""
        ng = C.c_int32(0)
        of = (C.c_int32 * self.count)()
        _check(lib().mg_batch_groups(self.b, C.byref(ng), of), "mg_batch_groups")
        return ng.value, list(of)

    def solve(self, us, Ws=None, tol=1e-10, max_outer=100, raise_on_failure=True):
        reps = (MgReport * self.count)()
        st = lib().mg_solve_batch(self.b, _ptr_array(us), _ptr_array(Ws) if Ws is not None else None,
                                  tol, max_outer, reps)
        out = [dict(status=r.status, outer_iters=r.outer_iters, h_rms=r.h_rms, m_rms=r.m_rms,
                    h_max=r.h_max, m_max=r.m_max, seconds=r.seconds) for r in reps]
        if raise_on_failure:
            _check(st, "mg_solve_batch")
        return st, out


def scalar_field_sources(p: MgParams, phi_modes: np.ndarray, pi_modes: np.ndarray,
                         mass: float = 1.0, device="cuda", want_K=True):
    """Sources (rho5, rho1, S) of the Fourier scalar field and, when want_K,
    the library's constant K (K^2 = 24 pi <rho>); returns (rho5, rho1, S, K)."""
    n = p.n
    rho5 = torch.empty((n, n, n), dtype=torch.float64, device=device)
    rho1 = torch.empty_like(rho5)
    S = torch.empty((3, n, n, n), dtype=torch.float64, device=device)
    phi = np.ascontiguousarray(phi_modes, dtype=np.float64).reshape(-1, 5)
    pim = np.ascontiguousarray(pi_modes, dtype=np.float64).reshape(-1, 5)
    dp = C.POINTER(C.c_double)
    K = C.c_double(0.0)
    scratch = torch.empty(SOURCES_SCRATCH_BYTES, dtype=torch.uint8, device=device) if want_K else None
    _check(lib().mg_scalar_field_sources(
        C.byref(p), len(phi), phi.ctypes.data_as(dp) if len(phi) else None,
        len(pim), pim.ctypes.data_as(dp) if len(pim) else None, mass,
        _dptr(rho5), _dptr(rho1), _dptr(S),
        C.c_void_p(scratch.data_ptr()) if want_K else None,
        SOURCES_SCRATCH_BYTES if want_K else 0, None,
        C.byref(K) if want_K else None, _stream(rho5.device)), "mg_scalar_field_sources")
    return rho5, rho1, S, (K.value if want_K else None)


def zero_start_contraction(solver: "Solver", u: torch.Tensor, W: Optional[torch.Tensor] = None) -> float:
    """Contraction of max(rms H, rms M) over one outer iteration from the zero start
    (the keep ratio of the warm start's like-with-like fallback); leaves u, W zero."""
    u.zero_()
    if W is not None:
        W.zero_()
    r = solver.solve(u, W, tol=1e-300, max_outer=1, raise_on_failure=False)
    h = r["history"]
    u.zero_()
    if W is not None:
        W.zero_()
    return float(max(h[1][0], h[1][1]) / max(h[0][0], h[0][1]))


def box_params(base: MgParams, b0: int, m: int, levels: int, precision: Optional[int] = None) -> MgParams:
    """Parameters of a box refined by 2 over the m^3 base cells from base cell (b0, b0, b0):
    2m cells, zero ghost rule, the base grid's physics."""
    h = base.length / base.n
    p = params(2 * m, levels, BC_ZERO, base.precision if precision is None else precision, m * h,
               tuple(base.origin[a] + b0 * h for a in range(3)), base.K, base.nu_pre, base.nu_post, False,
               base.puncture_mass, tuple(base.puncture_pos[a] for a in range(3)))
    p.flags = base.flags & (FLAG_CONFORMAL_MATTER | FLAG_CUBIC_PROLONG)
    return p


def refine_solve(base: "Solver", box: "Solver", b0: int, uc: torch.Tensor, uf: torch.Tensor, tol: float = 1e-10,
                 max_outer: int = 60, nu_box: int = 1, nu_base: int = 1, raise_on_failure: bool = True) -> dict:
    """Two-level composite solve (mg_refine_solve): in place on uc (base) and uf (box).
    Both solvers must have been built with a forcing array f, which this overwrites."""
    nbytes = C.c_size_t(0)
    _check(lib().mg_refine_workspace_size(C.byref(base.p), C.byref(box.p), b0, C.byref(nbytes)),
           "mg_refine_workspace_size")
    work = torch.empty(nbytes.value, dtype=torch.uint8, device=uc.device)
    hist = np.zeros((max_outer + 2, 4))
    rep = MgReport()
    rep.history = hist.ctypes.data_as(C.POINTER(C.c_double))
    rep.history_cap = max_outer + 2
    st = lib().mg_refine_solve(base.ctx, box.ctx, b0, _dptr(uc, numel=base.cells), _dptr(uf, numel=box.cells),
                               C.c_void_p(work.data_ptr()), nbytes.value, tol, max_outer, nu_box, nu_base,
                               C.byref(rep))
    out = dict(status=st, outer_iters=rep.outer_iters, vcycles_psi=rep.vcycles_psi, h_rms=rep.h_rms,
               h_max=rep.h_max, seconds=rep.seconds, history=hist[: rep.history_len].copy())
    if raise_on_failure:
        _check(st, "mg_refine_solve")
    return out


def refine_solve_nested(solvers, offsets, us, tol: float = 1e-10, max_outer: int = 60, nu_box: int = 1,
                        nu_base: int = 1, raise_on_failure: bool = True) -> dict:
    """Nested-box composite solve (mg_refine_solve_nested): solvers[0] the base, solvers[k]
    a box over solvers[k-1] at cell offsets[k] (offsets[0] unused); in place on us."""
    L = len(solvers)
    pp = (C.POINTER(MgParams) * L)(*[C.pointer(s.p) for s in solvers])
    off = (C.c_int32 * L)(*[int(b) for b in offsets])
    nbytes = C.c_size_t(0)
    _check(lib().mg_refine_nested_workspace_size(L, pp, off, C.byref(nbytes)), "mg_refine_nested_workspace_size")
    work = torch.empty(nbytes.value, dtype=torch.uint8, device=us[0].device)
    ctx = (C.c_void_p * L)(*[s.ctx.value for s in solvers])
    ua = (C.c_void_p * L)(*[_dptr(u, numel=s.cells).value for u, s in zip(us, solvers)])
    hist = np.zeros((max_outer + 2, 4))
    rep = MgReport()
    rep.history = hist.ctypes.data_as(C.POINTER(C.c_double))
    rep.history_cap = max_outer + 2
    st = lib().mg_refine_solve_nested(L, ctx, off, ua, C.c_void_p(work.data_ptr()), nbytes.value, tol, max_outer,
                                      nu_box, nu_base, C.byref(rep))
    out = dict(status=st, outer_iters=rep.outer_iters, vcycles_psi=rep.vcycles_psi, h_rms=rep.h_rms,
               h_max=rep.h_max, seconds=rep.seconds, history=hist[: rep.history_len].copy())
    if raise_on_failure:
        _check(st, "mg_refine_solve_nested")
    return out


def cttk_hybrid_sources(p: MgParams, rho5: torch.Tensor, rho1: torch.Tensor, S: torch.Tensor):
    """CTTK-Hybrid: transforms rho5 (-> 0) and S (-> S + D K / (12 pi)) in place and
    returns (K field, K0) with K^2 = 24 pi (rho5 + <rho1>), K0^2 = 24 pi <rho1>."""
    n = p.n
    K = torch.empty((n, n, n), dtype=torch.float64, device=rho5.device)
    scratch = torch.empty(SOURCES_SCRATCH_BYTES, dtype=torch.uint8, device=rho5.device)
    K0 = C.c_double(0.0)
    _check(lib().mg_cttk_hybrid_sources(C.byref(p), _dptr(rho5, numel=n ** 3), _dptr(rho1, numel=n ** 3),
                                        _dptr(S, numel=3 * n ** 3), _dptr(K), C.c_void_p(scratch.data_ptr()),
                                        SOURCES_SCRATCH_BYTES, C.byref(K0), _stream(rho5.device)),
           "mg_cttk_hybrid_sources")
    return K, K0.value


def bowen_york_sources(p: MgParams, table, device="cuda"):
    """psi0 = 1 + sum m/(2r) and A2 of the Bowen-York curvature of the punctures
    (rows m, C[3], P[3], S[3]) on p's grid."""
    n = p.n
    tab = np.ascontiguousarray(table, dtype=np.float64).reshape(-1, 10)
    psi0 = torch.empty((n, n, n), dtype=torch.float64, device=device)
    A2 = torch.empty_like(psi0)
    _check(lib().mg_bowen_york_sources(C.byref(p), len(tab), tab.ctypes.data_as(C.POINTER(C.c_double)),
                                       _dptr(psi0), _dptr(A2), _stream(psi0.device)), "mg_bowen_york_sources")
    return psi0, A2


def shell_field_sources(p: MgParams, amplitude: float, r0: float, width2: float,
                        mass: float = 1.0, device="cuda"):
    n = p.n
    rho5 = torch.empty((n, n, n), dtype=torch.float64, device=device)
    rho1 = torch.empty_like(rho5)
    S = torch.empty((3, n, n, n), dtype=torch.float64, device=device)
    _check(lib().mg_shell_field_sources(C.byref(p), amplitude, r0, width2, mass, _dptr(rho5),
                                        _dptr(rho1), _dptr(S), _stream(rho5.device)),
           "mg_shell_field_sources")
    return rho5, rho1, S


def interp_cubic(pc: MgParams, coarse: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    nc = pc.n
    fine = torch.empty((2 * nc,) * 3, dtype=torch.float64, device=coarse.device) if out is None else out
    _check(lib().mg_interp_cubic(C.byref(pc), _dptr(coarse, numel=nc ** 3), _dptr(fine, numel=8 * nc ** 3),
                                 _stream(coarse.device)), "mg_interp_cubic")
    return fine


def tune_key(p: MgParams) -> str:
    return f"n{p.n}_L{p.levels}_prec{p.precision}_bc{p.bc}_mom{p.solve_momentum}"


def autotune_cached(solver: "Solver", u: torch.Tensor, W: Optional[torch.Tensor] = None,
                    path: Optional[str] = None, reps: int = 20) -> list:
    """Apply the brick depths stored for this configuration in a JSON cache
    (path, else $GRTMG_TUNE_CACHE, else ~/.cache/grtmg_tune.json); tune and
    store them when the configuration is not in the cache yet."""
    import json
    path = path or os.environ.get("GRTMG_TUNE_CACHE") or os.path.join(os.path.expanduser("~"), ".cache",
                                                                         "grtmg_tune.json")
    try:
        with open(path) as f:
            cache = json.load(f)
    except (OSError, ValueError):
        cache = {}
    key = tune_key(solver.p)
    if key in cache:
        for e in cache[key]:
            solver.set_tile(e["family"], e["level"], e["chosen"])
        return cache[key]
    entries = solver.autotune(u, W, reps)
    cache[key] = [dict(family=e["family"], level=e["level"], chosen=e["chosen"]) for e in entries]
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1)
    os.replace(tmp, path)
    return entries


def fmg_start(coarse: "Solver", fine: "Solver", uc: torch.Tensor, Wc: Optional[torch.Tensor],
              uf: torch.Tensor, Wf: Optional[torch.Tensor], tol: float = 1e-10, max_outer: int = 100) -> dict:
    """Solve the coarse problem, then interpolate its state to the fine arrays."""
    rep = MgReport()
    st = lib().mg_fmg_start(coarse.ctx, fine.ctx, _dptr(uc, numel=coarse.cells), coarse._W(Wc), tol, max_outer,
                            _dptr(uf, numel=fine.cells), fine._W(Wf), C.byref(rep))
    _check(st, "mg_fmg_start", ok=(MG_OK, MG_ERR_NOT_CONVERGED))
    return dict(status=st, outer_iters=rep.outer_iters, h_rms=rep.h_rms, m_rms=rep.m_rms, seconds=rep.seconds)


def fmg_coarse_tol(coarse: "Solver", fine: "Solver", uc: torch.Tensor, Wc: Optional[torch.Tensor],
                   uf: torch.Tensor, Wf: Optional[torch.Tensor], fraction: float = 0.1) -> float:
    """Coarse tolerance of an FMG start: `fraction` of the rms Hamiltonian
    residual that the converged coarse solution, interpolated, leaves on the
    fine grid (the discretisation difference between the two grids, which no
    coarse iteration removes).  Solves the coarse problem once to 1e-10; the
    arrays are overwritten."""
    uc.zero_()
    if Wc is not None:
        Wc.zero_()
    fmg_start(coarse, fine, uc, Wc, uf, Wf, tol=1e-10)
    h = fine.residual_norm(uf, Wf)[0]
    return float(fraction * h)
