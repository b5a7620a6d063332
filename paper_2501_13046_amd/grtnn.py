"""ctypes binding of the warm-start network (the C ABI declared in include/grtnn.h).

Argument marshalling only: PyTorch supplies device memory and the current
stream; the forward and backward passes, the loss, the optimiser and the
packing of fields run in the library's HIP kernels.  BF16 tensors are
torch.bfloat16 (bit patterns identical to the ABI's uint16_t).
"""
from __future__ import annotations

import ctypes as C
from typing import Optional, Sequence

import torch

from . import grtmg as _mg
from .grtmg import MGError, _check, _dptr, _stream

DEFAULT_CH = (16, 32, 48, 64)


class NnConfig(C.Structure):
    _fields_ = [("n", C.c_int32), ("levels", C.c_int32), ("ch", C.c_int32 * 4),
                ("c_in", C.c_int32), ("c_out", C.c_int32)]


class NnNorm(C.Structure):
    _fields_ = [("in_mean", C.c_double * 4), ("in_std", C.c_double * 4),
                ("out_mean", C.c_double * 4), ("out_std", C.c_double * 4)]


_bound = False


def lib() -> C.CDLL:
    global _bound
    L = _mg.lib()
    if not _bound:
        vp, cp, i32, i64 = C.c_void_p, C.POINTER(NnConfig), C.c_int32, C.c_int64
        dp, np_ = C.POINTER(C.c_double), C.POINTER(NnNorm)
        L.nn_param_count.argtypes = [cp, C.POINTER(i64)]
        L.nn_workspace_size.argtypes = [cp, i32, C.POINTER(C.c_size_t)]
        L.nn_setup.argtypes = [cp, i32, vp, C.c_size_t, vp, C.POINTER(vp)]
        L.nn_load_params.argtypes = [vp, vp]
        L.nn_forward.argtypes = [vp, vp, vp]
        L.nn_mse.argtypes = [vp, vp, vp, dp]
        L.nn_backward.argtypes = [vp, vp]
        L.nn_adam_step.argtypes = [vp, vp, vp, vp, vp, i32, C.c_double, C.c_double, C.c_double,
                                   C.c_double, C.c_double]
        L.nn_pack_input.argtypes = [vp, vp, vp, vp, np_, vp]
        L.nn_pack_target.argtypes = [vp, vp, vp, np_, vp]
        L.nn_unpack_output.argtypes = [vp, vp, np_, vp, vp]
        L.nn_moments.argtypes = [vp, vp, vp, i64, dp]
        L.nn_warm_start.argtypes = [vp, vp, vp, vp, vp, np_, vp, vp, C.POINTER(i32), dp]
        L.nn_warm_start_ratio.argtypes = [vp, vp, vp, vp, vp, np_, vp, vp, C.c_double, C.POINTER(i32), dp]
        L.nn_destroy.argtypes = [vp]
        L.nn_destroy.restype = None
        L.nn_op_scratch_bytes.argtypes = [i32, i32, i32]
        L.nn_op_scratch_bytes.restype = C.c_size_t
        L.nn_conv3_forward.argtypes = [i32, i32, i32, vp, i32, vp, vp, vp, vp, C.c_size_t, vp]
        L.nn_conv3_backward_data.argtypes = [i32, i32, i32, vp, vp, vp, vp, C.c_size_t, vp]
        L.nn_conv3_backward_weight.argtypes = [i32, i32, i32, vp, i32, vp, vp, vp, vp, C.c_size_t, vp]
        for f in ("nn_param_count", "nn_workspace_size", "nn_setup", "nn_load_params", "nn_forward",
                  "nn_mse", "nn_backward", "nn_adam_step", "nn_pack_input", "nn_pack_target",
                  "nn_unpack_output", "nn_moments", "nn_warm_start", "nn_warm_start_ratio", "nn_conv3_forward",
                  "nn_conv3_backward_data", "nn_conv3_backward_weight"):
            getattr(L, f).restype = C.c_int
        _bound = True
    return L


def config(n: int, levels: int = 4, ch: Sequence[int] = DEFAULT_CH, c_in: int = 4,
           c_out: int = 4) -> NnConfig:
    c = NnConfig()
    c.n, c.levels, c.c_in, c.c_out = n, levels, c_in, c_out
    ch = list(ch) + [16] * (4 - len(ch))
    for q in range(4):
        c.ch[q] = ch[q]
    return c


def norm(in_mean, in_std, out_mean, out_std) -> NnNorm:
    m = NnNorm()
    for q in range(4):
        m.in_mean[q], m.in_std[q] = float(in_mean[q]), float(in_std[q])
        m.out_mean[q], m.out_std[q] = float(out_mean[q]), float(out_std[q])
    return m


def layer_shapes(cfg: NnConfig):
    """(c_in, c_out) of every convolution in the parameter order of grtnn.h."""
    L, ch = cfg.levels, list(cfg.ch)
    out, cin = [], cfg.c_in
    for l in range(L):
        out += [(cin, ch[l]), (ch[l], ch[l])]
        cin = ch[l]
    for l in range(L - 2, -1, -1):
        out += [(ch[l] + ch[l + 1], ch[l]), (ch[l], ch[l])]
    out.append((ch[0], cfg.c_out))
    return out


def param_count(cfg: NnConfig) -> int:
    c = C.c_int64(0)
    _check(lib().nn_param_count(C.byref(cfg), C.byref(c)), "nn_param_count")
    return c.value


def workspace_size(cfg: NnConfig, training: bool) -> int:
    b = C.c_size_t(0)
    _check(lib().nn_workspace_size(C.byref(cfg), int(training), C.byref(b)), "nn_workspace_size")
    return b.value


def _bf(t, numel=None):
    return _dptr(t, torch.bfloat16, numel)


def _f32(t, numel=None):
    return _dptr(t, torch.float32, numel)


class Net:
    """One nn_ctx on a torch-allocated workspace and the current stream."""

    def __init__(self, cfg: NnConfig, training: bool = False, device="cuda"):
        self.cfg = cfg
        self.training = training
        self.device = torch.device(device)
        self.cells = cfg.n ** 3
        nbytes = workspace_size(cfg, training)
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        ctx = C.c_void_p(None)
        _check(lib().nn_setup(C.byref(cfg), int(training), C.c_void_p(self.ws.data_ptr()), nbytes,
                              _stream(self.device), C.byref(ctx)), "nn_setup")
        self.ctx = ctx
        self.nparams = param_count(cfg)

    def close(self):
        if getattr(self, "ctx", None) is not None and self.ctx.value:
            lib().nn_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def load(self, params: torch.Tensor):
        _check(lib().nn_load_params(self.ctx, _f32(params, self.nparams)), "nn_load_params")

    def forward(self, x: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        if out is None:
            out = torch.empty((self.cells, self.cfg.c_out), dtype=torch.float32, device=self.device)
        _check(lib().nn_forward(self.ctx, _bf(x, self.cells * 8), _f32(out, self.cells * self.cfg.c_out)),
               "nn_forward")
        self._last_in = x  # read again by backward()
        return out

    def mse(self, out: torch.Tensor, target: torch.Tensor) -> float:
        loss = C.c_double(0.0)
        _check(lib().nn_mse(self.ctx, _f32(out, self.cells * self.cfg.c_out),
                            _bf(target, self.cells * self.cfg.c_out), C.byref(loss)), "nn_mse")
        return loss.value

    def backward(self, grad: torch.Tensor):
        _check(lib().nn_backward(self.ctx, _f32(grad, self.nparams)), "nn_backward")

    def adam(self, params, grad, m, v, step: int, lr: float, beta1=0.9, beta2=0.999, eps=1e-8,
             grad_scale=1.0):
        _check(lib().nn_adam_step(self.ctx, _f32(params, self.nparams), _f32(grad, self.nparams),
                                  _f32(m, self.nparams), _f32(v, self.nparams), step, lr, beta1, beta2,
                                  eps, grad_scale), "nn_adam_step")

    def pack_input(self, rho5, rho1, S, nm: NnNorm, x: Optional[torch.Tensor] = None):
        if x is None:
            x = torch.empty((self.cells, 8), dtype=torch.bfloat16, device=self.device)
        _check(lib().nn_pack_input(self.ctx, _dptr(rho5, numel=self.cells), _dptr(rho1, numel=self.cells),
                                   _dptr(S, numel=3 * self.cells), C.byref(nm), _bf(x, 8 * self.cells)),
               "nn_pack_input")
        return x

    def pack_target(self, u, W, nm: NnNorm, t: Optional[torch.Tensor] = None):
        if t is None:
            t = torch.empty((self.cells, 4), dtype=torch.bfloat16, device=self.device)
        _check(lib().nn_pack_target(self.ctx, _dptr(u, numel=self.cells), _dptr(W, numel=3 * self.cells),
                                    C.byref(nm), _bf(t, 4 * self.cells)), "nn_pack_target")
        return t

    def unpack_output(self, out, nm: NnNorm, u, W):
        _check(lib().nn_unpack_output(self.ctx, _f32(out, 4 * self.cells), C.byref(nm),
                                      _dptr(u, numel=self.cells), _dptr(W, numel=3 * self.cells)),
               "nn_unpack_output")

    def moments(self, x: torch.Tensor, y: Optional[torch.Tensor] = None):
        out = (C.c_double * 2)()
        _check(lib().nn_moments(self.ctx, _dptr(x), _dptr(y, numel=x.numel()) if y is not None else None,
                                x.numel(), out), "nn_moments")
        return out[0], out[1]

    def warm_start(self, solver: "_mg.Solver", rho5, rho1, S, nm: NnNorm, u, W, keep_ratio: float = None):
        """keep_ratio: the zero start's one-iteration contraction (nn_warm_start_ratio);
        None keeps a prediction that beats the zero state itself (nn_warm_start)."""
        if solver.cells != self.cells:
            raise MGError(_mg.MG_ERR_INVALID, "nn_warm_start: solver and network grids differ")
        used = C.c_int32(0)
        norms = (C.c_double * 4)()
        args = (self.ctx, solver.ctx, _dptr(rho5, numel=self.cells), _dptr(rho1, numel=self.cells),
                _dptr(S, numel=3 * self.cells), C.byref(nm), _dptr(u, numel=self.cells),
                _dptr(W, numel=3 * self.cells))
        if keep_ratio is None:
            _check(lib().nn_warm_start(*args, C.byref(used), norms), "nn_warm_start")
        else:
            _check(lib().nn_warm_start_ratio(*args, keep_ratio, C.byref(used), norms), "nn_warm_start_ratio")
        return bool(used.value), list(norms)


def _scratch(cin, cout, n, device):
    b = lib().nn_op_scratch_bytes(cin, cout, n)
    if b == 0:
        raise MGError(_mg.MG_ERR_INVALID, "nn_op_scratch_bytes")
    return torch.empty(b, dtype=torch.uint8, device=device), b


def conv3_forward(x: torch.Tensor, W: torch.Tensor, b: torch.Tensor, n: int, cin: int, cout: int,
                  act: bool = False) -> torch.Tensor:
    """y [n^3][cout] FP32 from x [n^3][cin] BF16, W [cout][cin][27], b [cout] FP32."""
    sc, nb = _scratch(cin, cout, n, x.device)
    y = torch.empty((n ** 3, cout), dtype=torch.float32, device=x.device)
    _check(lib().nn_conv3_forward(n, cin, cout, _bf(x, n ** 3 * cin), int(act), _f32(W, cout * cin * 27),
                                  _f32(b, cout), _f32(y), C.c_void_p(sc.data_ptr()), nb, _stream(x.device)),
           "nn_conv3_forward")
    return y


def conv3_backward_data(dy: torch.Tensor, W: torch.Tensor, n: int, cin: int, cout: int) -> torch.Tensor:
    """dx [n^3][cin] FP32 from dy [n^3][cout8] BF16."""
    sc, nb = _scratch(cin, cout, n, dy.device)
    dx = torch.empty((n ** 3, cin), dtype=torch.float32, device=dy.device)
    _check(lib().nn_conv3_backward_data(n, cin, cout, _bf(dy), _f32(W, cout * cin * 27), _f32(dx),
                                        C.c_void_p(sc.data_ptr()), nb, _stream(dy.device)),
           "nn_conv3_backward_data")
    return dx


def conv3_backward_weight(x: torch.Tensor, dy: torch.Tensor, n: int, cin: int, cout: int,
                          act: bool = False):
    """(dW [cout][cin][27], db [cout]) FP32."""
    sc, nb = _scratch(cin, cout, n, x.device)
    dW = torch.empty(cout * cin * 27, dtype=torch.float32, device=x.device)
    db = torch.empty(cout, dtype=torch.float32, device=x.device)
    _check(lib().nn_conv3_backward_weight(n, cin, cout, _bf(x, n ** 3 * cin), int(act), _bf(dy), _f32(dW),
                                          _f32(db), C.c_void_p(sc.data_ptr()), nb, _stream(x.device)),
           "nn_conv3_backward_weight")
    return dW, db
