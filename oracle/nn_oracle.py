"""CPU FP64 oracle of the warm-start network (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may use this module; it shares no code with the GPU library.

The paper starts every constraint solve from psi = 1, W = 0; the network here
is an addition that predicts a better starting point (u = psi - 1, W_a) from
the sources (rho = rho5 + rho1, S_a).  Its architecture is a reading, stated
once here and mirrored by the GPU library's documented parameter layout:

* a U-Net over ``levels`` resolution levels with widths ``ch[l]``;
* each level of the encoder applies two 3x3x3 convolutions with circular
  padding (the grids are periodic), each followed by SiLU, z * sigmoid(z);
* between encoder levels: 2x2x2 average pooling;
* the decoder, from level ``levels-2`` up to 0, upsamples the level below by
  cell-centred trilinear interpolation (weights 3/4 and 1/4 per axis, periodic),
  concatenates [encoder output of the level, upsampled tensor] along channels,
  and applies two 3x3x3 convolutions + SiLU;
* a final 3x3x3 convolution (no activation) gives ``c_out`` channels.

Parameter layout (one flat float array): for every convolution in the order
enc0a, enc0b, enc1a, enc1b, ..., dec(L-2)a, dec(L-2)b, ..., dec0a, dec0b, head,
the weights W[co][ci][kx][ky][kz] (kx = dx + 1 for the tap offset dx in -1..1)
followed by the bias b[co].  A convolution computes
    y[co](p) = b[co] + sum_ci sum_d W[co][ci][d + 1] x[ci](p + d)   (indices mod n).

Inputs and targets are standardised per channel: x_c = (v_c - mean_c) / std_c.
The loss is the mean squared error over all output channels and cells.

Gradients are taken with torch autograd in float64 (a library primitive);
they are pinned by central finite differences in the tests, and the
convolution by a brute-force loop over its definition.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import List, Sequence, Tuple

import numpy as np
import torch

DT = torch.float64


@dataclass
class NetConfig:
    n: int = 128
    levels: int = 4
    ch: Tuple[int, ...] = (16, 32, 48, 64)
    c_in: int = 4
    c_out: int = 4


def layer_shapes(cfg: NetConfig) -> List[Tuple[int, int]]:
    """(c_in, c_out) of every convolution in parameter order."""
    L = cfg.levels
    out = []
    cin = cfg.c_in
    for l in range(L):
        out.append((cin, cfg.ch[l]))
        out.append((cfg.ch[l], cfg.ch[l]))
        cin = cfg.ch[l]
    for l in range(L - 2, -1, -1):
        out.append((cfg.ch[l] + cfg.ch[l + 1], cfg.ch[l]))
        out.append((cfg.ch[l], cfg.ch[l]))
    out.append((cfg.ch[0], cfg.c_out))
    return out


def param_count(cfg: NetConfig) -> int:
    return sum(27 * ci * co + co for ci, co in layer_shapes(cfg))


def unpack(params, cfg: NetConfig):
    """Split the flat parameter vector into [(W, b)] (views when given a tensor)."""
    p = params if torch.is_tensor(params) else torch.as_tensor(np.asarray(params), dtype=DT)
    out, off = [], 0
    for ci, co in layer_shapes(cfg):
        W = p[off:off + 27 * ci * co].reshape(co, ci, 3, 3, 3)
        off += 27 * ci * co
        b = p[off:off + co]
        off += co
        out.append((W, b))
    assert off == p.numel()
    return out


def conv3(x: torch.Tensor, W: torch.Tensor, b: torch.Tensor) -> torch.Tensor:
    """3x3x3 convolution with circular padding; x: (ci, n, n, n) -> (co, n, n, n)."""
    y = b.reshape(-1, 1, 1, 1).expand(W.shape[0], *x.shape[1:]).clone()
    for dx in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dz in (-1, 0, 1):
                xs = torch.roll(x, shifts=(-dx, -dy, -dz), dims=(1, 2, 3))  # xs(p) = x(p + d)
                y = y + torch.einsum("oc,cxyz->oxyz", W[:, :, dx + 1, dy + 1, dz + 1], xs)
    return y


def silu(z: torch.Tensor) -> torch.Tensor:
    return z * torch.sigmoid(z)


def pool(x: torch.Tensor) -> torch.Tensor:
    """Mean over the 2x2x2 children of every coarse cell."""
    c, n = x.shape[0], x.shape[1]
    m = n // 2
    return x.reshape(c, m, 2, m, 2, m, 2).mean(dim=(2, 4, 6))


def _up_axis(x: torch.Tensor, axis: int) -> torch.Tensor:
    # fine cell 2I sits a quarter cell below coarse centre I, 2I+1 a quarter above
    lo = 0.75 * x + 0.25 * torch.roll(x, shifts=1, dims=axis)   # uses x[I-1]
    hi = 0.75 * x + 0.25 * torch.roll(x, shifts=-1, dims=axis)  # uses x[I+1]
    st = torch.stack((lo, hi), dim=axis + 1)
    shape = list(x.shape)
    shape[axis] *= 2
    return st.reshape(shape)


def up(x: torch.Tensor) -> torch.Tensor:
    """Cell-centred trilinear interpolation to the grid with twice the cells per axis."""
    return _up_axis(_up_axis(_up_axis(x, 1), 2), 3)


def forward(params, x: torch.Tensor, cfg: NetConfig, keep: bool = False):
    """Network output (c_out, n, n, n) for the standardised input x (c_in, n, n, n).
    With keep=True also returns the list of pre-activations in layer order."""
    layers = unpack(params, cfg)
    L = cfg.levels
    pre = []
    k = 0

    def cv(t, act=True):
        nonlocal k
        W, b = layers[k]
        k += 1
        z = conv3(t, W, b)
        pre.append(z)
        return silu(z) if act else z

    enc = []
    t = x
    for l in range(L):
        if l > 0:
            t = pool(t)
        t = cv(cv(t))
        enc.append(t)
    d = enc[L - 1]
    for l in range(L - 2, -1, -1):
        t = torch.cat((enc[l], up(d)), dim=0)
        d = cv(cv(t))
    out = cv(d, act=False)
    return (out, pre) if keep else out


def mse(out: torch.Tensor, target: torch.Tensor) -> torch.Tensor:
    return ((out - target) ** 2).mean()


def loss_and_grad(params, x, target, cfg: NetConfig):
    """(loss, d loss / d params) in float64."""
    p = torch.as_tensor(np.asarray(params), dtype=DT).clone().requires_grad_(True)
    out = forward(p, torch.as_tensor(np.asarray(x), dtype=DT), cfg)
    loss = mse(out, torch.as_tensor(np.asarray(target), dtype=DT))
    loss.backward()
    return float(loss.detach()), p.grad.detach().numpy().copy()


def conv3_vjp(x, W, b, dy):
    """Vector-Jacobian product of one convolution: (dx, dW, db) for output cotangent dy."""
    xt = torch.as_tensor(np.asarray(x), dtype=DT).clone().requires_grad_(True)
    Wt = torch.as_tensor(np.asarray(W), dtype=DT).clone().requires_grad_(True)
    bt = torch.as_tensor(np.asarray(b), dtype=DT).clone().requires_grad_(True)
    y = conv3(xt, Wt, bt)
    y.backward(torch.as_tensor(np.asarray(dy), dtype=DT))
    return xt.grad.numpy().copy(), Wt.grad.numpy().copy(), bt.grad.numpy().copy()


def adam(params, grad, m, v, step: int, lr: float, beta1: float = 0.9, beta2: float = 0.999,
         eps: float = 1e-8):
    """One Adam update (bias-corrected), float64; returns new (params, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v


# ---- inputs and targets ------------------------------------------------------------------

def net_input(rho5, rho1, S, mean: Sequence[float], std: Sequence[float]) -> np.ndarray:
    """Standardised network input: channels (rho5 + rho1, S_x, S_y, S_z)."""
    raw = [np.asarray(rho5) + np.asarray(rho1)] + [np.asarray(S)[a] for a in range(3)]
    return np.stack([(raw[c] - mean[c]) / std[c] for c in range(4)])


def net_target(u, W, mean: Sequence[float], std: Sequence[float]) -> np.ndarray:
    """Standardised target: channels (u, W_x, W_y, W_z)."""
    raw = [np.asarray(u)] + [np.asarray(W)[a] for a in range(3)]
    return np.stack([(raw[c] - mean[c]) / std[c] for c in range(4)])


def net_state(out, mean: Sequence[float], std: Sequence[float]):
    """Invert the target standardisation: (u, W) from the network output."""
    o = np.asarray(out)
    u = o[0] * std[0] + mean[0]
    W = np.stack([o[1 + a] * std[1 + a] + mean[1 + a] for a in range(3)])
    return u, W
