"""Parity of the warm-start network kernels with the FP64 oracle.

Operands are rounded to BF16 on the CPU before the oracle sees them, so that a
convolution without activation differs from the oracle only by FP32
accumulation order (tolerance 1e-4 of the output scale).  Where the GPU also
rounds intermediate values to BF16 (SiLU on load, stored activations), the
tolerance follows from the BF16 unit roundoff 2^-9 per stored value,
compounded over the layers (1e-2 for one layer, 3e-2 / 5e-2 for the
network's output / gradients in relative 2-norm).
"""
import numpy as np
import pytest
import torch

import synth
from oracle import nn_oracle as nn
from paper_2501_13046_amd import grtmg as g
from paper_2501_13046_amd import grtnn as gn
from gpu_helpers import dev

pytestmark = pytest.mark.gpu


def bf(a):
    """Round to BF16 (nearest even) and return float64 numpy."""
    return torch.as_tensor(np.asarray(a)).to(torch.bfloat16).to(torch.float64).numpy()


def cl(x):
    """(C, n, n, n) -> channels-last (n^3, C)."""
    return np.ascontiguousarray(np.moveaxis(np.asarray(x), 0, -1).reshape(-1, x.shape[0]))


def cf(y, n):
    """channels-last (n^3, C) -> (C, n, n, n)."""
    y = np.asarray(y)
    return np.moveaxis(y.reshape(n, n, n, -1), -1, 0)


def to_dev(a, dtype):
    return torch.as_tensor(np.ascontiguousarray(a)).to(dtype).to(dev())


def silu_bf(x):
    return bf(x / (1.0 + np.exp(-x)))


# n a multiple of 16 without SiLU on load runs the brick kernel (slices of 8, 16, 32
# channels; 7 K steps of weights in flight on grids under 1024 blocks, 2 from 64^3 on);
# the other cases run the general kernel
@pytest.mark.parametrize("n,cin,cout,act", [(6, 8, 4, False), (8, 16, 16, True), (5, 48, 48, False),
                                            (16, 32, 48, True), (4, 112, 48, False), (32, 48, 16, False),
                                            (16, 64, 64, False), (32, 8, 16, False), (16, 112, 80, False),
                                            (64, 48, 16, False), (64, 8, 16, False)])
def test_conv_forward(n, cin, cout, act):
    rng = np.random.default_rng(n * 1000 + cin + cout)
    x = bf(rng.standard_normal((cin, n, n, n)))
    W = bf(rng.standard_normal((cout, cin, 3, 3, 3)) * np.sqrt(2.0 / (27 * cin)))
    b = rng.uniform(-0.1, 0.1, cout).astype(np.float32).astype(np.float64)
    y = gn.conv3_forward(to_dev(cl(x), torch.bfloat16), to_dev(W.reshape(-1), torch.float32),
                         to_dev(b, torch.float32), n, cin, cout, act)
    xin = silu_bf(x) if act else x
    ref = nn.conv3(torch.tensor(xin), torch.tensor(W), torch.tensor(b)).numpy()
    got = cf(y.cpu().numpy(), n)
    scale = np.sqrt(np.mean(ref ** 2))
    err = np.abs(got - ref).max() / scale
    print(f"conv fwd n={n} {cin}->{cout} act={act}: max err / rms = {err:.2e}")
    assert err < (1e-2 if act else 1e-4)


@pytest.mark.parametrize("n,cin,cout", [(6, 16, 4), (8, 48, 16), (5, 80, 32), (16, 16, 16), (32, 48, 4),
                                        (16, 112, 32), (32, 16, 64), (64, 16, 16)])
def test_conv_backward_data(n, cin, cout):
    rng = np.random.default_rng(7 * n + cin + cout)
    cout8 = (cout + 7) // 8 * 8
    W = bf(rng.standard_normal((cout, cin, 3, 3, 3)) * 0.1)
    dy = np.zeros((cout8, n, n, n))
    dy[:cout] = bf(rng.standard_normal((cout, n, n, n)))
    dx = gn.conv3_backward_data(to_dev(cl(dy), torch.bfloat16), to_dev(W.reshape(-1), torch.float32), n, cin,
                                cout)
    x0 = np.zeros((cin, n, n, n))
    ref, _, _ = nn.conv3_vjp(x0, W, np.zeros(cout), dy[:cout])
    got = cf(dx.cpu().numpy(), n)
    err = np.abs(got - ref).max() / np.sqrt(np.mean(ref ** 2))
    print(f"conv bwd data n={n} {cin}->{cout}: max err / rms = {err:.2e}")
    assert err < 1e-4


@pytest.mark.parametrize("n,cin,cout,act", [(6, 8, 4, False), (8, 16, 16, False), (5, 48, 32, True),
                                            (16, 32, 16, False), (3, 16, 48, False), (32, 48, 4, False),
                                            (16, 8, 16, False), (32, 24, 48, False), (16, 16, 16, True)])
def test_conv_backward_weight(n, cin, cout, act):
    rng = np.random.default_rng(11 * n + cin + cout)
    cout8 = (cout + 7) // 8 * 8
    x = bf(rng.standard_normal((cin, n, n, n)))
    dy = np.zeros((cout8, n, n, n))
    dy[:cout] = bf(rng.standard_normal((cout, n, n, n)))
    dW, db = gn.conv3_backward_weight(to_dev(cl(x), torch.bfloat16), to_dev(cl(dy), torch.bfloat16), n, cin,
                                      cout, act)
    xin = silu_bf(x) if act else x
    _, rW, rb = nn.conv3_vjp(xin, np.zeros((cout, cin, 3, 3, 3)), np.zeros(cout), dy[:cout])
    eW = np.abs(dW.cpu().numpy().reshape(rW.shape) - rW).max() / np.sqrt(np.mean(rW ** 2))
    eb = np.abs(db.cpu().numpy() - rb).max() / np.sqrt(np.mean(rb ** 2))
    print(f"conv bwd weight n={n} {cin}->{cout} act={act}: dW {eW:.2e} db {eb:.2e}")
    assert eW < (1e-2 if act else 1e-4) and eb < 1e-4


def small_cfg(n=16, levels=3, ch=(16, 32, 48)):
    return nn.NetConfig(n=n, levels=levels, ch=tuple(ch), c_in=4, c_out=4), gn.config(n, levels, ch)


def net_inputs(cfg, seed):
    rng = np.random.default_rng(seed)
    p = synth.nn_init(nn.layer_shapes(cfg), seed=seed, bias_scale=0.05)
    x = bf(rng.standard_normal((4, cfg.n, cfg.n, cfg.n)))
    t = bf(rng.standard_normal((4, cfg.n, cfg.n, cfg.n)) * 0.5)
    return p, x, t


def gpu_x(x):
    x8 = np.zeros((8,) + x.shape[1:])
    x8[:4] = x
    return to_dev(cl(x8), torch.bfloat16)


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


# 64^3: upsampling into 64^3 takes one thread per coarse cell, the 64^3 convolutions 2 K steps
# of weights in flight
@pytest.mark.parametrize("n,levels,ch", [(16, 3, (16, 32, 48)), (8, 1, (16,)), (16, 2, (32, 16)),
                                         (32, 4, (16, 32, 48, 64)), (64, 4, (16, 32, 48, 64))])
def test_network_forward(n, levels, ch):
    cfg, gc = small_cfg(n, levels, ch)
    p, x, _ = net_inputs(cfg, 5)
    net = gn.Net(gc, training=False)
    net.load(to_dev(p, torch.float32))
    out = net.forward(gpu_x(x))
    pb = bf(p)  # the kernels use BF16 weights; biases stay FP32
    shapes = nn.layer_shapes(cfg)
    off = 0
    for ci, co in shapes:
        off += 27 * ci * co
        pb[off:off + co] = p[off:off + co]
        off += co
    ref = nn.forward(torch.tensor(pb), torch.tensor(x), cfg).numpy()
    got = cf(out.cpu().numpy(), n)
    e = rel(got, ref)
    print(f"network forward n={n} levels={levels} ch={ch}: rel err {e:.2e}")
    assert e < 3e-2


@pytest.mark.parametrize("n,levels,ch", [(16, 3, (16, 32, 48)), (8, 1, (16,)), (16, 4, (16, 32, 48, 64))])
def test_network_gradients(n, levels, ch):
    cfg, gc = small_cfg(n, levels, ch)
    p, x, t = net_inputs(cfg, 6)
    net = gn.Net(gc, training=True)
    net.load(to_dev(p, torch.float32))
    out = net.forward(gpu_x(x))
    loss = net.mse(out, to_dev(cl(t), torch.bfloat16))
    grad = torch.zeros(net.nparams, dtype=torch.float32, device=dev())
    net.backward(grad)
    pb = bf(p)
    off = 0
    for ci, co in nn.layer_shapes(cfg):
        off += 27 * ci * co
        pb[off:off + co] = p[off:off + co]
        off += co
    rloss, rgrad = nn.loss_and_grad(pb, x, t, cfg)
    gg = grad.cpu().numpy().astype(np.float64)
    print(f"network gradients n={n} levels={levels}: loss {loss:.6f} vs {rloss:.6f}, "
          f"grad rel err {rel(gg, rgrad):.2e}")
    # measured on MI355X: loss 1.2e-4 relative, gradient 7.1e-4, per layer 2.0e-3 (weights)
    # and 1.2e-3 (biases); bounds about 3x those
    assert abs(loss - rloss) <= 5e-4 * rloss
    assert rel(gg, rgrad) < 2.5e-3
    off = 0
    errs = []
    for k, (ci, co) in enumerate(nn.layer_shapes(cfg)):
        w = slice(off, off + 27 * ci * co)
        bsl = slice(off + 27 * ci * co, off + 27 * ci * co + co)
        off += 27 * ci * co + co
        errs.append((rel(gg[w], rgrad[w]), rel(gg[bsl], rgrad[bsl])))
    print("per-layer gradient rel err (max weight, max bias):",
          f"{max(e[0] for e in errs):.2e} {max(e[1] for e in errs):.2e}")
    for k, (ew, eb) in enumerate(errs):
        assert ew < 6e-3 and eb < 4e-3, (k, ew, eb)


def test_adam_matches_oracle():
    cfg, gc = small_cfg(8, 2, (16, 16))
    net = gn.Net(gc, training=True)
    rng = np.random.default_rng(3)
    N = net.nparams
    p = rng.standard_normal(N).astype(np.float32)
    gr = (rng.standard_normal(N) * 1e-3).astype(np.float32)
    m = (rng.standard_normal(N) * 1e-3).astype(np.float32)
    v = (rng.random(N) * 1e-6).astype(np.float32)
    tp, tg, tm, tv = (to_dev(a, torch.float32) for a in (p, gr, m, v))
    net.adam(tp, tg, tm, tv, step=3, lr=1e-3, grad_scale=0.5)
    rp, rm, rv = nn.adam(p.astype(np.float64), 0.5 * gr.astype(np.float64), m.astype(np.float64),
                         v.astype(np.float64), 3, 1e-3)
    assert np.abs(tp.cpu().numpy() - rp).max() < 1e-6
    assert np.abs(tm.cpu().numpy() - rm).max() <= 1e-7 * np.abs(rm).max() + 1e-12
    assert np.abs(tv.cpu().numpy() - rv).max() <= 1e-6 * np.abs(rv).max() + 1e-15


def test_field_packing_and_moments():
    n = 8
    cfg, gc = small_cfg(n, 2, (16, 16))
    net = gn.Net(gc, training=True)
    rng = np.random.default_rng(4)
    rho5, rho1 = rng.random((n, n, n)), rng.random((n, n, n))
    S, u, W = rng.standard_normal((3, n, n, n)), rng.standard_normal((n, n, n)), rng.standard_normal((3, n, n, n))
    mean_in, std_in = [1.0, 0.1, -0.1, 0.0], [0.3, 1.2, 0.9, 1.1]
    mean_out, std_out = [0.5, 0.0, 0.2, -0.2], [0.4, 2.0, 1.5, 0.7]
    nm = gn.norm(mean_in, std_in, mean_out, std_out)
    T = lambda a: to_dev(a, torch.float64)
    x = net.pack_input(T(rho5), T(rho1), T(S), nm)
    ref = bf(nn.net_input(rho5, rho1, S, mean_in, std_in))
    got = cf(x.float().cpu().numpy(), n)
    assert np.array_equal(got[:4], ref) and not got[4:].any()
    t = net.pack_target(T(u), T(W), nm)
    assert np.array_equal(cf(t.float().cpu().numpy(), n), bf(nn.net_target(u, W, mean_out, std_out)))
    out = rng.standard_normal((n ** 3, 4)).astype(np.float32)
    du, dW = torch.empty((n, n, n), dtype=torch.float64, device=dev()), torch.empty((3, n, n, n),
                                                                                    dtype=torch.float64,
                                                                                    device=dev())
    net.unpack_output(to_dev(out, torch.float32), nm, du, dW)
    ru, rW = nn.net_state(cf(out.astype(np.float64), n), mean_out, std_out)
    assert np.allclose(du.cpu().numpy(), ru, rtol=1e-6, atol=1e-6)
    assert np.allclose(dW.cpu().numpy(), rW, rtol=1e-6, atol=1e-6)
    s, s2 = net.moments(T(S))
    assert s == pytest.approx(S.sum(), rel=1e-12, abs=1e-12)
    assert s2 == pytest.approx((S ** 2).sum(), rel=1e-12)
    s, s2 = net.moments(T(rho5), T(rho1))
    assert s == pytest.approx((rho5 + rho1).sum(), rel=1e-12)
    assert s2 == pytest.approx(((rho5 + rho1) ** 2).sum(), rel=1e-12)


def test_forward_is_shift_equivariant_at_full_size():
    """At the 128^3 training size: rolling the input by a multiple of the
    coarsest spacing rolls the output exactly (periodic network, identical
    per-cell arithmetic)."""
    cfg, gc = small_cfg(128, 4, (16, 32, 48, 64))
    p, _, _ = net_inputs(nn.NetConfig(n=8, levels=4, ch=(16, 32, 48, 64)), 9)
    net = gn.Net(gc, training=False)
    net.load(to_dev(p, torch.float32))
    x = torch.randn((8, 128, 128, 128), generator=torch.Generator().manual_seed(1)).to(torch.bfloat16)
    x[4:] = 0
    xd = x.permute(1, 2, 3, 0).contiguous().reshape(-1, 8).to(dev())
    y0 = net.forward(xd).reshape(128, 128, 128, 4).clone()
    xs = torch.roll(x, shifts=(8, 16, 24), dims=(1, 2, 3)).permute(1, 2, 3, 0).contiguous().reshape(-1, 8).to(dev())
    y1 = net.forward(xs).reshape(128, 128, 128, 4)
    assert torch.equal(torch.roll(y0, shifts=(8, 16, 24), dims=(0, 1, 2)), y1)
    assert torch.isfinite(y0).all()


def test_training_steps_reduce_the_loss():
    cfg, gc = small_cfg(16, 3, (16, 32, 48))
    p, x, _ = net_inputs(cfg, 12)
    t = bf(np.stack([np.sin(2 * np.pi * np.arange(16) / 16)[:, None, None] * np.ones((16, 16, 16))] * 4) * 0.5)
    net = gn.Net(gc, training=True)
    params = to_dev(p, torch.float32)
    net.load(params)
    m, v = torch.zeros_like(params), torch.zeros_like(params)
    xd, td = gpu_x(x), to_dev(cl(t), torch.bfloat16)
    losses = []
    for step in range(1, 31):
        grad = torch.zeros_like(params)
        out = net.forward(xd)
        losses.append(net.mse(out, td))
        net.backward(grad)
        net.adam(params, grad, m, v, step, lr=1e-3)
    print("training losses", [f"{q:.4f}" for q in losses[::5]])
    assert np.isfinite(losses).all() and losses[-1] < 0.7 * losses[0]


def test_warm_start_falls_back_on_a_bad_prediction():
    w = synth.coupled(32, seed=3, precision=g.PREC_FP32_IR, levels=4)
    from gpu_helpers import gparams
    p = gparams(w, 0.0)
    r5, r1, S, p.K = g.scalar_field_sources(p, w.phi_modes, w.pi_modes, w.scalar_mass, dev())
    s = g.Solver(p, r5, r1, S)
    cfg, gc = small_cfg(32, 4, (16, 32, 48, 64))
    net = gn.Net(gc, training=False)
    # weights scaled far beyond their initialisation: a useless prediction
    bad = synth.nn_init(nn.layer_shapes(cfg), seed=1) * 50.0
    net.load(to_dev(bad, torch.float32))
    nm = gn.norm([1.0, 0, 0, 0], [1.0, 1, 1, 1], [0.0, 0, 0, 0], [1.0, 1, 1, 1])
    u = torch.empty((32, 32, 32), dtype=torch.float64, device=dev())
    W = torch.empty((3, 32, 32, 32), dtype=torch.float64, device=dev())
    used, norms = net.warm_start(s, r5, r1, S, nm, u, W)
    print("bad warm start norms", norms)
    assert not used
    assert not u.any() and not W.any()
    # the zero start's norms (evaluated beside the network) are those of the zero state
    with pytest.raises(g.MGError):  # the zeroed state is not the check iteration's
        s.solve(u, W, resume=True)
    zn = s.residual_norm(u, W)
    assert norms[2] == zn[0] and norms[3] == zn[1]
    rep = s.solve(u, W, tol=1e-10, max_outer=60)
    assert rep["h_rms"] <= 1e-10 and rep["m_rms"] <= 1e-10
