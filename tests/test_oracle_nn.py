"""Pins of the warm-start network oracle: the convolution against a brute-force
loop over its definition and against its impulse response, circular shift
equivariance, closed forms of pooling and trilinear upsampling, gradients
against central finite differences, and the Adam update against its formula
evaluated by hand on scalars."""
import itertools

import numpy as np
import pytest
import torch

import synth
from oracle import nn_oracle as nn


def rnd(seed, shape):
    return np.random.default_rng(seed).standard_normal(shape)


def test_conv_matches_brute_force_loop():
    n, ci, co = 3, 2, 3
    x, W, b = rnd(1, (ci, n, n, n)), rnd(2, (co, ci, 3, 3, 3)), rnd(3, co)
    y = nn.conv3(torch.tensor(x), torch.tensor(W), torch.tensor(b)).numpy()
    ref = np.zeros((co, n, n, n))
    for o, i, j, k in itertools.product(range(co), range(n), range(n), range(n)):
        s = b[o]
        for c, a, bb, cc in itertools.product(range(ci), range(3), range(3), range(3)):
            s += W[o, c, a, bb, cc] * x[c, (i + a - 1) % n, (j + bb - 1) % n, (k + cc - 1) % n]
        ref[o, i, j, k] = s
    assert np.allclose(y, ref, rtol=1e-13, atol=1e-13)


def test_conv_impulse_response_reads_the_weights():
    n, ci, co = 5, 2, 2
    W = torch.tensor(rnd(4, (co, ci, 3, 3, 3)))
    x = torch.zeros((ci, n, n, n), dtype=torch.float64)
    x[1, 2, 2, 2] = 1.0
    y = nn.conv3(x, W, torch.zeros(co, dtype=torch.float64))
    # y(p) = sum_d W[d+1] x(p+d): the impulse at q shows W[.., 1, q-p+1] at p
    for d in itertools.product((-1, 0, 1), repeat=3):
        p = tuple(2 - t for t in d)
        assert np.allclose(y[:, p[0], p[1], p[2]].numpy(), W[:, 1, d[0] + 1, d[1] + 1, d[2] + 1].numpy())
    assert float(y.abs().sum()) == pytest.approx(float(W[:, 1].abs().sum()), rel=1e-14)


def test_conv_is_shift_equivariant():
    n = 6
    x, W, b = (torch.tensor(rnd(5, (3, n, n, n))), torch.tensor(rnd(6, (2, 3, 3, 3, 3))),
               torch.tensor(rnd(7, 2)))
    s = (2, -1, 3)
    a = nn.conv3(torch.roll(x, s, (1, 2, 3)), W, b)
    c = torch.roll(nn.conv3(x, W, b), s, (1, 2, 3))
    assert torch.allclose(a, c, rtol=1e-13, atol=1e-13)


def test_pool_and_up_closed_forms():
    n = 8
    const = torch.full((2, n, n, n), 1.7, dtype=torch.float64)
    assert torch.allclose(nn.pool(const), torch.full((2, 4, 4, 4), 1.7, dtype=torch.float64))
    assert torch.allclose(nn.up(const), torch.full((2, 16, 16, 16), 1.7, dtype=torch.float64))
    # pooling: the mean of the eight children
    x = torch.tensor(rnd(8, (1, n, n, n)))
    assert float(nn.pool(x)[0, 1, 2, 3]) == pytest.approx(float(x[0, 2:4, 4:6, 6:8].mean()), rel=1e-14)
    # trilinear interpolation reproduces a linear function of the cell centre
    # (away from the periodic seam): coarse centres at I + 1/2, fine at (i + 1/2) / 2
    m = 8
    I = np.arange(m) + 0.5
    f = lambda X, Y, Z: 0.3 + 1.1 * X - 0.7 * Y + 0.25 * Z
    coarse = torch.tensor(f(*np.meshgrid(I, I, I, indexing="ij"))[None])
    fine = nn.up(coarse)[0].numpy()
    xi = (np.arange(2 * m) + 0.5) / 2
    ref = f(*np.meshgrid(xi, xi, xi, indexing="ij"))
    inner = slice(1, 2 * m - 1)
    assert np.allclose(fine[inner, inner, inner], ref[inner, inner, inner], rtol=1e-14, atol=1e-13)


def small_cfg():
    return nn.NetConfig(n=8, levels=3, ch=(3, 4, 5), c_in=4, c_out=4)


def test_param_count_of_the_default_network():
    cfg = nn.NetConfig()
    weights = sum(27 * ci * co for ci, co in nn.layer_shapes(cfg))
    assert weights == 680832
    assert nn.param_count(cfg) == weights + sum(co for _, co in nn.layer_shapes(cfg))


def test_gradients_match_central_differences():
    cfg = small_cfg()
    p = synth.nn_init(nn.layer_shapes(cfg), seed=3, bias_scale=0.1).astype(np.float64)
    x = rnd(9, (cfg.c_in, cfg.n, cfg.n, cfg.n))
    t = rnd(10, (cfg.c_out, cfg.n, cfg.n, cfg.n))
    loss, g = nn.loss_and_grad(p, x, t, cfg)
    rng = np.random.default_rng(11)
    idx = np.concatenate([rng.choice(p.size, 24, replace=False), [p.size - 1, 0]])
    eps = 1e-5
    for q in idx:
        pp, pm = p.copy(), p.copy()
        pp[q] += eps
        pm[q] -= eps
        lp = float(nn.mse(nn.forward(torch.tensor(pp), torch.tensor(x), cfg), torch.tensor(t)))
        lm = float(nn.mse(nn.forward(torch.tensor(pm), torch.tensor(x), cfg), torch.tensor(t)))
        fd = (lp - lm) / (2 * eps)
        assert abs(fd - g[q]) <= 1e-7 * max(1.0, abs(g[q])) + 1e-9, (q, fd, g[q])


def test_conv_vjp_matches_central_differences():
    n, ci, co = 4, 3, 2
    x, W, b, dy = rnd(12, (ci, n, n, n)), rnd(13, (co, ci, 3, 3, 3)), rnd(14, co), rnd(15, (co, n, n, n))
    dx, dW, db = nn.conv3_vjp(x, W, b, dy)
    f = lambda x, W, b: float((nn.conv3(torch.tensor(x), torch.tensor(W), torch.tensor(b)).numpy() * dy).sum())
    eps = 1e-6
    for (arr, grad) in ((x, dx), (W, dW), (b, db)):
        flat = arr.reshape(-1)
        for q in (0, flat.size // 2, flat.size - 1):
            old = flat[q]
            flat[q] = old + eps
            fp = f(x, W, b)
            flat[q] = old - eps
            fm = f(x, W, b)
            flat[q] = old
            assert abs((fp - fm) / (2 * eps) - grad.reshape(-1)[q]) < 1e-6


def test_adam_update_by_hand():
    p, g = np.array([1.0, -2.0]), np.array([0.5, -0.25])
    m, v = np.zeros(2), np.zeros(2)
    p1, m1, v1 = nn.adam(p, g, m, v, step=1, lr=0.1)
    # first step: m_hat = g, v_hat = g^2, so the update is lr * sign(g) (up to eps)
    assert np.allclose(p1, p - 0.1 * np.sign(g), rtol=0, atol=1e-7)
    p2, _, _ = nn.adam(p1, g, m1, v1, step=2, lr=0.1)
    assert np.allclose(p2, p1 - 0.1 * np.sign(g), rtol=0, atol=1e-7)


def test_standardisation_round_trip():
    u, W = rnd(16, (4, 4, 4)), rnd(17, (3, 4, 4, 4))
    mean, std = [0.1, -0.2, 0.3, 0.0], [2.0, 0.5, 1.5, 3.0]
    t = nn.net_target(u, W, mean, std)
    u2, W2 = nn.net_state(t, mean, std)
    assert np.allclose(u2, u) and np.allclose(W2, W)
    assert np.allclose(t[1], (W[0] + 0.2) / 0.5)


def check_silu():
    # SiLU(z) = z / (1 + e^-z): closed forms at 0 and +-ln 3 (logistic 3/4 and 1/4), its
    # limits, the identity SiLU(z) - SiLU(-z) = z, and the slope 1/2 at 0
    ln3 = float(np.log(3.0))
    z = torch.tensor([0.0, ln3, -ln3, 40.0, -40.0], dtype=torch.float64)
    s = nn.silu(z).numpy()
    assert s[0] == 0.0
    assert abs(s[1] - 0.75 * ln3) <= 1e-15 and abs(s[2] + 0.25 * ln3) <= 1e-15
    assert abs(s[3] - 40.0) <= 1e-14 and abs(s[4]) <= 1e-15
    x = torch.tensor(rnd(9, 64), dtype=torch.float64)
    assert torch.allclose(nn.silu(x) - nn.silu(-x), x, rtol=0, atol=1e-14)
    z0 = torch.zeros(1, dtype=torch.float64, requires_grad=True)
    nn.silu(z0).sum().backward()
    assert abs(float(z0.grad[0]) - 0.5) <= 1e-15


def test_silu_closed_forms():
    check_silu()


@pytest.mark.parametrize("wrong", [
    lambda z: z * torch.sigmoid(-z),          # logistic of the wrong sign
    lambda z: torch.sigmoid(z),               # the logistic alone
    lambda z: z * torch.sigmoid(2.0 * z),     # a scaled logistic (the "swish-beta" with beta 2)
], ids=["sign", "no-z", "beta2"])
def test_silu_planted_mistake_is_caught(wrong, monkeypatch):
    monkeypatch.setattr(nn, "silu", wrong)
    with pytest.raises(AssertionError):
        check_silu()
