"""Full-size parity: the 128^3 workloads in the launch configuration bench.py
times, compared at sampled cells with stored oracle results (written by
tests/golden/make_golden.py, which calls only the oracle), and the 256^3
puncture workload checked through properties (judge residuals at sampled
cells, Robin monopole fall-off, positivity)."""
import json
import os

import numpy as np
import pytest
import torch

import synth
from oracle import judge
from paper_2501_13046_amd import grtmg as g
from gpu_helpers import N, dev, gparams

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load(name):
    with open(os.path.join(GOLDEN, f"{name}.json")) as f:
        return json.load(f)


def gpu_sources(w):
    p = gparams(w)
    if w.shell is not None:
        rho5, rho1, S = g.shell_field_sources(p, w.shell["amplitude"], w.shell["r0"],
                                              w.shell["width2"], w.scalar_mass, dev())
        return rho5, rho1, S, 0.0
    return g.scalar_field_sources(p, w.phi_modes, w.pi_modes, w.scalar_mass, dev())


def sampled_hamiltonian(w, K, u, W, rho5, rho1, cells):
    gr = judge.Grid(w.n, w.length, w.bc, w.origin, w.puncture_pos)
    return judge.hamiltonian_at(gr, u, W, rho5, rho1, K, cells, w.puncture_mass,
                                conformal_matter=w.conformal_matter)


@pytest.mark.parametrize("precision", [g.PREC_FP32_IR, g.PREC_FP64])
def test_coupled_128_matches_oracle(precision):
    gold = load("coupled_128")
    w = synth.coupled_128(seed=0, precision=precision)
    rho5, rho1, S, K = gpu_sources(w)
    assert abs(K - gold["K"]) <= 1e-13 * gold["K"]
    s = g.Solver(gparams(w, K), rho5, rho1, S)
    n = w.n
    u = torch.zeros((n,) * 3, dtype=torch.float64, device=dev())
    W = torch.zeros((3, n, n, n), dtype=torch.float64, device=dev())
    rep = s.solve(u, W, tol=1e-10, max_outer=60)
    cells = np.asarray(gold["cells"])
    i, j, k = cells[:, 0], cells[:, 1], cells[:, 2]
    un = N(u)
    uo = np.asarray(gold["u"])
    err = np.max(np.abs(un[i, j, k] - uo) / np.abs(1.0 + uo))
    Wn = N(W)
    Wn -= Wn.mean(axis=(1, 2, 3), keepdims=True)
    werr = max(np.max(np.abs(Wn[a][i, j, k] - np.asarray(gold["W_meanfree"][a]))) for a in range(3))
    H = sampled_hamiltonian(w, K, un, N(W), N(rho5), N(rho1), cells)
    print(f"coupled_128 prec={precision}: iters={rep['outer_iters']} (oracle {gold['outer_iters']} "
          f"to 1e-11) psi_err={err:.2e} W_err={werr:.2e} rms H={rep['h_rms']:.2e} "
          f"rms M={rep['m_rms']:.2e} sampled |H|max={np.abs(H).max():.2e}")
    assert rep["h_rms"] <= 1e-10 and rep["m_rms"] <= 1e-10
    assert err < 1e-9
    assert werr < 1e-9
    # sampled judge residual: consistent with an RMS of 1e-10
    assert np.sqrt(np.mean(H ** 2)) < 3e-10


def test_puncture_shell_128_matches_oracle():
    gold = load("puncture_shell_128")
    w = synth.puncture_shell(128, precision=g.PREC_FP32_IR, levels=6)
    rho5, rho1, S, K = gpu_sources(w)
    s = g.Solver(gparams(w, K), rho5, rho1)
    n = w.n
    u = torch.zeros((n,) * 3, dtype=torch.float64, device=dev())
    rep10 = s.solve(u, None, tol=1e-10, max_outer=60)
    assert rep10["h_rms"] <= 1e-10
    cells = np.asarray(gold["cells"])
    i, j, k = cells[:, 0], cells[:, 1], cells[:, 2]
    gr = judge.Grid(n, w.length, w.bc, w.origin, w.puncture_pos)
    psi0 = judge.psi0(gr, w.puncture_mass)[i, j, k]
    uo = np.asarray(gold["u"])
    err10 = np.max(np.abs(N(u)[i, j, k] - uo) / (psi0 + uo))
    # psi is compared after the GPU reaches 1e-12 and the oracle 1e-13 (the wide Robin
    # box has a lowest eigenvalue ~5e-3, so a residual bounds psi only to ~200 times it:
    # 1e-10 to ~2e-8, 1e-12 to ~2e-10)
    rep = s.solve(u, None, tol=1e-12, max_outer=60)
    err = np.max(np.abs(N(u)[i, j, k] - uo) / (psi0 + uo))
    print(f"puncture_shell_128: psi error vs oracle {err10:.2e} at rms H {rep10['h_rms']:.2e} "
          f"({rep10['outer_iters']} iterations), {err:.2e} at rms H {rep['h_rms']:.2e} "
          f"(+{rep['outer_iters']} iterations; oracle {gold['outer_iters']} to {gold['tol']:.0e})")
    assert gold["tol"] <= 1e-13
    assert rep["h_rms"] <= 1e-12
    assert err < 1e-9


def test_puncture_shell_256_properties():
    w = synth.puncture_shell(256, precision=g.PREC_FP32_IR, levels=6)
    rho5, rho1, S, K = gpu_sources(w)
    s = g.Solver(gparams(w, K), rho5, rho1)
    n = w.n
    u = torch.zeros((n,) * 3, dtype=torch.float64, device=dev())
    rep = s.solve(u, None, tol=1e-10, max_outer=60)
    un = N(u)
    rng = np.random.default_rng(256)
    cells = rng.integers(0, n, size=(4096, 3))
    cells[:4] = [[0, 0, 0], [n - 1, n - 1, n - 1], [n // 2, n // 2, n // 2], [n // 2 - 1, n // 2, n // 2]]
    H = sampled_hamiltonian(w, K, un, None, N(rho5), N(rho1), cells)
    print(f"puncture_shell_256: iters={rep['outer_iters']} rms H={rep['h_rms']:.2e} "
          f"sampled rms H={np.sqrt(np.mean(H ** 2)):.2e} u range [{un.min():.3e}, {un.max():.3e}]")
    assert rep["h_rms"] <= 1e-10
    assert np.sqrt(np.mean(H ** 2)) < 3e-10
    # positive matter density raises psi: u > 0 everywhere, and decays ~1/r outside the shell
    assert un.min() > 0.0
    gr = judge.Grid(n, w.length, w.bc, w.origin, w.puncture_pos)
    r = gr.radius()
    far = r > 20.0
    q = un[far] * r[far]
    assert q.std() / q.mean() < 0.05
