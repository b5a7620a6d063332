"""Shared helpers of the GPU parity tests: seeded inputs on both sides."""
import numpy as np
import torch

import oracle
import synth
from paper_2501_13046_amd import grtmg as g


def dev():
    return torch.device("cuda:0")


def T(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device=dev(), dtype=dtype)


def N(t):
    return t.detach().to("cpu", torch.float64).numpy()


def gparams(w, K=0.0, precision=None, levels=None):
    return g.params(w.n, levels if levels is not None else w.levels, w.bc,
                    w.precision if precision is None else precision, w.length, w.origin, K,
                    w.nu_pre, w.nu_post, w.solve_momentum, w.puncture_mass, w.puncture_pos,
                    w.conformal_matter, nu_pre_W=w.nu_pre_W, nu_post_W=w.nu_post_W,
                    cubic_prolong=w.cubic_prolong, same_state=w.same_state)


def oracle_problem(w):
    """Oracle sources, K and params for a workload (the inputs both sides use)."""
    rho5, rho1, S, K = oracle.sources_for(w)
    return rho5, rho1, S, K, oracle.params_from_workload(w, K)


def rel_err(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def psi_rel_err(u_gpu, u_orc, psi0=1.0):
    pg = psi0 + u_gpu
    po = psi0 + u_orc
    return float(np.max(np.abs(pg - po) / np.abs(po)))


def mean_free(W):
    return W - W.mean(axis=(1, 2, 3), keepdims=True)


def random_state(n, seed, u_amp=0.05, w_amp=0.02):
    u = synth.uniform_random(seed, (n, n, n), -u_amp, u_amp)
    W = synth.uniform_random(seed + 1, (3, n, n, n), -w_amp, w_amp)
    return u, W
