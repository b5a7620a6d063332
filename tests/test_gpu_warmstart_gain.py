"""What the trained warm-start network gains over the zero start, on held-out
seeds of the 128^3 coupled workload (seeds 10000+; training used 0-1999):
fewer outer iterations (the one iteration spent by the fallback comparison
included), the same final residual, and the same solution as the zero start
(psi within 1e-9 relative, W mean-free within 1e-9).  The zero-start solve of
this workload is compared with the oracle in test_gpu_fullsize."""
import os

import numpy as np
import pytest
import torch

from paper_2501_13046_amd import grtnn as gn
from paper_2501_13046_amd import warmstart as ws
from gpu_helpers import N, dev

pytestmark = pytest.mark.gpu
WEIGHTS = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2501_13046_amd",
                       "weights", "warmstart_128.npz")


def test_trained_warm_start_cuts_outer_iterations():
    cfg, nm, params, meta = ws.load(WEIGHTS, dev())
    assert cfg.n == 128 and meta["train_seeds"] >= 2000
    net = gn.Net(cfg, training=False, device=dev())
    net.load(params)
    rows = []
    for seed in range(10000, 10004):
        p, r5, r1, S = ws.problem(seed, 128, dev())
        _, u0, W0, r0 = ws.solve(p, r5, r1, S)
        s = ws.g.Solver(p, r5, r1, S)
        u = torch.empty_like(u0)
        W = torch.empty_like(W0)
        used, norms = net.warm_start(s, r5, r1, S, nm, u, W)
        # odd seeds continue from the check iteration's state, even ones evaluate it again
        r = s.solve(u, W, tol=1e-10, max_outer=100, resume=used and seed % 2 == 1)
        psi_err = float(torch.max(torch.abs(u - u0) / (1.0 + u0)))
        Wm = W - W.mean(dim=(1, 2, 3), keepdim=True)
        W0m = W0 - W0.mean(dim=(1, 2, 3), keepdim=True)
        w_err = float(torch.max(torch.abs(Wm - W0m)))
        rows.append((r0["outer_iters"], r["outer_iters"] + 1, used, psi_err, w_err, r["h_rms"], r["m_rms"]))
        print(f"seed {seed}: zero start {r0['outer_iters']} iterations, warm start {r['outer_iters']} + 1 "
              f"(used {used}; residual after the first iteration H {norms[0]:.2e} vs zero start {norms[2]:.2e}); "
              f"psi diff {psi_err:.1e}, W diff {w_err:.1e}")
        assert r["h_rms"] <= 1e-10 and r["m_rms"] <= 1e-10
        assert psi_err < 1e-9 and w_err < 1e-9
    zero = np.mean([q[0] for q in rows])
    warm = np.mean([q[1] for q in rows])
    print(f"mean outer iterations: zero start {zero:.2f}, warm start {warm:.2f}")
    assert all(q[2] for q in rows)
    assert warm < zero
