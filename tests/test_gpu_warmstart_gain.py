"""What the trained warm-start networks gain over the zero start, on held-out
seeds of the 128^3 coupled workload (seeds 10000+; training used 0-1999).  The
network at 128^3: its prediction passes the fallback's bar (the zero state's residual),
and the solve from it reaches the same final residual and the same solution as the
zero start (psi within 1e-9 relative, W mean-free within 1e-9).  The network at 64^3
as the coarse start of the full-multigrid start: fewer coarse iterations.  Neither
saves time against the multigrid as it now converges (printed, not asserted).  The
zero-start solve of this workload is compared with the oracle in test_gpu_fullsize."""
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
WEIGHTS_64 = os.path.join(os.path.dirname(WEIGHTS), "warmstart_64.npz")


def test_trained_warm_start_reaches_the_zero_start_solution():
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


def _event_ms(fn):
    """Device time of fn() on the current stream (HIP events), in ms."""
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record()
    out = fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b), out


def test_learned_coarse_start_on_held_out_seeds():
    """The network trained on the 64^3 problem as the coarse start of the full-multigrid
    start of the 128^3 solve: on held-out seeds its prediction is kept, the coarse solve
    needs fewer iterations (its check iteration counted), and the 128^3 solution is the
    same.  The time it saves against the same start from zero is measured and printed:
    with cubic correction prolongation and V(2,2) cycles the start from zero needs 3
    coarse iterations and the learned start no longer saves time (the fine solve after it
    takes one iteration more)."""
    from paper_2501_13046_amd import grtmg as g
    import synth
    cfg, nm, params, meta = ws.load(WEIGHTS_64, dev())
    assert cfg.n == 64 and meta["train_seeds"] >= 2000
    net = gn.Net(cfg, training=False, device=dev())
    net.load(params)
    saved, its = [], []
    for seed in range(10000, 10004):
        pf, r5, r1, S = ws.problem(seed, 128, dev())
        wc = synth.coupled(64, seed=seed, precision=g.PREC_FP32_IR)
        pc = g.params(64, wc.levels, wc.bc, g.PREC_FP32_IR, wc.length, wc.origin, pf.K, wc.nu_pre, wc.nu_post, True,
                      nu_pre_W=wc.nu_pre_W, nu_post_W=wc.nu_post_W, cubic_prolong=wc.cubic_prolong,
                      same_state=wc.same_state)
        r5c, r1c, Sc, _ = g.scalar_field_sources(pc, wc.phi_modes, wc.pi_modes, wc.scalar_mass, dev())
        fine, coarse = g.Solver(pf, r5, r1, S), g.Solver(pc, r5c, r1c, Sc)
        z = lambda n: torch.zeros((n,) * 3, dtype=torch.float64, device=dev())
        zw = lambda n: torch.zeros((3, n, n, n), dtype=torch.float64, device=dev())
        uc, Wc, uf, Wf = z(64), zw(64), z(128), zw(128)
        tol_c = g.fmg_coarse_tol(coarse, fine, uc, Wc, uf, Wf)
        ratio = g.zero_start_contraction(coarse, uc, Wc)  # the like-with-like fallback's bar

        def plain():
            uc.zero_(); Wc.zero_()
            rc = g.fmg_start(coarse, fine, uc, Wc, uf, Wf, tol=tol_c)
            return rc, fine.solve(uf, Wf, tol=1e-10, max_outer=100)

        def learned():
            used, rc = ws.fmg_learned_start(net, nm, coarse, fine, r5c, r1c, Sc, uc, Wc, uf, Wf, tol_c,
                                            keep_ratio=ratio)
            return used, rc, fine.solve(uf, Wf, tol=1e-10, max_outer=100)

        plain(), learned()  # warm-up: graphs captured, kernels loaded
        t0 = []
        for _ in range(3):
            ms, (rc0, rf0) = _event_ms(plain)
            t0.append(ms)
        u0, W0 = uf.clone(), Wf.clone()
        t1 = []
        for _ in range(3):
            ms, (used, rc1, rf1) = _event_ms(learned)
            t1.append(ms)
        assert used and rf1["h_rms"] <= 1e-10 and rf1["m_rms"] <= 1e-10
        psi_err = float(torch.max(torch.abs(uf - u0) / (1.0 + u0)))
        assert psi_err < 1e-9
        saved.append(float(np.median(t0) - np.median(t1)))
        its.append((rc0["outer_iters"], rc1["outer_iters"] + 1, rf0["outer_iters"], rf1["outer_iters"]))
        print(f"seed {seed}: FMG from zero {np.median(t0):.3f} ms (coarse {rc0['outer_iters']} + fine "
              f"{rf0['outer_iters']}), learned coarse start {np.median(t1):.3f} ms (coarse {rc1['outer_iters']} + 1 "
              f"+ fine {rf1['outer_iters']}); psi diff {psi_err:.1e}", flush=True)
        fine.close()
        coarse.close()
    print(f"time saved per solve (median over seeds): {np.median(saved):.3f} ms")
    assert all(c1 < c0 for c0, c1, _, _ in its)  # the check iteration counted


def test_fallback_compares_with_one_zero_start_iteration():
    """The like-with-like fallback (nn_warm_start_ratio): the prediction is kept only if,
    after its check iteration, it beats what one outer iteration from the zero start
    achieves (keep_ratio = that iteration's measured contraction); an unreachable bar
    falls back to the zero state, and a bar outside (0, 1] is refused."""
    from paper_2501_13046_amd import grtmg as g
    import synth
    cfg, nm, params, meta = ws.load(WEIGHTS_64, dev())
    net = gn.Net(cfg, training=False, device=dev())
    net.load(params)
    seed = 10005
    pf, _, _, _ = ws.problem(seed, 128, dev())
    wc = synth.coupled(64, seed=seed, precision=g.PREC_FP32_IR)
    pc = g.params(64, wc.levels, wc.bc, g.PREC_FP32_IR, wc.length, wc.origin, pf.K, wc.nu_pre, wc.nu_post, True,
                  nu_pre_W=wc.nu_pre_W, nu_post_W=wc.nu_post_W, cubic_prolong=wc.cubic_prolong,
                  same_state=wc.same_state)
    r5c, r1c, Sc, _ = g.scalar_field_sources(pc, wc.phi_modes, wc.pi_modes, wc.scalar_mass, dev())
    coarse = g.Solver(pc, r5c, r1c, Sc)
    uc = torch.zeros((64,) * 3, dtype=torch.float64, device=dev())
    Wc = torch.zeros((3, 64, 64, 64), dtype=torch.float64, device=dev())
    ratio = g.zero_start_contraction(coarse, uc, Wc)
    used, norms = net.warm_start(coarse, r5c, r1c, Sc, nm, uc, Wc, keep_ratio=ratio)
    pred, zero = max(norms[0], norms[1]), max(norms[2], norms[3])
    print(f"zero-start contraction {ratio:.3f}; prediction after its check iteration {pred / zero:.4f} of the "
          f"zero state")
    assert 0.0 < ratio < 1.0
    assert used and pred < ratio * zero
    used, _ = net.warm_start(coarse, r5c, r1c, Sc, nm, uc, Wc, keep_ratio=1e-9)
    assert not used and not uc.any() and not Wc.any()
    with pytest.raises(gn.MGError):
        net.warm_start(coarse, r5c, r1c, Sc, nm, uc, Wc, keep_ratio=1.5)
    coarse.close()
