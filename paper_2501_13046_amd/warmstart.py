"""Learned warm start: training data from the solver, training and evaluation.

The paper starts every solve from psi = 1, W = 0.  Here a U-Net (grtnn.h)
predicts (u, W) from the sources; the multigrid solve always finishes the job.

* Data: for every seed a periodic coupled problem (scalar-field sources with
  8 Fourier modes of amplitude 0.05 in phi and 0.02 in Pi, 128^3 by default) is
  solved to RMS residual 1e-10 with the mixed-precision multigrid.  Its sources
  become the standardised BF16 input (rho5 + rho1, S_a) and its solution the
  standardised BF16 target (u, W_a), both kept resident in HBM.
* Training: per-sample forward, MSE, backward (gradients summed over a
  minibatch), Adam on FP32 master weights with a cosine learning rate; every
  step runs in the library's kernels.
* Evaluation: held-out seeds solved from the zero start and from the warm
  start (with the library's fallback); outer iterations (one V-cycle per
  equation each) and wall time are compared.

Run as a module: python -m paper_2501_13046_amd.warmstart --help
"""
from __future__ import annotations

import argparse
import json
import math
import time
from typing import List, Optional

import numpy as np
import torch

import synth
from . import grtmg as g
from . import grtnn as gn


def problem(seed: int, n: int, device, phi_amp: float = 0.05):
    """Solver params and sources of the coupled periodic problem of a seed."""
    w = synth.coupled(n, seed=seed, phi_amp=phi_amp, precision=g.PREC_FP32_IR)
    p = g.params(w.n, w.levels, w.bc, w.precision, w.length, w.origin, 0.0, w.nu_pre, w.nu_post,
                 w.solve_momentum, w.puncture_mass, w.puncture_pos, w.conformal_matter,
                 nu_pre_W=w.nu_pre_W, nu_post_W=w.nu_post_W, cubic_prolong=w.cubic_prolong,
                 same_state=w.same_state)
    r5, r1, S, p.K = g.scalar_field_sources(p, w.phi_modes, w.pi_modes, w.scalar_mass, device)
    return p, r5, r1, S


def solve(p, r5, r1, S, u=None, W=None, tol=1e-10):
    n = p.n
    dev = r5.device
    if u is None:
        u = torch.zeros((n,) * 3, dtype=torch.float64, device=dev)
        W = torch.zeros((3, n, n, n), dtype=torch.float64, device=dev)
    s = g.Solver(p, r5, r1, S)
    rep = s.solve(u, W, tol=tol, max_outer=100)
    return s, u, W, rep


def statistics(seeds: List[int], n: int, device, net: gn.Net) -> gn.NnNorm:
    """Per-channel mean and standard deviation of inputs and targets over the
    given seeds (device moments of the FP64 fields)."""
    acc = np.zeros((8, 2))
    count = 0
    for sd in seeds:
        p, r5, r1, S = problem(sd, n, device)
        _, u, W, _ = solve(p, r5, r1, S)
        fields = [(r5, r1)] + [(S[a], None) for a in range(3)] + [(u, None)] + [(W[a], None) for a in range(3)]
        for c, (x, y) in enumerate(fields):
            acc[c] += net.moments(x.contiguous(), y)
        count += n ** 3
    mean = acc[:, 0] / count
    std = np.sqrt(np.maximum(acc[:, 1] / count - mean ** 2, 1e-300))
    return gn.norm(mean[:4], std[:4], mean[4:], std[4:])


def norm_to_dict(nm: gn.NnNorm) -> dict:
    return {k: [float(v) for v in getattr(nm, k)] for k in ("in_mean", "in_std", "out_mean", "out_std")}


def norm_from_dict(d: dict) -> gn.NnNorm:
    return gn.norm(d["in_mean"], d["in_std"], d["out_mean"], d["out_std"])


def generate(seeds: List[int], n: int, device, net: gn.Net, nm: gn.NnNorm, log=print):
    """Dataset resident on the device: X [S, n^3, 8] and Y [S, n^3, 4], BF16."""
    V = n ** 3
    X = torch.empty((len(seeds), V, 8), dtype=torch.bfloat16, device=device)
    Y = torch.empty((len(seeds), V, 4), dtype=torch.bfloat16, device=device)
    iters = []
    t0 = time.time()
    for q, sd in enumerate(seeds):
        p, r5, r1, S = problem(sd, n, device)
        _, u, W, rep = solve(p, r5, r1, S)
        iters.append(rep["outer_iters"])
        net.pack_input(r5, r1, S, nm, X[q])
        net.pack_target(u, W, nm, Y[q])
        if (q + 1) % 100 == 0 or q + 1 == len(seeds):
            torch.cuda.synchronize(device)
            log(f"data {q + 1}/{len(seeds)} solves, {time.time() - t0:.1f} s, mean iters {np.mean(iters):.2f}")
    return X, Y, iters


def train(net: gn.Net, params: torch.Tensor, X: torch.Tensor, Y: torch.Tensor, epochs: float, batch: int,
          lr: float, lr_min: float, seed: int = 0, log=print, log_every: float = 30.0,
          time_limit: Optional[float] = None):
    """Adam with a cosine learning rate over epochs x samples / batch steps."""
    S = X.shape[0]
    steps = max(1, int(math.ceil(epochs * S / batch)))
    m = torch.zeros_like(params)
    v = torch.zeros_like(params)
    grad = torch.zeros_like(params)
    out = torch.empty((X.shape[1], 4), dtype=torch.float32, device=X.device)
    rng = np.random.default_rng(seed)
    order = np.concatenate([rng.permutation(S) for _ in range(int(math.ceil(epochs)) + 1)])
    losses = []
    t0 = last = time.time()
    k = 0
    for step in range(1, steps + 1):
        grad.zero_()
        ls = 0.0
        for _ in range(batch):
            q = int(order[k])
            k += 1
            net.forward(X[q], out)
            ls += net.mse(out, Y[q])
            net.backward(grad)
        lr_t = lr_min + 0.5 * (lr - lr_min) * (1.0 + math.cos(math.pi * (step - 1) / steps))
        net.adam(params, grad, m, v, step, lr_t, grad_scale=1.0 / batch)
        losses.append(ls / batch)
        now = time.time()
        if now - last > log_every or step == steps:
            last = now
            log(f"train step {step}/{steps} loss {np.mean(losses[-20:]):.5f} lr {lr_t:.2e} "
                f"{now - t0:.1f} s")
        if time_limit is not None and now - t0 > time_limit:
            log(f"train: time limit reached after {step} steps")
            break
    return losses


def evaluate(net: gn.Net, nm: gn.NnNorm, seeds: List[int], n: int, device, log=print):
    """Outer iterations and times from the zero start and from the warm start."""
    rows = []
    for sd in seeds:
        p, r5, r1, S = problem(sd, n, device)
        s = g.Solver(p, r5, r1, S)
        u = torch.zeros((n,) * 3, dtype=torch.float64, device=device)
        W = torch.zeros((3, n, n, n), dtype=torch.float64, device=device)
        s.solve(u, W, tol=1e-10, max_outer=100)  # warm-up of the graph
        u.zero_()
        W.zero_()
        net.warm_start(s, r5, r1, S, nm, u, W)  # warm-up of the network
        u.zero_()
        W.zero_()
        torch.cuda.synchronize(device)
        t0 = time.perf_counter()
        r0 = s.solve(u, W, tol=1e-10, max_outer=100)
        torch.cuda.synchronize(device)
        t_zero = time.perf_counter() - t0
        t0 = time.perf_counter()
        used, norms = net.warm_start(s, r5, r1, S, nm, u, W)
        r1_ = s.solve(u, W, tol=1e-10, max_outer=100)
        torch.cuda.synchronize(device)
        t_warm = time.perf_counter() - t0
        # the warm start applies one outer iteration itself
        rows.append(dict(seed=sd, iters_zero=r0["outer_iters"], iters_warm=r1_["outer_iters"] + 1, used=used,
                         h0_pred=norms[0], m0_pred=norms[1], h0_zero=norms[2], m0_zero=norms[3],
                         t_zero=t_zero, t_warm=t_warm, h_rms=r1_["h_rms"], m_rms=r1_["m_rms"]))
    iz = np.mean([r["iters_zero"] for r in rows])
    iw = np.mean([r["iters_warm"] for r in rows])
    tz = np.median([r["t_zero"] for r in rows])
    tw = np.median([r["t_warm"] for r in rows])
    log(f"eval {len(rows)} seeds: outer iterations zero {iz:.2f} warm {iw:.2f}; median time zero "
        f"{tz * 1e3:.2f} ms warm {tw * 1e3:.2f} ms; warm start used {sum(r['used'] for r in rows)}")
    return rows


def fmg_learned_start(net: gn.Net, nm: gn.NnNorm, coarse: g.Solver, fine: g.Solver, r5c, r1c, Sc, uc, Wc, uf, Wf,
                      tol_c: float, max_outer: int = 100, keep_ratio: float = None):
    """Full-multigrid start with a learned coarse start: the network (trained on the
    coarse problem) predicts (u, W) on the coarse grid, one coarse outer iteration
    checks it against the zero start (the library's fallback rule; keep_ratio: the zero
    start's one-iteration contraction, for the like-with-like form), the coarse solve
    continues to tol_c, and the cubic interpolation fills the fine arrays.  Returns
    (prediction kept, coarse report of the continued solve)."""
    used, _ = net.warm_start(coarse, r5c, r1c, Sc, nm, uc, Wc, keep_ratio)
    if not used:
        return used, g.fmg_start(coarse, fine, uc, Wc, uf, Wf, tol=tol_c, max_outer=max_outer)
    # a kept prediction continues from its check iteration's state (not evaluated again),
    # then the same cubic interpolation as the full-multigrid start
    rc = coarse.solve(uc, Wc, tol=tol_c, max_outer=max_outer, raise_on_failure=False, resume=True)
    if rc["status"] not in (g.MG_OK, g.MG_ERR_NOT_CONVERGED):
        raise g.MGError(rc["status"], "coarse solve after the learned start")
    g.interp_cubic(coarse.p, uc, out=uf)
    for a in range(3):
        g.interp_cubic(coarse.p, Wc[a], out=Wf[a])
    return used, rc


def save(path: str, params: torch.Tensor, nm: gn.NnNorm, cfg: gn.NnConfig, meta: dict):
    np.savez(path, params=params.detach().cpu().numpy().astype(np.float32),
             norm=json.dumps(norm_to_dict(nm)),
             config=json.dumps(dict(n=cfg.n, levels=cfg.levels, ch=list(cfg.ch), c_in=cfg.c_in,
                                    c_out=cfg.c_out)),
             meta=json.dumps(meta))


def load(path: str, device):
    z = np.load(path, allow_pickle=False)
    c = json.loads(str(z["config"]))
    cfg = gn.config(c["n"], c["levels"], c["ch"], c["c_in"], c["c_out"])
    nm = norm_from_dict(json.loads(str(z["norm"])))
    params = torch.from_numpy(z["params"]).to(device)
    return cfg, nm, params, json.loads(str(z["meta"]))


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--n", type=int, default=128)
    ap.add_argument("--train-seeds", type=int, default=2000, help="seeds 0 .. count-1")
    ap.add_argument("--eval-seeds", type=int, default=20, help="seeds 10000 .. 10000+count-1")
    ap.add_argument("--stat-seeds", type=int, default=16)
    ap.add_argument("--epochs", type=float, default=2.0)
    ap.add_argument("--batch", type=int, default=4)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--lr-min", type=float, default=1e-5)
    ap.add_argument("--init", type=str, default=None, help="continue from saved weights")
    ap.add_argument("--out", type=str, required=True)
    ap.add_argument("--time-limit", type=float, default=None, help="seconds of training at most")
    a = ap.parse_args(argv)
    device = torch.device("cuda:0")
    log = lambda s: print(s, flush=True)
    cfg = gn.config(a.n)
    net = gn.Net(cfg, training=True, device=device)
    if a.init:
        _, nm, params, _ = load(a.init, device)
    else:
        nm = statistics(list(range(a.stat_seeds)), a.n, device, net)
        params = torch.from_numpy(synth.nn_init(gn.layer_shapes(cfg), seed=0)).to(device)
    log(f"norm {json.dumps(norm_to_dict(nm))}")
    net.load(params)
    X, Y, iters = generate(list(range(a.train_seeds)), a.n, device, net, nm, log)
    losses = train(net, params, X, Y, a.epochs, a.batch, a.lr, a.lr_min, log=log, time_limit=a.time_limit)
    del X, Y
    infer = gn.Net(cfg, training=False, device=device)
    infer.load(params)
    rows = evaluate(infer, nm, list(range(10000, 10000 + a.eval_seeds)), a.n, device, log)
    save(a.out, params, nm, cfg, dict(train_seeds=a.train_seeds, epochs=a.epochs, batch=a.batch, lr=a.lr,
                                      final_loss=float(np.mean(losses[-20:])), eval=rows))
    log(f"saved {a.out}")


if __name__ == "__main__":
    main()
