"""Two-level static mesh refinement on the HIP path (Key features, "Adaptive Mesh
Refinement" and "Fast"): one composite iteration element by element against the
oracle (FP64), converged composite solves against the oracle's (FP64 and FP32
V-cycles in FP64 refinement), and the full-size pair (128^3 base, 128^3 box)
against the oracle's composite residual."""
import numpy as np
import pytest
import torch

import oracle
import synth
from oracle import refine
from paper_2501_13046_amd import grtmg as g
from gpu_helpers import N, T, dev, rel_err

pytestmark = pytest.mark.gpu


def pair(nc, m, lc, lf, precision):
    """Base grid of the isolated black hole with a scalar shell (the 64 M box, Robin
    rule) and a box of m^3 base cells refined by 2 around the puncture."""
    w = synth.puncture_shell(nc, precision=precision, levels=lc)
    b0 = (nc - m) // 2
    pb = g.params(nc, lc, w.bc, precision, w.length, w.origin, 0.0, w.nu_pre, w.nu_post, False, w.puncture_mass,
                  w.puncture_pos, True, cubic_prolong=w.cubic_prolong)
    px = g.box_params(pb, b0, m, lf)
    pbo = oracle.params_from_workload(w)
    h = w.length / nc
    pxo = oracle.params(2 * m, levels=lf, bc=oracle.BC_ZERO, length=m * h,
                        origin=tuple(w.origin[a] + b0 * h for a in range(3)), nu_pre=w.nu_pre, nu_post=w.nu_post,
                        puncture_mass=w.puncture_mass, puncture_pos=w.puncture_pos, conformal_matter=True,
                        cubic_prolong=w.cubic_prolong)
    sh = w.shell
    rc5, rc1, _ = oracle.shell_sources(pbo, sh["amplitude"], sh["r0"], sh["width2"], w.scalar_mass)
    rf5, rf1, _ = oracle.shell_sources(pxo, sh["amplitude"], sh["r0"], sh["width2"], w.scalar_mass)
    prob = refine.Problem(pbo, pxo, b0, rc5, rc1, rf5, rf1)
    keep = [T(rc5), T(rc1), torch.zeros((nc,) * 3, dtype=torch.float64, device=dev()),
            T(rf5), T(rf1), torch.zeros((2 * m,) * 3, dtype=torch.float64, device=dev())]
    sb = g.Solver(pb, keep[0], keep[1], None, keep[2])
    sx = g.Solver(px, keep[3], keep[4], None, keep[5])
    return prob, sb, sx, b0, keep


def test_one_composite_iteration_matches_oracle():
    nc, m = 24, 8
    prob, sb, sx, b0, _ = pair(nc, m, 3, 3, g.PREC_FP64)
    uc0 = 0.01 * synth.uniform_random(3, (nc,) * 3)
    uf0 = 0.01 * synth.uniform_random(4, (2 * m,) * 3)
    uc, uf = T(uc0), T(uf0)
    rep = g.refine_solve(sb, sx, b0, uc, uf, tol=1e-300, max_outer=1, raise_on_failure=False)
    assert rep["status"] == g.MG_ERR_NOT_CONVERGED and rep["outer_iters"] == 1
    uco, ufo = uc0.copy(), uf0.copy()
    it, hist, st = refine.solve(prob, uco, ufo, tol=1e-300, max_outer=1)
    assert it == 1
    # the composite norm of the start and of the result, and the fields themselves
    assert abs(rep["history"][0][0] - hist[0][0]) <= 1e-12 * hist[0][0]
    assert abs(rep["history"][1][0] - hist[1][0]) <= 1e-10 * hist[1][0]
    assert rel_err(N(uf), ufo) < 1e-11
    assert rel_err(N(uc), uco) < 1e-11


@pytest.mark.parametrize("precision", [g.PREC_FP64, g.PREC_FP32_IR])
def test_composite_solve_matches_oracle(precision):
    nc, m = 32, 16
    prob, sb, sx, b0, _ = pair(nc, m, 4, 4, precision)
    uc = torch.zeros((nc,) * 3, dtype=torch.float64, device=dev())
    uf = torch.zeros((2 * m,) * 3, dtype=torch.float64, device=dev())
    rep = g.refine_solve(sb, sx, b0, uc, uf, tol=1e-11, max_outer=60)
    uco, ufo = np.zeros((nc,) * 3), np.zeros((2 * m,) * 3)
    it, hist, st = refine.solve(prob, uco, ufo, tol=1e-11, max_outer=60)
    assert st == 0
    print(f"refine prec={precision}: {rep['outer_iters']} iterations (oracle {it}), rms {rep['h_rms']:.2e}")
    assert np.abs(N(uf) - ufo).max() <= 1e-9 * (1.0 + np.abs(ufo).max())
    assert np.abs(N(uc) - uco).max() <= 1e-9 * (1.0 + np.abs(uco).max())


def test_composite_solve_128_full_size():
    """Base 128^3 (h = 0.5) and a box of 64^3 base cells refined to 128^3 (h = 0.25)
    around the puncture, FP32 V-cycles in FP64 refinement: the oracle's composite
    residual of the result is below the tolerance."""
    nc, m = 128, 64
    prob, sb, sx, b0, _ = pair(nc, m, 6, 6, g.PREC_FP32_IR)
    uc = torch.zeros((nc,) * 3, dtype=torch.float64, device=dev())
    uf = torch.zeros((2 * m,) * 3, dtype=torch.float64, device=dev())
    rep = g.refine_solve(sb, sx, b0, uc, uf, tol=1e-10, max_outer=40)
    Hf, Hc, _ = prob.residuals(N(uc), N(uf))
    rms, mx = prob.norm(Hf, Hc)
    print(f"refine 128+128: {rep['outer_iters']} iterations, {rep['seconds'] * 1e3:.1f} ms, oracle composite rms "
          f"{rms:.2e} (GPU {rep['h_rms']:.2e})")
    assert rms <= 1.01e-10
    assert abs(rms - rep["h_rms"]) <= 1e-3 * rms + 1e-14


def test_refine_rejects_bad_geometry():
    nc, m = 24, 8
    prob, sb, sx, b0, keep = pair(nc, m, 3, 3, g.PREC_FP64)
    uc = torch.zeros((nc,) * 3, dtype=torch.float64, device=dev())
    uf = torch.zeros((2 * m,) * 3, dtype=torch.float64, device=dev())
    for bad_b0 in (2, nc - m - 2):  # margin below 3 base cells
        with pytest.raises(g.MGError):
            g.refine_solve(sb, sx, bad_b0, uc, uf, max_outer=1)
    with pytest.raises(g.MGError):  # the base grid as its own box
        g.refine_solve(sb, sb, b0, uc, uc, max_outer=1)


def nested(nc, boxes, levels, precision):
    """The black hole of the 64 M box on a base grid of nc^3 with nested boxes (m, b)
    around the puncture, on both sides."""
    w = synth.puncture_shell(nc, precision=precision, levels=levels[0])
    pb = g.params(nc, levels[0], w.bc, precision, w.length, w.origin, 0.0, w.nu_pre, w.nu_post, False,
                  w.puncture_mass, w.puncture_pos, True, cubic_prolong=w.cubic_prolong)
    ps, pos = [pb], [oracle.params_from_workload(w)]
    offs = [0]
    for (m, b), lv in zip(boxes, levels[1:]):
        ps.append(g.box_params(ps[-1], b, m, lv))
        q = ps[-1]
        pos.append(oracle.params(q.n, levels=lv, bc=oracle.BC_ZERO, length=q.length, origin=tuple(q.origin),
                                 nu_pre=w.nu_pre, nu_post=w.nu_post, puncture_mass=w.puncture_mass,
                                 puncture_pos=w.puncture_pos, conformal_matter=True,
                                 cubic_prolong=w.cubic_prolong))
        offs.append(b)
    sh = w.shell
    src = [oracle.shell_sources(po, sh["amplitude"], sh["r0"], sh["width2"], w.scalar_mass) for po in pos]
    prob = refine.Nested(pos, offs, [q[0] for q in src], [q[1] for q in src])
    keep, solvers = [], []
    for p, (r5, r1, _) in zip(ps, src):
        t = [T(r5), T(r1), torch.zeros((p.n,) * 3, dtype=torch.float64, device=dev())]
        keep.append(t)
        solvers.append(g.Solver(p, t[0], t[1], None, t[2]))
    return prob, solvers, offs, keep


@pytest.mark.parametrize("precision", [g.PREC_FP64, g.PREC_FP32_IR])
def test_nested_boxes_match_oracle(precision):
    prob, solvers, offs, _ = nested(32, [(16, 8), (16, 8)], [4, 4, 4], precision)
    us = [torch.zeros((s.p.n,) * 3, dtype=torch.float64, device=dev()) for s in solvers]
    rep = g.refine_solve_nested(solvers, offs, us, tol=1e-11, max_outer=60)
    uo = [np.zeros((p.n,) * 3) for p in prob.p]
    it, hist, st = refine.solve_nested(prob, uo, tol=1e-11, max_outer=60)
    assert st == 0
    print(f"nested prec={precision}: {rep['outer_iters']} iterations (oracle {it}), rms {rep['h_rms']:.2e}")
    for k in range(3):
        assert np.abs(N(us[k]) - uo[k]).max() <= 1e-9 * (1.0 + np.abs(uo[k]).max()), k


def test_nested_boxes_full_size():
    """Base 128^3 (h = 0.5) with boxes of 64^3 parent cells refined twice (128^3 at
    h = 0.25 over [-16, 16]^3, 128^3 at h = 0.125 over [-8, 8]^3): the oracle's composite
    residual of the result is below the tolerance."""
    prob, solvers, offs, _ = nested(128, [(64, 32), (64, 32)], [6, 6, 6], g.PREC_FP32_IR)
    us = [torch.zeros((s.p.n,) * 3, dtype=torch.float64, device=dev()) for s in solvers]
    rep = g.refine_solve_nested(solvers, offs, us, tol=1e-10, max_outer=40)
    u = [N(x) for x in us]
    rms, mx = refine.Nested.norm(prob, refine.Nested.residuals(prob, u))
    print(f"nested 3 x 128^3: {rep['outer_iters']} iterations, {rep['seconds'] * 1e3:.1f} ms, oracle composite rms "
          f"{rms:.2e} (GPU {rep['h_rms']:.2e})")
    assert rms <= 1.01e-10
    assert abs(rms - rep["h_rms"]) <= 1e-3 * rms + 1e-14
