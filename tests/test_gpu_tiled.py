"""Element-by-element parity of the 2.5D LDS-tiled finest-level kernels (the
launch configuration used from 128^3 up) with the CPU oracle."""
import numpy as np
import pytest
import torch

import oracle
import synth
from paper_2501_13046_amd import grtmg as g
from gpu_helpers import N, T, dev, rel_err

pytestmark = pytest.mark.gpu

n = 128


@pytest.mark.parametrize("precision", [g.PREC_FP64, g.PREC_FP32_IR])
@pytest.mark.parametrize("bc", [g.BC_PERIODIC, g.BC_ROBIN, g.BC_REFLECT, g.BC_EXTRAP, g.BC_ZERO])
def test_tiled_psi_pass(precision, bc):
    L, org = (1.0, (0.0,) * 3) if bc == g.BC_PERIODIC else (64.0, (-32.0,) * 3)
    p = g.params(n, 6, bc=bc, precision=precision, length=L, origin=org)
    po = oracle.params(n, 6, bc=bc, length=L, origin=org)
    z = torch.zeros((n,) * 3, dtype=torch.float64, device=dev())
    s = g.Solver(p, z, z)
    d = synth.uniform_random(60, (n,) * 3)
    r = synth.uniform_random(61, (n,) * 3)
    c = -1.0 - synth.uniform_random(62, (n,) * 3, 0, 2)
    vt = s.vtype
    if vt == torch.float32:  # compare on the same rounded inputs
        d, r, c = (a.astype(np.float32).astype(np.float64) for a in (d, r, c))
    tol = 1e-13 if vt == torch.float64 else 2e-6
    for colour in (0, 1):
        out = torch.empty((n,) * 3, dtype=vt, device=dev())
        s.kernel_op(g.OP_PASS_PSI, 0, colour, T(d, vt), out, T(r, vt), T(c, vt))
        assert rel_err(N(out), oracle.pass_psi(po, d, r, c, colour)) < tol, colour


@pytest.mark.parametrize("precision,depth", [(g.PREC_FP64, 1), (g.PREC_FP64, 2), (g.PREC_FP64, 8),
                                             (g.PREC_FP32_IR, 2), (g.PREC_FP32_IR, 4), (g.PREC_FP32_IR, 8),
                                             (g.PREC_FP32_IR, 16)])
def test_tiled_W_pass(precision, depth):
    """Every brick depth (staged bricks 1-4, x-marched columns 8 and 16) against the oracle."""
    p = g.params(n, 6, precision=precision, solve_momentum=True)
    po = oracle.params(n, 6)
    z = torch.zeros((n,) * 3, dtype=torch.float64, device=dev())
    S = torch.zeros((3, n, n, n), dtype=torch.float64, device=dev())
    s = g.Solver(p, z, z, S)
    s.set_tile(g.TUNE_PASS_W, 0, depth)
    d = synth.uniform_random(63, (3, n, n, n))
    r = synth.uniform_random(64, (3, n, n, n))
    vt = s.vtype
    if vt == torch.float32:
        d, r = (a.astype(np.float32).astype(np.float64) for a in (d, r))
    tol = 1e-13 if vt == torch.float64 else 2e-6
    for colour in (0, 1):
        out = torch.empty((3, n, n, n), dtype=vt, device=dev())
        s.kernel_op(g.OP_PASS_W, 0, colour, T(d, vt), out, T(r, vt))
        assert rel_err(N(out), oracle.pass_W(po, d, r, colour)) < tol, colour


@pytest.mark.parametrize("precision", [g.PREC_FP64, g.PREC_FP32_IR])
def test_marched_W_defect_restrict(precision):
    """W defect r - Delta_L d restricted to 64^3 by the x-marched kernel (finest level)."""
    p = g.params(n, 6, precision=precision, solve_momentum=True)
    po = oracle.params(n, 6)
    z = torch.zeros((n,) * 3, dtype=torch.float64, device=dev())
    S = torch.zeros((3, n, n, n), dtype=torch.float64, device=dev())
    s = g.Solver(p, z, z, S)
    d = synth.uniform_random(65, (3, n, n, n))
    r = synth.uniform_random(66, (3, n, n, n))
    vt = s.vtype
    if vt == torch.float32:
        d, r = (a.astype(np.float32).astype(np.float64) for a in (d, r))
    out = torch.empty((3,) + (n // 2,) * 3, dtype=vt, device=dev())
    s.kernel_op(g.OP_DEFECT_RESTRICT_W, 0, 0, T(d, vt), out, T(r, vt))
    defect = r - oracle.apply_deltaL(po, d)
    ref = np.stack([oracle.restrict(np.ascontiguousarray(defect[a])) for a in range(3)])
    tol = 1e-12 if vt == torch.float64 else 1e-5
    assert rel_err(N(out), ref) < tol


@pytest.mark.parametrize("precision", [g.PREC_FP64, g.PREC_FP32_IR])
def test_marched64_W_pass_and_defect(precision):
    """64^3 level: the W colour passes and the W defect restriction run as x-marched
    columns of 64-cell rows (two brick rows per wave)."""
    m = 64
    p = g.params(m, 5, precision=precision, solve_momentum=True)
    po = oracle.params(m, 5)
    z = torch.zeros((m,) * 3, dtype=torch.float64, device=dev())
    S = torch.zeros((3, m, m, m), dtype=torch.float64, device=dev())
    s = g.Solver(p, z, z, S)
    d = synth.uniform_random(67, (3, m, m, m))
    r = synth.uniform_random(68, (3, m, m, m))
    vt = s.vtype
    if vt == torch.float32:
        d, r = (a.astype(np.float32).astype(np.float64) for a in (d, r))
    tol = 1e-13 if vt == torch.float64 else 2e-6
    for colour in (0, 1):
        out = torch.empty((3, m, m, m), dtype=vt, device=dev())
        s.kernel_op(g.OP_PASS_W, 0, colour, T(d, vt), out, T(r, vt))
        assert rel_err(N(out), oracle.pass_W(po, d, r, colour)) < tol, colour
    out = torch.empty((3,) + (m // 2,) * 3, dtype=vt, device=dev())
    s.kernel_op(g.OP_DEFECT_RESTRICT_W, 0, 0, T(d, vt), out, T(r, vt))
    defect = r - oracle.apply_deltaL(po, d)
    ref = np.stack([oracle.restrict(np.ascontiguousarray(defect[a])) for a in range(3)])
    assert rel_err(N(out), ref) < (1e-12 if vt == torch.float64 else 1e-5)


@pytest.mark.parametrize("depth", [2, 4, 8, 16])
def test_tiled_residual_periodic_coupled(depth):
    """Bricks (depth 2, 4) and x-marched columns (8, 16) of the finest residual."""
    K = 2.3
    p = g.params(n, 6, K=K, solve_momentum=True)
    po = oracle.params(n, 6, K=K, solve_momentum=True)
    u = synth.uniform_random(70, (n,) * 3, -0.05, 0.05)
    W = synth.uniform_random(71, (3, n, n, n), -0.02, 0.02)
    rho5 = synth.uniform_random(72, (n,) * 3, 0, 1)
    rho1 = synth.uniform_random(73, (n,) * 3, 0, 1)
    S = synth.uniform_random(74, (3, n, n, n))
    s = g.Solver(p, T(rho5), T(rho1), T(S))
    s.set_tile(g.TUNE_RESIDUAL, 0, depth)
    H, M, c = s.residual_fields(T(u), T(W))
    Ho, Mo, co = oracle.residuals(po, u, W, rho5, rho1, S)
    assert rel_err(N(H), Ho) < 1e-12
    assert rel_err(N(M), Mo) < 1e-12
    assert rel_err(N(c), co) < 1e-13
    np.testing.assert_allclose(s.residual_norm(T(u), T(W)), oracle.norms(Ho, Mo), rtol=1e-11)
    # the psi step's form: H and c without the momentum part
    H2, _, c2 = s.residual_fields(T(u), T(W), want_M=False)
    assert np.array_equal(N(H2), N(H)) and np.array_equal(N(c2), N(c))


def test_tiled_residual_robin_puncture():
    p = g.params(n, 6, bc=g.BC_ROBIN, length=64.0, origin=(-32.0,) * 3, puncture_mass=1.0,
                 conformal_matter=True)
    po = oracle.params(n, 6, bc=oracle.BC_ROBIN, length=64.0, origin=(-32.0,) * 3, puncture_mass=1.0,
                       conformal_matter=True)
    u = synth.uniform_random(75, (n,) * 3, -0.05, 0.05)
    rho5 = synth.uniform_random(76, (n,) * 3, 0, 0.01)
    rho1 = synth.uniform_random(77, (n,) * 3, 0, 0.01)
    s = g.Solver(p, T(rho5), T(rho1))
    H, _, c = s.residual_fields(T(u), None, want_M=False)
    z3 = np.zeros((3, n, n, n))
    Ho, _, co = oracle.residuals(po, u, z3, rho5, rho1, z3)
    assert rel_err(N(H), Ho) < 1e-12
    assert rel_err(N(c), co) < 1e-13


@pytest.mark.parametrize("bc", [g.BC_REFLECT, g.BC_EXTRAP, g.BC_ZERO])
@pytest.mark.parametrize("depth", [2, 4])
def test_tiled_residual_reflect_extrap(bc, depth):
    """Residual bricks under the reflective and extrapolating rules, frozen W."""
    K = 1.7
    p = g.params(n, 6, bc=bc, K=K)
    po = oracle.params(n, 6, bc=bc, K=K)
    u = synth.uniform_random(80, (n,) * 3, -0.05, 0.05)
    W = synth.uniform_random(81, (3, n, n, n), -0.01, 0.01)
    rho5 = synth.uniform_random(82, (n,) * 3, 0, 0.5)
    rho1 = synth.uniform_random(83, (n,) * 3, 0, 0.5)
    s = g.Solver(p, T(rho5), T(rho1))
    s.set_tile(g.TUNE_RESIDUAL, 0, depth)
    H, _, c = s.residual_fields(T(u), T(W), want_M=False)
    z3 = np.zeros((3, n, n, n))
    Ho, _, co = oracle.residuals(po, u, W, rho5, rho1, z3)
    assert rel_err(N(H), Ho) < 1e-12
    assert rel_err(N(c), co) < 1e-13
