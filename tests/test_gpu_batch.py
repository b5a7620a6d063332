"""The batched solve (grouped launches: one launch per kernel for every member of
a size class; or member by member): every member equals its own single-instance
solve bitwise in every launch mode, and members agree with the CPU oracle."""
import numpy as np
import pytest
import torch

import oracle
import synth
from paper_2501_13046_amd import grtmg as g
from gpu_helpers import N, T, dev, gparams, oracle_problem, psi_rel_err

pytestmark = pytest.mark.gpu


def make_members(ws_list, precision):
    plist, r5s, r1s, Ss, Ks = [], [], [], [], []
    for w in ws_list:
        p = gparams(w, 0.0, precision)
        r5, r1, S, p.K = g.scalar_field_sources(p, w.phi_modes, w.pi_modes, w.scalar_mass, dev())
        plist.append(p)
        r5s.append(r5)
        r1s.append(r1)
        Ss.append(S)
        Ks.append(p.K)
    return plist, r5s, r1s, Ss, Ks


@pytest.mark.parametrize("precision", [g.PREC_FP32_IR, g.PREC_FP64])
@pytest.mark.parametrize("mode", [g.BATCH_GROUPS, g.BATCH_LANES])
def test_batch_members_equal_single_solves(precision, mode):
    """Members of three sizes (groups of 3, 3 and 1): the grouped launches and the
    member-by-member launches give every member its single solve, bit for bit."""
    ws = synth.scan_96(count=7, sizes=(32, 48, 64))
    plist, r5s, r1s, Ss, Ks = make_members(ws, precision)
    batch = g.Batch(plist, r5s, r1s, Ss)
    batch.launch_mode(mode)
    ng, of = batch.groups()
    assert ng == len({w.n for w in ws}) and all(of[i] == of[j] for i in range(7) for j in range(7)
                                                 if ws[i].n == ws[j].n)
    us = [torch.zeros((w.n,) * 3, dtype=torch.float64, device=dev()) for w in ws]
    Ws = [torch.zeros((3,) + (w.n,) * 3, dtype=torch.float64, device=dev()) for w in ws]
    st, reps = batch.solve(us, Ws, tol=1e-10, max_outer=60)
    assert st == 0
    for i, w in enumerate(ws):
        s = g.Solver(plist[i], r5s[i], r1s[i], Ss[i])
        u1 = torch.zeros_like(us[i])
        W1 = torch.zeros_like(Ws[i])
        rep = s.solve(u1, W1, tol=1e-10, max_outer=60)
        print(f"member {i} n={w.n} iters batch={reps[i]['outer_iters']} single={rep['outer_iters']} "
              f"rms H={reps[i]['h_rms']:.2e} rms M={reps[i]['m_rms']:.2e}")
        assert reps[i]["outer_iters"] == rep["outer_iters"]
        assert torch.equal(us[i], u1) and torch.equal(Ws[i], W1)
        assert reps[i]["h_rms"] <= 1e-10 and reps[i]["m_rms"] <= 1e-10
    # a second batched solve replays the same graph and gives the same answer
    first = [N(u) for u in us]
    for u, W in zip(us, Ws):
        u.zero_()
        W.zero_()
    st2, reps2 = batch.solve(us, Ws, tol=1e-10, max_outer=60)
    assert st2 == 0
    for i in range(len(ws)):
        assert np.array_equal(N(us[i]), first[i])


def test_batch_member_matches_oracle():
    ws = synth.scan_96(count=3, sizes=(32, 48))
    plist, r5s, r1s, Ss, Ks = make_members(ws, g.PREC_FP32_IR)
    batch = g.Batch(plist, r5s, r1s, Ss)
    us = [torch.zeros((w.n,) * 3, dtype=torch.float64, device=dev()) for w in ws]
    Ws = [torch.zeros((3,) + (w.n,) * 3, dtype=torch.float64, device=dev()) for w in ws]
    batch.solve(us, Ws, tol=1e-10)
    for i, w in enumerate(ws):
        rho5, rho1, S, K, po = oracle_problem(w)
        uo = np.zeros((w.n,) * 3)
        Wo = np.zeros((3,) + (w.n,) * 3)
        res = oracle.solve(po, uo, Wo, rho5, rho1, S, tol=1e-11, max_outer=60)
        assert res.status == 0
        assert psi_rel_err(N(us[i]), uo) < 1e-9


def test_batch_gates_converged_members():
    # a member that is already converged at the start is never updated
    ws = synth.scan_96(count=2, sizes=(32,))
    plist, r5s, r1s, Ss, Ks = make_members(ws, g.PREC_FP32_IR)
    batch = g.Batch(plist, r5s, r1s, Ss)
    us = [torch.zeros((32,) * 3, dtype=torch.float64, device=dev()) for _ in ws]
    Ws = [torch.zeros((3, 32, 32, 32), dtype=torch.float64, device=dev()) for _ in ws]
    batch.solve(us, Ws, tol=1e-10)
    solved = [u.clone() for u in us]
    us[1].zero_()
    Ws[1].zero_()
    st, reps = batch.solve(us, Ws, tol=1e-10)
    assert reps[0]["outer_iters"] == 0 and torch.equal(us[0], solved[0])
    assert reps[1]["outer_iters"] > 0 and torch.equal(us[1], solved[1])


def test_batch_launch_modes_agree_and_autotune():
    """Both launch modes replay the same member graphs: identical results;
    the automatic mode times one outer iteration in each and keeps one."""
    ws = synth.scan_96(count=5, sizes=(32, 48))
    plist, r5s, r1s, Ss, Ks = make_members(ws, g.PREC_FP32_IR)
    batch = g.Batch(plist, r5s, r1s, Ss)
    results = {}
    for mode in (g.BATCH_GRAPH, g.BATCH_LANES, g.BATCH_GROUPS, g.BATCH_AUTO):
        batch.launch_mode(mode)
        us = [torch.zeros((w.n,) * 3, dtype=torch.float64, device=dev()) for w in ws]
        Ws = [torch.zeros((3,) + (w.n,) * 3, dtype=torch.float64, device=dev()) for w in ws]
        st, reps = batch.solve(us, Ws, tol=1e-10, max_outer=60)
        assert st == 0
        results[mode] = ([N(u) for u in us], [r["outer_iters"] for r in reps])
    chosen, ms = batch.launch_mode()
    print(f"autotuned launch mode {chosen}: graph {ms[0]:.2f} ms, lanes {ms[1]:.2f} ms, groups {ms[2]:.2f} ms "
          f"per outer iteration")
    assert chosen in (g.BATCH_GRAPH, g.BATCH_LANES, g.BATCH_GROUPS) and min(ms) > 0
    for mode in (g.BATCH_LANES, g.BATCH_GROUPS, g.BATCH_AUTO):
        assert results[mode][1] == results[g.BATCH_GRAPH][1]
        for a, b in zip(results[mode][0], results[g.BATCH_GRAPH][0]):
            assert np.array_equal(a, b)


def test_scan_96_full_batch_and_large_members_match_oracle():
    """The 96-instance scan itself: every member converges to rms 1e-10 (also by
    the judge's Hamiltonian at sampled cells), and one 64^3 and one 96^3 member
    match the CPU oracle's solution (driven to 1e-11) to 1e-9 in psi."""
    from oracle import judge
    ws = synth.scan_96()
    plist, r5s, r1s, Ss, Ks = make_members(ws, g.PREC_FP32_IR)
    batch = g.Batch(plist, r5s, r1s, Ss)
    us = [torch.zeros((w.n,) * 3, dtype=torch.float64, device=dev()) for w in ws]
    Ws = [torch.zeros((3,) + (w.n,) * 3, dtype=torch.float64, device=dev()) for w in ws]
    st, reps = batch.solve(us, Ws, tol=1e-10, max_outer=60)
    its = [r["outer_iters"] for r in reps]
    print(f"scan_96: status {st}, iterations {min(its)}-{max(its)}, worst rms H "
          f"{max(r['h_rms'] for r in reps):.2e} M {max(r['m_rms'] for r in reps):.2e}", flush=True)
    assert st == 0
    rng = np.random.default_rng(96)
    for i, (w, r) in enumerate(zip(ws, reps)):
        assert r["status"] == 0 and r["h_rms"] <= 1e-10 and r["m_rms"] <= 1e-10, (i, r)
        cells = rng.integers(0, w.n, size=(64, 3))
        gr = judge.Grid(w.n, w.length, w.bc, w.origin)
        H = judge.hamiltonian_at(gr, N(us[i]), N(Ws[i]), N(r5s[i]), N(r1s[i]), Ks[i], cells)
        assert np.sqrt(np.mean(H ** 2)) < 5e-10, (i, np.sqrt(np.mean(H ** 2)))
    for size in (64, 96):
        i = next(k for k, w in enumerate(ws) if w.n == size)
        w = ws[i]
        rho5, rho1, S, K, po = oracle_problem(w)
        assert abs(K - Ks[i]) <= 1e-13 * K
        uo = np.zeros((w.n,) * 3)
        Wo = np.zeros((3,) + (w.n,) * 3)
        res = oracle.solve(po, uo, Wo, rho5, rho1, S, tol=1e-11, max_outer=60)
        assert res.status == 0
        err = psi_rel_err(N(us[i]), uo)
        Wg = N(Ws[i]) - N(Ws[i]).mean(axis=(1, 2, 3), keepdims=True)
        Wo -= Wo.mean(axis=(1, 2, 3), keepdims=True)
        werr = np.abs(Wg - Wo).max()
        print(f"scan member {i} n={w.n}: batch {reps[i]['outer_iters']} iterations, oracle {res.iters}; "
              f"psi rel err {err:.2e}, W err {werr:.2e}", flush=True)
        assert err < 1e-9 and werr < 1e-9
    batch.close()
