"""Brick-depth autotuning of the tiled kernels: every candidate gives bitwise
the same solve (the depth does not change per-cell arithmetic), the tuner
reports a time for every candidate and keeps the fastest, and choices apply
from a cache file."""
import json

import numpy as np
import pytest
import torch

import synth
from paper_2501_13046_amd import grtmg as g
from gpu_helpers import N, dev, gparams

pytestmark = pytest.mark.gpu


def setup(precision):
    w = synth.coupled(128, seed=2, precision=precision)
    p = gparams(w)
    r5, r1, S, p.K = g.scalar_field_sources(p, w.phi_modes, w.pi_modes, w.scalar_mass, dev())
    return g.Solver(p, r5, r1, S)


def solve(s):
    u = torch.zeros((128,) * 3, dtype=torch.float64, device=dev())
    W = torch.zeros((3, 128, 128, 128), dtype=torch.float64, device=dev())
    rep = s.solve(u, W, tol=1e-10, max_outer=60)
    return N(u), N(W), rep["outer_iters"]


@pytest.mark.parametrize("precision", [g.PREC_FP32_IR, g.PREC_FP64])
def test_every_candidate_gives_the_same_solve(precision, tmp_path):
    s = setup(precision)
    u0, W0, it0 = solve(s)
    entries = s.autotune(torch.zeros((128,) * 3, dtype=torch.float64, device=dev()),
                         torch.zeros((3, 128, 128, 128), dtype=torch.float64, device=dev()), reps=10)
    fams = {e["family"] for e in entries}
    expected = {g.TUNE_PASS_PSI, g.TUNE_PASS_W, g.TUNE_RESIDUAL}
    if not s.p.flags & g.FLAG_CUBIC_PROLONG:  # the tails prolong trilinearly
        expected |= {g.TUNE_TAIL_PSI, g.TUNE_TAIL_W}
    if precision == g.PREC_FP32_IR:
        expected.add(g.TUNE_FOURIER_W)  # the exact W bottom
    assert fams == expected
    # the tails change the grouping of restriction sums and the exact W bottom the
    # V-cycle itself (results agree to rounding or to the tolerance, not bitwise): back to
    # their defaults (tails off, exact bottom on) while checking that every brick depth
    # gives bitwise the same solve
    whole = (g.TUNE_TAIL_PSI, g.TUNE_TAIL_W, g.TUNE_FOURIER_W)
    for e in entries:
        if e["family"] in whole:
            s.set_tile(e["family"], e["level"], 1 if e["family"] == g.TUNE_FOURIER_W else 0)
    entries_tiles = [e for e in entries if e["family"] not in whole]
    for e in entries:
        print(f"family {e['family']} level {e['level']}: chosen {e['chosen']}, us {e['candidates']}")
        times = {k: v for k, v in e["candidates"].items() if v > 0}
        assert e["chosen"] in times and times[e["chosen"]] == min(times.values())
    u1, W1, it1 = solve(s)
    assert it1 == it0 and np.array_equal(u1, u0) and np.array_equal(W1, W0)
    for e in entries_tiles:
        for tx in e["candidates"]:
            s.set_tile(e["family"], e["level"], tx)
            u2, W2, it2 = solve(s)
            assert it2 == it0 and np.array_equal(u2, u0) and np.array_equal(W2, W0), (e["family"], tx)
        s.set_tile(e["family"], e["level"], e["chosen"])
    with pytest.raises(g.MGError):
        s.set_tile(g.TUNE_PASS_PSI, 0, 3)
    # the cache: first call tunes and stores, the second applies the stored choice
    path = str(tmp_path / "tune.json")
    z = torch.zeros((128,) * 3, dtype=torch.float64, device=dev())
    zw = torch.zeros((3, 128, 128, 128), dtype=torch.float64, device=dev())
    first = g.autotune_cached(s, z, zw, path=path, reps=5)
    stored = json.load(open(path))[g.tune_key(s.p)]
    assert [e["chosen"] for e in stored] == [e["chosen"] for e in first]
    again = g.autotune_cached(s, z, zw, path=path)
    assert again == stored
