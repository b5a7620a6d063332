"""The allocation-free source entry point (device scratch inside the library)
against the entry point that takes a caller-owned scratch: same fields and the
same mean density and K, bit for bit, on two calls in a row with the second
on a smaller grid; K also against the oracle's."""
import ctypes as C

import numpy as np
import pytest
import torch

import synth
from paper_2501_13046_amd import grtmg as g
from gpu_helpers import dev, gparams, oracle_problem

pytestmark = pytest.mark.gpu


def _ptr(t):
    return C.c_void_p(t.data_ptr())


def test_static_scratch_sources_match_scratch_argument():
    lib = g.lib()
    dp = C.POINTER(C.c_double)
    for n, seed in ((48, 5), (20, 6)):
        w = synth.coupled(n, seed=seed)
        p = gparams(w)
        print(f"no-alloc sources: n={n} seed={seed}", flush=True)
        ref5, ref1, refS, refK = g.scalar_field_sources(p, w.phi_modes, w.pi_modes, w.scalar_mass, dev())
        phi = np.ascontiguousarray(w.phi_modes, dtype=np.float64).reshape(-1, 5)
        pim = np.ascontiguousarray(w.pi_modes, dtype=np.float64).reshape(-1, 5)
        rho5 = torch.full((n, n, n), np.nan, dtype=torch.float64, device=dev())
        rho1 = torch.full_like(rho5, np.nan)
        S = torch.full((3, n, n, n), np.nan, dtype=torch.float64, device=dev())
        mean, K = C.c_double(-1.0), C.c_double(-1.0)
        stream = C.c_void_p(torch.cuda.current_stream(rho5.device).cuda_stream)
        st = lib.mg_scalar_field_sources_static(
            C.byref(p), len(phi), phi.ctypes.data_as(dp) if len(phi) else None,
            len(pim), pim.ctypes.data_as(dp) if len(pim) else None, w.scalar_mass,
            _ptr(rho5), _ptr(rho1), _ptr(S), C.byref(mean), C.byref(K), stream)
        assert st == g.MG_OK, g.status_str(st)
        torch.cuda.synchronize()
        assert torch.equal(rho5, ref5) and torch.equal(rho1, ref1) and torch.equal(S, refS)
        assert K.value == refK
        o5, o1, _, oK = oracle_problem(w)[:4]
        assert abs(mean.value - np.mean(o5 + o1)) <= 1e-14 * np.mean(o5 + o1)
        assert abs(K.value - oK) <= 1e-14 * oK


def test_static_scratch_rejects_bad_arguments_before_any_launch():
    lib = g.lib()
    p = g.params(8, 1)
    z = torch.zeros(8 ** 3 * 3, dtype=torch.float64, device=dev())
    mean = C.c_double(0.0)
    # too many modes and a missing mode table: refused before the device is touched
    assert lib.mg_scalar_field_sources_static(C.byref(p), 40, None, 0, None, 1.0, _ptr(z), _ptr(z), _ptr(z),
                                              C.byref(mean), None, None) == g.MG_ERR_INVALID
    p.n = 5000
    assert lib.mg_scalar_field_sources_static(C.byref(p), 0, None, 0, None, 1.0, _ptr(z), _ptr(z), _ptr(z),
                                              C.byref(mean), None, None) == g.MG_ERR_INVALID
