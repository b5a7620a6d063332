"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function include/grtmg.h declares, struct layouts match, and argument
validation happens before any HIP call."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def g():
    from paper_2501_13046_amd import grtmg
    if not os.path.exists(grtmg.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    return grtmg


def declared_functions():
    names = set()
    for h in ("grtmg.h", "grtnn.h"):
        text = open(os.path.join(ROOT, "include", h)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names |= set(re.findall(r"\b((?:mg|nn)_[a-z_0-9]+)\s*\(", text))
    return sorted(names)


def test_exports_every_declared_symbol(g):
    names = declared_functions()
    assert len(names) >= 30, names
    lib = C.CDLL(g.LIB_PATH)
    for name in names:
        assert hasattr(lib, name), name


def test_struct_layouts(g):
    assert C.sizeof(g.MgParams) == 8 * 4 + 9 * 8 + 3 * 4 + 4  # padded to the 8-byte alignment of its doubles
    assert g.MgParams.nu_pre_W.offset == 8 * 4 + 9 * 8
    assert g.MgParams.length.offset == 32
    assert C.sizeof(g.MgReport) == 4 * 4 + 5 * 8 + 8 + 8


def test_workspace_size_and_validation(g):
    ok = g.workspace_size(g.params(32, 4))
    assert ok > 0
    big = g.workspace_size(g.params(128, 6, solve_momentum=True, precision=g.PREC_FP32_IR))
    assert big > ok
    # the W step's own partial sums when it runs beside the psi step
    assert g.workspace_size(g.params(128, 6, solve_momentum=True, precision=g.PREC_FP32_IR,
                                     same_state=True)) > big
    bad = [g.params(30, 4),  # 30 -> 15 -> 7.5
           g.params(32, 6),  # coarsest 1
           g.params(32, 1),  # coarsest 32^3 too large for the dense solve
           g.params(32, 4, bc=g.BC_ROBIN, solve_momentum=True),
           g.params(32, 4, nu_pre=0, nu_post=0),
           g.params(32, 4, nu_pre=0, nu_post=2),  # the first pre-sweep pass comes with the residual
           g.params(32, 4, solve_momentum=True, nu_post_W=17),
           g.params(32, 4, solve_momentum=True, nu_pre_W=-1),
           g.params(32, 4, solve_momentum=True, cttk=True, mix_depth=7)]
    unknown = g.params(32, 4, solve_momentum=True)
    unknown.flags = 32  # no such flag
    bad.append(unknown)
    for p in bad:
        with pytest.raises(g.MGError) as e:
            g.workspace_size(p)
        assert e.value.status == g.MG_ERR_INVALID


def test_setup_rejects_before_any_hip_call(g):
    lib = g.lib()
    ctx = C.c_void_p(None)
    p = g.params(32, 4)
    # null sources -> invalid; no device memory is touched
    st = lib.mg_setup(C.byref(p), None, 0, None, None, None, None, None, C.byref(ctx))
    assert st == g.MG_ERR_INVALID and not ctx.value
    # sources given, workspace missing -> workspace error
    fake = C.c_void_p(0x1000)
    st = lib.mg_setup(C.byref(p), None, 0, None, fake, fake, None, None, C.byref(ctx))
    assert st == g.MG_ERR_WORKSPACE
    st = lib.mg_setup(C.byref(p), C.c_void_p(0x1001), 1 << 40, None, fake, fake, None, None,
                      C.byref(ctx))
    assert st == g.MG_ERR_WORKSPACE  # misaligned
    assert g.status_str(g.MG_ERR_DIVERGED).startswith("diverged")


def test_entry_points_reject_null_context(g):
    lib = g.lib()
    assert lib.mg_vcycle(None, 1, None, None) == g.MG_ERR_INVALID
    assert lib.mg_solve_constraints(None, None, None, 1e-10, 10, None) == g.MG_ERR_INVALID
    assert lib.mg_residual_norm(None, None, None, None) == g.MG_ERR_INVALID
    assert lib.mg_kernel_op(None, 1, 0, 0, None, None, None, None) == g.MG_ERR_INVALID
    p = g.params(8, 1)
    assert lib.mg_interp_cubic(C.byref(p), None, None, None) == g.MG_ERR_INVALID
    assert lib.mg_scalar_field_sources(C.byref(p), 40, None, 0, None, 1.0, None, None, None,
                                       None, 0, None, None, None) == g.MG_ERR_INVALID


def test_network_abi(g):
    from paper_2501_13046_amd import grtnn as gn
    from oracle import nn_oracle as nn
    assert C.sizeof(gn.NnConfig) == 8 * 4
    assert C.sizeof(gn.NnNorm) == 16 * 8
    for n, levels, ch in ((128, 4, (16, 32, 48, 64)), (16, 3, (16, 32, 48)), (8, 1, (16,))):
        cfg = nn.NetConfig(n=n, levels=levels, ch=ch)
        assert gn.param_count(gn.config(n, levels, ch)) == nn.param_count(cfg)
    assert gn.workspace_size(gn.config(32), True) > gn.workspace_size(gn.config(32), False) > 0
    for bad in (gn.config(30), gn.config(8, 4), gn.config(32, 4, (16, 24, 48, 64)),
                gn.config(32, 4, c_in=9), gn.config(32, 5)):
        with pytest.raises(g.MGError) as e:
            gn.workspace_size(bad, False)
        assert e.value.status == g.MG_ERR_INVALID
    lib = gn.lib()
    ctx = C.c_void_p(None)
    cfg = gn.config(32)
    # null / misaligned workspace: rejected before any HIP call
    assert lib.nn_setup(C.byref(cfg), 0, None, 0, None, C.byref(ctx)) == g.MG_ERR_WORKSPACE
    assert lib.nn_setup(C.byref(cfg), 0, C.c_void_p(256 * 3 + 8), 1 << 40, None, C.byref(ctx)) == g.MG_ERR_WORKSPACE
    assert lib.nn_forward(None, None, None) == g.MG_ERR_INVALID
    assert lib.nn_op_scratch_bytes(12, 16, 8) == 0
    assert lib.nn_conv3_forward(8, 12, 16, None, 0, None, None, None, None, 0, None) == g.MG_ERR_INVALID


def test_network_layer_shapes_follow_the_documented_order(g):
    from paper_2501_13046_amd import grtnn as gn
    from oracle import nn_oracle as nn
    for n, levels, ch in ((128, 4, (16, 32, 48, 64)), (16, 2, (32, 16))):
        assert gn.layer_shapes(gn.config(n, levels, ch)) == nn.layer_shapes(nn.NetConfig(n=n, levels=levels, ch=ch))
