"""The C-ABI library: loads, exports what include/mpp.h declares, validates
arguments on the host (no GPU calls are made by these tests)."""
import ctypes
import os
import re

import pytest

import paper_2312_11740_amd as M

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "mpp.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mpp_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_exports():
    assert declared_functions() == sorted(M.EXPORTS)


def test_library_exports_every_declared_symbol():
    L = M.load_library()
    for name in declared_functions():
        assert hasattr(L, name), name


@pytest.mark.parametrize("n,batch,ok", [
    (0, 1, False), (1, 1, False), (2, 1, True), (3, 1, True), (8, 1, True), (11, 1, False),
    (20, 1, True), (36, 1, True), (44, 1, False), (256, 1, True), (1024, 1, True),
    (2048, 1, False), (64, 0, False), (64, 64, True), (64, 70000, False)])
def test_workspace_bytes_validates_shapes(n, batch, ok):
    nb = M.workspace_bytes(n, batch)
    assert (nb > 0) == ok
    if ok:
        assert nb >= 6 * 8 * n ** 3 * batch


def test_workspace_grows_with_batch():
    assert M.workspace_bytes(32, 4) > 3 * M.workspace_bytes(32, 1)


def test_build_rejects_bad_arguments_before_device_work():
    L = M.load_library()
    d = M.Desc(16, 1, 0)
    h = ctypes.c_void_p()
    one = (ctypes.c_double * 1)(1.0)
    neg = (ctypes.c_double * 1)(-1.0)
    nan = (ctypes.c_double * 1)(float("nan"))
    fake = ctypes.c_void_p(0x1000)   # never dereferenced: validation fails first
    nbytes = M.workspace_bytes(16)
    # null phi
    assert L.mpp_build_operator(ctypes.byref(d), None, one, one, one, fake, nbytes, None,
                                ctypes.byref(h)) == M.EINVAL
    # non-positive or non-finite density, negative sigma
    for rn, rp, sg in ((neg, one, one), (one, nan, one), (one, one, neg)):
        assert L.mpp_build_operator(ctypes.byref(d), fake, rn, rp, sg, fake, nbytes, None,
                                    ctypes.byref(h)) == M.EINVAL
    # workspace too small
    assert L.mpp_build_operator(ctypes.byref(d), fake, one, one, one, fake, 100, None,
                                ctypes.byref(h)) == M.ENOMEM
    # bad shape
    bad = M.Desc(11, 1, 0)
    assert L.mpp_build_operator(ctypes.byref(bad), fake, one, one, one, fake, nbytes, None,
                                ctypes.byref(h)) == M.EINVAL
    assert h.value is None


def test_calls_on_null_operator():
    L = M.load_library()
    assert L.mpp_apply_stencil(None, None, None, None) == M.EINVAL
    assert L.mpp_solve(None, None, None, None, None, None) == M.EINVAL
    assert L.mpp_vcycle(None, None, None, 2, None) == M.EINVAL
    L.mpp_destroy_operator(None)


def test_default_opts_and_strerror():
    L = M.load_library()
    o = M.SolveOpts()
    L.mpp_default_opts(ctypes.byref(o))
    assert o.rtol == 1e-10 and o.mode == M.MODE_FP64 and o.nu == 2
    assert o.deflate == 1 and o.reuse_rhs == 0
    assert M.strerror(M.ENOTCONVERGED) == "not converged within max_iter"


def test_level_set_calls_reject_bad_arguments_before_device_work():
    L = M.load_library()
    a, b, c = (ctypes.c_void_p(0x1000 * k) for k in (1, 2, 3))   # never dereferenced
    u = [ctypes.c_void_p(0x8000)] * 3
    assert L.mpp_ls_advect(1, 1, a, *u, 0.1, b, None) == M.EINVAL         # n < 2
    assert L.mpp_ls_advect(8, 0, a, *u, 0.1, b, None) == M.EINVAL         # batch < 1
    assert L.mpp_ls_advect(8, 1, a, *u, 0.0, b, None) == M.EINVAL         # dt <= 0
    assert L.mpp_ls_advect(8, 1, a, *u, float("inf"), b, None) == M.EINVAL
    assert L.mpp_ls_advect(8, 1, a, *u, 0.1, a, None) == M.EINVAL         # out aliases phi
    assert L.mpp_ls_advect(8, 1, None, *u, 0.1, b, None) == M.EINVAL
    assert L.mpp_ls_reinit(8, 1, a, b, c, -1, 0.1, None) == M.EINVAL      # iters < 0
    assert L.mpp_ls_reinit(8, 1, a, b, c, 3, 0.0, None) == M.EINVAL       # dtau <= 0
    assert L.mpp_ls_reinit(8, 1, a, a, c, 3, 0.1, None) == M.EINVAL       # phi0 aliases phi
    assert L.mpp_ls_reinit(8, 1, a, b, b, 3, 0.1, None) == M.EINVAL       # work aliases phi
    assert L.mpp_ls_reinit(2048, 1, a, b, c, 3, 0.1, None) == M.EINVAL    # n too large


def test_heat_solve_rejects_bad_arguments_before_device_work():
    L = M.load_library()
    op, a, b = (ctypes.c_void_p(0x1000 * k) for k in (1, 2, 3))   # never dereferenced
    opts = M.SolveOpts()
    L.mpp_default_opts(ctypes.byref(opts))
    info = (M.SolveInfo * 1)()
    assert L.mpp_heat_solve(None, a, None, 0.1, b, ctypes.byref(opts), info, None) == M.EINVAL
    assert L.mpp_heat_solve(op, None, None, 0.1, b, ctypes.byref(opts), info, None) == M.EINVAL
    assert L.mpp_heat_solve(op, a, None, 0.1, None, ctypes.byref(opts), info, None) == M.EINVAL
    assert L.mpp_heat_solve(op, a, b, 0.1, b, ctypes.byref(opts), info, None) == M.EINVAL  # src = t
    assert L.mpp_heat_solve(op, a, None, -1.0, b, ctypes.byref(opts), info, None) == M.EINVAL
    assert L.mpp_heat_solve(op, a, None, float("nan"), b, ctypes.byref(opts), info,
                            None) == M.EINVAL
    assert L.mpp_heat_solve(op, a, None, float("inf"), b, ctypes.byref(opts), info,
                            None) == M.EINVAL
    assert L.mpp_heat_solve(op, a, None, 0.1, b, None, info, None) == M.EINVAL
    opts.rtol = 0.0
    assert L.mpp_heat_solve(op, a, None, 0.1, b, ctypes.byref(opts), info, None) == M.EINVAL
    L.mpp_default_opts(ctypes.byref(opts))
    opts.check_every = 0
    assert L.mpp_heat_solve(op, a, None, 0.1, b, ctypes.byref(opts), info, None) == M.EINVAL


def test_block_layout_calls_reject_bad_arguments_before_device_work():
    L = M.load_library()
    a, b, op = (ctypes.c_void_p(0x1000 * k) for k in (1, 2, 3))   # never dereferenced
    for fn in (L.mpp_blocks_scatter, L.mpp_blocks_gather):
        assert fn(32, 1, 16, 1, a, a, None) == M.EINVAL      # aliasing
        assert fn(30, 1, 16, 1, a, b, None) == M.EINVAL      # n % nb
        assert fn(32, 1, 16, 17, a, b, None) == M.EINVAL     # g > nb
        assert fn(32, 1, 16, -1, a, b, None) == M.EINVAL
        assert fn(32, 0, 16, 1, a, b, None) == M.EINVAL      # batch
        assert fn(32, 1, 1, 1, a, b, None) == M.EINVAL       # nb < 2
        assert fn(2048, 1, 16, 1, a, b, None) == M.EINVAL    # n too large
        assert fn(32, 1, 16, 1, None, b, None) == M.EINVAL
    assert L.mpp_blocks_fill_guards(32, 1, 16, 1, None, None) == M.EINVAL
    assert L.mpp_blocks_fill_guards(32, 1, 12, 1, a, None) == M.EINVAL
    assert L.mpp_blocks_fill_guards(32, 1, 16, 0, a, None) == M.OK        # nothing to do
    assert L.mpp_blocks_apply(None, 16, 1, a, b, None) == M.EINVAL
    assert L.mpp_blocks_apply(op, 16, 1, a, a, None) == M.EINVAL


def test_amr_host_validation():
    L = M.load_library()
    assert L.mpp_amr_workspace_bytes(30, 8) == 0          # 30 % 8
    assert L.mpp_amr_workspace_bytes(1024, 16) == 0       # n0 > 512
    assert L.mpp_amr_workspace_bytes(32, 8) > 0
    flags = (ctypes.c_uint8 * 64)()
    h = ctypes.c_void_p()
    ws = ctypes.c_void_p(1 << 20)   # never touched: every call below fails its checks first
    nbytes = L.mpp_amr_workspace_bytes(32, 8)
    for n0, nb, g in ((32, 8, 0), (32, 8, 9), (30, 8, 1), (32, 1, 1)):
        assert L.mpp_amr_create(n0, nb, g, flags, ws, nbytes, None, ctypes.byref(h)) == M.EINVAL
        assert not h.value
    assert L.mpp_amr_create(32, 8, 1, flags, ws, 16, None, ctypes.byref(h)) == -2   # ENOMEM
    assert L.mpp_amr_create(32, 8, 1, None, ws, nbytes, None, ctypes.byref(h)) == M.EINVAL
    cnt = ctypes.c_int32(0)
    assert L.mpp_amr_level1_blocks(None, ctypes.byref(cnt), None) == M.EINVAL
    assert L.mpp_amr_fill_guards(None, ws, None, None) == M.EINVAL
    assert L.mpp_amr_apply(None, ws, None, ws, None, 1.0, 1.0, ws, None, None) == M.EINVAL
    assert L.mpp_amr_coarse_operator(None, None, ws, None, 1.0, 1.0, None) == M.EINVAL


def test_net_train_rejects_bad_arguments_before_device_work():
    """mpp_net_train checks its arguments before it reads the handle or touches memory
    (the pointers below are never dereferenced)."""
    L = M.load_library()
    net, x, t, lo = (ctypes.c_void_p(0x1000 * k) for k in (1, 2, 3, 4))

    def opts(**kw):
        o = M.NetTrainOpts(batch=4, steps=2, first_step=0, total_steps=2, lr0=1e-3, lr1=1e-4,
                           beta1=0.9, beta2=0.999, eps=1e-8, reserved=0, seed=7)
        for k, v in kw.items():
            setattr(o, k, v)
        return ctypes.byref(o)
    nan, inf = float("nan"), float("inf")
    assert L.mpp_net_train(None, x, t, 10, opts(), lo, None) == M.EINVAL
    assert L.mpp_net_train(net, None, t, 10, opts(), lo, None) == M.EINVAL
    assert L.mpp_net_train(net, x, None, 10, opts(), lo, None) == M.EINVAL
    assert L.mpp_net_train(net, x, t, 10, None, lo, None) == M.EINVAL
    assert L.mpp_net_train(net, x, t, 0, opts(), lo, None) == M.EINVAL          # count
    for bad in (dict(batch=0), dict(steps=-1), dict(first_step=-3), dict(total_steps=-1),
                dict(lr0=0.0), dict(lr0=-1e-3), dict(lr0=nan), dict(lr1=0.0), dict(lr1=inf),
                dict(beta1=1.0), dict(beta1=-0.1), dict(beta2=1.0), dict(eps=0.0),
                dict(eps=nan)):
        assert L.mpp_net_train(net, x, t, 10, opts(**bad), lo, None) == M.EINVAL, bad


def test_reinit_noalloc_rejects_bad_and_oversized_arguments_before_device_work():
    """The allocation-free re-distancing call refuses a batch beyond its fixed scratch field
    (2^24 cells) with MPP_ENOMEM, and the usual bad arguments with MPP_EINVAL, before any
    device call (the pointers are never dereferenced)."""
    L = M.load_library()
    a, b = (ctypes.c_void_p(0x1000 * k) for k in (1, 2))
    assert L.mpp_ls_reinit_noalloc(256, 2, a, b, 2, 0.001, None) == M.ENOMEM    # 2 x 256^3
    assert L.mpp_ls_reinit_noalloc(512, 1, a, b, 2, 0.001, None) == M.ENOMEM
    assert L.mpp_ls_reinit_noalloc(1, 1, a, b, 2, 0.001, None) == M.EINVAL      # n < 2
    assert L.mpp_ls_reinit_noalloc(8, 0, a, b, 2, 0.001, None) == M.EINVAL      # batch
    assert L.mpp_ls_reinit_noalloc(8, 1, a, a, 2, 0.001, None) == M.EINVAL      # aliasing
    assert L.mpp_ls_reinit_noalloc(8, 1, None, b, 2, 0.001, None) == M.EINVAL
    assert L.mpp_ls_reinit_noalloc(8, 1, a, b, -1, 0.001, None) == M.EINVAL     # iters
    assert L.mpp_ls_reinit_noalloc(8, 1, a, b, 2, 0.0, None) == M.EINVAL        # dtau
    assert L.mpp_ls_reinit_noalloc(8, 1, a, b, 2, float("nan"), None) == M.EINVAL
