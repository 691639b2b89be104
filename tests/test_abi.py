"""The C-ABI library without a GPU: it loads, exports every function that
include/tl.h declares, and rejects bad arguments before touching the device.

Fake (never dereferenced) host addresses are used: every call here returns an
argument error before anything is launched.
"""
import ctypes
import os
import re

import pytest

from paper_1804_10120_amd import _abi
from paper_1804_10120_amd._abi import CField, Domain, Field, Tune

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tl.h")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tl_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(_abi.LIB_PATH):
        from paper_1804_10120_amd import build
        build.build()
    return _abi.lib()


def test_header_declares_the_hot_path():
    names = declared()
    for n in ("tl_sym_inverse", "tl_christoffel", "tl_cov_deriv", "tl_dtg", "tl_dtg_chain",
              "tl_dtg_chain_bwd", "tl_dtg_chain_fwd_bwd", "tl_batch_plan_create", "tl_batch_plan_launch",
              "tl_batch_plan_destroy"):
        assert n in names


def test_every_declared_symbol_is_exported(L):
    missing = [n for n in declared() if not hasattr(L, n)]
    assert missing == []
    assert set(declared()) <= set(_abi.SIGNATURES)


def test_binding_constants_match_the_header():
    text = open(HEADER).read()
    for name in ("TL_ABI_VERSION", "TL_NOALLOC_MAX_DOMAINS", "TL_NOALLOC_MAX_TILES",
                 "TL_BW_READ_BLOCKS", "TL_TUNE_NT", "TL_TUNE_XCD", "TL_TUNE_PTR64"):
        m = re.search(rf"#define {name} (\d+)", text)
        assert m, name
        py = _abi.ABI_VERSION if name == "TL_ABI_VERSION" else getattr(_abi, name)
        assert int(m.group(1)) == py, name


def test_version_and_strings(L):
    assert L.tl_abi_version() == _abi.ABI_VERSION
    for s, name in enumerate(["TL_OK", "TL_ERR_NULL", "TL_ERR_SIZE", "TL_ERR_ALIAS",
                              "TL_ERR_ALIGN", "TL_ERR_HIP", "TL_ERR_INVALID"]):
        assert L.tl_status_string(s).decode() == name


BASE = 1 << 40          # fake, 256-byte aligned, never dereferenced
MB = 1 << 20


def cf(addr, ld):
    return CField(addr, ld)


def f(addr, ld):
    return Field(addr, ld)


def chain_args(n, ld=None, out_addr=None, alpha_addr=None):
    ld = n if ld is None else ld
    a = [cf(BASE + i * 64 * MB, ld) for i in range(6)]
    if alpha_addr is not None:
        a[5] = cf(alpha_addr, ld)
    out = f(BASE + 6 * 64 * MB if out_addr is None else out_addr, ld)
    return a, out


def call_chain(L, n, a, out, tune=None):
    return L.tl_dtg_chain(n, *a, out, None, tune)


def test_zero_points_is_a_noop(L):
    a, out = chain_args(0)
    assert call_chain(L, 0, [cf(None, 0)] * 6, f(None, 0)) == _abi.TL_OK


def test_negative_n(L):
    a, out = chain_args(16)
    assert call_chain(L, -1, a, out) == _abi.TL_ERR_SIZE
    assert b"n=-1" in L.tl_last_error()


def test_null_pointer(L):
    a, out = chain_args(16)
    a[2] = cf(None, 16)
    assert call_chain(L, 16, a, out) == _abi.TL_ERR_NULL
    assert b"beta" in L.tl_last_error()
    a, out = chain_args(16)
    assert call_chain(L, 16, a, f(None, 16)) == _abi.TL_ERR_NULL


def test_ld_smaller_than_n(L):
    a, out = chain_args(100)
    a[1] = cf(a[1].ptr, 99)
    assert call_chain(L, 100, a, out) == _abi.TL_ERR_SIZE
    assert b"dg" in L.tl_last_error()


def test_misaligned(L):
    a, out = chain_args(16)
    a[0] = cf(BASE + 4, 16)
    assert call_chain(L, 16, a, out) == _abi.TL_ERR_ALIGN


def test_output_overlapping_input(L):
    n = 1000
    a, _ = chain_args(n)
    # dtg starts inside the last component of dg
    out = f(a[1].ptr + (17 * n + 10) * 8, n)
    assert call_chain(L, n, a, out) == _abi.TL_ERR_ALIAS
    # touching but not overlapping is fine up to validation (would launch): check the
    # boundary on the unfused inverse, whose only other check is the tuning
    g = cf(BASE, n)
    ginv = f(BASE + (5 * n + n - 1) * 8, n)        # starts on g's last element
    assert L.tl_sym_inverse(n, g, ginv, None, None) == _abi.TL_ERR_ALIAS


def test_inputs_may_alias_each_other(L):
    # identical input pointers are allowed; with an invalid tuning the call stops
    # after validation, before any device work
    n = 64
    a = [cf(BASE, n)] * 6
    out = f(BASE + 64 * MB, n)
    bad = ctypes.pointer(Tune(96, 0, 0, 0))
    assert call_chain(L, n, a, out, bad) == _abi.TL_ERR_INVALID


@pytest.mark.parametrize("tune", [(96, 0, 0, 0), (256, 3, 0, 0), (256, 8, 0, 0), (256, 1, 8, 0), (256, 1, 0, -1),
                                  (256, 1, 0, 0, 4), (256, 1, 0, 0, 3)])
def test_invalid_tuning(L, tune):
    a, out = chain_args(64)
    assert call_chain(L, 64, a, out, ctypes.pointer(Tune(*tune))) == _abi.TL_ERR_INVALID


def test_bwd_needs_an_output(L):
    n = 32
    ins = [cf(BASE + i * MB, n) for i in range(6)]
    outs = [f(None, 0)] * 6
    assert L.tl_dtg_chain_bwd(n, *ins, *outs, None, None) == _abi.TL_ERR_NULL


def test_bwd_outputs_may_not_overlap(L):
    n = 32
    ins = [cf(BASE + i * MB, n) for i in range(6)]
    outs = [f(BASE + 10 * MB, n), f(BASE + 10 * MB + 8 * 40, n)] + [f(None, 0)] * 4
    assert L.tl_dtg_chain_bwd(n, *ins, *outs, None, None) == _abi.TL_ERR_ALIAS


def test_fwd_bwd_validation(L):
    n = 32
    ins = [cf(BASE + i * MB, n) for i in range(7)]
    none = [f(None, 0)] * 7
    assert L.tl_dtg_chain_fwd_bwd(n, *ins, *none, None, None) == _abi.TL_ERR_NULL
    outs = [f(BASE + 10 * MB, n)] + [f(None, 0)] * 6
    bad = list(ins)
    bad[6] = cf(None, n)                             # the cotangent w
    assert L.tl_dtg_chain_fwd_bwd(n, *bad, *outs, None, None) == _abi.TL_ERR_NULL
    assert b"w" in L.tl_last_error()
    # d_t g overlapping g_bar
    outs = [f(BASE + 10 * MB, n), f(BASE + 10 * MB + 8 * 100, n)] + [f(None, 0)] * 5
    assert L.tl_dtg_chain_fwd_bwd(n, *ins, *outs, None, None) == _abi.TL_ERR_ALIAS
    # d beta (read here, unlike in the adjoint) overlapping an output
    outs = [f(BASE + 3 * MB + 8, n)] + [f(None, 0)] * 6
    assert L.tl_dtg_chain_fwd_bwd(n, *ins, *outs, None, None) == _abi.TL_ERR_ALIAS
    assert L.tl_dtg_chain_fwd_bwd(-2, *ins, *outs, None, None) == _abi.TL_ERR_SIZE
    assert L.tl_dtg_chain_fwd_bwd(0, *ins, *none, None, None) == _abi.TL_OK


def test_unfused_validation(L):
    n = 10
    assert L.tl_christoffel(n, cf(BASE, n), cf(None, n), f(BASE + MB, n), None, None) == _abi.TL_ERR_NULL
    assert L.tl_cov_deriv(n, cf(BASE, n), cf(BASE + MB, n), cf(BASE + 2 * MB, 9),
                          f(BASE + 3 * MB, n), None, None) == _abi.TL_ERR_SIZE
    assert L.tl_dtg(n, cf(BASE, 0), cf(BASE + MB, n), cf(BASE + 2 * MB, n),
                    f(BASE + 8 * 3, n), None, None) == _abi.TL_ERR_ALIAS


def test_batch_plan_validation(L):
    plan = ctypes.c_void_p()
    assert L.tl_batch_plan_create(None, 1, None, ctypes.byref(plan)) == _abi.TL_ERR_NULL
    doms = (Domain * 2)()
    assert L.tl_batch_plan_create(doms, 0, None, ctypes.byref(plan)) == _abi.TL_ERR_SIZE
    n = 100
    for d in range(2):
        a, out = chain_args(n)
        base = d * 512 * MB
        doms[d] = Domain(n, *[cf(x.ptr + base, n) for x in a], f(out.ptr + base, n))
    doms[1].dtg = Field(doms[0].g.ptr, n)         # second domain writes the first one's g
    assert L.tl_batch_plan_create(doms, 2, None, ctypes.byref(plan)) == _abi.TL_ERR_ALIAS
    assert not plan.value
    doms[1].n = -5
    assert L.tl_batch_plan_create(doms, 2, None, ctypes.byref(plan)) == _abi.TL_ERR_SIZE
    assert L.tl_batch_plan_destroy(None) == _abi.TL_OK


def test_noalloc_batch_limits(L):
    """tl_batch_run_noalloc rejects a batch beyond its fixed tables (too many
    subgrids, too many tiles) and bad domains before launching anything."""
    assert L.tl_batch_run_noalloc(None, 1, None, None) == _abi.TL_ERR_NULL
    doms = (Domain * (_abi.TL_NOALLOC_MAX_DOMAINS + 1))()
    assert L.tl_batch_run_noalloc(doms, 0, None, None) == _abi.TL_ERR_SIZE
    assert L.tl_batch_run_noalloc(doms, _abi.TL_NOALLOC_MAX_DOMAINS + 1, None, None) == \
        _abi.TL_ERR_SIZE
    assert b"TL_NOALLOC_MAX_DOMAINS" in L.tl_last_error()
    # one subgrid of more tiles than the table holds (blocks of 64 points)
    n = 64 * _abi.TL_NOALLOC_MAX_TILES + 1
    gib = 1 << 30
    one = (Domain * 1)()
    one[0] = Domain(n, *[cf(BASE + i * 8 * gib, n) for i in range(6)], f(BASE + 6 * 8 * gib, n))
    tune = Tune(64, 1, _abi.TL_TUNE_NT, 0, 0)
    assert L.tl_batch_run_noalloc(one, 1, ctypes.byref(tune), None) == _abi.TL_ERR_SIZE
    assert b"TL_NOALLOC_MAX_TILES" in L.tl_last_error()
    one[0].dtg = Field(one[0].K.ptr, n)      # output over an input
    assert L.tl_batch_run_noalloc(one, 1, ctypes.byref(tune), None) == _abi.TL_ERR_ALIAS


def test_kernel_info_unknown(L):
    a = _abi.KernelAttr()
    assert L.tl_kernel_info(b"nope", None, ctypes.byref(a)) == _abi.TL_ERR_INVALID


def test_python_binding_rejects_host_tensors():
    import torch
    from paper_1804_10120_amd import tl_sym_inverse
    with pytest.raises(ValueError, match="HIP device"):
        tl_sym_inverse(torch.zeros(6, 4, dtype=torch.float64))
    with pytest.raises(TypeError, match="float64"):
        tl_sym_inverse(torch.zeros(6, 4, dtype=torch.float32))


def test_twin_rejects_unknown_shapes(L):
    assert L.tl_bw_twin(16, 5, cf(BASE, 16), 5, f(BASE + MB, 16), None, None) == _abi.TL_ERR_INVALID
    assert L.tl_bw_twin(16, 43, cf(BASE, 16), 6, f(BASE + 8 * 16, 16), None, None) == _abi.TL_ERR_ALIAS


def test_expr_shapes_match_the_oracle(L):
    import oracle
    from paper_1804_10120_amd import tl_expr_shape
    for name in _abi.EXPRS:
        assert tl_expr_shape(name) == oracle.expr_shape(name)


def test_expr_validation(L):
    n = 16
    ins = (CField * 2)(cf(BASE, n), cf(BASE + MB, n))
    assert L.tl_expr(99, n, ins, 2, f(BASE + 2 * MB, n), None, None) == _abi.TL_ERR_INVALID
    assert L.tl_expr(_abi.EXPRS.index("contract1"), n, ins, 3, f(BASE + 2 * MB, n), None,
                     None) == _abi.TL_ERR_INVALID
    # contract1 reads 81 components of E: an output 1 MiB after E's base overlaps it
    bad = (CField * 2)(cf(BASE, 4096), cf(BASE + MB, 4096))
    assert L.tl_expr(_abi.EXPRS.index("contract1"), 4096, bad, 2, f(BASE + 2 * MB, 4096), None,
                     None) == _abi.TL_ERR_ALIAS
    assert L.tl_expr(0, 0, None, 1, f(None, 0), None, None) == _abi.TL_OK


def test_batch_overlap_check_scales(L):
    """20000 subgrids (140000 fields): the overlap check is a sort and a sweep,
    and it finds the one output that overlaps another subgrid's input."""
    import time
    nd, n = 20000, 64
    doms = (Domain * nd)()
    stride = 64 * 1024
    for d in range(nd):
        base = BASE + d * 8 * stride
        doms[d] = Domain(n, *[cf(base + f * stride, n) for f in range(6)], f(base + 6 * stride, n))
    doms[nd - 1].dtg = Field(doms[0].dbeta.ptr + 8, n)
    plan = ctypes.c_void_p()
    t0 = time.perf_counter()
    assert L.tl_batch_plan_create(doms, nd, None, ctypes.byref(plan)) == _abi.TL_ERR_ALIAS
    assert time.perf_counter() - t0 < 5.0
    assert b"dtg" in L.tl_last_error() and b"dbeta" in L.tl_last_error()


def test_padded_fields():
    import numpy as np
    import torch
    from paper_1804_10120_amd import empty_field, padded_ld, to_field
    assert [padded_ld(n) for n in (0, 1, 16, 17, 19683)] == [16, 16, 16, 32, 19696]
    f = empty_field(18, 1000)
    assert f.shape == (18, 1000) and f.stride() == (1008, 1) and f.dtype == torch.float64
    x = np.random.default_rng(0).standard_normal((6, 27 ** 3))
    t = to_field(x)
    assert t.stride(0) % 16 == 0 and np.array_equal(t.numpy(), x)
    a = to_field(np.arange(5.0))
    assert a.shape == (1, 5) and a.stride(0) == 16


def test_bw_stream_validation(L):
    n = 4096
    assert L.tl_bw_stream(n, 3, BASE, BASE + MB, None) == _abi.TL_ERR_INVALID
    assert L.tl_bw_stream(-1, _abi.TL_BW_READ, BASE, BASE + MB, None) == _abi.TL_ERR_SIZE
    assert L.tl_bw_stream(n, _abi.TL_BW_READ, None, BASE + MB, None) == _abi.TL_ERR_NULL
    assert L.tl_bw_stream(n, _abi.TL_BW_READ, BASE, None, None) == _abi.TL_ERR_NULL
    # the partial sums may not overlap the source
    assert L.tl_bw_stream(n, _abi.TL_BW_READ, BASE, BASE + 8 * 100, None) == _abi.TL_ERR_ALIAS
    assert L.tl_bw_stream(n, _abi.TL_BW_WRITE, None, None, None) == _abi.TL_ERR_NULL
    assert L.tl_bw_stream(n, _abi.TL_BW_WRITE, None, BASE + 4, None) == _abi.TL_ERR_ALIGN
    assert L.tl_bw_stream(0, _abi.TL_BW_WRITE, None, None, None) == _abi.TL_OK


def test_interleaved_fields_are_not_overlapping(L):
    """Fields interleaved in one buffer (components of one in the gaps of the
    other's leading dimension) share no element and are accepted; the call
    then stops at the invalid tuning, before any launch.  A single shared
    element is still caught."""
    n = 100
    a = [cf(BASE + i * 64 * MB, n) for i in range(6)]
    a[1] = cf(BASE + 7 * 64 * MB, 2 * n)                    # dg, ld = 2n
    bad = ctypes.pointer(Tune(96, 0, 0, 0))
    out = f(BASE + 7 * 64 * MB + 8 * n, 2 * n)              # dtg in dg's gaps
    assert call_chain(L, n, a, out, bad) == _abi.TL_ERR_INVALID
    out = f(BASE + 7 * 64 * MB + 8 * (n - 1), 2 * n)        # one element of dg shared
    assert call_chain(L, n, a, out, bad) == _abi.TL_ERR_ALIAS
    assert b"dtg" in L.tl_last_error() and b"dg" in L.tl_last_error()


def test_lanes_only_for_christoffel(L):
    """lanes > 1 passes tl_christoffel's checks (the call then stops at the
    invalid block size, which is checked after lanes) and is refused by
    every other entry point."""
    n = 64
    lanes6_bad_block = ctypes.pointer(Tune(96, 0, 0, 0, 6))
    assert L.tl_christoffel(n, cf(BASE, n), cf(BASE + MB, n), f(BASE + 2 * MB, n), None,
                            lanes6_bad_block) == _abi.TL_ERR_INVALID
    assert b"block" in L.tl_last_error()
    a, out = chain_args(n)
    assert call_chain(L, n, a, out, lanes6_bad_block) == _abi.TL_ERR_INVALID
    assert b"lanes" in L.tl_last_error()


def test_bwd_plan_validation(L):
    from paper_1804_10120_amd._abi import DomainBwd
    n = 32
    plan = ctypes.c_void_p()

    def dom(base, outs=True, w=True):
        ins = [cf(base + i * MB, n) for i in range(6)]
        if not w:
            ins[5] = cf(None, n)
        grads = [f(base + (10 + i) * MB, n) if outs else f(None, 0) for i in range(6)]
        return DomainBwd(n, *ins, *grads)

    arr = (DomainBwd * 2)(dom(BASE), dom(BASE + 64 * MB))
    assert L.tl_batch_plan_bwd_create(None, 2, None, ctypes.byref(plan)) == _abi.TL_ERR_NULL
    assert L.tl_batch_plan_bwd_create(arr, 0, None, ctypes.byref(plan)) == _abi.TL_ERR_SIZE
    bad = ctypes.pointer(Tune(96, 0, 0, 0))
    assert L.tl_batch_plan_bwd_create(arr, 2, bad, ctypes.byref(plan)) == _abi.TL_ERR_INVALID
    arr[1] = dom(BASE + 64 * MB, outs=False)
    assert L.tl_batch_plan_bwd_create(arr, 2, bad, ctypes.byref(plan)) == _abi.TL_ERR_NULL
    assert b"domain 1" in L.tl_last_error()
    arr[1] = dom(BASE + 64 * MB, w=False)
    assert L.tl_batch_plan_bwd_create(arr, 2, bad, ctypes.byref(plan)) == _abi.TL_ERR_NULL
    # domain 1 writes its g_bar onto domain 0's dg
    arr[1] = dom(BASE + 64 * MB)
    arr[1].g_bar = Field(BASE + 1 * MB + 8, n)
    assert L.tl_batch_plan_bwd_create(arr, 2, bad, ctypes.byref(plan)) == _abi.TL_ERR_ALIAS
    assert not plan.value


def test_missing_library_raises(monkeypatch, tmp_path):
    """Without libtl.so every entry point fails loudly: there is no fallback."""
    from paper_1804_10120_amd import _abi
    monkeypatch.setattr(_abi, "LIB_PATH", str(tmp_path / "libtl.so"))
    monkeypatch.setattr(_abi, "_lib", None)
    with pytest.raises(RuntimeError, match="no fallback"):
        _abi.lib()

