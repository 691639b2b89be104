"""Randomised parity: the fused chain, the adjoint, the one-pass forward +
adjoint and the Christoffel kernel against the oracle on layouts, sizes and
launch shapes drawn by hypothesis (derandomised, so every run draws the same
cases).  Each case also checks that nothing outside the outputs was written."""
import numpy as np
import pytest
import torch
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

import oracle
from gpu_util import DevField, assert_close, need_gpu
from paper_1804_10120_amd import (tl_christoffel, tl_dtg_chain, tl_dtg_chain_bwd,
                                  tl_dtg_chain_fwd_bwd)
from paper_1804_10120_amd.synth import make_fields

pytestmark = pytest.mark.gpu

KEYS = ("g", "dg", "beta", "dbeta", "K", "alpha")
GRADS = (6, 18, 3, 9, 6, 1)

tunes = st.one_of(
    st.none(),
    st.fixed_dictionaries({"block": st.sampled_from([64, 128, 256, 512, 1024]),
                           "ppt": st.sampled_from([1, 2, 4]), "nt": st.booleans(),
                           "xcd": st.booleans(), "ptr64": st.booleans(),
                           "grid_mult": st.sampled_from([0, 0, 1, 3])}))
layouts = st.tuples(st.integers(0, 37), st.integers(0, 5))     # (pad, offset) in doubles
SETTINGS = settings(max_examples=40, deadline=None, derandomize=True,
                    suppress_health_check=list(HealthCheck))


@SETTINGS
@given(n=st.integers(1, 5000), tune=tunes, lay=layouts, seed=st.integers(0, 10 ** 6))
def test_chain_random(n, tune, lay, seed):
    need_gpu()
    f = make_fields(n, seed=seed)
    ins = [DevField(f[k], pad=lay[0], offset=lay[1]) for k in KEYS]
    out = DevField.empty(6, n, pad=lay[0] + 1, offset=lay[1])
    tl_dtg_chain(*[x.view for x in ins], out.view, tune=tune)
    torch.cuda.synchronize()
    assert_close(out.view, oracle.dtg_chain(*[f[k] for k in KEYS]), what=f"chain n={n} {tune}")
    assert out.canaries_intact()


@SETTINGS
@given(n=st.integers(1, 5000), tune=tunes, lay=layouts, seed=st.integers(0, 10 ** 6),
       one_pass=st.booleans())
def test_adjoint_random(n, tune, lay, seed, one_pass):
    need_gpu()
    f = make_fields(n, seed=seed)
    ref = oracle.dtg_chain_vjp(tuple(f[k] for k in KEYS), f["W"])
    dev = {k: DevField(f[k], pad=lay[0], offset=lay[1]).view for k in KEYS + ("W",)}
    outs = [DevField.empty(c, n, pad=lay[0] + 2, offset=lay[1]) for c in GRADS]
    if one_pass:
        dtg = DevField.empty(6, n, pad=lay[0], offset=lay[1] + 1)
        tl_dtg_chain_fwd_bwd(*[dev[k] for k in KEYS], dev["W"], dtg.view,
                             [o.view for o in outs], tune=tune)
    else:
        tl_dtg_chain_bwd(dev["g"], dev["dg"], dev["beta"], dev["K"], dev["alpha"], dev["W"],
                         *[o.view for o in outs], tune=tune)
    torch.cuda.synchronize()
    for k, o in zip(KEYS, outs):
        assert_close(o.view, ref[k], what=f"{k}_bar n={n} {tune} one_pass={one_pass}")
        assert o.canaries_intact()
    if one_pass:
        assert_close(dtg.view, oracle.dtg_chain(*[f[k] for k in KEYS]), what="d_t g one pass")
        assert dtg.canaries_intact()


@SETTINGS
@given(n=st.integers(1, 5000), block=st.sampled_from([64, 256, 1024]),
       lanes=st.sampled_from([0, 1, 2, 3, 6, 9, 18]), lay=layouts, seed=st.integers(0, 10 ** 6))
def test_christoffel_random(n, block, lanes, lay, seed):
    need_gpu()
    f = make_fields(n, seed=seed)
    gi = oracle.sym_inverse(f["g"])
    ginv = DevField(gi, pad=lay[0], offset=lay[1])
    dg = DevField(f["dg"], pad=lay[0], offset=lay[1])
    out = DevField.empty(18, n, pad=lay[0], offset=lay[1] + 2)
    tl_christoffel(ginv.view, dg.view, out.view, tune=dict(block=block, nt=True, lanes=lanes))
    torch.cuda.synchronize()
    assert_close(out.view, oracle.christoffel(gi, f["dg"]), what=f"gamma n={n} lanes={lanes}")
    assert out.canaries_intact()
