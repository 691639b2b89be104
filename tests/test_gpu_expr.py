"""The paper's benchmark expressions (Sec. 5.1) on the GPU against the oracle."""
import numpy as np
import pytest
import torch

import oracle
import oracle_par
from gpu_util import DevField, assert_close, dev, need_gpu
from paper_1804_10120_amd import tl_expr, tl_expr_shape
from paper_1804_10120_amd.synth import EXPR_INPUTS, make_expr_inputs

pytestmark = pytest.mark.gpu

EXPRS = tuple(EXPR_INPUTS)
TUNES = [None, dict(block=64, ppt=1), dict(block=256, ppt=2, nt=True, xcd=True),
         dict(block=128, ppt=1, nt=True, grid_mult=1), dict(block=512, ppt=2),
         dict(block=256, ppt=1, nt=True, xcd=True, ptr64=True), dict(block=256, ppt=4, nt=True),
         dict(block=64, ppt=4, xcd=True, grid_mult=1)]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


def _tid(t):
    return "default" if t is None else "-".join(f"{k}{v}" for k, v in t.items())


def test_shapes_match_synth():
    for name in EXPRS:
        assert tl_expr_shape(name) == (EXPR_INPUTS[name], oracle.expr_shape(name)[1])


@pytest.mark.parametrize("name", EXPRS)
@pytest.mark.parametrize("n", [1, 63, 65, 1000, 4097])
@pytest.mark.parametrize("tune", TUNES, ids=_tid)
def test_expr_vs_oracle(name, n, tune):
    xs = make_expr_inputs(name, n, seed=n)
    out = tl_expr(name, *[dev(x) for x in xs], tune=tune)
    assert_close(out, oracle.expr(name, *xs), what=name)


@pytest.mark.parametrize("name", EXPRS)
def test_expr_layout_and_guard_bands(name):
    n = 777
    xs = make_expr_inputs(name, n, seed=3)
    ins = [DevField(x, pad=5, offset=1) for x in xs]
    oc = tl_expr_shape(name)[1]
    out = DevField.empty(oc, n, pad=3, offset=2)
    tl_expr(name, *[x.view for x in ins], out=out.view)
    torch.cuda.synchronize()
    assert_close(out.view, oracle.expr(name, *xs), what=name)
    assert out.canaries_intact()


@pytest.mark.parametrize("name", EXPRS)
def test_expr_large(name):
    """2^20 points with the default (large-grid) launch shape, every output
    element against the oracle (run on host threads)."""
    n = 1 << 20
    xs = make_expr_inputs(name, n, seed=11)
    out = tl_expr(name, *[dev(x) for x in xs])
    assert_close(out, oracle_par.expr(name, *xs), what=f"{name} 2^20")


def test_assign_is_bitwise_and_exact_integer_products():
    n = 500
    rng = np.random.default_rng(1)
    B = rng.integers(-9, 10, size=(27, n)).astype(np.float64)
    assert torch.equal(tl_expr("assign3", dev(B)).cpu(), torch.from_numpy(B))
    v = [rng.integers(-9, 10, size=(3, n)).astype(np.float64) for _ in range(4)]
    exp = np.einsum("in,jn,kn,ln->ijkln", *v).reshape(81, n)
    assert np.array_equal(tl_expr("mult3", *[dev(x) for x in v]).cpu().numpy(), exp)
