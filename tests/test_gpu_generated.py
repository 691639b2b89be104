"""Kernels generated from index notation against the oracle and against the
hand-written kernels of the same expressions."""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import DevField, assert_close, dev, need_gpu
from paper_1804_10120_amd import tl_christoffel, tl_dtg_chain, tl_expr
from paper_1804_10120_amd.generated import call, programs
from paper_1804_10120_amd.synth import make_expr_inputs, make_fields

pytestmark = pytest.mark.gpu

SIZES = [1, 65, 1000, 4097]
TUNES = [None, dict(block=64, nt=True), dict(block=512, nt=True, xcd=True, grid_mult=1),
         dict(block=256, nt=True, xcd=True, ptr64=True), dict(block=128, ppt=4, nt=True)]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


def _tid(t):
    return "default" if t is None else "-".join(f"{k}{v}" for k, v in t.items())


def _f(n, seed):
    return make_fields(n, seed=seed)


@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("tune", TUNES, ids=_tid)
def test_christoffel(n, tune):
    f = _f(n, 1)
    gi = oracle.sym_inverse(f["g"])
    (gam,) = call("christoffel", dev(gi), dev(f["dg"]), tune=tune)
    assert_close(gam, oracle.christoffel(gi, f["dg"]), what="generated Gamma")
    hand = tl_christoffel(dev(gi), dev(f["dg"]))
    assert_close(gam, hand.cpu().numpy(), what="generated vs hand-written")


@pytest.mark.parametrize("n", SIZES)
def test_cov_deriv_and_dtg(n):
    f = _f(n, 2)
    gam = oracle.christoffel(oracle.sym_inverse(f["g"]), f["dg"])
    (nb,) = call("cov_deriv", dev(f["dbeta"]), dev(gam), dev(f["beta"]))
    ref = oracle.cov_deriv(gam, f["beta"], f["dbeta"])
    assert_close(nb, ref, what="generated nabla beta")
    (dtg,) = call("dtg", dev(f["alpha"]), dev(f["K"]), dev(ref))
    assert_close(dtg, oracle.dtg(f["alpha"], f["K"], ref), what="generated dtg")


@pytest.mark.parametrize("n", SIZES + [64 ** 3])
@pytest.mark.parametrize("tune", TUNES, ids=_tid)
def test_generated_fused_chain(n, tune):
    f = _f(n, 3)
    gi = oracle.sym_inverse(f["g"])
    (dtg,) = call("dtg_chain_invg", dev(gi), dev(f["dg"]), dev(f["dbeta"]), dev(f["beta"]),
                  dev(f["alpha"]), dev(f["K"]), tune=tune)
    ref = oracle.dtg_chain(f["g"], f["dg"], f["beta"], f["dbeta"], f["K"], f["alpha"])
    assert_close(dtg, ref, what="generated chain")
    hand = tl_dtg_chain(*[dev(f[k]) for k in ("g", "dg", "beta", "dbeta", "K", "alpha")])
    assert_close(dtg, hand.cpu().numpy(), what="generated vs hand-written chain")


FAMILY = ("assign1", "assign2", "assign3", "add1", "add2", "add3", "mult1", "mult2", "mult3",
          "contract1", "contract2", "contract3", "kij")


@pytest.mark.parametrize("name", ["contract1", "contract2", "contract3"])
def test_wide_programs_full_size(name):
    """The programs whose inputs are loaded slice by slice, at 2^21 points and
    a ragged tail in the default launch shape: every element against the
    hand-written kernel, sampled points against the oracle."""
    n = (1 << 21) + 5
    ins = [torch.rand(c, n, dtype=torch.float64, device="cuda") * 2 - 1
           for c in (t["ncomp"] for t in programs()[name]["inputs"])]
    (out,) = call(name, *ins)
    hand = tl_expr(name, *ins)
    assert_close(out, hand, what=f"generated {name} vs hand-written, 2^21 + 5 points")
    idx = torch.tensor([0, 1, 4095, 1 << 20, n - 2, n - 1], device="cuda")
    sub = [np.ascontiguousarray(x[:, idx].cpu().numpy()) for x in ins]
    assert_close(out[:, idx], oracle.expr(name, *sub), what=f"generated {name} vs oracle")


@pytest.mark.parametrize("name", FAMILY)
@pytest.mark.parametrize("n", SIZES)
def test_against_the_expression_kernels(name, n):
    xs = make_expr_inputs(name, n, seed=n)
    (out,) = call(name, *[dev(x) for x in xs])
    assert_close(out, oracle.expr(name, *xs), what=f"generated {name}")
    assert_close(out, tl_expr(name, *[dev(x) for x in xs]).cpu().numpy(), what=name)


@pytest.mark.parametrize("n", SIZES)
def test_listing_examples_and_spacetime_split(n):
    rng = np.random.default_rng(n)
    A, B = rng.uniform(-1, 1, (16, n)), rng.uniform(-1, 1, (16, n))
    (C,) = call("lst_sym_contract", dev(A), dev(B))
    assert_close(C, oracle.expr("lst_sym_contract", A, B), what="symmetric contraction")
    prev = rng.uniform(-1, 1, (10, n))
    D = DevField(prev, pad=3)
    call("lst_fixed_offset", dev(A), dev(B), outs=[D.view])
    torch.cuda.synchronize()
    assert_close(D.view, oracle.expr("lst_fixed_offset", A, B, out=prev), what="fixed/offset")
    assert D.canaries_intact()
    psi = rng.uniform(-1, 1, (10, n))
    g, beta = call("spacetime_split", dev(psi))
    assert np.array_equal(g.cpu().numpy(), oracle.expr("spacetime_g", psi))
    assert np.array_equal(beta.cpu().numpy(), oracle.expr("spacetime_beta", psi))


def test_every_generated_program_is_exercised():
    tested = {"christoffel", "cov_deriv", "dtg", "dtg_chain_invg", "lst_sym_contract",
              "lst_fixed_offset", "spacetime_split"} | set(FAMILY)
    assert set(programs()) == tested


@pytest.mark.parametrize("name", ["contract3", "mult3"])
@pytest.mark.parametrize("block", [512, 1024])
def test_wide_programs_in_large_blocks(name, block):
    """A wide program asked for more threads per block than its cap runs in
    the capped block size, with the same results."""
    n = 3001
    xs = make_expr_inputs(name, n, seed=9)
    (out,) = call(name, *[dev(x) for x in xs], tune=dict(block=block, nt=True))
    assert_close(out, oracle.expr(name, *xs), what=f"generated {name} block={block}")
