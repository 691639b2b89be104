"""The adjoint kernel and the autograd wrapper against the oracle's
reverse-mode gradients, closed forms and central finite differences."""
import numpy as np
import pytest
import torch

import oracle
import oracle_par
from gpu_util import DevField, assert_close, dev, need_gpu
from paper_1804_10120_amd import dtg_chain, tl_dtg_chain, tl_dtg_chain_bwd, tl_dtg_chain_fwd_bwd
from paper_1804_10120_amd.synth import config_seed, make_fields

pytestmark = pytest.mark.gpu

KEYS = ("g", "dg", "beta", "dbeta", "K", "alpha")
TUNES = [None, dict(block=64, ppt=1), dict(block=128, ppt=2), dict(block=256, ppt=2, nt=True),
         dict(block=512, ppt=1, grid_mult=1), dict(block=256, ppt=1, nt=True, xcd=True),
         dict(block=64, ppt=2, nt=True, xcd=True, grid_mult=1),
         dict(block=256, ppt=1, nt=True, xcd=True, ptr64=True), dict(block=512, ppt=2, nt=True, ptr64=True)]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


def _vjp_ref(f):
    return oracle.dtg_chain_vjp(tuple(f[k] for k in KEYS), f["W"])


def _bwd(f, tune=None, want=None, **kw):
    return tl_dtg_chain_bwd(dev(f["g"]), dev(f["dg"]), dev(f["beta"]), dev(f["K"]),
                            dev(f["alpha"]), dev(f["W"]), want=want, tune=tune, **kw)


def _tid(t):
    return "default" if t is None else "-".join(f"{k}{v}" for k, v in t.items())


@pytest.mark.parametrize("n", [1, 2, 63, 65, 512, 4097, 10007, 40000])
@pytest.mark.parametrize("tune", TUNES, ids=_tid)
def test_bwd_vs_oracle_vjp(n, tune):
    f = make_fields(n, seed=100 + n)
    ref = _vjp_ref(f)
    got = _bwd(f, tune)
    for k, x in zip(KEYS, got):
        assert_close(x, ref[k], what=f"{k}_bar")


def test_bwd_closed_forms_exact():
    n = 1000
    f = make_fields(n, seed=7)
    gb, dgb, bb, dbb, Kb, ab = _bwd(f)
    assert np.array_equal(Kb.cpu().numpy(), -2.0 * f["alpha"] * f["W"])
    S = np.array([[0, 1, 2], [1, 3, 4], [2, 4, 5]])
    exp = np.stack([f["W"][S[i, j]] * (2.0 if i == j else 1.0) for j in range(3) for i in range(3)])
    assert np.array_equal(dbb.cpu().numpy(), exp)


def test_bwd_full_size():
    """Adjoint at 64^3 points in the benchmark's launch shape."""
    n = 64 ** 3
    f = make_fields(n, seed=config_seed(5))
    ref = _vjp_ref(f)
    got = _bwd(f)
    for k, x in zip(KEYS, got):
        assert_close(x, ref[k], what=f"{k}_bar 64^3")


def test_bwd_full_size_128():
    """Adjoint at 128^3 points, the benchmark's dominant kernel in the launch
    shape the benchmark times: every one of the 43 gradient components at
    every point against the oracle (run on host threads)."""
    n = 128 ** 3
    f = make_fields(n, seed=config_seed(3))
    got = [x.cpu().numpy() for x in _bwd(f)]
    ref = oracle_par.dtg_chain_vjp(f)
    for k, x in zip(KEYS, got):
        assert_close(x, ref[k], what=f"{k}_bar 128^3")


@pytest.mark.parametrize("tune", [dict(block=1024, ppt=2, nt=True, xcd=True),
                                  dict(block=512, ppt=2, nt=True)], ids=_tid)
def test_bwd_two_point_shapes_full_size(tune):
    """Two points per lane (16-byte loads and stores) at 128^3 points against
    one point per lane, element by element: the 16-byte stores are written with
    explicit wait states, and a missing one shows only at this size, as a
    fraction of a percent of wrong points."""
    n = 128 ** 3
    f = make_fields(n, seed=config_seed(3) + 1)
    ref = _bwd(f)
    got = _bwd(f, tune)
    for k, x, r in zip(KEYS, got, ref):
        assert_close(x, r, what=f"{k}_bar 128^3 {_tid(tune)}")


@pytest.mark.parametrize("want", [(1, 0, 0, 0, 0, 0), (0, 1, 0, 0, 0, 0), (0, 0, 1, 0, 1, 0),
                                  (0, 0, 0, 1, 0, 1), (1, 1, 1, 1, 1, 1)])
@pytest.mark.parametrize("tune", [None, dict(block=128, ppt=2, nt=True, xcd=True)], ids=_tid)
def test_bwd_output_subsets(want, tune):
    n = 999
    f = make_fields(n, seed=13)
    ref = _vjp_ref(f)
    got = _bwd(f, want=want, tune=tune)
    for k, w, x in zip(KEYS, want, got):
        if w:
            assert_close(x, ref[k], what=f"{k}_bar subset")
        else:
            assert x is None


def test_bwd_guard_bands_and_padding():
    n = 1553
    f = make_fields(n, seed=17)
    ref = _vjp_ref(f)
    outs = [DevField.empty(c, n, pad=3, offset=1) for c in (6, 18, 3, 9, 6, 1)]
    tl_dtg_chain_bwd(dev(f["g"]), dev(f["dg"]), dev(f["beta"]), dev(f["K"]), dev(f["alpha"]),
                     dev(f["W"]), *[o.view for o in outs])
    torch.cuda.synchronize()
    for k, o in zip(KEYS, outs):
        assert_close(o.view, ref[k], what=f"{k}_bar padded")
        assert o.canaries_intact()


def _leafs(f, requires=KEYS):
    return {k: dev(f[k]).requires_grad_(k in requires) for k in KEYS}


def test_autograd_matches_oracle():
    n = 4097
    f = make_fields(n, seed=19)
    t = _leafs(f)
    out = dtg_chain(*[t[k] for k in KEYS])
    out.backward(dev(f["W"]))
    ref = _vjp_ref(f)
    for k in KEYS:
        assert_close(t[k].grad, ref[k], what=f"autograd {k}")


def test_autograd_subset_and_alpha_1d():
    n = 300
    f = make_fields(n, seed=23)
    t = _leafs(f, requires=("K", "alpha"))
    t["alpha"] = torch.from_numpy(f["alpha"][0].copy()).cuda().requires_grad_(True)
    out = dtg_chain(*[t[k] for k in KEYS])
    (out * dev(f["W"])).sum().backward()
    ref = _vjp_ref(f)
    assert_close(t["K"].grad, ref["K"], what="K grad")
    assert t["alpha"].grad.shape == (n,)
    assert_close(t["alpha"].grad[None], ref["alpha"], what="alpha grad")
    assert t["g"].grad is None


def test_finite_differences_8cubed():
    """Central differences (h = 1e-6) of L_p = sum_s W_s d_t g_s(p) computed with
    the GPU forward, one component perturbed at all points at once."""
    n = 8 ** 3
    h = 1e-6
    f = make_fields(n, seed=config_seed(5))
    W = f["W"]
    got = dict(zip(KEYS, _bwd(f)))

    def loss(ff):
        out = tl_dtg_chain(*[dev(ff[k]) for k in KEYS]).cpu().numpy()
        return (W * out).sum(0)

    for k in KEYS:
        fd = np.empty_like(f[k])
        for c in range(f[k].shape[0]):
            fp = {kk: v.copy() for kk, v in f.items()}
            fm = {kk: v.copy() for kk, v in f.items()}
            fp[k][c] += h
            fm[k][c] -= h
            fd[c] = (loss(fp) - loss(fm)) / (2 * h)
        assert_close(got[k], fd, tol=1e-6, what=f"FD {k}")


# --------------------------------------------------------------------------- fused forward + adjoint

def _fwd_bwd(f, tune=None, want=None, **kw):
    return tl_dtg_chain_fwd_bwd(*[dev(f[k]) for k in KEYS], dev(f["W"]), want=want, tune=tune,
                                **kw)


@pytest.mark.parametrize("n", [1, 3, 64, 1000, 4097, 40001])
@pytest.mark.parametrize("tune", TUNES, ids=_tid)
def test_fwd_bwd_vs_oracle(n, tune):
    f = make_fields(n, seed=300 + n)
    ref = _vjp_ref(f)
    dtg, grads = _fwd_bwd(f, tune)
    assert_close(dtg, oracle.dtg_chain(*[f[k] for k in KEYS]), what="d_t g")
    for k, x in zip(KEYS, grads):
        assert_close(x, ref[k], what=f"{k}_bar")


def test_fwd_bwd_matches_the_two_kernels():
    """Same values as tl_dtg_chain followed by tl_dtg_chain_bwd (the same
    per-point arithmetic, though the compiler may contract it differently)."""
    n = 20000
    f = make_fields(n, seed=31)
    dtg, grads = _fwd_bwd(f)
    assert_close(dtg, tl_dtg_chain(*[dev(f[k]) for k in KEYS]), what="d_t g vs forward kernel")
    for k, a, b in zip(KEYS, grads, _bwd(f)):
        assert_close(a, b, what=f"{k}_bar vs adjoint kernel")


@pytest.mark.parametrize("want", [(1, 0, 0, 0, 0, 0, 0), (0, 1, 1, 0, 0, 0, 0),
                                  (0, 0, 0, 1, 1, 1, 1), (1, 0, 1, 0, 1, 0, 1)])
def test_fwd_bwd_output_subsets(want):
    n = 777
    f = make_fields(n, seed=37)
    ref = _vjp_ref(f)
    dtg, grads = _fwd_bwd(f, want=want)
    if want[0]:
        assert_close(dtg, oracle.dtg_chain(*[f[k] for k in KEYS]), what="d_t g subset")
    else:
        assert dtg is None
    for k, w, x in zip(KEYS, want[1:], grads):
        if w:
            assert_close(x, ref[k], what=f"{k}_bar subset")
        else:
            assert x is None


def test_fwd_bwd_guard_bands_and_padding():
    n = 2111
    f = make_fields(n, seed=41)
    ref = _vjp_ref(f)
    ins = [DevField(f[k], pad=5, offset=3) for k in KEYS + ("W",)]
    dtg = DevField.empty(6, n, pad=2, offset=1)
    outs = [DevField.empty(c, n, pad=3, offset=1) for c in (6, 18, 3, 9, 6, 1)]
    tl_dtg_chain_fwd_bwd(*[x.view for x in ins], dtg.view, [o.view for o in outs])
    torch.cuda.synchronize()
    assert_close(dtg.view, oracle.dtg_chain(*[f[k] for k in KEYS]), what="d_t g padded")
    assert dtg.canaries_intact()
    for k, o in zip(KEYS, outs):
        assert_close(o.view, ref[k], what=f"{k}_bar padded")
        assert o.canaries_intact()


def test_fwd_bwd_full_size():
    """Forward and adjoint in one kernel at 128^3 points in the default launch
    shape: d_t g and all 43 gradient components at every point against the
    oracle (run on host threads)."""
    n = 128 ** 3
    f = make_fields(n, seed=config_seed(3) + 2, fields=KEYS + ("W",))
    dtg, grads = _fwd_bwd(f)
    assert_close(dtg, oracle_par.dtg_chain(f), what="d_t g 128^3")
    del dtg
    ref = oracle_par.dtg_chain_vjp(f)
    for k, x in zip(KEYS, grads):
        assert_close(x, ref[k], what=f"{k}_bar 128^3")


def test_bwd_output_spanning_more_than_4_GiB():
    """dg_bar in a buffer whose 18 components span more than 4 GiB: the call
    takes the 64-bit pointer path; values match the oracle and nothing outside
    the written components changes."""
    n = 2049
    ld = (1 << 25) + 32
    f = make_fields(n, seed=43)
    big = torch.full((18 * ld,), 3.25, dtype=torch.float64, device="cuda")
    dgb = big.view(18, ld)[:, :n]
    tl_dtg_chain_bwd(dev(f["g"]), dev(f["dg"]), dev(f["beta"]), dev(f["K"]), dev(f["alpha"]),
                     dev(f["W"]), dg_bar=dgb, want=(0, 1, 0, 0, 0, 0))
    torch.cuda.synchronize()
    assert_close(dgb, _vjp_ref(f)["dg"], what="dg_bar over 4 GiB")
    rest = big.view(18, ld)[:, n:n + 4096]
    assert bool((rest == 3.25).all())
    del big, dgb, rest
    torch.cuda.empty_cache()


def test_autograd_step_captured_in_a_graph():
    """Forward and backward through the autograd Function captured once into a
    HIP graph and replayed on new inputs (copied into the captured tensors
    between replays, with synchronisation): every replay matches the oracle."""
    n = 3001
    f0 = make_fields(n, seed=61)
    leaf = {k: torch.from_numpy(f0[k]).cuda().requires_grad_(True) for k in KEYS}
    w = torch.from_numpy(f0["W"]).cuda()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):           # warm-up outside the capture
        for _ in range(2):
            for t in leaf.values():
                t.grad = None
            dtg_chain(*[leaf[k] for k in KEYS]).backward(w)
    torch.cuda.current_stream().wait_stream(side)
    for t in leaf.values():
        t.grad = None
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        out = dtg_chain(*[leaf[k] for k in KEYS])
        out.backward(w)
    for rep in range(3):
        f = make_fields(n, seed=62 + rep)
        with torch.no_grad():
            for k in KEYS:
                leaf[k].copy_(torch.from_numpy(f[k]))
            w.copy_(torch.from_numpy(f["W"]))
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert_close(out, oracle.dtg_chain(*[f[k] for k in KEYS]), what=f"replay {rep} d_t g")
        ref = _vjp_ref(f)
        for k in KEYS:
            assert_close(leaf[k].grad, ref[k], what=f"replay {rep} grad {k}")
