"""tl_batch_run_noalloc (the batched forward chain with its tables in the
library's fixed per-device array) against the batch plan it varies: the same
launch on the same subgrids must give bitwise the same d_t g, and both must
match the oracle.  Two calls in a row, the second with fewer and smaller
subgrids, so the second call runs over tables the first one left behind."""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import assert_close, dev, need_gpu
from paper_1804_10120_amd import BatchPlan, TLError, empty_field, tl_batch_run_noalloc
from paper_1804_10120_amd import _abi
from paper_1804_10120_amd.synth import make_fields

pytestmark = pytest.mark.gpu

KEYS = ("g", "dg", "beta", "dbeta", "K", "alpha")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


def _domains(sizes, seed):
    hosts, devs = [], []
    for d, n in enumerate(sizes):
        f = make_fields(int(n), seed=seed * 1000 + d)
        hosts.append(f)
        devs.append({k: dev(f[k]) for k in KEYS})
    return hosts, devs


def _run_both(hosts, devs, tune):
    """d_t g of every subgrid from a batch plan (direct launch) and from the
    no-allocation entry point, each into its own output fields."""
    plan = BatchPlan(devs, tune=tune)
    plan.run_direct()
    torch.cuda.synchronize()
    ref = [o.clone() for o in plan.outputs]
    plan.close()
    outs = [dict(d, dtg=empty_field(6, h["g"].shape[1], device="cuda")) for h, d in zip(hosts, devs)]
    for o in outs:
        o["dtg"].fill_(np.nan)
    got = tl_batch_run_noalloc(outs, tune=tune)
    torch.cuda.synchronize()
    return ref, got


def _check(hosts, ref, got, what):
    assert len(ref) == len(got)
    for i, (f, a, b) in enumerate(zip(hosts, ref, got)):
        assert torch.equal(a, b), f"{what}: subgrid {i} (n={a.shape[1]}) differs from the plan"
        assert_close(b, oracle.dtg_chain(*[f[k] for k in KEYS]),
                     what=f"{what}: subgrid {i} vs oracle")


@pytest.mark.parametrize("tune", [None, dict(block=64, ppt=2, nt=True, xcd=True, grid_mult=1),
                                  dict(block=256, ppt=1, nt=True, ptr64=True)],
                         ids=["default", "b64ppt2xcd_persistent", "b256ptr64"])
def test_noalloc_matches_plan_two_calls(tune):
    rng = np.random.default_rng(11)
    # first call: 70 subgrids (more than three table-writing launches of
    # descriptors), empty and one-point ones among them, about 1.2 M points
    big = [int(x) ** 3 for x in rng.integers(8, 40, size=60)]
    sizes1 = big + [0, 1, 0, 17, 63, 64, 65, 1000, 4097, 3]
    hosts1, devs1 = _domains(sizes1, seed=21)
    ref1, got1 = _run_both(hosts1, devs1, tune)
    _check(hosts1, ref1, got1, "first call")
    # second call: fewer, smaller subgrids, over the tables of the first
    sizes2 = [5, 0, 700, 8 ** 3, 2]
    hosts2, devs2 = _domains(sizes2, seed=22)
    ref2, got2 = _run_both(hosts2, devs2, tune)
    _check(hosts2, ref2, got2, "second call")


def test_noalloc_on_a_side_stream_and_repeated():
    """On a stream of its own, called again on the same fields: the results do
    not change."""
    sizes = [9 ** 3, 0, 30 ** 3, 1]
    hosts, devs = _domains(sizes, seed=23)
    outs = [dict(d, dtg=empty_field(6, h["g"].shape[1], device="cuda")) for h, d in zip(hosts, devs)]
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        first = [o.clone() for o in tl_batch_run_noalloc(outs, stream=s)]
        for o in outs:
            o["dtg"].zero_()
        again = tl_batch_run_noalloc(outs, stream=s)
    s.synchronize()
    for f, a, b in zip(hosts, first, again):
        assert torch.equal(a, b)
        assert_close(b, oracle.dtg_chain(*[f[k] for k in KEYS]), what="side stream")


def test_noalloc_rejects_beyond_its_limits():
    sizes = [10] * 3
    hosts, devs = _domains(sizes, seed=24)
    outs = [dict(d, dtg=empty_field(6, 10, device="cuda")) for d in devs]
    with pytest.raises(TLError) as e:
        tl_batch_run_noalloc(outs * 342)      # 1026 subgrids
    assert e.value.status == _abi.TL_ERR_SIZE
    with pytest.raises(ValueError):
        tl_batch_run_noalloc([dict(devs[0])])  # no output given


def test_noalloc_captured_in_a_graph():
    """Captured into a HIP graph (it launches kernels only: no allocation, copy
    or memset) and replayed several times, with eager work and
    synchronisation between the replays: every replay equals the eager call."""
    sizes = [20 ** 3, 7, 0, 33 ** 3]
    hosts, devs = _domains(sizes, seed=25)
    outs = [dict(d, dtg=empty_field(6, h["g"].shape[1], device="cuda")) for h, d in zip(hosts, devs)]
    eager = [o.clone() for o in tl_batch_run_noalloc(outs)]
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        tl_batch_run_noalloc(outs)
    for rep in range(3):
        for o in outs:
            o["dtg"].fill_(np.nan)
        # other eager work on the same device between the replays
        other = [dict(d, dtg=empty_field(6, h["g"].shape[1], device="cuda"))
                 for h, d in zip(hosts[:2], devs[:2])]
        tl_batch_run_noalloc(other)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        for i, (a, o) in enumerate(zip(eager, outs)):
            assert torch.equal(a, o["dtg"]), f"replay {rep}: subgrid {i} differs from the eager call"
    for f, o in zip(hosts, outs):
        assert_close(o["dtg"], oracle.dtg_chain(*[f[k] for k in KEYS]), what="graph replay")


def test_noalloc_at_its_limits():
    """The largest batches the fixed array holds: 1024 subgrids (34 table-writing
    launches), and one subgrid of exactly 262144 tiles of 64 points (16.8 M
    points, fields made on the device); each bitwise equal to a plan, the
    oracle checked on every subgrid of the first and on sampled points of the
    second."""
    rng = np.random.default_rng(31)
    sizes = [int(x) for x in rng.integers(0, 40, size=_abi.TL_NOALLOC_MAX_DOMAINS)]
    hosts, devs = _domains(sizes, seed=26)
    ref, got = _run_both(hosts, devs, None)
    _check(hosts, ref, got, "1024 subgrids")
    del hosts, devs, ref, got

    tune = dict(block=64, ppt=1, nt=True)
    n = 64 * _abi.TL_NOALLOC_MAX_TILES
    gen = torch.Generator(device="cuda").manual_seed(7)
    d = {}
    for k, c in (("g", 6), ("dg", 18), ("beta", 3), ("dbeta", 9), ("K", 6), ("alpha", 1)):
        d[k] = torch.rand(c, n, dtype=torch.float64, device="cuda", generator=gen) - 0.5
    d["g"][[0, 3, 5]] += 2.5      # diagonal entries: a well-conditioned, diagonally dominant g
    d["alpha"] += 1.0
    plan = BatchPlan([d], tune=tune)
    plan.run_direct()
    torch.cuda.synchronize()
    ref = plan.outputs[0].clone()
    plan.close()
    out = dict(d, dtg=empty_field(6, n, device="cuda"))
    tl_batch_run_noalloc([out], tune=tune)
    torch.cuda.synchronize()
    assert torch.equal(ref, out["dtg"]), "max-tiles batch differs from the plan"
    idx = np.unique(np.concatenate([np.arange(64), n - 64 + np.arange(64),
                                    np.random.default_rng(3).integers(0, n, 4096)]))
    ti = torch.from_numpy(idx).cuda()
    sub = [d[k][:, ti].cpu().numpy() for k in KEYS]
    assert_close(out["dtg"][:, ti], oracle.dtg_chain(*sub), what="max-tiles batch vs oracle")
