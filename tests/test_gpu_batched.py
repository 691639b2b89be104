"""Many subgrids in one graph-captured persistent launch: every subgrid equals
the plain fused kernel on that subgrid and the oracle."""
import numpy as np
import pytest
import torch

import oracle
import oracle_par
from gpu_util import assert_close, dev, need_gpu
from paper_1804_10120_amd import BatchPlan, tl_dtg_chain, tl_dtg_chain_bwd
from paper_1804_10120_amd.synth import config_seed, domain_edges, make_fields

pytestmark = pytest.mark.gpu

KEYS = ("g", "dg", "beta", "dbeta", "K", "alpha")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


def _domains(sizes, seed=0):
    hosts, devs = [], []
    for d, n in enumerate(sizes):
        f = make_fields(int(n), seed=seed * 1000 + d)
        hosts.append(f)
        devs.append({k: dev(f[k]) for k in KEYS})
    return hosts, devs


def _check(plan, hosts, devs, tune=None):
    for f, d, out in zip(hosts, devs, plan.outputs):
        ref = oracle.dtg_chain(*[f[k] for k in KEYS])
        assert_close(out, ref, what=f"domain n={out.shape[1]}")
        plain = tl_dtg_chain(*[d[k] for k in KEYS], tune=tune)
        if not torch.equal(plain, out):     # same per-point body: expected bitwise
            assert_close(out, plain.cpu().numpy(), what="batched vs plain kernel")


@pytest.mark.parametrize("tune", [None, dict(block=64, ppt=1, grid_mult=1),
                                  dict(block=256, ppt=2, nt=True, grid_mult=2),
                                  dict(block=128, ppt=1, grid_mult=0),
                                  dict(block=64, ppt=1, nt=True, xcd=True, grid_mult=1),
                                  dict(block=128, ppt=1, nt=True, ptr64=True)],
                         ids=["default", "b64", "b256ppt2nt", "b128grid", "b64xcd", "b128ptr64"])
def test_small_batch(tune):
    sizes = [1, 0, 63, 64, 65, 512, 1000, 4097, 0, 27, 8 ** 3, 12 ** 3, 3]
    hosts, devs = _domains(sizes, seed=1)
    plan = BatchPlan(devs, tune=tune)
    assert plan.points == sum(sizes)
    plan.run()
    torch.cuda.synchronize()
    _check(plan, hosts, devs, tune)
    plan.close()


@pytest.mark.parametrize("tune", [dict(block=64, ppt=1, grid_mult=1),
                                  dict(block=64, ppt=2, nt=True, xcd=True, grid_mult=1)],
                         ids=["b64", "b64xcd"])
def test_persistent_chunks_cross_subgrids(tune):
    """More tiles than blocks: each block walks a chunk of tiles that spans
    several subgrids (including empty and one-point ones)."""
    rng = np.random.default_rng(5)
    sizes = [int(x) for x in rng.integers(0, 2500, size=40)] + [0, 1, 1]
    hosts, devs = _domains(sizes, seed=6)
    plan = BatchPlan(devs, tune=tune)
    assert plan.tiles > plan.blocks
    plan.run()
    torch.cuda.synchronize()
    _check(plan, hosts, devs, tune)
    plan.close()


def test_replay_and_direct_are_idempotent():
    sizes = [100, 2000, 30000, 7]
    hosts, devs = _domains(sizes, seed=2)
    plan = BatchPlan(devs)
    plan.run()
    torch.cuda.synchronize()
    first = [o.clone() for o in plan.outputs]
    for o in plan.outputs:
        o.fill_(0.0)
    for _ in range(3):
        plan.run()
        torch.cuda.synchronize()
        assert all(torch.equal(a, b) for a, b in zip(first, plan.outputs))
    for o in plan.outputs:
        o.fill_(0.0)
    plan.run_direct()
    torch.cuda.synchronize()
    assert all(torch.equal(a, b) for a, b in zip(first, plan.outputs))
    _check(plan, hosts, devs)


def test_new_plan_after_pointer_change():
    sizes = [500, 700]
    hosts, devs = _domains(sizes, seed=3)
    plan = BatchPlan(devs)
    plan.run()
    hosts2, devs2 = _domains(sizes, seed=4)
    plan.close()
    plan2 = BatchPlan(devs2)
    plan2.run()
    torch.cuda.synchronize()
    _check(plan2, hosts2, devs2)


def _oracle_per_domain(hosts, fn):
    """The oracle (on host threads) over all subgrids at once, split back per
    subgrid."""
    sizes = [f["g"].shape[1] for f in hosts]
    cut = np.cumsum(sizes)[:-1]
    res = fn({k: np.concatenate([f[k] for f in hosts], axis=1) for k in hosts[0]})
    if isinstance(res, dict):
        parts = {k: np.split(v, cut, axis=1) for k, v in res.items()}
        return [{k: parts[k][d] for k in res} for d in range(len(sizes))]
    return np.split(res, cut, axis=1)


def test_full_multidomain_workload():
    """256 subgrids with edges uniform on 8..48 (the benchmark's batch, its
    fields with the leading dimension padded to 16 doubles as the benchmark
    stores them): every subgrid against the oracle element by element, and
    against the plain kernel."""
    from paper_1804_10120_amd import to_field
    edges = domain_edges(256, seed=config_seed(4))
    sizes = [int(e) ** 3 for e in edges]
    hosts = [make_fields(n, seed=config_seed(4) * 1000 + d, fields=KEYS)
             for d, n in enumerate(sizes)]
    devs = [{k: to_field(f[k], device="cuda") for k in KEYS} for f in hosts]
    plan = BatchPlan(devs)
    plan.run()
    torch.cuda.synchronize()
    refs = _oracle_per_domain(hosts, oracle_par.dtg_chain)
    for d in range(256):
        assert_close(plan.outputs[d], refs[d], what=f"subgrid {d} vs oracle")
        plain = tl_dtg_chain(*[devs[d][k] for k in KEYS])
        if not torch.equal(plain, plan.outputs[d]):
            assert_close(plan.outputs[d], plain.cpu().numpy(), what=f"subgrid {d} vs plain")
    plan.close()


def test_padded_subgrids():
    """Subgrids in fields whose leading dimension is padded to 16 doubles (the
    layout the benchmark uses), outputs allocated by the plan the same way."""
    from paper_1804_10120_amd import to_field
    sizes = [27, 1000, 4913, 17 ** 3, 1, 16]
    hosts = [make_fields(n, seed=5000 + d) for d, n in enumerate(sizes)]
    devs = [{k: to_field(f[k], device="cuda") for k in KEYS} for f in hosts]
    plan = BatchPlan(devs)
    plan.run()
    torch.cuda.synchronize()
    for out, n in zip(plan.outputs, sizes):
        assert out.shape == (6, n) and out.stride(0) % 16 == 0
    _check(plan, hosts, devs)
    plan.close()


def test_autotuned_plan(tmp_path, monkeypatch):
    """The autotuner picks one of the candidate shapes for a set of subgrids,
    caches it, and tune="auto" builds the plan from the cache; the outputs
    equal the default plan's (same per-point body)."""
    from paper_1804_10120_amd import autotune
    monkeypatch.setenv("TLMI_TUNE_CACHE", str(tmp_path / "tune.json"))
    sizes = [8 ** 3, 13 ** 3, 1000, 65, 20 ** 3, 1]
    hosts, devs = _domains(sizes, seed=9)
    cands = [dict(block=128, ppt=1, nt=True), dict(block=256, ppt=1, nt=True, xcd=True),
             dict(block=64, ppt=2, nt=True, grid_mult=2)]
    res = autotune.tune_plan(devs, tunes=cands, reps=3, warmup=1)
    assert res["tune"] in cands and len(res["table"]) == 3
    assert autotune.lookup_plan(devs) == res["tune"]

    def no_retune(*a, **k):
        raise AssertionError("tune='auto' re-tuned although the shape is cached")
    monkeypatch.setattr(autotune, "tune_plan", no_retune)
    auto = BatchPlan(devs, tune="auto")
    ref = BatchPlan(devs)
    auto.run()
    ref.run()
    torch.cuda.synchronize()
    for a, b in zip(auto.outputs, ref.outputs):
        assert torch.equal(a, b)
    _check(auto, hosts, devs)
    auto.close()
    ref.close()


# --------------------------------------------------------------------------- the adjoint

GRADS = ("g", "dg", "beta", "dbeta", "K", "alpha")


def _bwd_domains(sizes, seed):
    hosts, devs = [], []
    for d, n in enumerate(sizes):
        f = make_fields(int(n), seed=seed * 1000 + d)
        hosts.append(f)
        devs.append({k: dev(f[k]) for k in ("g", "dg", "beta", "K", "alpha", "W")})
    return hosts, devs


@pytest.mark.parametrize("tune", [None, dict(block=64, ppt=1, nt=True),
                                  dict(block=256, ppt=2, nt=True, grid_mult=2),
                                  dict(block=128, ppt=1, nt=True, xcd=True, ptr64=True)],
                         ids=["default", "b64", "b256ppt2grid", "b128xcdptr64"])
def test_bwd_plan_small_batch(tune):
    """Each subgrid's gradients equal the oracle's VJP and the plain adjoint
    kernel's (same per-point body)."""
    sizes = [1, 0, 63, 64, 65, 1000, 4097, 0, 27, 9 ** 3, 3]
    hosts, devs = _bwd_domains(sizes, seed=21)
    plan = BatchPlan(devs, tune=tune, kind="bwd")
    assert plan.points == sum(sizes)
    plan.run()
    torch.cuda.synchronize()
    for f, d, outs in zip(hosts, devs, plan.outputs):
        if f["g"].shape[1] == 0:
            continue
        ref = oracle.dtg_chain_vjp(tuple(f[k] for k in KEYS), f["W"])
        plain = tl_dtg_chain_bwd(d["g"], d["dg"], d["beta"], d["K"], d["alpha"], d["W"])
        for k, o, p in zip(GRADS, outs, plain):
            assert_close(o, ref[k], what=f"batched {k}_bar n={f['g'].shape[1]}")
            assert_close(o, p, what=f"batched vs plain {k}_bar")
    plan.close()


def test_bwd_plan_wanted_subset_and_graph_replay():
    sizes = [500, 1, 2048, 77]
    hosts, devs = _bwd_domains(sizes, seed=22)
    want = (0, 1, 0, 0, 1, 1)
    plan = BatchPlan(devs, kind="bwd", want=want)
    for rep in range(3):                    # replays with eager work in between
        for outs in plan.outputs:
            for o in outs:
                if o is not None:
                    o.fill_(-1.0)
        torch.cuda.synchronize()
        plan.run()
        torch.cuda.synchronize()
        for f, outs in zip(hosts, plan.outputs):
            ref = oracle.dtg_chain_vjp(tuple(f[k] for k in KEYS), f["W"])
            for k, w, o in zip(GRADS, want, outs):
                if w:
                    assert_close(o, ref[k], what=f"replay {rep} {k}_bar")
                else:
                    assert o is None
    plan.close()


def test_bwd_plan_full_multidomain_workload():
    """256 subgrids with edges uniform on 8..48: every gradient component of
    every subgrid against the oracle element by element, and against the plain
    adjoint kernel."""
    edges = domain_edges(256, seed=config_seed(4))
    sizes = [int(e) ** 3 for e in edges]
    hosts, devs = _bwd_domains(sizes, seed=23)
    plan = BatchPlan(devs, kind="bwd")
    plan.run()
    torch.cuda.synchronize()
    refs = _oracle_per_domain(hosts, oracle_par.dtg_chain_vjp)
    for i, (d, outs, ref) in enumerate(zip(devs, plan.outputs, refs)):
        plain = tl_dtg_chain_bwd(d["g"], d["dg"], d["beta"], d["K"], d["alpha"], d["W"])
        for k, o, p in zip(GRADS, outs, plain):
            assert_close(o, ref[k], what=f"subgrid {i} {k}_bar vs oracle")
            assert_close(o, p, what=f"subgrid {i} {k}_bar vs plain")
    plan.close()


def test_blocked_layout_through_plans():
    """A grid cut into blocks of T points whose fields lie next to each other
    in one allocation per block ([blocks][components][T]), run as one plan
    per direction: equal to the plain kernels on the same values stored
    component-major, and to the oracle."""
    T, nb = 4096, 6
    ncin = {"g": 6, "dg": 18, "beta": 3, "dbeta": 9, "K": 6, "alpha": 1, "W": 6}
    f = make_fields(T * nb, seed=31)
    blk = torch.empty(nb, sum(ncin.values()) * T, dtype=torch.float64, device="cuda")
    fwd_out = torch.empty(nb, 6 * T, dtype=torch.float64, device="cuda")
    bwd_out = torch.empty(nb, 43 * T, dtype=torch.float64, device="cuda")
    fdoms, bdoms = [], []
    for b in range(nb):
        views, o = {}, 0
        for k, c in ncin.items():
            views[k] = blk[b, o * T:(o + c) * T].view(c, T)
            views[k].copy_(torch.from_numpy(np.ascontiguousarray(f[k][:, b * T:(b + 1) * T])))
            o += c
        fdoms.append(dict({k: views[k] for k in KEYS}, dtg=fwd_out[b].view(6, T)))
        grads, o = {}, 0
        for k, c in zip(GRADS, (6, 18, 3, 9, 6, 1)):
            grads[k + "_bar"] = bwd_out[b, o * T:(o + c) * T].view(c, T)
            o += c
        bdoms.append(dict({k: views[k] for k in ("g", "dg", "beta", "K", "alpha", "W")}, **grads))
    pf, pb = BatchPlan(fdoms), BatchPlan(bdoms, kind="bwd")
    pf.run()
    pb.run()
    torch.cuda.synchronize()
    flat = {k: dev(f[k]) for k in ncin}
    dtg = tl_dtg_chain(*[flat[k] for k in KEYS])
    grads = tl_dtg_chain_bwd(flat["g"], flat["dg"], flat["beta"], flat["K"], flat["alpha"],
                             flat["W"])
    ref_fwd = oracle.dtg_chain(*[f[k] for k in KEYS])
    ref_bwd = oracle.dtg_chain_vjp(tuple(f[k] for k in KEYS), f["W"])
    got_fwd = torch.cat(pf.outputs, dim=1)
    assert_close(got_fwd, dtg.cpu().numpy(), what="blocked d_t g vs plain")
    assert_close(got_fwd, ref_fwd, what="blocked d_t g vs oracle")
    for i, k in enumerate(GRADS):
        got = torch.cat([outs[i] for outs in pb.outputs], dim=1)
        assert_close(got, grads[i].cpu().numpy(), what=f"blocked {k}_bar vs plain")
        assert_close(got, ref_bwd[k], what=f"blocked {k}_bar vs oracle")
    pf.close()
    pb.close()
