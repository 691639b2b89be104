"""GPU kernels against the CPU oracle, element by element (FP64, per-component
relative error <= 1e-12), across launch shapes, ragged sizes, padded and
misaligned layouts, and at the full workload sizes."""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import TOL, DevField, assert_close, dev, need_gpu
from paper_1804_10120_amd import (tl_christoffel, tl_cov_deriv, tl_dtg, tl_dtg_chain,
                                  tl_kernel_info, tl_sym_inverse)
from paper_1804_10120_amd.synth import config_seed, make_fields

pytestmark = pytest.mark.gpu

SIZES = [1, 2, 63, 64, 65, 127, 129, 512, 1553, 4096, 4097, 10007]
TUNES = [None, dict(block=64, ppt=1), dict(block=128, ppt=2), dict(block=256, ppt=2, nt=True),
         dict(block=512, ppt=1, nt=True), dict(block=1024, ppt=1), dict(block=256, ppt=1, grid_mult=1),
         dict(block=256, ppt=1, nt=True, xcd=True), dict(block=64, ppt=2, xcd=True, grid_mult=1),
         dict(block=256, ppt=1, nt=True, xcd=True, ptr64=True), dict(block=512, ppt=2, nt=True, ptr64=True),
         # four points per lane (the kernels with more streams run two)
         dict(block=256, ppt=4, nt=True), dict(block=128, ppt=4),
         dict(block=64, ppt=4, nt=True, xcd=True, grid_mult=1), dict(block=512, ppt=4, nt=True, ptr64=True)]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


def _fields(n, seed=1):
    return make_fields(n, seed=seed + n)


def _tid(t):
    return "default" if t is None else "-".join(f"{k}{v}" for k, v in t.items())


@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("tune", TUNES, ids=_tid)
def test_sym_inverse(n, tune):
    f = _fields(n)
    out = tl_sym_inverse(dev(f["g"]), tune=tune)
    assert_close(out, oracle.sym_inverse(f["g"]), what="ginv")


@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("tune", TUNES, ids=_tid)
def test_christoffel(n, tune):
    f = _fields(n)
    ginv = oracle.sym_inverse(f["g"])
    out = tl_christoffel(dev(ginv), dev(f["dg"]), tune=tune)
    assert_close(out, oracle.christoffel(ginv, f["dg"]), what="gamma")


@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("tune", TUNES, ids=_tid)
def test_cov_deriv(n, tune):
    f = _fields(n)
    gam = oracle.christoffel(oracle.sym_inverse(f["g"]), f["dg"])
    out = tl_cov_deriv(dev(gam), dev(f["beta"]), dev(f["dbeta"]), tune=tune)
    assert_close(out, oracle.cov_deriv(gam, f["beta"], f["dbeta"]), what="nabla beta")


@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("tune", TUNES, ids=_tid)
def test_dtg(n, tune):
    f = _fields(n)
    nb = oracle.cov_deriv(oracle.christoffel(oracle.sym_inverse(f["g"]), f["dg"]),
                          f["beta"], f["dbeta"])
    out = tl_dtg(dev(f["alpha"][0]), dev(f["K"]), dev(nb), tune=tune)
    assert_close(out, oracle.dtg(f["alpha"], f["K"], nb), what="dtg")


def _chain_dev(f, **kw):
    return [DevField(f[k], **kw) for k in ("g", "dg", "beta", "dbeta", "K", "alpha")]


def _oracle_chain(f):
    return oracle.dtg_chain(f["g"], f["dg"], f["beta"], f["dbeta"], f["K"], f["alpha"])


@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("tune", TUNES, ids=_tid)
def test_chain(n, tune):
    f = _fields(n)
    ins = _chain_dev(f)
    out = tl_dtg_chain(*[x.view for x in ins], tune=tune)
    assert_close(out, _oracle_chain(f), what="fused chain")


@pytest.mark.parametrize("n", [1, 65, 4097, 10007])
def test_unfused_chain_matches_oracle_and_fused(n):
    f = _fields(n, seed=3)
    d = {k: dev(v) for k, v in f.items()}
    ginv = tl_sym_inverse(d["g"])
    gam = tl_christoffel(ginv, d["dg"])
    nb = tl_cov_deriv(gam, d["beta"], d["dbeta"])
    unfused = tl_dtg(d["alpha"], d["K"], nb)
    fused = tl_dtg_chain(d["g"], d["dg"], d["beta"], d["dbeta"], d["K"], d["alpha"])
    ref = _oracle_chain(f)
    assert_close(unfused, ref, what="unfused chain")
    assert_close(fused, unfused.cpu().numpy(), what="fused vs unfused")


@pytest.mark.parametrize("pad,offset", [(0, 0), (1, 0), (3, 1), (64, 2), (5, 3)])
@pytest.mark.parametrize("tune", [None, dict(block=128, ppt=2, nt=True)], ids=_tid)
def test_layouts_and_guard_bands(pad, offset, tune):
    n = 1553
    f = _fields(n, seed=5)
    ins = _chain_dev(f, pad=pad, offset=offset)
    out = DevField.empty(6, n, pad=pad, offset=offset + 1)
    tl_dtg_chain(*[x.view for x in ins], out.view, tune=tune)
    torch.cuda.synchronize()
    assert_close(out.view, _oracle_chain(f), what=f"chain pad={pad} offset={offset}")
    assert out.canaries_intact()
    assert all(x.canaries_intact() for x in ins)
    g = DevField(f["g"], pad=pad, offset=offset)
    gi = DevField.empty(6, n, pad=pad + 2, offset=offset)
    tl_sym_inverse(g.view, gi.view, tune=tune)
    torch.cuda.synchronize()
    assert_close(gi.view, oracle.sym_inverse(f["g"]), what="ginv layout")
    assert gi.canaries_intact()


def test_zero_points_touches_nothing():
    f = _fields(0)
    out = DevField.empty(6, 0)
    tl_dtg_chain(*[dev(f[k]) for k in ("g", "dg", "beta", "dbeta", "K", "alpha")], out.view)
    torch.cuda.synchronize()
    assert out.canaries_intact()


def test_points_are_independent():
    n = 777
    f = _fields(n, seed=9)
    base = tl_dtg_chain(*[dev(f[k]) for k in ("g", "dg", "beta", "dbeta", "K", "alpha")])
    p = 400
    f2 = {k: v.copy() for k, v in f.items()}
    for k in ("g", "dg", "beta", "dbeta", "K", "alpha"):
        f2[k][:, p] *= 1.01
    pert = tl_dtg_chain(*[dev(f2[k]) for k in ("g", "dg", "beta", "dbeta", "K", "alpha")])
    diff = (pert != base).any(dim=0).cpu().numpy()
    assert diff[p] and diff.sum() == 1


@pytest.mark.parametrize("edge", [64, 128])
def test_full_size_chain(edge):
    """The fused chain at 64^3 and 128^3 points in the benchmark's launch shape."""
    n = edge ** 3
    f = make_fields(n, seed=config_seed(2 if edge == 64 else 3))
    ins = _chain_dev(f)
    out = tl_dtg_chain(*[x.view for x in ins])
    assert_close(out, _oracle_chain(f), what=f"chain {edge}^3")


def test_full_size_christoffel_config():
    """Inverse and Christoffel symbols at 16^3 points (unfused)."""
    n = 16 ** 3
    f = make_fields(n, seed=config_seed(1))
    ginv = tl_sym_inverse(dev(f["g"]))
    gam = tl_christoffel(ginv, dev(f["dg"]))
    gi_ref = oracle.sym_inverse(f["g"])
    assert_close(ginv, gi_ref, what="ginv 16^3")
    assert_close(gam, oracle.christoffel(gi_ref, f["dg"]), what="gamma 16^3")


def test_singular_metric_propagates_nonfinite():
    n = 64
    f = _fields(n, seed=11)
    f["g"][:, 5] = 0.0                    # g = 0 at point 5: det = 0
    out = tl_dtg_chain(*[dev(f[k]) for k in ("g", "dg", "beta", "dbeta", "K", "alpha")]).cpu().numpy()
    ref = _oracle_chain(f)
    assert not np.isfinite(out[:, 5]).all()
    assert not np.isfinite(ref[:, 5]).all()
    keep = np.ones(n, bool)
    keep[5] = False
    assert_close(out[:, keep], ref[:, keep], what="finite points")


@pytest.mark.parametrize("kernel", ["sym_inverse", "christoffel", "cov_deriv", "dtg", "dtg_chain",
                                    "dtg_chain_bwd", "dtg_chain_batched", "dtg_chain_fwd_bwd",
                                    "dtg_chain_bwd_batched", "assign1", "contract3", "kij"])
def test_kernel_info(kernel):
    """Registers and occupancy of the default large-grid instantiation: the
    runtime's VGPR count equals the compiler's report compiled into the
    library, nothing spills, and the runtime's occupancy at the launch block
    size is the compiler's register-bound occupancy (blocks of 256 threads
    fill whole SIMD slots)."""
    a = tl_kernel_info(kernel)
    assert a["vgprs"] > 0 and a["max_threads"] >= a["block"]
    assert a["scratch_bytes"] == 0, f"{kernel} spills to scratch"
    assert 0 < a["sgprs"] <= 128 and a["agprs"] == 0, a
    assert 1 <= a["waves_per_simd"] <= a["max_waves_per_simd"] <= 8, a
    if a["block"] % 256 == 0:
        assert a["waves_per_simd"] == a["max_waves_per_simd"], a


def test_kernel_info_headline_kernels():
    """The benchmark step's kernels (one point per lane, 256 threads, buffer
    addressing): the forward fits 8 waves per SIMD, the adjoint 5, from their
    62 and 84 VGPRs (512 per SIMD lane, allocated in granules of 8)."""
    f = tl_kernel_info("dtg_chain")
    b = tl_kernel_info("dtg_chain_bwd")
    assert (f["block"], f["ppt"]) == (256, 1) and (b["block"], b["ppt"]) == (256, 1)
    assert f["vgprs"] <= 64 and f["waves_per_simd"] == 8, f
    assert 80 < b["vgprs"] <= 88 and b["waves_per_simd"] == 5, b


@pytest.mark.parametrize("kernel,ppt", [("sym_inverse", 4), ("dtg", 4), ("assign1", 4),
                                        ("kij", 4), ("assign3", 2), ("christoffel", 2),
                                        ("dtg_chain", 2), ("dtg_chain_bwd", 2),
                                        ("dtg_chain_batched", 2)])
def test_kernel_info_four_points(kernel, ppt):
    """A request of four points per lane runs with four only for bodies of at
    most 24 component streams, otherwise with two, and kernel_info says so."""
    a = tl_kernel_info(kernel, tune=dict(block=256, ppt=4, nt=True))
    assert a["ppt"] == ppt and a["block"] == 256 and a["scratch_bytes"] == 0, a


@pytest.mark.parametrize("lanes", [2, 3, 6, 9, 18])
def test_kernel_info_lanes(lanes):
    a = tl_kernel_info("christoffel", tune=dict(block=64, lanes=lanes))
    assert a["vgprs"] > 0 and a["block"] == 64 and a["scratch_bytes"] == 0
    assert a["sgprs"] > 0 and a["waves_per_simd"] >= 1


def test_graph_capture_replays():
    """Library launches captured in a HIP graph replay correctly, with eager
    work and synchronisation between replays (every replay is checked)."""
    n = 4097
    f = _fields(n, seed=13)
    d = {k: dev(f[k]) for k in ("g", "dg", "beta", "dbeta", "K", "alpha")}
    eager = tl_dtg_chain(*[d[k] for k in ("g", "dg", "beta", "dbeta", "K", "alpha")])
    ginv_e = tl_sym_inverse(d["g"])
    out = torch.empty_like(eager)
    ginv = torch.empty_like(ginv_e)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        tl_sym_inverse(d["g"], ginv)
        tl_dtg_chain(*[d[k] for k in ("g", "dg", "beta", "dbeta", "K", "alpha")], out)
    for rep in range(4):
        out.fill_(float("nan"))
        ginv.fill_(float("nan"))
        tl_sym_inverse(d["K"])            # unrelated eager work between replays
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, eager), f"replay {rep}"
        assert torch.equal(ginv, ginv_e), f"replay {rep}"
    assert_close(out, _oracle_chain(f), what="graph replay vs oracle")


def test_autotuner_picks_a_valid_shape(tmp_path, monkeypatch):
    """The autotuner times candidate shapes and caches the fastest; the cached
    shape gives the same results."""
    from paper_1804_10120_amd import autotune
    monkeypatch.setenv("TLMI_TUNE_CACHE", str(tmp_path / "tune.json"))
    n = 1 << 16
    cands = list(autotune.candidates(blocks=(64, 256), ppts=(1, 2), nts=(True,), xcds=(False,),
                                     grid_mults=(0,)))
    res = autotune.tune("dtg_chain", n, tunes=cands, reps=5)
    assert res["tune"] in cands and len(res["table"]) == len(cands)
    assert autotune.lookup("dtg_chain", n) == res["tune"]
    f = _fields(4097, seed=17)
    out = tl_dtg_chain(*[dev(f[k]) for k in ("g", "dg", "beta", "dbeta", "K", "alpha")],
                       tune=res["tune"])
    assert_close(out, _oracle_chain(f), what="tuned shape")


def test_auto_tune_uses_the_cache(tmp_path, monkeypatch):
    import json
    from paper_1804_10120_amd import autotune
    monkeypatch.setenv("TLMI_TUNE_CACHE", str(tmp_path / "tune.json"))
    n = 3000
    f = _fields(n, seed=19)
    ref = tl_sym_inverse(dev(f["g"]))                      # nothing cached: default shape
    assert torch.equal(tl_sym_inverse(dev(f["g"]), tune="auto"), ref)
    with open(tmp_path / "tune.json", "w") as fh:
        json.dump({autotune.cache_key("sym_inverse", n):
                   {"tune": {"block": 128, "ppt": 2, "nt": True}, "us": 1.0, "GB_s": 1.0}}, fh)
    assert autotune.lookup("sym_inverse", n) == {"block": 128, "ppt": 2, "nt": True}
    assert_close(tl_sym_inverse(dev(f["g"]), tune="auto"), oracle.sym_inverse(f["g"]),
                 what="auto-tuned inverse")
    with pytest.raises(ValueError, match="auto"):
        tl_sym_inverse(dev(f["g"]), tune="fast")


def test_fields_spanning_more_than_4_GiB():
    """A field whose components are spread over more than 4 GiB (a large
    leading dimension) cannot use 32-bit buffer offsets: the call must take the
    64-bit pointer path and still match the oracle; its neighbours with small
    extents in the same call are unaffected."""
    n = 3001
    ld = (1 << 25) + 64                       # 18 components span 4.3 GiB
    f = _fields(n, seed=77)
    big = torch.empty(18 * ld, dtype=torch.float64, device="cuda")
    dg = big.view(18, ld)[:, :n]
    dg.copy_(torch.from_numpy(f["dg"]))
    assert (17 * ld + n) * 8 > 1 << 32
    ins = [dev(f[k]) for k in ("g", "beta", "dbeta", "K", "alpha")]
    out = tl_dtg_chain(ins[0], dg, *ins[1:])
    assert_close(out, _oracle_chain(f), what="chain, dg over 4 GiB")
    gi = tl_sym_inverse(ins[0])
    gam = tl_christoffel(gi, dg)
    assert_close(gam, oracle.christoffel(oracle.sym_inverse(f["g"]), f["dg"]),
                 what="christoffel, dg over 4 GiB")
    del big, dg
    torch.cuda.empty_cache()


@pytest.mark.parametrize("lanes", [2, 3, 6, 9, 18])
@pytest.mark.parametrize("n", [1, 7, 64, 65, 1553, 4097])
@pytest.mark.parametrize("block", [64, 256, 1024])
def test_christoffel_lanes_per_point(lanes, n, block):
    """The 18 components of a point spread over `lanes` lanes: the one-lane
    kernel's result and the oracle's, to 1e-12 (the same per-point body, which
    the compiler may contract differently in the two kernels)."""
    f = _fields(n, seed=91)
    gi = oracle.sym_inverse(f["g"])
    ginv, dg = dev(gi), dev(f["dg"])
    out = DevField.empty(18, n, pad=3, offset=1)
    tl_christoffel(ginv, dg, out.view, tune=dict(block=block, lanes=lanes))
    one = tl_christoffel(ginv, dg)
    torch.cuda.synchronize()
    assert_close(out.view, one, what=f"christoffel lanes={lanes} vs one lane")
    assert out.canaries_intact()
    assert_close(out.view, oracle.christoffel(gi, f["dg"]), what=f"christoffel lanes={lanes}")
