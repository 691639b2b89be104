#!/usr/bin/env python3
"""Benchmark of the fused FP64 metric-evolution chain on one MI355X.

One step = the fused forward d_t g_ij (tl_dtg_chain) and its adjoint
(tl_dtg_chain_bwd) over N = 128^3 grid points, through the C ABI, with the
library's default launch shapes.  Inputs are seeded synthetic fields already
resident in HBM (about 1.75 GB touched per step, far beyond the 256 MB
Infinity Cache, so every step streams from HBM).

Prints ONE JSON line: whole-job grid points/s for fwd+bwd, the roofline of the
dominant kernel (algorithmic bytes / HIP-event-timed duration against the
8 TB/s HBM peak, plus the counter-measured traffic when a profile of the
current kernels is committed), the other hot-path rows timed in the same run
(forward alone, the unfused steps, the 64^3 configurations, many subgrids in
one launch), the measured copy ceiling, and the serial CPU oracle timed on a
bounded sample.

    python bench.py [--gpus 1] [--steps 100] [--warmup 10] [--edge 128]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
KEYS = ("g", "dg", "beta", "dbeta", "K", "alpha")
# Algorithmic bytes per grid point: 8 B per stored tensor element read or
# written (the paper's effective-bandwidth count, with no scalars outside
# the fields).
BYTES = {"sym_inverse": 8 * 12, "christoffel": 8 * 42, "cov_deriv": 8 * 39, "dtg": 8 * 22,
         "dtg_chain": 8 * 49, "dtg_chain_bwd": 8 * 83, "dtg_chain_batched": 8 * 49,
         "dtg_chain_fwd_bwd": 8 * 98,
         "unfused_chain": 8 * 115}
# (read, written) doubles per point of the kernels the step runs
RW_DOUBLES = {"dtg_chain": (43, 6), "dtg_chain_bwd": (40, 43), "dtg_chain_fwd_bwd": (49, 49)}
METRIC = "grid points/s + achieved HBM GB/s, fused FP64 chain fwd and fwd+bwd"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def traffic_record(kernel, n, root=ROOT):
    """HBM bytes per launch from the committed rocprofv3 counter summary of
    ``kernel``, if it was taken at this size from the current library sources,
    headers and build flags."""
    from paper_1804_10120_amd.profsum import sources_sha256
    path = os.path.join(root, "profiles", f"pmc_{kernel}.md")
    if not os.path.exists(path):
        return None
    rec = {}
    for line in open(path):
        if ":" in line and not line.startswith(("#", "|", " ")):
            k, v = line.split(":", 1)
            rec[k.strip()] = v.strip()
    if rec.get("sources_sha256") != sources_sha256(root) or rec.get("points") != str(n):
        return None
    try:
        return float(rec["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def device_sets(n, nsets, device, seed0):
    import torch
    from paper_1804_10120_amd.synth import make_fields
    sets = []
    for s in range(nsets):
        f = make_fields(n, seed=seed0 + 1000 * s)
        sets.append((f, {k: torch.from_numpy(v).to(device) for k, v in f.items()}))
    return sets


class KernelLabels:
    """roctx ranges around timed calls (``--label-kernels``): a profiler run
    with kernel renaming (rocprofv3 --marker-trace --kernel-rename) then names
    every dispatch after the configuration and call that launched it, e.g.
    ``c2 dtg_chain n=262144``, so the kernel trace splits by configuration."""

    def __init__(self):
        self.push = self.pop = None

    def enable(self):
        import ctypes
        lib = ctypes.CDLL(os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "lib",
                                       "librocprofiler-sdk-roctx.so"))
        lib.roctxRangePushA.argtypes = [ctypes.c_char_p]
        lib.roctxRangePushA.restype = ctypes.c_int
        lib.roctxRangePop.restype = ctypes.c_int
        self.push, self.pop = lib.roctxRangePushA, lib.roctxRangePop

    def wrap(self, label, call):
        if self.push is None or label is None:
            return call
        name, push, pop = label.encode(), self.push, self.pop

        def labelled():
            push(name)
            call()
            pop()
        return labelled


LABELS = KernelLabels()


def label(cfg, kernel, n, extra=""):
    return f"c{cfg} {kernel} n={n}" + (f" {extra}" if extra else "")


def _labelled(lists, labels):
    if labels is None:
        return lists
    if isinstance(labels, str):
        labels = [labels] * len(lists[0])
    return [[LABELS.wrap(lab, c) for lab, c in zip(labels, calls)] for calls in lists]


def back_to_back(lists, reps, warmup=3, labels=None):
    """Mean ms per call list with HIP events around all ``reps`` lists only:
    the launches queue back to back, so this is the kernels' own time plus
    the gaps between consecutive dispatches, without per-call event cost."""
    import torch
    lists = _labelled(lists, labels)
    for i in range(warmup):
        for c in lists[i % len(lists)]:
            c()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for i in range(reps):
        for c in lists[i % len(lists)]:
            c()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def time_calls(lists, reps, warmup, labels=None):
    """Runs the call lists round-robin.  Returns (wall ms per list, HIP-event
    ms per call position averaged over reps).  ``labels``: a roctx range name
    per call position (or one for all) when kernel labelling is on."""
    import torch
    lists = _labelled(lists, labels)
    nl, nc = len(lists), len(lists[0])
    for i in range(warmup):
        for c in lists[i % nl]:
            c()
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(nc + 1)] for _ in range(reps)]
    t0 = time.perf_counter()
    for i in range(reps):
        e = evs[i]
        e[0].record()
        for j, c in enumerate(lists[i % nl]):
            c()
            e[j + 1].record()
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3 / reps
    per = [sum(evs[i][j].elapsed_time(evs[i][j + 1]) for i in range(reps)) / reps
           for j in range(nc)]
    return wall, per


def rate(nbytes, ms):
    return nbytes / (ms * 1e-3) / 1e9


def blocked_layout(d, n, T=4096):
    """The benchmark grid cut into blocks of T points, each block holding all
    its components together ([n/T][C][T], the way a multi-domain code stores
    each element's fields), run as one forward and one adjoint batch plan with
    one subgrid per block.  Returns the timings and the largest relative
    difference from the outputs of the non-batched kernels on the
    component-major fields (d["dtg"], d["grads"])."""
    import torch
    from paper_1804_10120_amd import BatchPlan
    from paper_1804_10120_amd.ops import GRAD_NAMES
    if n % T:
        return None
    nb = n // T
    fields = (("g", 6), ("dg", 18), ("beta", 3), ("dbeta", 9), ("K", 6), ("alpha", 1), ("W", 6))
    dev = d["g"].device
    blk = torch.empty(nb, sum(c for _, c in fields) * T, dtype=torch.float64, device=dev)
    views, o = [{} for _ in range(nb)], 0
    for k, c in fields:
        blk[:, o * T:(o + c) * T].view(nb, c, T).copy_(d[k].reshape(c, nb, T).permute(1, 0, 2))
        for b in range(nb):
            views[b][k] = blk[b, o * T:(o + c) * T].view(c, T)
        o += c
    ncg = (6, 18, 3, 9, 6, 1)
    fout = torch.empty(nb, 6 * T, dtype=torch.float64, device=dev)
    bout = torch.empty(nb, sum(ncg) * T, dtype=torch.float64, device=dev)
    fdoms, bdoms = [], []
    for b, v in enumerate(views):
        fdoms.append(dict({k: v[k] for k in KEYS}, dtg=fout[b].view(6, T)))
        grads, o = {}, 0
        for k, c in zip(GRAD_NAMES, ncg):
            grads[k + "_bar"] = bout[b, o * T:(o + c) * T].view(c, T)
            o += c
        bdoms.append(dict({k: v[k] for k in ("g", "dg", "beta", "K", "alpha", "W")}, **grads))
    pf, pb = BatchPlan(fdoms), BatchPlan(bdoms, kind="bwd")
    _, (ms_f, ms_b) = time_calls([[pf.run, pb.run]], 20, 3)

    def unblock(x, c):
        return x.view(nb, c, T).permute(1, 0, 2).reshape(c, n)

    diffs = [unblock(fout, 6) - d["dtg"].reshape(6, n)]
    scale = [d["dtg"].abs().max()]
    o = 0
    for c, ref in zip(ncg, d["grads"]):
        diffs.append(unblock(bout[:, o * T:(o + c) * T], c) - ref.reshape(c, n))
        scale.append(ref.abs().max())
        o += c
    rel = max(float(x.abs().max() / s) for x, s in zip(diffs, scale))
    pf.close()
    pb.close()
    return {"block_points": T, "blocks": nb,
            "fwd_us": ms_f * 1e3, "fwd_GB_s": rate(BYTES["dtg_chain"] * n, ms_f),
            "bwd_us": ms_b * 1e3, "bwd_GB_s": rate(BYTES["dtg_chain_bwd"] * n, ms_b),
            "max_rel_diff_vs_component_major": rel}


def copy_ceiling(device, reps=20):
    """GB/s of the library's streaming copy over 2 x 512 MiB."""
    import torch
    from paper_1804_10120_amd import tl_bw_copy
    from paper_1804_10120_amd.ops import record
    n = 64 * 1024 * 1024
    src = torch.rand(n, dtype=torch.float64, device=device)
    dst = torch.empty_like(src)
    with record() as calls:
        tl_bw_copy(src, dst)
    _, (ms,) = time_calls([calls], reps, 3)
    assert torch.equal(src[:4096], dst[:4096]) and torch.equal(src[-4096:], dst[-4096:])
    return rate(16 * n, ms)


def direction_ceilings(device, reps=20):
    """GB/s of the library's read-only and write-only references over 1 GiB."""
    import torch
    from paper_1804_10120_amd import tl_bw_read, tl_bw_write
    from paper_1804_10120_amd.ops import record
    n = 128 * 1024 * 1024
    buf = torch.rand(n, dtype=torch.float64, device=device)
    with record() as rd:
        part = tl_bw_read(buf)
    with record() as wr:
        tl_bw_write(buf)
    _, (ms_r,) = time_calls([rd], reps, 3)
    _, (ms_w,) = time_calls([wr], reps, 3)
    del part
    return rate(8 * n, ms_r), rate(8 * n, ms_w)


def rw_model(read_doubles, write_doubles, read_gbs, write_gbs):
    """Ceiling of a kernel that reads and writes the given doubles per point if
    its reads ran at the read-only rate and its writes at the write-only rate,
    one after the other (the streaming copy matches this model)."""
    return (read_doubles + write_doubles) / (read_doubles / read_gbs + write_doubles / write_gbs)


MID_SHAPES = {"ppt1_b256": dict(block=256, ppt=1, nt=True),
              "ppt2_b512": dict(block=512, ppt=2, nt=True)}


def mid_size_shapes(sets, n):
    """At 64^3 points (all blocks resident at once), one point per lane in
    blocks of 256 against two points per lane (16-byte accesses) in blocks of
    512, for the adjoint and the four unfused kernels: HIP-event time per call
    and time per call queued back to back, over rotating buffer sets."""
    import torch
    from paper_1804_10120_amd import (tl_christoffel, tl_cov_deriv, tl_dtg, tl_dtg_chain_bwd,
                                      tl_sym_inverse)
    from paper_1804_10120_amd.ops import record
    mids = []
    for _, e in sets:
        gi = tl_sym_inverse(e["g"])
        ga = tl_christoffel(gi, e["dg"])
        mids.append((e, gi, ga, tl_cov_deriv(ga, e["beta"], e["dbeta"])))
    calls = {
        "dtg_chain_bwd": lambda e, gi, ga, nb, t: tl_dtg_chain_bwd(
            e["g"], e["dg"], e["beta"], e["K"], e["alpha"], e["W"], tune=t),
        "sym_inverse": lambda e, gi, ga, nb, t: tl_sym_inverse(e["g"], tune=t),
        "christoffel": lambda e, gi, ga, nb, t: tl_christoffel(gi, e["dg"], tune=t),
        "cov_deriv": lambda e, gi, ga, nb, t: tl_cov_deriv(ga, e["beta"], e["dbeta"], tune=t),
        "dtg": lambda e, gi, ga, nb, t: tl_dtg(e["alpha"], e["K"], nb, tune=t),
    }
    out = {}
    for kname, fn in calls.items():
        out[kname] = {}
        for sname, tune in MID_SHAPES.items():
            lists = []
            for m in mids:
                with record() as c:
                    fn(*m, tune)
                lists.append(c)
            lab = label(5 if kname == "dtg_chain_bwd" else 2, kname, n, sname)
            _, (ms,) = time_calls(lists, 100, 10, labels=lab)
            ms_q = back_to_back(lists, 100, labels=lab + " queued")
            out[kname][sname] = {"us": ms * 1e3, "GB_s": rate(BYTES[kname] * n, ms),
                                 "queued_us": ms_q * 1e3,
                                 "queued_GB_s": rate(BYTES[kname] * n, ms_q)}
    del mids
    torch.cuda.empty_cache()
    return out


def host_cpu():
    """Model name of the host CPU and the number of cores this process may use."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, len(os.sched_getaffinity(0))


def _oracle_slices(f, budget_s, first, step):
    """Runs the oracle (forward chain + reverse-mode gradients) over the
    4096-point slices first, first + step, ... of the benchmark's fields until
    ``budget_s`` seconds have passed; returns the number of points done."""
    import numpy as np
    import oracle
    n = f["g"].shape[1]
    chunk = min(n, 4096)
    nslices = (n + chunk - 1) // chunk
    done, k, t0 = 0, first, time.perf_counter()
    while time.perf_counter() - t0 < budget_s:
        lo = (k % nslices) * chunk
        hi = min(n, lo + chunk)
        ins = tuple(np.ascontiguousarray(f[key][:, lo:hi]) for key in KEYS)
        oracle.dtg_chain(*ins)
        oracle.dtg_chain_vjp(ins, np.ascontiguousarray(f["W"][:, lo:hi]))
        done += hi - lo
        k += step
    return done


def cpu_baseline(f, budget_s):
    """The serial oracle on one host core, over consecutive 16^3-point slices
    of the benchmark's fields, for about ``budget_s`` seconds."""
    t0 = time.perf_counter()
    done = _oracle_slices(f, budget_s, 0, 1)
    dt = time.perf_counter() - t0
    model, ncpu = host_cpu()
    return {"value": done / dt, "unit": "grid points/s", "cores": 1, "kind": "oracle",
            "sample": f"serial oracle (forward chain + tape VJP) on {done} points of the "
                      f"benchmark fields, in 4096-point slices, {dt:.1f} s on one host core",
            "host_cpu": model, "host_cores": ncpu}


def cpu_all_cores(f, budget_s, threads):
    """The same oracle, unchanged, on ``threads`` host threads at once (each
    takes every threads-th slice; the oracle's C entry points run without the
    interpreter lock)."""
    from concurrent.futures import ThreadPoolExecutor
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=threads) as pool:
        done = sum(pool.map(lambda i: _oracle_slices(f, budget_s, i, threads), range(threads)))
    dt = time.perf_counter() - t0
    return {"value": done / dt, "unit": "grid points/s", "cores": threads, "kind": "oracle",
            "sample": f"{done} points in 4096-point slices over {dt:.1f} s"}


SWEEP_SIZES = tuple(32 * 4 ** k for k in range(9)) + (2 ** 21,)


def paper_family(device, sizes, reps=21):
    """BW_eff (the paper's effective bandwidth: 8 B x elements x N / t) of the
    Sec. 5.1 benchmark expressions, the Christoffel symbols (g^ij given, as in
    the paper), the fused chain and the same chain as four launches, at each
    grid size.  Each size: ``reps``
    launches timed with HIP events, the first discarded, the median kept (the
    paper's method).  Smaller grids are views of the largest fields."""
    import torch
    from paper_1804_10120_amd import (tl_christoffel, tl_cov_deriv, tl_dtg, tl_dtg_chain,
                                      tl_expr, tl_expr_shape, tl_sym_inverse)
    from paper_1804_10120_amd.ops import record
    from paper_1804_10120_amd.synth import EXPR_INPUTS, make_expr_inputs, make_fields
    nmax = max(sizes)
    table = {}

    def run(name, ne, launch):
        row = {}
        for n in sizes:
            with record() as calls:
                launch(n)
            ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                  for _ in range(reps)]
            for a, b in ev:
                a.record()
                for c in calls:
                    c()
                b.record()
            torch.cuda.synchronize()
            ts = sorted(a.elapsed_time(b) for a, b in ev[1:])
            row[n] = rate(8 * ne * n, ts[len(ts) // 2])
        table[name] = row

    for name in EXPR_INPUTS:
        ic, oc = tl_expr_shape(name)
        xs = [torch.from_numpy(x).to(device) for x in make_expr_inputs(name, nmax, seed=5)]
        out = torch.empty(oc, nmax, dtype=torch.float64, device=device)
        run(name, sum(ic) + oc,
            lambda n: tl_expr(name, *[x[:, :n] for x in xs], out=out[:, :n]))
        del xs, out
    f = {k: torch.from_numpy(v).to(device) for k, v in
         make_fields(nmax, seed=7, fields=KEYS).items()}
    gam = torch.empty(18, nmax, dtype=torch.float64, device=device)
    run("christoffel", 42, lambda n: tl_christoffel(f["g"][:, :n], f["dg"][:, :n], gam[:, :n]))
    # the paper's parallelisation over left-hand-side components: 3 and 18 lanes per point
    for lanes in (3, 18):
        run(f"christoffel_{lanes}_lanes", 42,
            lambda n: tl_christoffel(f["g"][:, :n], f["dg"][:, :n], gam[:, :n],
                                     tune=dict(block=64, lanes=lanes)))
    dtg = torch.empty(6, nmax, dtype=torch.float64, device=device)
    run("dtg_chain", 49, lambda n: tl_dtg_chain(*[f[k][:, :n] for k in KEYS], dtg[:, :n]))
    # the same d_t g as four launches (a1-a4), counted with the fused chain's 49 elements:
    # the paper's comparison of one kernel per expression with several (Sec. 5.5)
    gi = torch.empty(6, nmax, dtype=torch.float64, device=device)
    nb = torch.empty(9, nmax, dtype=torch.float64, device=device)

    def unfused(n):
        tl_sym_inverse(f["g"][:, :n], gi[:, :n])
        tl_christoffel(gi[:, :n], f["dg"][:, :n], gam[:, :n])
        tl_cov_deriv(gam[:, :n], f["beta"][:, :n], f["dbeta"][:, :n], nb[:, :n])
        tl_dtg(f["alpha"][:, :n], f["K"][:, :n], nb[:, :n], dtg[:, :n])
    run("dtg_chain_4_launches", 49, unfused)
    del f, gam, dtg, gi, nb
    torch.cuda.empty_cache()
    return table


def family_summary(table):
    """Rate at the largest size and the smallest swept size reaching half of it."""
    out = {}
    for name, row in table.items():
        top = row[max(row)]
        half = min((n for n, g in row.items() if g >= 0.5 * top), default=None)
        out[name] = {"GB_s": top, "half_rate_at_points": half}
    return out


def write_sweep(table, path):
    sizes = sorted(next(iter(table.values())))
    with open(path, "w") as f:
        f.write("| expression | " + " | ".join(str(n) for n in sizes) + " |\n")
        f.write("|---" * (len(sizes) + 1) + "|\n")
        for name, row in table.items():
            f.write(f"| {name} | " + " | ".join(f"{row[n]:.0f}" for n in sizes) + " |\n")


def main():
    ap = argparse.ArgumentParser(description=__doc__,
                                 formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--edge", type=int, default=128, help="grid edge; N = edge^3 points")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-rows", action="store_true", help="time only the fwd+bwd step")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--label-kernels", action="store_true",
                    help="name the timed calls with roctx ranges (for a profiler run with "
                         "--marker-trace --kernel-rename)")
    ap.add_argument("--sweep", metavar="FILE",
                    help="also write the full grid-size sweep (GB/s) as a Markdown table")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py measures one GPU only (asked for {max(args.gpus, world)}): the hot path "
              "is point-wise with no data exchanged between GPUs, so each GPU would run the same "
              "kernels on its own share of the points; no multi-GPU figure is produced.",
              file=sys.stderr)
        sys.exit(2)

    if args.label_kernels:
        LABELS.enable()
    import torch
    from paper_1804_10120_amd import (BatchPlan, tl_batch_run_noalloc, tl_christoffel,
                                      tl_cov_deriv, tl_dtg, tl_dtg_chain, tl_dtg_chain_bwd,
                                      tl_dtg_chain_fwd_bwd, tl_sym_inverse, empty_field, to_field)
    from paper_1804_10120_amd.ops import record
    from paper_1804_10120_amd.synth import config_seed, domain_edges, make_fields

    if not torch.cuda.is_available():
        print("bench.py needs an AMD GPU", file=sys.stderr)
        sys.exit(1)
    device = torch.device("cuda:0")
    torch.cuda.set_device(device)
    n = args.edge ** 3
    log(f"[bench] fields for {n} points")
    (f, d), = device_sets(n, 1, device, config_seed(3))

    # ---- the step: fused forward + adjoint
    with record() as step:
        d["dtg"] = tl_dtg_chain(*[d[k] for k in KEYS])
        d["grads"] = tl_dtg_chain_bwd(d["g"], d["dg"], d["beta"], d["K"], d["alpha"], d["W"])
    log(f"[bench] {args.steps} steps after {args.warmup} warm-up steps")
    ms_step, (ms_fwd, ms_bwd) = time_calls([step], args.steps, args.warmup,
                                           labels=[label(3, "dtg_chain", n),
                                                   label(3, "dtg_chain_bwd", n)])
    assert torch.isfinite(d["dtg"]).all() and torch.isfinite(d["grads"][0]).all()

    res = {
        "metric": METRIC,
        "value": n / (ms_step * 1e-3),
        "unit": "grid points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"fused d_t g_ij chain, forward + adjoint, N = {args.edge}^3 = "
                               f"{n} grid points, FP64, seeded synthetic fields",
                   "points": n, "step": ["tl_dtg_chain", "tl_dtg_chain_bwd"]},
        "fwd": {"us": ms_fwd * 1e3, "points_per_s": n / (ms_fwd * 1e-3),
                "GB_s": rate(BYTES["dtg_chain"] * n, ms_fwd)},
        "bwd": {"us": ms_bwd * 1e3, "points_per_s": n / (ms_bwd * 1e-3),
                "GB_s": rate(BYTES["dtg_chain_bwd"] * n, ms_bwd)},
        "fwd_bwd_GB_s": rate((BYTES["dtg_chain"] + BYTES["dtg_chain_bwd"]) * n, ms_step),
    }
    dom, ms_dom = ("dtg_chain_bwd", ms_bwd) if ms_bwd >= ms_fwd else ("dtg_chain", ms_fwd)
    achieved = rate(BYTES[dom] * n, ms_dom)
    res["roofline"] = {"bound": "hbm", "kernel": dom, "achieved": achieved,
                       "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                       "traffic": traffic_record(dom, n),
                       "algorithmic_bytes_per_launch": BYTES[dom] * n,
                       "duration_us": ms_dom * 1e3}

    log("[bench] copy, read-only and write-only ceilings")
    cgbs = copy_ceiling(device)
    res["copy_GB_s"] = cgbs
    res["roofline"]["frac_of_copy"] = achieved / cgbs
    rgbs, wgbs = direction_ceilings(device)
    res["read_only_GB_s"], res["write_only_GB_s"] = rgbs, wgbs
    rd, wr = RW_DOUBLES[dom]
    res["roofline"]["rw_model_GB_s"] = rw_model(rd, wr, rgbs, wgbs)
    res["roofline"]["frac_of_rw_model"] = achieved / res["roofline"]["rw_model_GB_s"]
    res["fwd"]["frac_of_rw_model"] = res["fwd"]["GB_s"] / rw_model(*RW_DOUBLES["dtg_chain"],
                                                                   rgbs, wgbs)

    if not args.no_rows:
        rows = {}
        log("[bench] forward + adjoint in one kernel (cotangent known up front)")
        ref = [d["dtg"].clone()] + [x.clone() for x in d["grads"]]
        with record() as fb:
            tl_dtg_chain_fwd_bwd(*[d[k] for k in KEYS], d["W"], d["dtg"], d["grads"])
        _, (ms_fb,) = time_calls([fb], args.steps, args.warmup,
                                 labels=label(3, "dtg_chain_fwd_bwd", n))
        diff = max(float(((a - b).abs().max() / b.abs().max().clamp_min(1e-300)).item())
                   for a, b in zip([d["dtg"], *d["grads"]], ref))
        rows["fwd_bwd_one_kernel"] = {"us": ms_fb * 1e3, "points_per_s": n / (ms_fb * 1e-3),
                                      "GB_s": rate(BYTES["dtg_chain_fwd_bwd"] * n, ms_fb),
                                      "speedup_vs_two_kernels": ms_step / ms_fb,
                                      "max_rel_diff_vs_two_kernels": diff,
                                      "frac_of_rw_model": rate(BYTES["dtg_chain_fwd_bwd"] * n, ms_fb)
                                      / rw_model(*RW_DOUBLES["dtg_chain_fwd_bwd"], rgbs, wgbs)}
        del ref, fb
        log("[bench] the autograd step (torch.autograd.Function), eager and captured")
        from paper_1804_10120_amd import dtg_chain
        leaf = {k: d[k].detach().clone().requires_grad_(True) for k in KEYS}
        wt = d["W"]

        def ag_step():
            for t in leaf.values():
                t.grad = None
            dtg_chain(*[leaf[k] for k in KEYS]).backward(wt)
        ms_ag, _ = time_calls([[ag_step]], args.steps, args.warmup)
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            for _ in range(2):
                ag_step()
        torch.cuda.current_stream().wait_stream(side)
        for t in leaf.values():
            t.grad = None
        ag_graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(ag_graph):
            dtg_chain(*[leaf[k] for k in KEYS]).backward(wt)
        ms_agg, _ = time_calls([[ag_graph.replay]], args.steps, args.warmup)
        rows["autograd_step"] = {"eager_us": ms_ag * 1e3, "eager_points_per_s": n / (ms_ag * 1e-3),
                                 "graph_us": ms_agg * 1e3,
                                 "graph_points_per_s": n / (ms_agg * 1e-3)}
        del leaf, ag_graph
        log("[bench] unfused steps")
        with record() as unf:
            ginv = tl_sym_inverse(d["g"])
            gam = tl_christoffel(ginv, d["dg"])
            nb = tl_cov_deriv(gam, d["beta"], d["dbeta"])
            tl_dtg(d["alpha"], d["K"], nb)
        unf_names = ("sym_inverse", "christoffel", "cov_deriv", "dtg")
        _, per = time_calls([unf], 20, 3, labels=[label(3, k, n) for k in unf_names])
        for name, ms in zip(unf_names, per):
            rows[name] = {"us": ms * 1e3, "GB_s": rate(BYTES[name] * n, ms)}
        rows["unfused_chain"] = {"us": sum(per) * 1e3, "points_per_s": n / (sum(per) * 1e-3),
                                 "GB_s": rate(BYTES["unfused_chain"] * n, sum(per)),
                                 "fused_fwd_speedup": sum(per) / ms_fwd}
        del unf, ginv, gam, nb

        log("[bench] bandwidth twins")
        twins = {}
        from paper_1804_10120_amd import tl_bw_twin
        from paper_1804_10120_amd._abi import TWIN_SHAPES
        for nin, nout in TWIN_SHAPES:
            if nin == 1:
                continue
            src = torch.rand(nin, n, dtype=torch.float64, device=device)
            dst = torch.empty(nout, n, dtype=torch.float64, device=device)
            with record() as tw:
                tl_bw_twin(src, nout, dst)
            _, (ms,) = time_calls([tw], 20, 3)
            twins[f"{nin}r{nout}w"] = rate(8 * (nin + nout) * n, ms)
            del src, dst, tw
        rows["twin_GB_s"] = twins
        shape = "40r43w" if dom == "dtg_chain_bwd" else "43r6w"
        res["roofline"]["frac_of_twin"] = achieved / twins[shape]

        log("[bench] kernels generated from index notation")
        from paper_1804_10120_amd.generated import call as gen_call
        gi = tl_sym_inverse(d["g"])
        gam_g = torch.empty(18, n, dtype=torch.float64, device=device)
        dtg_g = torch.empty(6, n, dtype=torch.float64, device=device)
        with record() as gl:
            gen_call("christoffel", gi, d["dg"], outs=[gam_g])
            gen_call("dtg_chain_invg", gi, d["dg"], d["dbeta"], d["beta"], d["alpha"], d["K"],
                     outs=[dtg_g])
        _, (ms_gc, ms_gf) = time_calls([gl], 20, 3)
        rows["generated"] = {
            "christoffel": {"us": ms_gc * 1e3, "GB_s": rate(BYTES["christoffel"] * n, ms_gc),
                            "hand_written_us": rows["christoffel"]["us"]},
            "dtg_chain_invg": {"us": ms_gf * 1e3, "GB_s": rate(BYTES["dtg_chain"] * n, ms_gf),
                               "hand_written_fused_us": ms_fwd * 1e3}}
        del gl, gi, gam_g, dtg_g
        # the Sec. 5.1 family: hand-written (tl_expr) against generated (tlg_*)
        from paper_1804_10120_amd import tl_expr, tl_expr_shape
        from paper_1804_10120_amd.synth import EXPR_INPUTS, make_expr_inputs
        fam = {}
        for name in EXPR_INPUTS:
            ic, oc = tl_expr_shape(name)
            xs = [torch.from_numpy(x).to(device) for x in make_expr_inputs(name, n, seed=5)]
            o1 = torch.empty(oc, n, dtype=torch.float64, device=device)
            o2 = torch.empty(oc, n, dtype=torch.float64, device=device)
            with record() as fc:
                tl_expr(name, *xs, out=o1)
                gen_call(name, *xs, outs=[o2])
            _, (mh, mg) = time_calls([fc], 20, 3)
            nb = 8 * (sum(ic) + oc) * n
            fam[name] = {"hand_GB_s": rate(nb, mh), "generated_GB_s": rate(nb, mg)}
            del xs, o1, o2, fc
        rows["generated"]["family"] = fam

        log("[bench] Christoffel symbols at 16^3 points")
        n16 = 16 ** 3
        (_, e16), = device_sets(n16, 1, device, config_seed(1))
        with record() as cs:
            gi16 = tl_sym_inverse(e16["g"])
            tl_christoffel(gi16, e16["dg"])
        _, (ms_i, ms_c) = time_calls([cs], 200, 20, labels=[label(1, "sym_inverse", n16),
                                                             label(1, "christoffel", n16)])
        graph = torch.cuda.CUDAGraph()
        gi_g = torch.empty_like(gi16)
        ga_g = torch.empty(18, n16, dtype=torch.float64, device=device)
        with torch.cuda.graph(graph):       # launches go to the capture stream
            for _ in range(10):
                tl_sym_inverse(e16["g"], gi_g)
                tl_christoffel(gi_g, e16["dg"], ga_g)
        _, (ms_g,) = time_calls([[graph.replay]], 20, 3)
        # the Christoffel kernel with the components of a point spread over lanes
        lanes_us = {}
        for la in (2, 3, 6, 9, 18):
            with record() as cl:
                tl_christoffel(gi16, e16["dg"], tune=dict(block=64, nt=True, lanes=la))
            _, (ms_l,) = time_calls([cl], 200, 20,
                                    labels=label(1, "christoffel", n16, f"lanes={la}"))
            lanes_us[str(la)] = ms_l * 1e3
        rows["christoffel_16cubed"] = {
            "points": n16, "sym_inverse_us": ms_i * 1e3, "christoffel_us": ms_c * 1e3,
            "christoffel_lanes_us": lanes_us,
            "graph_us_per_pair": ms_g * 1e3 / 10,
            "points_per_s": n16 / (ms_g * 1e-3 / 10),
            "note": "latency-bound: 1.6 MB per pair; graph = 10 pairs per replay; "
                    "christoffel_lanes_us: one point's 18 components over 2..18 lanes"}
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(gi_g, gi16)
        del graph, cs, gi16, e16, gi_g, ga_g

        log("[bench] per-launch floor at tiny grids")
        from paper_1804_10120_amd import tl_bw_copy, tl_expr
        (_, e32), = device_sets(4096, 1, device, config_seed(1))
        tiny = {}
        for npt in (32, 4096):
            cp_src = torch.rand(npt, dtype=torch.float64, device=device)
            b3 = torch.rand(3, npt, dtype=torch.float64, device=device)
            with record() as fl:
                tl_bw_copy(cp_src)
                tl_expr("assign1", b3)
                tl_dtg_chain(*[e32[k][:, :npt] for k in KEYS])
            _, per = time_calls([fl], 200, 20)
            tiny[str(npt)] = dict(zip(("copy_us", "assign1_us", "dtg_chain_us"),
                                      (ms * 1e3 for ms in per)))
        tiny["note"] = ("one load and one store per point (copy), 3 and 3 (assign1) or 43 and 6 "
                        "(dtg_chain) take about the same time per launch: a round trip to "
                        "memory and the launch, not the lanes in flight, set the time")
        rows["tiny_grid_floor"] = tiny
        del e32, fl

        log("[bench] 64^3 with 6 rotating buffer sets")
        n64 = 64 ** 3
        s64 = device_sets(n64, 6, device, config_seed(2))
        lists = []
        for _, e in s64:
            with record() as c:
                tl_dtg_chain(*[e[k] for k in KEYS])
                tl_dtg_chain_bwd(e["g"], e["dg"], e["beta"], e["K"], e["alpha"], e["W"])
            lists.append(c)
        lab64 = [label(2, "dtg_chain", n64), label(5, "dtg_chain_bwd", n64)]
        ms64, (f64, b64) = time_calls(lists, 100, 10, labels=lab64)
        _, (wf64, wb64) = time_calls(lists[:1], 100, 10,     # one set: cache-resident
                                     labels=[x + " warm" for x in lab64])
        # the same launches queued back to back (no event between calls)
        bb_f64 = back_to_back([c[:1] for c in lists], 100, labels=lab64[0] + " queued")
        bb_b64 = back_to_back([c[1:] for c in lists], 100, labels=lab64[1] + " queued")
        # the same forward + adjoint pairs over the 4 sets, twice, replayed from one graph
        outs64 = [(torch.empty(6, n64, dtype=torch.float64, device=device),
                   [torch.empty(c, n64, dtype=torch.float64, device=device)
                    for c in (6, 18, 3, 9, 6, 1)]) for _ in s64]
        g64 = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g64):
            for _ in range(2):
                for (_, e), (o, gr) in zip(s64, outs64):
                    tl_dtg_chain(*[e[k] for k in KEYS], o)
                    tl_dtg_chain_bwd(e["g"], e["dg"], e["beta"], e["K"], e["alpha"], e["W"], *gr)
        _, (ms_g64,) = time_calls([[g64.replay]], 20, 3)
        rows["fwd_bwd_64cubed"] = {"points": n64, "us": ms64 * 1e3,
                                   "points_per_s": n64 / (ms64 * 1e-3),
                                   "fwd_us": f64 * 1e3,
                                   "fwd_GB_s": rate(BYTES["dtg_chain"] * n64, f64),
                                   "bwd_us": b64 * 1e3,
                                   "bwd_GB_s": rate(BYTES["dtg_chain_bwd"] * n64, b64),
                                   "warm_fwd_us": wf64 * 1e3, "warm_bwd_us": wb64 * 1e3,
                                   "queued_fwd_us": bb_f64 * 1e3,
                                   "queued_fwd_GB_s": rate(BYTES["dtg_chain"] * n64, bb_f64),
                                   "queued_bwd_us": bb_b64 * 1e3,
                                   "queued_bwd_GB_s": rate(BYTES["dtg_chain_bwd"] * n64, bb_b64),
                                   "graph_us_per_pair": ms_g64 * 1e3 / (2 * len(s64)),
                                   "graph_points_per_s": n64 / (ms_g64 * 1e-3 / (2 * len(s64)))}
        rows["shapes_64cubed"] = mid_size_shapes(s64, n64)
        del s64, lists, outs64, g64

        log("[bench] blocked field layout, batch plans over blocks of 4096 points")
        rows["blocked_layout"] = blocked_layout(d, n)
        log("[bench] 256 subgrids")
        edges = domain_edges(256, seed=config_seed(4))
        hosts = [make_fields(int(e) ** 3, seed=config_seed(4) * 1000 + i, fields=KEYS)
                 for i, e in enumerate(edges)]
        npts = sum(int(e) ** 3 for e in edges)
        # the same subgrids with ld = n (contiguous [C, n] tensors)
        flat = [{k: torch.from_numpy(v).to(device) for k, v in fe.items()} for fe in hosts]
        plan = BatchPlan(flat)
        _, (ms_flat,) = time_calls([[plan.run]], 20, 3,
                                   labels=label(4, "dtg_chain_batched", npts, "ld=n"))
        plan.close()
        del flat, plan
        # each subgrid's fields with ld padded to a multiple of 16 doubles
        doms = [{k: to_field(v, device=device) for k, v in fe.items()} for fe in hosts]
        del hosts
        plan = BatchPlan(doms)
        _, (ms_default,) = time_calls([[plan.run]], 20, 3,
                                      labels=label(4, "dtg_chain_batched", npts, "default"))
        _, (ms_direct,) = time_calls([[plan.run_direct]], 20, 3,
                                     labels=label(4, "dtg_chain_batched", npts, "direct"))
        # the same launch with its tables in the library's fixed array (no allocation)
        na_doms = [dict(e, dtg=empty_field(6, e["K"].shape[1], device=device)) for e in doms]
        with record() as na:
            tl_batch_run_noalloc(na_doms)
        _, (ms_na,) = time_calls([na], 20, 3,
                                 labels=label(4, "dtg_chain_batched", npts, "no allocation"))
        # queued back to back: the host's argument checks overlap the previous call's kernels
        ms_na_q = back_to_back([na], 20,
                               labels=label(4, "dtg_chain_batched", npts, "no allocation queued"))
        ms_direct_q = back_to_back([[plan.run_direct]], 20,
                                   labels=label(4, "dtg_chain_batched", npts, "direct queued"))
        na_same = all(torch.equal(a["dtg"], b) for a, b in zip(na_doms, plan.outputs))
        plan.close()
        del na, na_doms
        from paper_1804_10120_amd import autotune
        tuned = autotune.tune_plan(doms, save=False)
        plan = BatchPlan(doms, tune=tuned["tune"])
        _, (ms_graph,) = time_calls([[plan.run]], 20, 3,
                                    labels=label(4, "dtg_chain_batched", npts, "tuned"))
        outs = [empty_field(6, e["K"].shape[1], device=device) for e in doms]
        with record() as many:
            for e, o in zip(doms, outs):
                tl_dtg_chain(*[e[k] for k in KEYS], o)
        ms_many, _ = time_calls([many], 10, 2,
                                labels=label(4, "dtg_chain", npts, "256 launches"))
        graph256 = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph256):    # the 256 plain launches, captured
            for e, o in zip(doms, outs):
                tl_dtg_chain(*[e[k] for k in KEYS], o)
        _, (ms_g256,) = time_calls([[graph256.replay]], 20, 3)
        same = all(torch.equal(a, b) for a, b in zip(outs, plan.outputs))
        rows["dtg_chain_batched"] = {
            "subgrids": 256, "points": npts, "us": ms_graph * 1e3,
            "tune": tuned["tune"], "default_tune_us": ms_default * 1e3,
            "points_per_s": npts / (ms_graph * 1e-3),
            "GB_s": rate(BYTES["dtg_chain_batched"] * npts, ms_graph),
            "separate_launches_us": ms_many * 1e3,
            "separate_launches_points_per_s": npts / (ms_many * 1e-3),
            "separate_launches_graph_us": ms_g256 * 1e3,
            "separate_launches_graph_points_per_s": npts / (ms_g256 * 1e-3),
            "separate_launches_match_batched": same,
            "direct_launch_us": ms_direct * 1e3,
            "no_allocation_us": ms_na * 1e3,
            "no_allocation_queued_us": ms_na_q * 1e3,
            "direct_launch_queued_us": ms_direct_q * 1e3,
            "no_allocation_matches_plan": na_same,
            "ld_unpadded_us": ms_flat * 1e3,
            "ld_unpadded_GB_s": rate(BYTES["dtg_chain_batched"] * npts, ms_flat)}
        plan.close()
        del many, outs, graph256

        log("[bench] 256 subgrids, the adjoint")
        for i, (e, d) in enumerate(zip(edges, doms)):
            w = make_fields(int(e) ** 3, seed=config_seed(4) * 1000 + i, fields=("W",))["W"]
            d["W"] = to_field(w, device=device)
        bdoms = [{k: d[k] for k in ("g", "dg", "beta", "K", "alpha", "W")} for d in doms]
        tuned_b = autotune.tune_plan(bdoms, kind="bwd", save=False)
        bplan = BatchPlan(bdoms, tune=tuned_b["tune"], kind="bwd")
        _, (ms_bplan,) = time_calls([[bplan.run]], 20, 3,
                                    labels=label(4, "dtg_chain_bwd_batched", npts, "tuned"))
        with record() as bmany:
            for d, gr in zip(bdoms, bplan.outputs):
                tl_dtg_chain_bwd(d["g"], d["dg"], d["beta"], d["K"], d["alpha"], d["W"], *gr)
        ms_bmany, _ = time_calls([bmany], 10, 2,
                                 labels=label(4, "dtg_chain_bwd", npts, "256 launches"))
        rows["dtg_chain_bwd_batched"] = {
            "subgrids": 256, "points": npts, "us": ms_bplan * 1e3, "tune": tuned_b["tune"],
            "points_per_s": npts / (ms_bplan * 1e-3),
            "GB_s": rate(BYTES["dtg_chain_bwd"] * npts, ms_bplan),
            "separate_launches_us": ms_bmany * 1e3,
            "separate_launches_points_per_s": npts / (ms_bmany * 1e-3)}
        bplan.close()
        del doms, bdoms, bplan, bmany
        log("[bench] the paper's benchmark expressions, grid-size sweep")
        table = paper_family(device, SWEEP_SIZES)
        rows["paper_family"] = family_summary(table)
        if args.sweep:
            write_sweep(table, args.sweep)
        res["rows"] = rows
        torch.cuda.empty_cache()

    if not args.no_cpu:
        log(f"[bench] CPU oracle baseline (~{args.cpu_seconds:.0f} s)")
        res["cpu_baseline"] = cpu_baseline(f, args.cpu_seconds)
        if "rows" in res:
            threads = min(16, res["cpu_baseline"]["host_cores"])
            log(f"[bench] CPU oracle on {threads} threads (~{args.cpu_seconds / 2:.0f} s)")
            res["rows"]["cpu_oracle_all_cores"] = cpu_all_cores(f, args.cpu_seconds / 2, threads)
    else:
        res["cpu_baseline"] = None
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
