"""Launch-shape autotuner for the library's kernels.

The paper picks a block size per kernel from a fixed rule tuned for its GPUs;
here the shape is measured instead.  ``tune(kernel, n)`` times every candidate
(block size, points per thread, non-temporal hint, persistent grid multiple)
on seeded synthetic fields of ``n`` points with HIP events, rotating over
enough buffer sets that the working set exceeds the last-level cache, and
returns the fastest.  Results are cached as JSON keyed by kernel, GPU
architecture and size class (``TLMI_TUNE_CACHE`` overrides the file).
"""
from __future__ import annotations

import itertools
import json
import math
import os
import threading

import torch

from .ops import (record, tl_christoffel, tl_cov_deriv, tl_dtg, tl_dtg_chain, tl_dtg_chain_bwd,
                  tl_dtg_chain_fwd_bwd, tl_sym_inverse)
from .synth import make_fields

KERNELS = ("sym_inverse", "christoffel", "cov_deriv", "dtg", "dtg_chain", "dtg_chain_bwd",
           "dtg_chain_fwd_bwd")
BLOCKS = (64, 128, 256, 512, 1024)
PPTS = (1, 2)
# kernels whose bodies also run four points per lane (few component streams)
PPT4_KERNELS = ("sym_inverse", "dtg")
NTS = (False, True)
XCDS = (False, True)
GRID_MULTS = (0, 1, 2, 4, 8)
# stored doubles read + written per point
DOUBLES = {"sym_inverse": 12, "christoffel": 42, "cov_deriv": 39, "dtg": 22, "dtg_chain": 49,
           "dtg_chain_bwd": 83, "dtg_chain_fwd_bwd": 98}
CACHE_BYTES = 256 << 20


def cache_path():
    return os.environ.get("TLMI_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "tlmi", "tune.json"))


def _arch():
    try:
        return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    except Exception:
        return "unknown"


def cache_key(kernel, n):
    """Size class of a tuning: the power of two below n, and whether n is a
    power of two itself (the tile order that pays differs between 2^21
    points and the sizes just above, measured)."""
    n = max(int(n), 1)
    pow2 = "|pow2" if n & (n - 1) == 0 else ""
    return f"{kernel}|{_arch()}|log2n={n.bit_length() - 1}{pow2}"


_loaded = {}     # cache path -> (modification time, contents): tune="auto" looks up per call


def load_cache():
    p = cache_path()
    try:
        mtime = os.stat(p).st_mtime_ns
    except OSError:
        return {}
    hit = _loaded.get(p)
    if hit is not None and hit[0] == mtime:
        return dict(hit[1])
    try:
        with open(p) as f:
            c = json.load(f)
    except (OSError, ValueError):
        return {}
    _loaded[p] = (mtime, c)
    return dict(c)


def save_cache(c):
    """Writes the cache atomically (a private temporary file, then a rename), so
    concurrent tuners never leave a partial file."""
    p = cache_path()
    os.makedirs(os.path.dirname(p), exist_ok=True)
    tmp = f"{p}.{os.getpid()}.{threading.get_ident()}.tmp"
    with open(tmp, "w") as f:
        json.dump(c, f, indent=1, sort_keys=True)
    os.replace(tmp, p)


def lookup(kernel, n):
    """The cached best tuning for (kernel, size class), or None."""
    e = load_cache().get(cache_key(kernel, n))
    return None if e is None else e["tune"]


def candidates(blocks=BLOCKS, ppts=PPTS, nts=NTS, xcds=XCDS, grid_mults=GRID_MULTS):
    for b, p, nt, x, gm in itertools.product(blocks, ppts, nts, xcds, grid_mults):
        if b == 1024 and p >= 2:
            continue    # this shape exceeds the register budget and spills
        yield {"block": b, "ppt": p, "nt": nt, "xcd": x, "grid_mult": gm}


def _calls(kernel, d, tune):
    """One recorded call of ``kernel`` on the device fields ``d``."""
    with record() as calls:
        if kernel == "sym_inverse":
            tl_sym_inverse(d["g"], d["_o6"], tune=tune)
        elif kernel == "christoffel":
            tl_christoffel(d["g"], d["dg"], d["_o18"], tune=tune)
        elif kernel == "cov_deriv":
            tl_cov_deriv(d["dg"], d["beta"], d["dbeta"], d["_o9"], tune=tune)
        elif kernel == "dtg":
            tl_dtg(d["alpha"], d["K"], d["dbeta"], d["_o6"], tune=tune)
        elif kernel == "dtg_chain":
            tl_dtg_chain(d["g"], d["dg"], d["beta"], d["dbeta"], d["K"], d["alpha"], d["_o6"],
                         tune=tune)
        elif kernel == "dtg_chain_bwd":
            tl_dtg_chain_bwd(d["g"], d["dg"], d["beta"], d["K"], d["alpha"], d["W"], *d["_grads"],
                             tune=tune)
        elif kernel == "dtg_chain_fwd_bwd":
            tl_dtg_chain_fwd_bwd(d["g"], d["dg"], d["beta"], d["dbeta"], d["K"], d["alpha"],
                                 d["W"], d["_o6"], d["_grads"], tune=tune)
        else:
            raise KeyError(kernel)
    return calls[0]


def _device_sets(n, nsets, device):
    sets = []
    for s in range(nsets):
        f = make_fields(n, seed=7000 + s)
        d = {k: torch.from_numpy(v).to(device) for k, v in f.items()}
        d["_o6"] = torch.empty(6, n, dtype=torch.float64, device=device)
        d["_o9"] = torch.empty(9, n, dtype=torch.float64, device=device)
        d["_o18"] = torch.empty(18, n, dtype=torch.float64, device=device)
        d["_grads"] = [torch.empty(c, n, dtype=torch.float64, device=device)
                       for c in (6, 18, 3, 9, 6, 1)]
        sets.append(d)
    return sets


def time_tunes(kernel, n, tunes, reps=20, warmup=3, device="cuda", sets=None):
    """Median kernel time in microseconds for each tuning (HIP events)."""
    if sets is None:
        per_set = DOUBLES[kernel] * 8 * n
        nsets = max(1, min(8, math.ceil(3 * CACHE_BYTES / max(per_set, 1))))
        sets = _device_sets(n, nsets, device)
    out = []
    for t in tunes:
        calls = [_calls(kernel, d, t) for d in sets]
        for i in range(warmup):
            calls[i % len(calls)]()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(reps)]
        for i, (a, b) in enumerate(ev):
            a.record()
            calls[i % len(calls)]()
            b.record()
        torch.cuda.synchronize()
        ts = sorted(a.elapsed_time(b) * 1e3 for a, b in ev)
        out.append(ts[len(ts) // 2])
    return out


def tune(kernel, n, tunes=None, reps=20, save=True, device="cuda"):
    """Times every candidate shape of ``kernel`` at ``n`` points; returns
    {"tune": best, "us": time, "GB_s": algorithmic bandwidth, "table": [...]}."""
    if tunes is None:
        tunes = list(candidates(ppts=PPTS + ((4,) if kernel in PPT4_KERNELS else ())))
        if kernel == "christoffel":     # components of a point spread over lanes
            tunes += [{"block": b, "nt": True, "lanes": la}
                      for b in (64, 256) for la in (2, 3, 6, 9, 18)]
    tunes = list(tunes)
    us = time_tunes(kernel, n, tunes, reps=reps, device=device)
    table = sorted(zip(us, range(len(tunes))))
    best_us, bi = table[0]
    res = {"tune": tunes[bi], "us": best_us,
           "GB_s": DOUBLES[kernel] * 8 * n / (best_us * 1e-6) / 1e9,
           "table": [{"tune": tunes[i], "us": u} for u, i in table]}
    if save:
        c = load_cache()
        c[cache_key(kernel, n)] = {k: res[k] for k in ("tune", "us", "GB_s")}
        save_cache(c)
    return res


# --------------------------------------------------------------------------- batch plans

PLAN_BLOCKS = (64, 128, 256, 512)
PLAN_GRID_MULTS = (0, 2, 4, 8)


def plan_candidates(blocks=PLAN_BLOCKS, ppts=PPTS, xcds=XCDS, grid_mults=PLAN_GRID_MULTS):
    """Shapes of a batch plan: threads per block, points per lane, XCD order,
    one block per tile (grid_mult 0) or a persistent grid; all non-temporal."""
    for b, p, x, gm in itertools.product(blocks, ppts, xcds, grid_mults):
        yield {"block": b, "ppt": p, "nt": True, "xcd": x, "grid_mult": gm}


def plan_key(domains, kind="fwd"):
    """Cache key of a set of subgrids: plan kind, architecture, number of
    subgrids and the size class of the total and of the mean subgrid."""
    sizes = [int(d["K"].shape[-1]) for d in domains]
    total = max(1, sum(sizes))
    mean = max(1, total // max(1, len(sizes)))
    return (f"batch_plan_{kind}|{_arch()}|ndom={len(sizes)}|log2n={int(math.log2(total))}"
            f"|log2mean={int(math.log2(mean))}")


def lookup_plan(domains, kind="fwd"):
    """The cached best shape for subgrids like ``domains``, or None."""
    e = load_cache().get(plan_key(domains, kind))
    return None if e is None else e["tune"]


def tune_plan(domains, tunes=None, reps=10, warmup=2, save=True, kind="fwd", want=None):
    """Builds a plan of ``kind`` over ``domains`` for every candidate shape,
    times its graph replay with HIP events (median of ``reps``) and returns
    {"tune", "us", "table"} for the fastest; caches it under plan_key."""
    from .ops import BatchPlan
    tunes = list(plan_candidates()) if tunes is None else list(tunes)
    us = []
    for t in tunes:
        plan = BatchPlan(domains, tune=t, kind=kind, want=want)
        try:
            for _ in range(warmup):
                plan.run()
            ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                  for _ in range(reps)]
            for a, b in ev:
                a.record()
                plan.run()
                b.record()
            torch.cuda.synchronize()
            ts = sorted(a.elapsed_time(b) * 1e3 for a, b in ev)
            us.append(ts[len(ts) // 2])
        finally:
            plan.close()
    table = sorted(zip(us, range(len(tunes))))
    best_us, bi = table[0]
    res = {"tune": tunes[bi], "us": best_us,
           "table": [{"tune": tunes[i], "us": u} for u, i in table]}
    if save:
        c = load_cache()
        c[plan_key(domains, kind)] = {"tune": res["tune"], "us": best_us}
        save_cache(c)
    return res
