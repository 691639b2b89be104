"""The oracle over millions of points, on several host threads (test helper).

Every output point depends only on the inputs at the same point, so the
oracle's unchanged serial functions can run on contiguous point ranges in
parallel (its C entry points run without the interpreter lock, and its
operation tape is per thread) and the results are joined back in point
order.  Nothing here computes any part of the method.
"""
from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

import oracle

CHUNK = 1 << 16


def threads():
    """Host threads to use: the cores this process may run on, at most 16."""
    return max(1, min(16, len(os.sched_getaffinity(0))))


def over_points(fn, *arrays, chunk=CHUNK):
    """fn(*slices) on every range of ``chunk`` points of the [C, n] arrays
    (contiguous copies), joined along the point axis.  fn returns an array,
    a tuple of arrays or a dict of arrays."""
    n = arrays[0].shape[-1]
    bounds = [(lo, min(n, lo + chunk)) for lo in range(0, n, chunk)] or [(0, 0)]

    def one(b):
        lo, hi = b
        return fn(*[np.ascontiguousarray(a[..., lo:hi]) for a in arrays])

    with ThreadPoolExecutor(max_workers=threads()) as pool:
        parts = list(pool.map(one, bounds))
    first = parts[0]
    if isinstance(first, dict):
        return {k: np.concatenate([p[k] for p in parts], axis=-1) for k in first}
    if isinstance(first, tuple):
        return tuple(np.concatenate([p[i] for p in parts], axis=-1) for i in range(len(first)))
    return np.concatenate(parts, axis=-1)


KEYS = ("g", "dg", "beta", "dbeta", "K", "alpha")


def dtg_chain(f):
    """The oracle's fused-chain forward over the fields ``f`` (dict)."""
    return over_points(oracle.dtg_chain, *[f[k] for k in KEYS])


def dtg_chain_vjp(f):
    """The oracle's reverse-mode gradients of L = sum W . d_t g (dict by field)."""
    return over_points(lambda *x: oracle.dtg_chain_vjp(tuple(x[:6]), x[6]),
                       *[f[k] for k in KEYS], f["W"])


def expr(name, *inputs):
    """A benchmark expression of the oracle over [C, n] inputs."""
    return over_points(lambda *x: oracle.expr(name, *x), *inputs)
