"""Python binding of the C ABI over torch device tensors.

Each ``tl_*`` function has the name and argument order of the C entry point
in ``include/tl.h``.  It only checks and marshals arguments -- dtype float64,
one HIP device, shape [C, n] with unit stride along points (``alpha`` may be
[n]) -- allocates missing outputs with ``torch.empty`` and calls the library on
the current torch stream of the tensors' device.  Every step of the
computation runs in the library's HIP kernels.
"""
from __future__ import annotations

import ctypes
import threading

import torch

from . import _abi
from ._abi import CField, Domain, DomainBwd, Field, KernelAttr, TLError, Tune, check, lib

NCOMP = {"g": 6, "ginv": 6, "K": 6, "dtg": 6, "w": 6, "dg": 18, "gamma": 18, "beta": 3,
         "dbeta": 9, "nabla_beta": 9, "alpha": 1}


def _points(t, ncomp, name):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name}: expected a torch.Tensor")
    if t.dtype != torch.float64:
        raise TypeError(f"{name}: expected torch.float64, got {t.dtype}")
    if t.device.type != "cuda":
        raise ValueError(f"{name}: expected a HIP device tensor, got device {t.device}")
    if ncomp == 1 and t.dim() == 1:
        n = t.shape[0]
    elif t.dim() == 2 and t.shape[0] == ncomp:
        n = t.shape[1]
    else:
        raise ValueError(f"{name}: expected shape [{ncomp}, n]" + (" or [n]" if ncomp == 1 else "")
                         + f", got {tuple(t.shape)}")
    if n > 1 and t.stride(-1) != 1:
        raise ValueError(f"{name}: points must be contiguous (stride(-1) == 1)")
    return n


def _ld(t, ncomp):
    if ncomp == 1 or t.dim() == 1:
        return max(1, t.shape[-1])
    return t.stride(0)


def _cf(t, ncomp):
    return CField(t.data_ptr(), _ld(t, ncomp))


def _f(t, ncomp):
    if t is None:
        return Field(None, 0)
    return Field(t.data_ptr(), _ld(t, ncomp))


class _Call:
    """Collects the tensors of one call: common n, common device."""

    def __init__(self):
        self.n = None
        self.device = None
        self.keep = []

    def add(self, t, name, ncomp=None):
        ncomp = NCOMP[name] if ncomp is None else ncomp
        n = _points(t, ncomp, name)
        self.keep.append(t)
        if self.n is None:
            self.n, self.device = n, t.device
        else:
            if n != self.n:
                raise ValueError(f"{name}: {n} points, expected {self.n}")
            if t.device != self.device:
                raise ValueError(f"{name}: on {t.device}, expected {self.device}")
        return t

    def out(self, t, name, like, ncomp=None):
        ncomp = NCOMP[name] if ncomp is None else ncomp
        if t is None:
            shape = (self.n,) if ncomp == 1 and like.dim() == 1 else (ncomp, self.n)
            return torch.empty(shape, dtype=torch.float64, device=self.device)
        return self.add(t, name, ncomp)


LD_ALIGN = 16   # doubles: one 128-byte cache line


def padded_ld(n, align=LD_ALIGN):
    """n rounded up to a multiple of ``align`` (at least ``align``)."""
    return max(align, (int(n) + align - 1) // align * align)


def empty_field(ncomp, n, *, device=None, align=LD_ALIGN):
    """An uninitialised [ncomp, n] float64 field whose leading dimension is
    padded_ld(n): every component then starts on a 128-byte line (torch's
    allocations are at least that aligned), so no cache line is shared by two
    components.  With ld = n and n not a multiple of 16, the lines at the
    ends of each tile of each component are fetched by two tiles; measured on
    the 256-subgrid batch this costs about 9 % of the bandwidth."""
    buf = torch.empty(int(ncomp), padded_ld(n, align), dtype=torch.float64, device=device)
    return buf[:, :int(n)]


def to_field(x, *, device=None, align=LD_ALIGN):
    """Copies a [ncomp, n] (or [n]) array into an empty_field on ``device``."""
    x = torch.as_tensor(x, dtype=torch.float64)
    if x.dim() == 1:
        x = x[None]
    f = empty_field(x.shape[0], x.shape[1], device=device, align=align)
    f.copy_(x)
    return f


def _stream(device, stream):
    if stream is None:
        stream = torch.cuda.current_stream(device)
    return ctypes.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


def make_tune(tune):
    """None (library default), a Tune, a dict with keys block, ppt, nt, xcd,
    ptr64, grid_mult, lanes (missing numbers mean the default; flags default to
    off), or a tuple (block, ppt, flags, grid_mult[, lanes]) -> Tune pointer or None.  (The tl_*
    functions also accept tune="auto", the autotuner's cached shape.)"""
    if tune is None:
        return None
    if isinstance(tune, Tune):
        t = tune
    elif isinstance(tune, dict):
        t = Tune(int(tune.get("block", 0)), int(tune.get("ppt", 0)),
                 int(tune.get("flags", 0)) | (_abi.TL_TUNE_NT if tune.get("nt") else 0)
                 | (_abi.TL_TUNE_XCD if tune.get("xcd") else 0)
                 | (_abi.TL_TUNE_PTR64 if tune.get("ptr64") else 0),
                 int(tune.get("grid_mult", 0)), int(tune.get("lanes", 0)))
    else:
        t = Tune(*[int(v) for v in tune])
    return ctypes.pointer(t)


class Prepared:
    """One fully marshalled C-ABI call: calling it re-enters the library with
    the same arguments (validation included) and no Python-side checks.  It
    holds references to the tensors it names.  The stream is bound when the
    call is recorded: to capture into a graph, call the tl_* function inside
    the capture instead."""

    def __init__(self, fn, args, keep, device):
        self.fn, self.args, self.keep, self.device = fn, args, keep, device

    def __call__(self):
        st = self.fn(*self.args)
        if st:
            check(st)


_local = threading.local()     # per thread: the list being recorded into, or None


def _recording():
    return getattr(_local, "calls", None)


class record:
    """Context manager: tl_* calls made inside, on this thread, are marshalled
    into Prepared objects (outputs are still allocated) instead of being
    launched; other threads are unaffected.

        with record() as calls:
            tl_dtg_chain(...)
        for c in calls: c()
    """

    def __enter__(self):
        if _recording() is not None:
            raise RuntimeError("record() does not nest")
        _local.calls = []
        return _local.calls

    def __exit__(self, *exc):
        _local.calls = None
        return False


def _auto(tune, kernel, n):
    """tune="auto": the autotuner's cached shape for (kernel, size class), or
    the library default when nothing is cached."""
    if isinstance(tune, str):
        if tune != "auto":
            raise ValueError(f"tune={tune!r}: expected None, 'auto', a dict, a tuple or a Tune")
        from . import autotune
        return autotune.lookup(kernel, n)
    return tune


def _run(fn, c, *args, stream=None, tune=None, kernel=None):
    tune = _auto(tune, kernel, c.n)
    with torch.cuda.device(c.device):
        full = (c.n, *args, _stream(c.device, stream), make_tune(tune))
        if _recording() is not None:
            _recording().append(Prepared(fn, full, c.keep, c.device))
            return
        check(fn(*full))


def tl_sym_inverse(g, ginv=None, *, stream=None, tune=None):
    """g^ij = inverse of the symmetric g_ij: [6,n] -> [6,n]."""
    c = _Call()
    c.add(g, "g")
    ginv = c.out(ginv, "ginv", g)
    _run(lib().tl_sym_inverse, c, _cf(g, 6), _f(ginv, 6), stream=stream, tune=tune,
         kernel="sym_inverse")
    return ginv


def tl_christoffel(ginv, dg, gamma=None, *, stream=None, tune=None):
    """Gamma^i_jk from g^ij [6,n] and d_k g_ij [18,n] -> [18,n]."""
    c = _Call()
    c.add(ginv, "ginv")
    c.add(dg, "dg")
    gamma = c.out(gamma, "gamma", dg)
    _run(lib().tl_christoffel, c, _cf(ginv, 6), _cf(dg, 18), _f(gamma, 18), stream=stream,
         tune=tune,
         kernel="christoffel")
    return gamma


def tl_cov_deriv(gamma, beta, dbeta, nabla_beta=None, *, stream=None, tune=None):
    """nabla_j beta_i from Gamma [18,n], beta_i [3,n], d_j beta_i [9,n] -> [9,n]."""
    c = _Call()
    c.add(gamma, "gamma")
    c.add(beta, "beta")
    c.add(dbeta, "dbeta")
    nabla_beta = c.out(nabla_beta, "nabla_beta", dbeta)
    _run(lib().tl_cov_deriv, c, _cf(gamma, 18), _cf(beta, 3), _cf(dbeta, 9), _f(nabla_beta, 9),
         stream=stream, tune=tune,
         kernel="cov_deriv")
    return nabla_beta


def tl_dtg(alpha, K, nabla_beta, dtg=None, *, stream=None, tune=None):
    """d_t g_ij from alpha [n], K_ij [6,n], nabla_j beta_i [9,n] -> [6,n]."""
    c = _Call()
    c.add(alpha, "alpha")
    c.add(K, "K")
    c.add(nabla_beta, "nabla_beta")
    dtg = c.out(dtg, "dtg", K)
    _run(lib().tl_dtg, c, _cf(alpha, 1), _cf(K, 6), _cf(nabla_beta, 9), _f(dtg, 6),
         stream=stream, tune=tune,
         kernel="dtg")
    return dtg


def tl_dtg_chain(g, dg, beta, dbeta, K, alpha, dtg=None, *, stream=None, tune=None):
    """Fused d_t g_ij from g, d g, beta, d beta, K, alpha -> [6,n]."""
    c = _Call()
    for t, name in ((g, "g"), (dg, "dg"), (beta, "beta"), (dbeta, "dbeta"), (K, "K"),
                    (alpha, "alpha")):
        c.add(t, name)
    dtg = c.out(dtg, "dtg", K)
    _run(lib().tl_dtg_chain, c, _cf(g, 6), _cf(dg, 18), _cf(beta, 3), _cf(dbeta, 9), _cf(K, 6),
         _cf(alpha, 1), _f(dtg, 6), stream=stream, tune=tune,
         kernel="dtg_chain")
    return dtg


GRAD_NAMES = ("g", "dg", "beta", "dbeta", "K", "alpha")


def tl_dtg_chain_bwd(g, dg, beta, K, alpha, w, g_bar=None, dg_bar=None, beta_bar=None,
                     dbeta_bar=None, K_bar=None, alpha_bar=None, *, want=None, stream=None,
                     tune=None):
    """Adjoint of the fused chain for w = dL/d(d_t g) [6,n].

    Returns the tuple (g_bar, dg_bar, beta_bar, dbeta_bar, K_bar, alpha_bar).
    ``want`` is a 6-tuple of booleans in that order; an unwanted gradient is
    neither computed into memory nor allocated and comes back as None.
    """
    c = _Call()
    for t, name in ((g, "g"), (dg, "dg"), (beta, "beta"), (K, "K"), (alpha, "alpha"), (w, "w")):
        c.add(t, name)
    want = (True,) * 6 if want is None else tuple(bool(x) for x in want)
    if len(want) != 6:
        raise ValueError("tl_dtg_chain_bwd: want has 6 entries")
    outs = [g_bar, dg_bar, beta_bar, dbeta_bar, K_bar, alpha_bar]
    ncomp = (6, 18, 3, 9, 6, 1)
    likes = (g, dg, beta, dg, K, alpha)
    for i in range(6):
        if outs[i] is not None or want[i]:
            outs[i] = c.out(outs[i], GRAD_NAMES[i] + "_bar", likes[i], ncomp[i])
    if all(o is None for o in outs):
        raise ValueError("tl_dtg_chain_bwd: no gradient requested")
    fields = [_f(o, nc) for o, nc in zip(outs, ncomp)]
    _run(lib().tl_dtg_chain_bwd, c, _cf(g, 6), _cf(dg, 18), _cf(beta, 3), _cf(K, 6),
         _cf(alpha, 1), _cf(w, 6), *fields, stream=stream, tune=tune,
         kernel="dtg_chain_bwd")
    return tuple(outs)


def tl_dtg_chain_fwd_bwd(g, dg, beta, dbeta, K, alpha, w, dtg=None, grads=None, *, want=None,
                         stream=None, tune=None):
    """tl_dtg_chain and tl_dtg_chain_bwd in one pass, for a cotangent w [6,n]
    known up front (a loss linear in d_t g).

    Returns (dtg, (g_bar, dg_bar, beta_bar, dbeta_bar, K_bar, alpha_bar)).
    ``grads`` optionally gives the six gradient outputs (None entries are
    allocated when wanted); ``want`` is a 7-tuple of booleans for d_t g and the
    six gradients; an unwanted output is not written and comes back as None.
    """
    c = _Call()
    for t, name in ((g, "g"), (dg, "dg"), (beta, "beta"), (dbeta, "dbeta"), (K, "K"),
                    (alpha, "alpha"), (w, "w")):
        c.add(t, name)
    want = (True,) * 7 if want is None else tuple(bool(x) for x in want)
    if len(want) != 7:
        raise ValueError("tl_dtg_chain_fwd_bwd: want has 7 entries")
    outs = [dtg] + (list(grads) if grads is not None else [None] * 6)
    if len(outs) != 7:
        raise ValueError("tl_dtg_chain_fwd_bwd: grads has 6 entries")
    ncomp = (6, 6, 18, 3, 9, 6, 1)
    likes = (K, g, dg, beta, dbeta, K, alpha)
    names = ("dtg",) + tuple(x + "_bar" for x in GRAD_NAMES)
    for i in range(7):
        if outs[i] is not None or want[i]:
            outs[i] = c.out(outs[i], names[i], likes[i], ncomp[i])
    if all(o is None for o in outs):
        raise ValueError("tl_dtg_chain_fwd_bwd: no output requested")
    fields = [_f(o, nc) for o, nc in zip(outs, ncomp)]
    _run(lib().tl_dtg_chain_fwd_bwd, c, _cf(g, 6), _cf(dg, 18), _cf(beta, 3), _cf(dbeta, 9),
         _cf(K, 6), _cf(alpha, 1), _cf(w, 6), *fields, stream=stream, tune=tune,
         kernel="dtg_chain_fwd_bwd")
    return outs[0], tuple(outs[1:])


def tl_bw_copy(src, dst=None, *, stream=None):
    """dst = src for a contiguous float64 device tensor (bandwidth reference)."""
    if src.dtype != torch.float64 or not src.is_contiguous() or src.device.type != "cuda":
        raise ValueError("tl_bw_copy: src must be a contiguous float64 device tensor")
    if dst is None:
        dst = torch.empty_like(src)
    if dst.shape != src.shape or not dst.is_contiguous() or dst.dtype != torch.float64 \
            or dst.device != src.device:
        raise ValueError("tl_bw_copy: dst must match src")
    with torch.cuda.device(src.device):
        args = (src.numel(), ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()),
                _stream(src.device, stream))
        if _recording() is not None:
            _recording().append(Prepared(lib().tl_bw_copy, args, [src, dst], src.device))
        else:
            check(lib().tl_bw_copy(*args))
    return dst


def tl_bw_read(src, partial=None, *, stream=None):
    """Reads a contiguous float64 device tensor (the read-only bandwidth
    reference); returns the per-block partial sums [TL_BW_READ_BLOCKS]
    (entries past the number of blocks are left as they were)."""
    if src.dtype != torch.float64 or not src.is_contiguous() or src.device.type != "cuda":
        raise ValueError("tl_bw_read: src must be a contiguous float64 device tensor")
    if partial is None:
        partial = torch.zeros(_abi.TL_BW_READ_BLOCKS, dtype=torch.float64, device=src.device)
    if partial.numel() < _abi.TL_BW_READ_BLOCKS or not partial.is_contiguous() \
            or partial.dtype != torch.float64 or partial.device != src.device:
        raise ValueError("tl_bw_read: partial must be a contiguous float64 tensor of "
                         f"{_abi.TL_BW_READ_BLOCKS} elements on src's device")
    _bw_stream(src.numel(), _abi.TL_BW_READ, src, partial, stream)
    return partial


def tl_bw_write(dst, *, stream=None):
    """dst[:] = 1 for a contiguous float64 device tensor (the write-only
    bandwidth reference)."""
    if dst.dtype != torch.float64 or not dst.is_contiguous() or dst.device.type != "cuda":
        raise ValueError("tl_bw_write: dst must be a contiguous float64 device tensor")
    _bw_stream(dst.numel(), _abi.TL_BW_WRITE, None, dst, stream)
    return dst


def _bw_stream(n, kind, src, dst, stream):
    dev = dst.device
    keep = [t for t in (src, dst) if t is not None]
    with torch.cuda.device(dev):
        args = (n, kind, ctypes.c_void_p(src.data_ptr() if src is not None else None),
                ctypes.c_void_p(dst.data_ptr()), _stream(dev, stream))
        if _recording() is not None:
            _recording().append(Prepared(lib().tl_bw_stream, args, keep, dev))
            return
        check(lib().tl_bw_stream(*args))


def tl_bw_twin(src, nout, dst=None, *, stream=None, tune=None):
    """Bandwidth twin: reads every component of ``src`` [nin, n], writes
    ``nout`` components (out_c = sum of the inputs + c)."""
    c = _Call()
    nin = src.shape[0] if src.dim() == 2 else 0
    c.add(src, "in", nin)
    dst = c.out(dst, "out", src, nout)
    with torch.cuda.device(c.device):
        full = (c.n, nin, _cf(src, nin), nout, _f(dst, nout), _stream(c.device, stream),
                make_tune(tune))
        if _recording() is not None:
            _recording().append(Prepared(lib().tl_bw_twin, full, c.keep, c.device))
        else:
            check(lib().tl_bw_twin(*full))
    return dst


def tl_expr_shape(expr):
    """(input component counts, output component count) of a Sec. 5.1
    benchmark expression, by name ("assign1" ... "kij") or id."""
    eid = _abi.EXPRS.index(expr) if isinstance(expr, str) else int(expr)
    nin, oc = ctypes.c_int32(), ctypes.c_int32()
    ic = (ctypes.c_int32 * 4)()
    check(lib().tl_expr_shape(eid, ctypes.byref(nin), ic, ctypes.byref(oc)))
    return tuple(ic[:nin.value]), oc.value


def tl_expr(expr, *inputs, out=None, stream=None, tune=None):
    """A Sec. 5.1 benchmark expression over [C, n] device fields given in the
    order of its right-hand side; returns (or fills) the left-hand side."""
    eid = _abi.EXPRS.index(expr) if isinstance(expr, str) else int(expr)
    ic, oc = tl_expr_shape(eid)
    if len(inputs) != len(ic):
        raise ValueError(f"{_abi.EXPRS[eid]}: expected {len(ic)} inputs, got {len(inputs)}")
    c = _Call()
    for k, (t, nc) in enumerate(zip(inputs, ic)):
        c.add(t, f"in[{k}]", nc)
    out = c.out(out, "out", inputs[-1], oc)
    arr = (CField * len(inputs))(*[_cf(t, nc) for t, nc in zip(inputs, ic)])
    with torch.cuda.device(c.device):
        full = (eid, c.n, arr, len(inputs), _f(out, oc), _stream(c.device, stream),
                make_tune(tune))
        if _recording() is not None:
            _recording().append(Prepared(lib().tl_expr, full, c.keep + [arr], c.device))
        else:
            check(lib().tl_expr(*full))
    return out


def tl_kernel_info(kernel, tune=None):
    """Attributes (registers, scratch, ...) of the kernel a call would run."""
    a = KernelAttr()
    check(lib().tl_kernel_info(kernel.encode(), make_tune(tune), ctypes.byref(a)))
    return {k: getattr(a, k) for k, _ in KernelAttr._fields_}


def _fwd_domain(c, d):
    """The tl_domain of one forward subgrid (its inputs already added to the
    call ``c``), allocating d_t g with empty_field when it is not given."""
    out = d.get("dtg")
    out = c.out(empty_field(6, c.n, device=c.device) if out is None else out, "dtg", d["K"])
    return (Domain(c.n, _cf(d["g"], 6), _cf(d["dg"], 18), _cf(d["beta"], 3), _cf(d["dbeta"], 9),
                   _cf(d["K"], 6), _cf(d["alpha"], 1), _f(out, 6)), dict(d, dtg=out))


def tl_batch_run_noalloc(domains, *, stream=None, tune=None):
    """tl_batch_run_noalloc: d_t g over many subgrids with the batched kernel,
    its tables in the library's fixed device array (no device allocation).

    ``domains``: dicts with the tensors g, dg, beta, dbeta, K, alpha and dtg
    (the output, which must be given: nothing is allocated here).  Calls that
    overlap on one device race (they share the array); order them on one
    stream.
    """
    arr = (Domain * len(domains))()
    device = None
    for i, d in enumerate(domains):
        if d.get("dtg") is None:
            raise ValueError(f"domain {i}: dtg (the output) must be given")
        c = _Call()
        for name in ("g", "dg", "beta", "dbeta", "K", "alpha"):
            c.add(d[name], name)
        if device is None:
            device = c.device
        elif c.device != device:
            raise ValueError("all subgrids must be on one device")
        arr[i], _ = _fwd_domain(c, d)
    if device is None:
        raise ValueError("tl_batch_run_noalloc needs at least one subgrid")
    with torch.cuda.device(device):
        full = (arr, len(domains), make_tune(tune), _stream(device, stream))
        if _recording() is not None:
            _recording().append(Prepared(lib().tl_batch_run_noalloc, full,
                                         [arr] + [d[k] for d in domains for k in
                                                  ("g", "dg", "beta", "dbeta", "K", "alpha",
                                                   "dtg")], device))
        else:
            check(lib().tl_batch_run_noalloc(*full))
    return [d["dtg"] for d in domains]


class BatchPlan:
    """tl_batch_plan_*: d_t g (kind="fwd") or its adjoint (kind="bwd") over
    many subgrids in one graph-captured launch.

    kind="fwd": ``domains`` is a sequence of dicts with the tensors g, dg,
    beta, dbeta, K, alpha and (optionally) dtg of one subgrid each.
    kind="bwd": dicts with g, dg, beta, K, alpha, the cotangent W and
    (optionally) g_bar, dg_bar, beta_bar, dbeta_bar, K_bar, alpha_bar; ``want``
    (6 booleans in that order) selects the gradients computed.
    Missing outputs are allocated with empty_field (leading dimension padded
    to 16 doubles).  ``tune="auto"`` takes the autotuner's cached shape for
    subgrids like these (autotune.plan_key), tuning them first if nothing is
    cached.  The plan keeps references to every tensor, so the buffers it
    borrows outlive it.
    """

    def __init__(self, domains, tune=None, kind="fwd", want=None):
        self._plan = None
        self.domains = []
        if kind not in ("fwd", "bwd"):
            raise ValueError(f"kind={kind!r}: expected 'fwd' or 'bwd'")
        self.kind = kind
        if isinstance(tune, str):
            if tune != "auto":
                raise ValueError(f"tune={tune!r}: expected None, 'auto', a dict, a tuple or a Tune")
            from . import autotune
            tune = autotune.lookup_plan(domains, kind=kind)
            if tune is None:
                tune = autotune.tune_plan(domains, kind=kind, want=want)["tune"]
        want = (True,) * 6 if want is None else tuple(bool(x) for x in want)
        if len(want) != 6 or not any(want):
            raise ValueError("want: 6 booleans, at least one true")
        arr = ((Domain if kind == "fwd" else DomainBwd) * len(domains))()
        device = None
        for i, d in enumerate(domains):
            c = _Call()
            names = ("g", "dg", "beta", "dbeta", "K", "alpha") if kind == "fwd" else \
                ("g", "dg", "beta", "K", "alpha", "W")
            for name in names:
                c.add(d[name], "w" if name == "W" else name)
            if device is None:
                device = c.device
            elif c.device != device:
                raise ValueError("all subgrids must be on one device")
            if kind == "fwd":
                arr[i], dd = _fwd_domain(c, d)
                self.domains.append(dd)
            else:
                grads = []
                for k, nc, w in zip(GRAD_NAMES, (6, 18, 3, 9, 6, 1), want):
                    o = d.get(k + "_bar")
                    if o is None and w:
                        o = empty_field(nc, c.n, device=c.device)
                    grads.append(c.out(o, k + "_bar", d["K"], nc) if o is not None else None)
                self.domains.append(dict(d, **{k + "_bar": o for k, o in zip(GRAD_NAMES, grads)}))
                arr[i] = DomainBwd(c.n, _cf(d["g"], 6), _cf(d["dg"], 18), _cf(d["beta"], 3),
                                   _cf(d["K"], 6), _cf(d["alpha"], 1), _cf(d["W"], 6),
                                   *[_f(o, nc) for o, nc in zip(grads, (6, 18, 3, 9, 6, 1))])
        if device is None:
            raise ValueError("BatchPlan needs at least one subgrid")
        self.device = device
        plan = ctypes.c_void_p()
        create = lib().tl_batch_plan_create if kind == "fwd" else lib().tl_batch_plan_bwd_create
        with torch.cuda.device(device):
            check(create(arr, len(domains), make_tune(tune), ctypes.byref(plan)))
        self._plan = plan
        p, t, b = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        check(lib().tl_batch_plan_info(plan, ctypes.byref(p), ctypes.byref(t), ctypes.byref(b)))
        self.points, self.tiles, self.blocks = p.value, t.value, b.value

    @property
    def outputs(self):
        """kind="fwd": each subgrid's d_t g; kind="bwd": each subgrid's tuple
        (g_bar, dg_bar, beta_bar, dbeta_bar, K_bar, alpha_bar), None where not
        wanted."""
        if self.kind == "fwd":
            return [d["dtg"] for d in self.domains]
        return [tuple(d[k + "_bar"] for k in GRAD_NAMES) for d in self.domains]

    def run(self, stream=None):
        """Replay the captured graph on ``stream`` (default: current stream)."""
        with torch.cuda.device(self.device):
            check(lib().tl_batch_plan_launch(self._plan, _stream(self.device, stream)))

    def run_direct(self, stream=None):
        """Launch the persistent kernel directly (no graph)."""
        with torch.cuda.device(self.device):
            check(lib().tl_batch_plan_launch_direct(self._plan, _stream(self.device, stream)))

    def close(self):
        if self._plan is not None:
            with torch.cuda.device(self.device):
                check(lib().tl_batch_plan_destroy(self._plan))
            self._plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


__all__ = ["record", "Prepared", "tl_sym_inverse", "tl_christoffel", "tl_cov_deriv", "tl_dtg",
           "tl_dtg_chain", "tl_dtg_chain_bwd", "tl_dtg_chain_fwd_bwd", "tl_bw_copy", "tl_bw_read",
           "tl_bw_write", "tl_bw_twin", "tl_expr", "tl_expr_shape", "tl_kernel_info", "BatchPlan",
           "tl_batch_run_noalloc",
           "TLError", "empty_field", "to_field", "padded_ld", "LD_ALIGN"]
