"""Serial FP64 CPU oracle (test infrastructure only).

This package is the plain, slow, obviously correct reference implementation of
the per-grid-point tensor expressions of Lewis & Pfeiffer (arXiv:1804.10120):
the inverse metric, the Christoffel symbols (Sec. 1, eq:SpatialChristoffel),
the covariant derivative of the shift (Sec. 1, footnote) and the metric
evolution d_t g_ij (Sec. 1, eq:dtg_ij), forward- and reverse-mode derivatives
of their chain, and the benchmark expressions of Sec. 5.1 (assignments,
additions, outer products, chained contractions, K_ij).  The arithmetic lives in ``tl_oracle.cpp`` (plain
serial loops, IEEE double, no FP contraction); this module only marshals numpy
arrays into it.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import
this package.  It shares no code with the GPU library and never imports it.

Layouts: every field is a C-contiguous float64 array of shape [C, n] (``alpha``
may be [n]); component orders are documented in ``tl_oracle.cpp``.

Parity pins: every function here is pinned by the CPU tests (closed-form
metrics, invariants, an independent linear-system solve for Gamma, finite
differences and a dot-product test for the derivatives); none is unpinned.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")

_P = ctypes.c_void_p
_I = ctypes.c_int64
_SIGS = {
    "tlo_sym_inverse": [_I, _P, _P],
    "tlo_christoffel": [_I, _P, _P, _P],
    "tlo_christoffel_full": [_I, _P, _P, _P],
    "tlo_cov_deriv": [_I, _P, _P, _P, _P],
    "tlo_dtg": [_I, _P, _P, _P, _P],
    "tlo_dtg_chain": [_I] + [_P] * 7,
    "tlo_dtg_chain_jvp": [_I] + [_P] * 14,
    "tlo_dtg_chain_vjp": [_I] + [_P] * 13,
}
EXPRS = ("assign1", "assign2", "assign3", "add1", "add2", "add3", "mult1", "mult2", "mult3",
         "contract1", "contract2", "contract3", "kij",
         "lst_sym_contract", "lst_fixed_offset", "spacetime_g", "spacetime_beta")
GRAD_KEYS = (("g", 6), ("dg", 18), ("beta", 3), ("dbeta", 9), ("K", 6), ("alpha", 1))


def _field(x, ncomp, n=None, name="field"):
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    if ncomp == 1 and a.ndim == 1:
        a = a.reshape(1, -1)
    if a.ndim != 2 or a.shape[0] != ncomp:
        raise ValueError(f"{name}: expected shape [{ncomp}, n], got {a.shape}")
    if n is not None and a.shape[1] != n:
        raise ValueError(f"{name}: expected n={n}, got {a.shape[1]}")
    return a


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


class Oracle:
    """The oracle functions bound to one build of ``tl_oracle.cpp``."""

    def __init__(self, path=LIB_PATH):
        path = os.path.abspath(path)
        if not os.path.exists(path):
            raise RuntimeError(
                f"oracle library {path} is not built; run oracle.build.build() first")
        self.path = path
        self.lib = ctypes.CDLL(path)
        for name, args in _SIGS.items():
            fn = getattr(self.lib, name)
            fn.argtypes = args
            fn.restype = None
        self.lib.tlo_expr_shape.argtypes = [ctypes.c_int] + [ctypes.POINTER(ctypes.c_int)] * 3
        self.lib.tlo_expr_shape.restype = ctypes.c_int
        self.lib.tlo_expr.argtypes = [ctypes.c_int, _I, ctypes.POINTER(ctypes.c_void_p), _P]
        self.lib.tlo_expr.restype = ctypes.c_int

    def expr_shape(self, name):
        """(input component counts, output component count) of a benchmark
        expression of Sec. 5.1."""
        nin, oc = ctypes.c_int(), ctypes.c_int()
        ic = (ctypes.c_int * 4)()
        if self.lib.tlo_expr_shape(EXPRS.index(name), ctypes.byref(nin), ic, ctypes.byref(oc)):
            raise ValueError(name)
        return tuple(ic[:nin.value]), oc.value

    def expr(self, name, *inputs, out=None):
        """Expression ``name`` (the benchmark expressions of Sec. 5.1, the
        examples of Sec. 4, the spacetime split of Sec. 2.2) over [C, n] inputs
        given in the order of its right-hand side -> [C_out, n].  Components an
        expression does not write keep their values from ``out`` (NaN if no
        ``out`` is given)."""
        ic, oc = self.expr_shape(name)
        if len(inputs) != len(ic):
            raise ValueError(f"{name}: expected {len(ic)} inputs")
        ins = [_field(x, c, name=f"{name} input {k}") for k, (x, c) in enumerate(zip(inputs, ic))]
        n = ins[0].shape[1]
        if any(a.shape[1] != n for a in ins):
            raise ValueError(f"{name}: inputs differ in n")
        out = np.full((oc, n), np.nan) if out is None else np.array(out, dtype=np.float64)
        if out.shape != (oc, n):
            raise ValueError(f"{name}: out must be [{oc}, {n}]")
        ptrs = (ctypes.c_void_p * len(ins))(*[a.ctypes.data for a in ins])
        if self.lib.tlo_expr(EXPRS.index(name), n, ptrs, _ptr(out)):
            raise ValueError(name)
        return out

    def sym_inverse(self, g):
        """g [6,n] -> g^ij [6,n] (Cramer's rule: adjugate / determinant)."""
        g = _field(g, 6, name="g")
        n = g.shape[1]
        out = np.empty((6, n))
        self.lib.tlo_sym_inverse(n, _ptr(g), _ptr(out))
        return out

    def christoffel(self, ginv, dg, full=False):
        """g^ij [6,n], d_k g_ij [18,n] -> Gamma^i_jk [18,n] (all 27 if ``full``)."""
        ginv = _field(ginv, 6, name="ginv")
        n = ginv.shape[1]
        dg = _field(dg, 18, n, "dg")
        out = np.empty((27 if full else 18, n))
        fn = self.lib.tlo_christoffel_full if full else self.lib.tlo_christoffel
        fn(n, _ptr(ginv), _ptr(dg), _ptr(out))
        return out

    def cov_deriv(self, gamma, beta, dbeta):
        """Gamma [18,n], beta_i [3,n], d_j beta_i [9,n] -> nabla_j beta_i [9,n]."""
        gamma = _field(gamma, 18, name="gamma")
        n = gamma.shape[1]
        beta = _field(beta, 3, n, "beta")
        dbeta = _field(dbeta, 9, n, "dbeta")
        out = np.empty((9, n))
        self.lib.tlo_cov_deriv(n, _ptr(gamma), _ptr(beta), _ptr(dbeta), _ptr(out))
        return out

    def dtg(self, alpha, K, nabla):
        """alpha [n], K_ij [6,n], nabla_j beta_i [9,n] -> d_t g_ij [6,n]."""
        K = _field(K, 6, name="K")
        n = K.shape[1]
        alpha = _field(alpha, 1, n, "alpha")
        nabla = _field(nabla, 9, n, "nabla")
        out = np.empty((6, n))
        self.lib.tlo_dtg(n, _ptr(alpha), _ptr(K), _ptr(nabla), _ptr(out))
        return out

    @staticmethod
    def _chain_inputs(g, dg, beta, dbeta, K, alpha):
        g = _field(g, 6, name="g")
        n = g.shape[1]
        return n, (g, _field(dg, 18, n, "dg"), _field(beta, 3, n, "beta"),
                   _field(dbeta, 9, n, "dbeta"), _field(K, 6, n, "K"),
                   _field(alpha, 1, n, "alpha"))

    def dtg_chain(self, g, dg, beta, dbeta, K, alpha):
        """The whole chain, step by step (inverse, Gamma, nabla beta, dtg) -> [6,n]."""
        n, ins = self._chain_inputs(g, dg, beta, dbeta, K, alpha)
        out = np.empty((6, n))
        self.lib.tlo_dtg_chain(n, *[_ptr(a) for a in ins], _ptr(out))
        return out

    def dtg_chain_jvp(self, inputs, tangents):
        """Forward-mode derivative (dual numbers) of the chain along the tangent
        fields.  ``inputs`` and ``tangents`` are 6-tuples (g, dg, beta, dbeta,
        K, alpha).  Returns (dtg, d dtg), both [6,n]."""
        n, ins = self._chain_inputs(*inputs)
        m, tans = self._chain_inputs(*tangents)
        if m != n:
            raise ValueError("tangent size mismatch")
        out = np.empty((6, n))
        dot = np.empty((6, n))
        self.lib.tlo_dtg_chain_jvp(n, *[_ptr(a) for a in ins], *[_ptr(a) for a in tans],
                                   _ptr(out), _ptr(dot))
        return out, dot

    def dtg_chain_vjp(self, inputs, W):
        """Reverse-mode gradient (operation tape) of L = sum_p sum_s W_s dtg_s
        with respect to every stored input component.  Returns a dict with keys
        g, dg, beta, dbeta, K, alpha (shapes [6|18|3|9|6|1, n])."""
        n, ins = self._chain_inputs(*inputs)
        W = _field(W, 6, n, "W")
        outs = {k: np.empty((c, n)) for k, c in GRAD_KEYS}
        self.lib.tlo_dtg_chain_vjp(n, *[_ptr(a) for a in ins], _ptr(W),
                                   *[_ptr(outs[k]) for k, _ in GRAD_KEYS])
        return outs


_default = None


def default() -> Oracle:
    """The oracle built beside this file."""
    global _default
    if _default is None:
        _default = Oracle()
    return _default


def sym_inverse(g):
    return default().sym_inverse(g)


def christoffel(ginv, dg, full=False):
    return default().christoffel(ginv, dg, full)


def cov_deriv(gamma, beta, dbeta):
    return default().cov_deriv(gamma, beta, dbeta)


def dtg(alpha, K, nabla):
    return default().dtg(alpha, K, nabla)


def dtg_chain(g, dg, beta, dbeta, K, alpha):
    return default().dtg_chain(g, dg, beta, dbeta, K, alpha)


def dtg_chain_jvp(inputs, tangents):
    return default().dtg_chain_jvp(inputs, tangents)


def dtg_chain_vjp(inputs, W):
    return default().dtg_chain_vjp(inputs, W)


def expr(name, *inputs, out=None):
    return default().expr(name, *inputs, out=out)


def expr_shape(name):
    return default().expr_shape(name)
