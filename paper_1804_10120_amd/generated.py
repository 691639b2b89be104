"""Python binding of the generated entry points (include/tl_generated.h).

``call(name, *inputs)`` marshals the input fields (in the order the manifest
lists them), allocates missing outputs and calls ``tlg_<name>`` on the current
torch stream.  The manifest (generated.json) is written by the code generator
together with the kernels and the header.
"""
from __future__ import annotations

import ctypes
import json
import os

import torch

from . import ops
from ._abi import CField, Field, Tune, check, lib

MANIFEST = os.path.join(os.path.dirname(os.path.abspath(__file__)), "generated.json")
_programs = None
_fns = {}


def programs():
    """{name: manifest entry} of every generated entry point."""
    global _programs
    if _programs is None:
        with open(MANIFEST) as f:
            _programs = {p["name"]: p for p in json.load(f)["programs"]}
    return _programs


def _fn(name):
    if name not in _fns:
        fn = getattr(lib(), f"tlg_{name}")
        fn.argtypes = [ctypes.c_int64, ctypes.POINTER(CField), ctypes.c_int32,
                       ctypes.POINTER(Field), ctypes.c_int32, ctypes.c_void_p,
                       ctypes.POINTER(Tune)]
        fn.restype = ctypes.c_int
        _fns[name] = fn
    return _fns[name]


def call(name, *inputs, outs=None, stream=None, tune=None):
    """Runs generated program ``name``; returns the tuple of output fields.
    Output components that the program does not write are left untouched (so
    pass ``outs`` when they matter)."""
    p = programs()[name]
    if len(inputs) != len(p["inputs"]):
        raise ValueError(f"{name}: expected inputs {[t['name'] for t in p['inputs']]}")
    c = ops._Call()
    for t, spec in zip(inputs, p["inputs"]):
        c.add(t, spec["name"], spec["ncomp"])
    outs = list(outs) if outs is not None else [None] * len(p["outputs"])
    if len(outs) != len(p["outputs"]):
        raise ValueError(f"{name}: expected outputs {[t['name'] for t in p['outputs']]}")
    outs = [c.out(o, spec["name"], inputs[0], spec["ncomp"]) for o, spec in zip(outs, p["outputs"])]
    cin = (CField * len(inputs))(*[ops._cf(t, s["ncomp"]) for t, s in zip(inputs, p["inputs"])])
    cout = (Field * len(outs))(*[ops._f(t, s["ncomp"]) for t, s in zip(outs, p["outputs"])])
    with torch.cuda.device(c.device):
        full = (c.n, cin, len(inputs), cout, len(outs), ops._stream(c.device, stream),
                ops.make_tune(tune))
        if ops._recording() is not None:
            ops._recording().append(ops.Prepared(_fn(name), full, c.keep + [cin, cout], c.device))
        else:
            check(_fn(name)(*full))
    return tuple(outs)
