"""FP64 per-grid-point tensor expressions of arXiv:1804.10120 on AMD MI355X.

The compute path is the C-ABI library ``libtl.so`` (hand-written HIP kernels
for gfx950, declared in ``include/tl.h``); this package only marshals torch
device tensors into it.  The library is loaded on first use, and every entry
point raises if it is missing: there is no CPU fallback.
"""
__all__ = ["synth"]
