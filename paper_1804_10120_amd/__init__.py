"""FP64 per-grid-point tensor expressions of arXiv:1804.10120 on AMD MI355X.

The compute path is the C-ABI library ``libtl.so`` (hand-written HIP kernels
for gfx950, declared in ``include/tl.h``); this package only marshals torch
device tensors into it.  The library is loaded on first use, and every entry
point raises if it is missing: there is no CPU fallback.
"""
from .ops import (BatchPlan, TLError, tl_batch_run_noalloc, empty_field, padded_ld, tl_bw_copy,
                  tl_bw_read, tl_bw_twin, tl_bw_write, tl_christoffel, tl_cov_deriv, tl_dtg, tl_dtg_chain, tl_dtg_chain_bwd,
                  tl_dtg_chain_fwd_bwd, tl_expr, tl_expr_shape, tl_kernel_info, tl_sym_inverse,
                  to_field)
from .autograd import DtgChainFn, dtg_chain

__all__ = ["tl_sym_inverse", "tl_christoffel", "tl_cov_deriv", "tl_dtg", "tl_dtg_chain",
           "tl_dtg_chain_bwd", "tl_dtg_chain_fwd_bwd", "tl_bw_copy", "tl_bw_read", "tl_bw_write",
           "tl_bw_twin", "tl_expr", "tl_expr_shape", "tl_kernel_info", "BatchPlan", "TLError",
           "tl_batch_run_noalloc",
           "empty_field", "to_field", "padded_ld", "DtgChainFn", "dtg_chain"]
