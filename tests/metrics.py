"""Error metric shared by every numerical comparison in the tests.

Per-component relative error, scaled by the component's magnitude:
err_c = max_p |X[c,p] - R[c,p]| / max_p |R[c,p]|; a component that is
identically zero is scaled by the largest magnitude of the whole tensor (or by 1
if that is zero too).  The reported error is max_c err_c.  A NaN or inf in one
array but not at the same place in the other counts as an infinite error.
"""
import numpy as np


def rel_err(x, r, scale="component"):
    """``scale="tensor"`` divides every component by the tensor-wide maximum
    instead (for closed forms whose exact zeros come out as rounding noise)."""
    x = np.asarray(x, dtype=np.float64)
    r = np.asarray(r, dtype=np.float64)
    if x.shape != r.shape:
        raise ValueError(f"shape mismatch {x.shape} vs {r.shape}")
    if x.ndim == 1:
        x, r = x[None], r[None]
    x = x.reshape(x.shape[0], -1)
    r = r.reshape(r.shape[0], -1)
    if x.size == 0:
        return 0.0
    fx, fr = np.isfinite(x), np.isfinite(r)
    if np.any(fx != fr):
        return np.inf
    if not np.all(fr):
        same = (x == r) | (np.isnan(x) & np.isnan(r))
        if np.any(~fr & ~same):
            return np.inf
        x = np.where(fr, x, 0.0)
        r = np.where(fr, r, 0.0)
    whole = np.abs(r).max()
    if scale == "tensor":
        sc = np.full(r.shape[0], whole if whole > 0 else 1.0)
    else:
        sc = np.abs(r).max(axis=1)
        sc = np.where(sc > 0, sc, whole if whole > 0 else 1.0)
    return float((np.abs(x - r).max(axis=1) / sc).max())
