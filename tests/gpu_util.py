"""Helpers for the GPU tests: device fields with chosen layouts, canary
guard bands, and the comparison against the oracle."""
from __future__ import annotations

import numpy as np
import pytest
import torch

from metrics import rel_err

TOL = 1e-12     # per-component relative error gate for FP64 parity
CANARY = 1234.5678e300


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


class DevField:
    """A [C, n] field on the device inside a larger buffer: leading dimension
    ``ld = n + pad`` and ``offset`` leading doubles, everything outside the
    field initialised to a canary value that must survive every call."""

    def __init__(self, host, pad=0, offset=0, device="cuda"):
        host = np.asarray(host, dtype=np.float64)
        if host.ndim == 1:
            host = host[None]
        self.ncomp, self.n = host.shape
        self.ld = self.n + pad
        self.offset = offset
        total = offset + self.ncomp * self.ld + 64
        self.buf = torch.full((total,), CANARY, dtype=torch.float64, device=device)
        self.view = self.buf[offset:offset + self.ncomp * self.ld].view(self.ncomp, self.ld)[:, :self.n]
        if self.n:
            self.view.copy_(torch.from_numpy(host))

    @classmethod
    def empty(cls, ncomp, n, pad=0, offset=0, device="cuda"):
        return cls(np.full((ncomp, n), CANARY), pad, offset, device)

    def numpy(self):
        return self.view.cpu().numpy()

    def canaries_intact(self):
        mask = torch.ones_like(self.buf, dtype=torch.bool)
        if self.n:
            inner = self.buf[self.offset:self.offset + self.ncomp * self.ld].view(self.ncomp, self.ld)
            m_inner = mask[self.offset:self.offset + self.ncomp * self.ld].view(self.ncomp, self.ld)
            m_inner[:, :self.n] = False
            del inner
        return bool((self.buf[mask] == CANARY).all())


def dev(host, **kw):
    return DevField(host, **kw).view


def assert_close(x, r, tol=TOL, what=""):
    x = x.detach().cpu().numpy() if isinstance(x, torch.Tensor) else np.asarray(x)
    r = r.detach().cpu().numpy() if isinstance(r, torch.Tensor) else np.asarray(r)
    e = rel_err(x, r)
    assert e <= tol, f"{what}: relative error {e:.3e} > {tol:.1e}"
    return e
