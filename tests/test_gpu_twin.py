"""The bandwidth-twin and copy kernels (the measured memory ceilings)."""
import numpy as np
import pytest
import torch

from gpu_util import DevField, need_gpu
from paper_1804_10120_amd import tl_bw_copy, tl_bw_twin
from paper_1804_10120_amd._abi import TWIN_SHAPES

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


@pytest.mark.parametrize("nin,nout", TWIN_SHAPES)
@pytest.mark.parametrize("n", [1, 129, 4097])
@pytest.mark.parametrize("tune", [None, dict(block=64, ppt=2, nt=True, xcd=True),
                                  dict(block=256, ppt=4, nt=True)],
                         ids=["default", "b64ppt2", "b256ppt4"])
def test_twin(nin, nout, n, tune):
    x = np.random.default_rng(nin * 1000 + n).standard_normal((nin, n))
    src = DevField(x, pad=2)
    dst = DevField.empty(nout, n, pad=4, offset=2)
    tl_bw_twin(src.view, nout, dst.view, tune=tune)
    torch.cuda.synchronize()
    s = np.zeros(n)
    for i in range(nin):          # the kernel's summation order
        s = s + x[i]
    exp = np.stack([s + c for c in range(nout)])
    assert np.array_equal(dst.numpy(), exp)
    assert dst.canaries_intact()


@pytest.mark.parametrize("nin,nout", [(40, 43), (24, 18)])
@pytest.mark.parametrize("tune", [dict(block=1024, ppt=2, nt=True, xcd=True),
                                  dict(block=512, ppt=2, nt=True)], ids=["b1024ppt2", "b512ppt2"])
def test_twin_two_point_stores_full_size(nin, nout, tune):
    """Two points per lane (16-byte stores with explicit wait states) over 2^21
    points and a ragged tail, every element exact."""
    n = (1 << 21) + 6
    gen = torch.Generator(device="cuda").manual_seed(nin * 7 + nout)
    src = torch.randn(nin, n, dtype=torch.float64, device="cuda", generator=gen)
    dst = tl_bw_twin(src, nout, tune=tune)
    s = torch.zeros(n, dtype=torch.float64, device="cuda")
    for i in range(nin):          # the kernel's summation order
        s = s + src[i]
    for c in range(nout):
        assert torch.equal(dst[c], s + c), f"component {c}"


def test_more_than_2_31_points():
    """The streaming template's index arithmetic beyond 2^31 points (one
    component in and out, 17 GB each, 64-bit addressing), every element, in
    the default shape and with two points per lane."""
    n = (1 << 31) + 1029
    src = torch.arange(n, dtype=torch.float64, device="cuda").view(1, n)
    dst = torch.empty(1, n, dtype=torch.float64, device="cuda")
    for tune in (None, dict(block=512, ppt=2, nt=True)):
        dst.fill_(-1.0)
        tl_bw_twin(src, 1, dst, tune=tune)
        assert torch.equal(dst, src), tune
    del src, dst
    torch.cuda.empty_cache()


@pytest.mark.parametrize("n", [1, 2, 3, 1001, 1 << 20])
def test_copy(n):
    src = torch.randn(n, dtype=torch.float64, device="cuda")
    assert torch.equal(tl_bw_copy(src), src)


@pytest.mark.parametrize("n", [1, 2, 511, 513, 4097, 1 << 22])
@pytest.mark.parametrize("offset", [0, 1])
def test_read_reference(n, offset):
    from paper_1804_10120_amd import tl_bw_read
    buf = torch.rand(n + offset, dtype=torch.float64, device="cuda")
    src = buf[offset:]
    partial = torch.full((2048,), 7.0, dtype=torch.float64, device="cuda")
    tl_bw_read(src, partial)
    nblk = min(2048, (n + 511) // 512)
    got = partial[:nblk].sum().item()
    ref = src.double().sum().item()
    assert abs(got - ref) <= 1e-12 * abs(ref)
    assert torch.all(partial[nblk:] == 7.0)


@pytest.mark.parametrize("n", [1, 2, 511, 4097, 1 << 22])
@pytest.mark.parametrize("offset", [0, 1])
def test_write_reference(n, offset):
    from paper_1804_10120_amd import tl_bw_write
    buf = DevField.empty(1, n + offset, pad=0, offset=0)
    dst = buf.buf[offset:offset + n]
    tl_bw_write(dst)
    torch.cuda.synchronize()
    assert torch.all(dst == 1.0)
    assert buf.buf[:offset].eq(1234.5678e300).all() and buf.buf[offset + n:].eq(1234.5678e300).all()
