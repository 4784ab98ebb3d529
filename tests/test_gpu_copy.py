"""The streaming copy the benchmark prices its kernels against
(pcad_stream_copy): byte-exact copies of several sizes, and its refusals."""
from __future__ import annotations

import ctypes

import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pcad():
    import paper_2310_03568_amd as p
    p.lib()
    assert torch.cuda.is_available()
    return p


@pytest.mark.parametrize("nbytes", [16, 4096 + 16, (1 << 20) + 48, 3 << 24])
def test_stream_copy_exact(pcad, nbytes):
    g = torch.Generator(device="cuda").manual_seed(nbytes)
    src = torch.randint(0, 256, (nbytes,), dtype=torch.uint8, device="cuda", generator=g)
    dst = torch.zeros_like(src)
    pcad.stream_copy(dst, src)
    torch.cuda.synchronize()
    assert torch.equal(dst, src)


def test_stream_copy_refusals(pcad):
    L = pcad.lib()
    buf = torch.zeros(1024, dtype=torch.uint8, device="cuda")
    p = buf.data_ptr()
    assert L.pcad_stream_copy(p, p + 512, 0, None) == 0          # nothing to do
    assert L.pcad_stream_copy(None, p, 16, None) == 3           # PCAD_E_NULLPTR
    assert L.pcad_stream_copy(p + 4, p + 512, 16, None) == 4    # PCAD_E_MISALIGNED
    assert L.pcad_stream_copy(p, p + 512, 24, None) == 1        # PCAD_E_INVALID_ARG
    torch.cuda.synchronize()
    assert int(buf.sum()) == 0
