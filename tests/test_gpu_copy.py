"""The bandwidth probe (isb_stream_copy) copies exactly, including the 8-byte tail of an odd length
and lengths that leave some lanes of the unrolled trip without work."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n", [0, 1, 2, 7, 256 * 2 + 1, 1 << 20, (1 << 22) + 3])
def test_stream_copy_exact(n):
    import torch
    from paper_2102_05791_amd import isb
    g = torch.Generator(device="cuda:0").manual_seed(n)
    src = torch.randn(max(n, 1), dtype=torch.float64, device="cuda:0", generator=g)[:n]
    dst = torch.full((max(n, 1) + 1,), -7.0, dtype=torch.float64, device="cuda:0")
    isb.stream_copy(src, dst[:n])
    torch.cuda.synchronize()
    assert torch.equal(dst[:n], src)
    assert float(dst[n]) == -7.0  # nothing past the end
