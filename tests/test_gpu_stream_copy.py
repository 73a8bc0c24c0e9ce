"""The reference streaming copy (roofline context): bytes copied exactly, bad arguments rejected
from the host before any launch."""
import sys

import pytest

pytestmark = pytest.mark.gpu


def test_stream_copy_exact_and_argument_checks():
    import torch
    from paper_1903_10367_amd import AdafacError, stream_copy
    print("case stream copy", file=sys.stderr, flush=True)
    g = torch.Generator(device="cpu").manual_seed(5)
    for n in (2, 1000, (1 << 20) + 6, 3 * (1 << 22)):          # doubles: 16 B .. 96 MiB, ragged tails
        src = torch.randn(n, generator=g, dtype=torch.float64).cuda()
        dst = torch.zeros_like(src)
        stream_copy(src, dst)
        torch.cuda.synchronize()
        assert torch.equal(src, dst), n
    src = torch.zeros(8, dtype=torch.float64, device="cuda")
    with pytest.raises(AdafacError):
        stream_copy(src[1:7], torch.zeros(6, dtype=torch.float64, device="cuda"))      # src off 16-byte alignment
    with pytest.raises(AdafacError):
        stream_copy(src[:3], torch.zeros(3, dtype=torch.float64, device="cuda"))       # 24 bytes
    with pytest.raises(AdafacError):
        stream_copy(src, torch.zeros(4, dtype=torch.float64, device="cuda"))           # sizes differ
