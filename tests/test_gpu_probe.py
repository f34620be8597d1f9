"""The measurement probes compute what they claim (their rates are only
meaningful if the work is really done)."""
import numpy as np
import pytest
import torch

import paper_1302_5586_amd as pf

pytestmark = pytest.mark.gpu


def _sdot4(a: int, b: int, c: int) -> int:
    """Signed 4 x int8 dot product plus c, wrapped to int32."""
    s = c
    for i in range(4):
        x = (a >> (8 * i)) & 0xFF
        y = (b >> (8 * i)) & 0xFF
        s += (x - 256 if x > 127 else x) * (y - 256 if y > 127 else y)
    return (s + 2**31) % 2**32 - 2**31


def test_probe_dot4_values():
    out = torch.empty(256, dtype=torch.int32, device="cuda")
    assert pf.probe_alu(pf.PROBE_DOT4, 1, 1, out) == 256 * 128
    got = out.cpu().numpy()
    b = 0x01020304
    for lane in (0, 1, 63, 64, 200, 255):
        a = [lane + k for k in range(8)]
        for _ in range(16):
            a = [_sdot4(a[k], b + k, a[k]) for k in range(8)]
        want = (sum(a) + 2**31) % 2**32 - 2**31
        assert got[lane] == want, lane


@pytest.mark.parametrize("n", [0, 1, 5, 4096, 1_000_003])
def test_probe_copy_exact(n):
    g = torch.Generator().manual_seed(n)
    x = torch.randn(n, generator=g).cuda()
    out = torch.full((n,), -1.0, device="cuda")
    pf.probe_copy(x, out)
    torch.cuda.synchronize()
    assert torch.equal(out.cpu(), x.cpu())


def test_probe_rejects():
    out = torch.empty(256, dtype=torch.int32, device="cuda")
    with pytest.raises(pf.PFError):
        pf.probe_alu(7, 1, 1, out)
    with pytest.raises(pf.PFError):
        pf.probe_alu(pf.PROBE_FMA, 1, 0, out)
