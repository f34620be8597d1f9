"""pf_sum_f32_noalloc (the sum for callers that cannot allocate) against
pf_sum_f32 with a caller workspace: the same bits, on two calls in a row
through the C ABI, the second with a smaller input (its scratch then holds
the first call's partials past the second's chunks), and its host-side
rejections."""
import ctypes

import numpy as np
import pytest

import oracle
import paper_1302_5586_amd as pf
from gpu_util import device

pytestmark = pytest.mark.gpu


def _t(a, dev):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def _noalloc(lib, x, out, stream):
    return lib.pf_sum_f32_noalloc(x.numel(), x.data_ptr(), out.data_ptr(), stream)


def test_noalloc_matches_workspace_sum_twice():
    dev = device()
    import torch
    lib = pf.load()
    stream = torch.cuda.current_stream().cuda_stream
    rng = np.random.default_rng(2024)
    for n in (5 * 65536 + 123, 70001, 1):
        x = _t((rng.standard_normal(n) * 100).astype(np.float32), dev)
        want = pf.sum_f32(x)
        got = torch.full((2,), float("nan"), dtype=torch.float64, device=dev)
        pf._check(_noalloc(lib, x, got, stream))
        torch.cuda.synchronize()
        g, w = got.cpu().numpy(), want.cpu().numpy()
        assert np.array_equal(g, w), (n, g, w)
        ref = oracle.sum_f32(x.cpu().numpy())
        tol = 2.0 * max(n - 1, 1) * 2.0 ** -53 * float(np.abs(x.cpu().numpy().astype(np.float64)).sum())
        assert abs(g[0] - ref) <= tol


def test_noalloc_largest_and_rejects():
    dev = device()
    import torch
    lib = pf.load()
    stream = torch.cuda.current_stream().cuda_stream
    n = 1 << 29  # the documented maximum: 8192 chunks of 65536
    x = torch.ones(n, dtype=torch.float32, device=dev)
    out = torch.empty(2, dtype=torch.float64, device=dev)
    pf._check(_noalloc(lib, x, out, stream))
    assert out.cpu().numpy().tolist() == [float(n), 1.0]
    del x
    y = torch.zeros(16, dtype=torch.float32, device=dev)
    st = lib.pf_sum_f32_noalloc((1 << 29) + 1, y.data_ptr(), out.data_ptr(), stream)
    assert st == pf.PF_EUNSUPPORTED
    st = lib.pf_sum_f32_noalloc(16, y.data_ptr(), y.data_ptr() + 8, stream)
    assert st == pf.PF_EALIAS
    st = lib.pf_sum_f32_noalloc(0, y.data_ptr(), out.data_ptr(), stream)
    assert st == pf.PF_EINVAL
    torch.cuda.synchronize()
