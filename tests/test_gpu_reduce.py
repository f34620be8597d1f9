"""Sum/mean and the 256-bin histogram on the GPU against the oracle.

The sum is float64 over a fixed tree, the oracle's a float64 left-to-right
loop: both are within (n - 1) * 2^-53 * sum|x| of the exact sum, so they
differ by at most twice that. Sums of integers below 2^53 are exact on both
sides and must match bit for bit, as must every histogram."""
import numpy as np
import pytest

import oracle
import paper_1302_5586_amd as pf
import synth
from gpu_util import device

pytestmark = pytest.mark.gpu

# 65536 is the chunk length: one full chunk, one short of it, one past it.
SIZES = [1, 3, 4, 5, 1023, 16383, 16384, 16385, 65535, 65536, 65537, 2 * 65536, 3 * 65536 + 5, 1 << 20]


def _t(a, dev):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


@pytest.mark.parametrize("n", SIZES)
def test_sum_against_oracle(n):
    dev = device()
    rng = np.random.default_rng(n)
    x = (rng.standard_normal(n) * 10).astype(np.float32)
    got = pf.sum_f32(_t(x, dev)).cpu().numpy()
    ref = oracle.sum_f32(x)
    tol = 2.0 * max(n - 1, 1) * 2.0 ** -53 * float(np.sum(np.abs(x.astype(np.float64))))
    assert abs(got[0] - ref) <= tol, (got[0], ref, tol)
    assert got[1] == got[0] / n


@pytest.mark.parametrize("n", [1, 65535, 65536, 65537, 3 * 65536 + 5, 1 << 22])
def test_sum_integers_exact(n):
    dev = device()
    rng = np.random.default_rng(7 + n)
    x = rng.integers(-1000, 1000, n).astype(np.float32)
    got = pf.sum_f32(_t(x, dev)).cpu().numpy()
    assert got[0] == oracle.sum_f32(x) == float(np.sum(x.astype(np.int64)))


def test_sum_reproducible_and_special_values():
    dev = device()
    rng = np.random.default_rng(11)
    x = rng.random(5 * 65536 + 77, dtype=np.float32)
    xt = _t(x, dev)
    a = pf.sum_f32(xt).cpu().numpy()
    for _ in range(3):
        assert np.array_equal(pf.sum_f32(xt).cpu().numpy(), a)
    y = x.copy()
    y[70000] = np.nan
    assert np.isnan(pf.sum_f32(_t(y, dev)).cpu().numpy()[0])
    y = x.copy()
    y[5] = np.inf
    assert pf.sum_f32(_t(y, dev)).cpu().numpy()[0] == np.inf


def test_sum_config_large():
    dev = device()
    cfg = synth.config_large()
    got = pf.sum_f32(_t(cfg.image, dev)).cpu().numpy()
    ref = oracle.sum_f32(cfg.image)
    n = cfg.image.size
    assert abs(got[0] - ref) <= 2.0 * n * 2.0 ** -53 * ref


@pytest.mark.parametrize("n", [1, 2, 3, 5, 4095, (1 << 20) - 1, 1 << 20, (1 << 20) + 3, 5 * (1 << 20) + 7])
def test_hist_against_oracle(n):
    dev = device()
    rng = np.random.default_rng(100 + n)
    x = rng.integers(0, 256, n).astype(np.uint8)
    got = pf.hist256_u8(_t(x, dev)).cpu().numpy()
    assert np.array_equal(got, oracle.hist256_u8(x))
    assert got.sum() == n


def test_hist_constant_unaligned_and_rgb():
    dev = device()
    import torch
    x = np.full(3 * (1 << 20) + 1, 200, np.uint8)
    got = pf.hist256_u8(_t(x, dev)).cpu().numpy()
    assert got[200] == x.size and got.sum() == x.size
    # an unaligned start: a view one byte into a buffer
    rng = np.random.default_rng(3)
    y = rng.integers(0, 256, (1 << 20) + 9).astype(np.uint8)
    yt = _t(y, dev)
    view = yt[1:]
    assert view.data_ptr() % 4 != 0
    got = pf.hist256_u8(view).cpu().numpy()
    assert np.array_equal(got, oracle.hist256_u8(y[1:]))
    # a start aligned to 4 bytes but not to 16 (the word path)
    view = yt[4:]
    assert view.data_ptr() % 16 != 0
    got = pf.hist256_u8(view).cpu().numpy()
    assert np.array_equal(got, oracle.hist256_u8(y[4:]))
    cfg = synth.config_rgb()
    got = pf.hist256_u8(_t(cfg.image, dev)).cpu().numpy()
    assert np.array_equal(got, oracle.hist256_u8(cfg.image.reshape(-1)))
    del torch


def test_reduce_rejects():
    dev = device()
    import torch
    x = torch.zeros(100, device=dev)
    ws = torch.empty(1, dtype=torch.float64, device=dev)
    small = torch.empty(0, dtype=torch.float64, device=dev)
    out = torch.empty(2, dtype=torch.float64, device=dev)
    with pytest.raises(pf.PFInvalid):
        pf.load()
        pf._check(pf.load().pf_sum_f32(100, x.data_ptr(), out.data_ptr(), small.data_ptr(), 0, None))
    with pytest.raises(pf.PFAlias):
        pf._check(pf.load().pf_sum_f32(100, x.data_ptr(), x.data_ptr() + 8, ws.data_ptr(), 8, None))
