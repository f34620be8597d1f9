"""Border rules and fused filter chains on the GPU against the oracle.

Exact mode (separate FP32 multiply and add, definition order) must equal the
oracle bit for bit at every pass and under every border rule. The default
mode (one FMA per tap) is held to a per-pass tolerance: with non-negative
weights and data each pass is within 1e-5 relative of its exact value, and
errors pass through a normalised filter without growing, so a chain of P
passes is within P * 1e-5 of the oracle's chain."""
import numpy as np
import pytest

import oracle
import paper_1302_5586_amd as pf
import synth
from gpu_util import device

pytestmark = pytest.mark.gpu

BORDERS = [pf.BORDER_CLAMP, pf.BORDER_ZERO, pf.BORDER_REFLECT, pf.BORDER_MIRROR]


def _t(a, dev):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


# Shapes: single tile, ragged multi-tile (64 x 32 tiles), narrower than a
# tile and than the halo, one row, one column.
SHAPES = [(1, 1), (1, 7), (5, 1), (3, 3), (31, 65), (70, 129), (33, 200), (100, 2)]


@pytest.mark.parametrize("border", BORDERS)
@pytest.mark.parametrize("r,passes", [(0, 1), (1, 1), (1, 3), (2, 2), (3, 1), (4, 4), (8, 2), (1, 16)])
def test_chain_exact_bitwise(border, r, passes):
    dev = device()
    rng = np.random.default_rng(100 + 10 * r + passes + 1000 * border)
    for (h, w) in SHAPES:
        img = rng.random((h, w), dtype=np.float32)
        f = rng.standard_normal((2 * r + 1, 2 * r + 1)).astype(np.float32)
        got = pf.filter_chain(_t(img, dev), _t(f, dev), passes, border, exact=True).cpu().numpy()
        ref = oracle.filter_chain_f32(img, f, passes, border)
        assert np.array_equal(got, ref), "chain %dx%d r=%d passes=%d border=%d" % (h, w, r, passes, border)


@pytest.mark.parametrize("border", BORDERS)
@pytest.mark.parametrize("r,passes", [(1, 4), (2, 3), (4, 2)])
def test_chain_fma_tolerance(border, r, passes):
    dev = device()
    rng = np.random.default_rng(7 + r * passes + 100 * border)
    f = synth.gaussian_2d(r, 1.0)
    for (h, w) in [(97, 301), (64, 64), (2, 9)]:
        img = rng.random((h, w), dtype=np.float32)
        got = pf.filter_chain(_t(img, dev), _t(f, dev), passes, border).cpu().numpy()
        ref = oracle.filter_chain_f32(img, f, passes, border)
        tol = passes * 1e-5 * np.abs(ref) + 1e-30
        assert np.all(np.abs(got - ref) <= tol), "chain %dx%d r=%d passes=%d border=%d max err %g" % (
            h, w, r, passes, border, float(np.max(np.abs(got - ref) - tol)))


@pytest.mark.parametrize("border", BORDERS)
@pytest.mark.parametrize("r", [0, 1, 2, 4, 8])
def test_border_filter_exact(border, r):
    dev = device()
    rng = np.random.default_rng(300 + r + 20 * border)
    for (h, w) in [(1, 1), (9, 4), (37, 300), (66, 3)]:
        img = rng.standard_normal((h, w)).astype(np.float32)
        f = rng.standard_normal((2 * r + 1, 2 * r + 1)).astype(np.float32)
        got = pf.filter2d_border(_t(img, dev), _t(f, dev), border, exact=True).cpu().numpy()
        ref = oracle.filter2d_f32_border(img, f, border)
        assert np.array_equal(got, ref), "border %dx%d r=%d border=%d" % (h, w, r, border)


def test_clamp_border_is_the_plain_filter():
    dev = device()
    cfg = synth.config_small()
    x, f = _t(cfg.image, dev), _t(cfg.f2d, dev)
    a = pf.filter2d_border(x, f, pf.BORDER_CLAMP).cpu().numpy()
    b = pf.filter2d(x, f).cpu().numpy()
    assert np.array_equal(a, b)
    # one-pass chain, exact, equals the plain exact filter
    c = pf.filter_chain(x, f, 1, pf.BORDER_CLAMP, exact=True).cpu().numpy()
    d = pf.filter2d(x, f, exact=True).cpu().numpy()
    assert np.array_equal(c, d)


def test_chain_4096_full():
    """The benchmark's chain (4096 x 4096, 3 x 3 Gaussian, 4 passes, clamp):
    exact mode equals the oracle's chain bit for bit at every pixel, and the
    default (FMA) mode is within 4 * 1e-5 relative of it everywhere."""
    dev = device()
    cfg = synth.config_large()
    f = synth.gaussian_2d(1, 1.0)
    passes = 4
    x, fd = _t(cfg.image, dev), _t(f, dev)
    ref = oracle.filter_chain_f32(cfg.image, f, passes, pf.BORDER_CLAMP)
    got = pf.filter_chain(x, fd, passes, pf.BORDER_CLAMP, exact=True).cpu().numpy()
    bad = np.flatnonzero(got != ref)
    assert bad.size == 0, "%d pixels differ, first at %s" % (bad.size, np.unravel_index(bad[0], got.shape))
    fma = pf.filter_chain(x, fd, passes, pf.BORDER_CLAMP).cpu().numpy()
    err = np.abs(fma.astype(np.float64) - ref)
    assert np.all(err <= passes * 1e-5 * np.abs(ref) + 1e-30), float(err.max())
    print("chain 4096^2 x 4: exact bit-identical; FMA max abs %.3g" % float(err.max()))


def test_chain_rejects():
    dev = device()
    import torch
    x = torch.zeros((8, 8), device=dev)
    f = torch.zeros((9, 9), device=dev)
    with pytest.raises(pf.PFError):
        pf.filter_chain(x, f, 5)  # r * passes = 20
    with pytest.raises(pf.PFInvalid):
        pf.filter_chain(x, f[:3, :3].contiguous(), 0)
