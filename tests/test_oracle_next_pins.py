"""Pins of the oracle's extensions: border rules, chains of passes,
reductions, the histogram and the OP2 edge increment.

Every expected value comes from a library routine or a closed form, never
from the oracle: scipy.ndimage.correlate (modes 'nearest', 'constant',
'reflect', 'mirror') and numpy.pad (modes 'edge', 'constant', 'symmetric',
'reflect'), math.fsum for exact sums, numpy.bincount for histograms, and
integer-valued data for exact mesh increments.
"""
import math

import numpy as np
import pytest
import scipy.ndimage as ndi

import oracle

U = 2.0 ** -24


def gamma(n):
    return n * U / (1.0 - n * U)


SCIPY_MODE = {oracle.BORDER_CLAMP: "nearest", oracle.BORDER_ZERO: "constant",
              oracle.BORDER_REFLECT: "reflect", oracle.BORDER_MIRROR: "mirror"}
NUMPY_MODE = {oracle.BORDER_CLAMP: "edge", oracle.BORDER_ZERO: "constant",
              oracle.BORDER_REFLECT: "symmetric", oracle.BORDER_MIRROR: "reflect"}


def padded_sum(img, f, r, border):
    h, w = img.shape
    p = np.pad(img.astype(np.float64), r, mode=NUMPY_MODE[border])
    acc = np.zeros((h, w))
    for dy in range(2 * r + 1):
        for dx in range(2 * r + 1):
            acc += float(f[dy, dx]) * p[dy:dy + h, dx:dx + w]
    return acc


@pytest.mark.parametrize("border", [0, 1, 2, 3])
def test_border_modes_brute_force(border):
    rng = np.random.default_rng(50 + border)
    for h in range(1, 8):
        for w in range(1, 8):
            for r in range(0, 5):
                if border == oracle.BORDER_MIRROR and (h == 1 or w == 1):
                    continue   # numpy's 'reflect' pad is undefined on one element
                img = rng.random((h, w), dtype=np.float32)
                f = rng.standard_normal((2 * r + 1, 2 * r + 1)).astype(np.float32)
                out = oracle.filter2d_f32_border(img, f, border).astype(np.float64)
                e = padded_sum(img, f, r, border)
                bound = gamma((2 * r + 1) ** 2) * (np.abs(f).sum() * np.abs(img).max()) + 1e-30
                assert np.all(np.abs(out - e) <= bound), (h, w, r, border)
                if min(h, w) > r:   # scipy's extension agrees once the window fits
                    e2 = ndi.correlate(img.astype(np.float64), f.astype(np.float64), mode=SCIPY_MODE[border], cval=0.0)
                    np.testing.assert_allclose(e, e2, rtol=0, atol=1e-12)


def test_border_mirror_single_element():
    img = np.array([[2.0]], np.float32)
    f = np.ones((3, 3), np.float32)
    assert oracle.filter2d_f32_border(img, f, oracle.BORDER_MIRROR)[0, 0] == 18.0


def test_border_clamp_matches_base():
    rng = np.random.default_rng(60)
    img = rng.random((11, 13), dtype=np.float32)
    f = rng.standard_normal((5, 5)).astype(np.float32)
    np.testing.assert_array_equal(oracle.filter2d_f32_border(img, f, oracle.BORDER_CLAMP), oracle.filter2d_f32(img, f))


@pytest.mark.parametrize("border", [0, 1, 2])
def test_chain(border):
    rng = np.random.default_rng(70 + border)
    img = rng.random((12, 14), dtype=np.float32)
    f = rng.random((3, 3)).astype(np.float32)
    one = oracle.filter_chain_f32(img, f, 1, border)
    np.testing.assert_array_equal(one, oracle.filter2d_f32_border(img, f, border))
    passes = 4
    out = oracle.filter_chain_f32(img, f, passes, border).astype(np.float64)
    e = img.astype(np.float64)
    d = np.abs(img.astype(np.float64))
    for _ in range(passes):
        e = padded_sum(e, f, 1, border)
        d = padded_sum(d, np.abs(f), 1, border)
    g = gamma(9)
    assert np.all(np.abs(out - e) <= passes * g * (1 + g) ** passes * d + 1e-30)


def test_sum_f32():
    rng = np.random.default_rng(80)
    for n in (1, 7, 1000, 123457):
        x = (rng.standard_normal(n) * 1e3).astype(np.float32)
        exact = math.fsum(float(v) for v in x)
        got = oracle.sum_f32(x)
        assert abs(got - exact) <= n * 2.0 ** -53 * float(np.abs(x.astype(np.float64)).sum()) + 1e-300
    assert oracle.sum_f32(np.full(1 << 20, 0.5, np.float32)) == float(1 << 19)


def test_hist256():
    rng = np.random.default_rng(81)
    for n in (1, 255, 100003):
        x = rng.integers(0, 256, n, dtype=np.uint8)
        np.testing.assert_array_equal(oracle.hist256_u8(x), np.bincount(x, minlength=256))
    np.testing.assert_array_equal(oracle.hist256_u8(np.full(10, 7, np.uint8)), np.eye(256, dtype=np.int64)[7] * 10)


def test_edge_inc_exact():
    rng = np.random.default_rng(82)
    ncells, nedges = 50, 400
    e2c = rng.integers(0, ncells, (nedges, 2)).astype(np.int32)
    edge = rng.integers(-1000, 1000, nedges).astype(np.float64)   # integers: every order is exact
    cells0 = rng.integers(-5, 5, ncells).astype(np.float64)
    out = oracle.edge_inc_f64(ncells, e2c, edge, cells0)
    expect = cells0.copy()
    np.add.at(expect, e2c[:, 0], edge)
    np.add.at(expect, e2c[:, 1], edge)
    np.testing.assert_array_equal(out, expect)


def test_edge_inc_paper_example_shape():
    # A 1-to-2 map on a ring of cells: edge i joins cells i and i+1, so each
    # cell receives its two incident edges' values.
    ncells = 6
    e2c = np.array([[i, (i + 1) % ncells] for i in range(ncells)], np.int32)
    edge = np.arange(1, ncells + 1, dtype=np.float64)
    out = oracle.edge_inc_f64(ncells, e2c, edge, np.zeros(ncells))
    expect = np.array([edge[i] + edge[(i - 1) % ncells] for i in range(ncells)])
    np.testing.assert_array_equal(out, expect)
