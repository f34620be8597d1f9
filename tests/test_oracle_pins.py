"""Pins of the oracle against facts that do not come from the oracle itself.

The paper prints no worked example or number, so the oracle is pinned by
closed forms, invariants of correlation, a library routine that computes
the same definition (scipy.ndimage.correlate with mode='nearest' is
clamp-to-edge correlation), and brute force on tiny images in exact
float64/int64 arithmetic.

Each pin is chosen so that a plausible mistake in the oracle fails it:
a transposed filter (K6, K11), a flipped kernel (K6, K11 with random
non-symmetric filters), a wrong border rule (K6, K7, K11 on images smaller
than the window), a dropped tap or radius off by one (K7, K11), swapped
row and column weights (K9), a logical instead of arithmetic shift or a
missing saturation (K3, K11u8), and wrong plane indexing (K11u8 with
distinct planes).
"""
import os

import numpy as np
import pytest
import scipy.ndimage as ndi

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
U = 2.0 ** -24


def gamma(n: int) -> float:
    """Higham's gamma_n = n u / (1 - n u): the relative bound of a recursive
    FP32 sum of n products (round-to-nearest)."""
    return n * U / (1.0 - n * U)


def exact_2d(img, f):
    """Clamp-to-edge correlation in float64 by scipy (exact for FP32 inputs
    up to float64 rounding, which is far below the FP32 bound)."""
    return ndi.correlate(np.asarray(img, np.float64), np.asarray(f, np.float64), mode="nearest")


def abs_bound(img, f):
    """D = sum |w| |x| over each window, the scale of the inner-product bound."""
    return ndi.correlate(np.abs(np.asarray(img, np.float64)), np.abs(np.asarray(f, np.float64)), mode="nearest")


def read_golden(name):
    sections = {}
    cur = None
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            if line.isalpha():
                cur = line
                sections[cur] = []
            else:
                sections[cur].append([float(v) for v in line.split()])
    return {k: np.array(v) for k, v in sections.items()}


# ---- K6 / K7: worked examples ---------------------------------------------

@pytest.mark.parametrize("name", ["k6_orientation.txt", "k7_box.txt"])
def test_worked_examples(name):
    g = read_golden(name)
    out = oracle.filter2d_f32(g["input"].astype(np.float32), g["filter"].astype(np.float32))
    np.testing.assert_array_equal(out, g["expected"].astype(np.float32))


def test_k6_orientation_u8():
    g = read_golden("k6_orientation.txt")
    img = g["input"].astype(np.uint8)[None]
    f = (g["filter"] * 64).astype(np.int8)       # tap weight 64 with shift 6 is the identity
    out = oracle.filter2d_u8(img, f, 6)
    np.testing.assert_array_equal(out[0], g["expected"].astype(np.uint8))


# ---- K1: identity ---------------------------------------------------------

@pytest.mark.parametrize("r", [0, 1, 2, 3, 4])
def test_k1_identity_f32(r):
    rng = np.random.default_rng(100 + r)
    img = rng.random((13, 17), dtype=np.float32)
    f = np.zeros((2 * r + 1, 2 * r + 1), np.float32)
    f[r, r] = 1.0
    np.testing.assert_array_equal(oracle.filter2d_f32(img, f), img)
    d = np.zeros(2 * r + 1, np.float32)
    d[r] = 1.0
    np.testing.assert_array_equal(oracle.filter_sep_f32(img, d, d), img)


@pytest.mark.parametrize("r", [0, 1, 3])
def test_k1_identity_u8(r):
    rng = np.random.default_rng(200 + r)
    img = rng.integers(0, 256, (2, 9, 11), dtype=np.uint8)
    f = np.zeros((2 * r + 1, 2 * r + 1), np.int8)
    f[r, r] = 64
    np.testing.assert_array_equal(oracle.filter2d_u8(img, f, 6), img)


# ---- K2 / K3: constant images ---------------------------------------------

@pytest.mark.parametrize("r,sigma", [(1, 1.0), (2, 1.5), (3, 0.7), (4, 2.0)])
def test_k2_constant_normalised(r, sigma):
    c = np.float32(0.7310586)
    img = np.full((10, 12), c, np.float32)
    f = synth.gaussian_2d(r, sigma)
    out = oracle.filter2d_f32(img, f)
    n = (2 * r + 1) ** 2
    # the weights sum to 1 only up to their own rounding: bound both errors
    wsum = float(np.asarray(f, np.float64).sum())
    expect = float(c) * wsum
    assert np.all(np.abs(out.astype(np.float64) - expect) <= gamma(n) * float(c) * wsum + 1e-12)
    assert abs(wsum - 1.0) <= n * U


def test_k2_constant_all_ones_exact():
    img = np.full((5, 4), 3.0, np.float32)
    out = oracle.filter2d_f32(img, np.ones((3, 3), np.float32))
    np.testing.assert_array_equal(out, np.full((5, 4), 27.0, np.float32))


def test_k3_u8_constant_golden():
    rows = np.loadtxt(os.path.join(GOLDEN, "k3_u8_constant.txt"), comments="#", dtype=np.int64)
    for v, wv, expect in rows:
        img = np.full((1, 6, 9), v, np.uint8)
        f = np.full((7, 7), wv, np.int8)
        out = oracle.filter2d_u8(img, f, 6)
        assert np.all(out == expect), (v, wv, expect)


# ---- K4: linearity --------------------------------------------------------

def test_k4_linearity():
    rng = np.random.default_rng(7)
    x = rng.random((20, 23), dtype=np.float32)
    y = rng.random((20, 23), dtype=np.float32)
    f = rng.standard_normal((5, 5)).astype(np.float32)
    a, b = np.float32(0.75), np.float32(-1.5)
    lhs = oracle.filter2d_f32(a * x + b * y, f).astype(np.float64)
    rhs = float(a) * oracle.filter2d_f32(x, f).astype(np.float64) + float(b) * oracle.filter2d_f32(y, f).astype(np.float64)
    d = abs_bound(np.abs(a * x) + np.abs(b * y), f)
    assert np.all(np.abs(lhs - rhs) <= 3 * gamma(26) * d + 1e-12)


# ---- K5: interior translation equivariance --------------------------------

def test_k5_translation():
    rng = np.random.default_rng(8)
    big = rng.random((40, 50), dtype=np.float32)
    f = rng.standard_normal((5, 5)).astype(np.float32)
    r, sy, sx = 2, 3, 5
    a = big[:30, :40]
    b = big[sy:sy + 30, sx:sx + 40]
    oa = oracle.filter2d_f32(a, f)
    ob = oracle.filter2d_f32(b, f)
    # interior where both windows stay inside their images
    np.testing.assert_array_equal(oa[sy + r:30 - r, sx + r:40 - r], ob[r:30 - r - sy, r:40 - r - sx])


# ---- K8 / K11: library routine and brute force ----------------------------

def test_k8_library_config_small():
    cfg = synth.config_small()
    out = oracle.filter2d_f32(cfg.image, cfg.f2d).astype(np.float64)
    e = exact_2d(cfg.image, cfg.f2d)
    assert np.all(np.abs(out - e) <= gamma(9) * abs_bound(cfg.image, cfg.f2d))


def _edge_window_sum(img, f, r):
    """Brute force by padding with numpy's edge mode and summing shifted
    slices in float64: a second formulation of clamp-to-edge correlation."""
    h, w = img.shape
    p = np.pad(np.asarray(img, np.float64), r, mode="edge")
    acc = np.zeros((h, w))
    for dy in range(2 * r + 1):
        for dx in range(2 * r + 1):
            acc += float(f[dy, dx]) * p[dy:dy + h, dx:dx + w]
    return acc


def test_k11_brute_force_f32():
    rng = np.random.default_rng(11)
    for h in range(1, 9):
        for w in range(1, 9):
            for r in range(0, 5):
                img = rng.random((h, w), dtype=np.float32)
                f = rng.standard_normal((2 * r + 1, 2 * r + 1)).astype(np.float32)
                out = oracle.filter2d_f32(img, f).astype(np.float64)
                e1 = exact_2d(img, f)
                e2 = _edge_window_sum(img, f, r)
                np.testing.assert_allclose(e1, e2, rtol=0, atol=1e-12)
                bound = gamma((2 * r + 1) ** 2) * abs_bound(img, f) + 1e-30
                assert np.all(np.abs(out - e1) <= bound), (h, w, r)


def test_k11_brute_force_u8():
    rng = np.random.default_rng(12)
    for h in range(1, 8):
        for w in range(1, 8):
            for r in (0, 1, 2, 3):
                for shift in (0, 3, 6):
                    img = rng.integers(0, 256, (3, h, w), dtype=np.uint8)
                    f = rng.integers(-8, 9, (2 * r + 1, 2 * r + 1)).astype(np.int8)
                    out = oracle.filter2d_u8(img, f, shift)
                    for c in range(3):
                        acc = np.rint(_edge_window_sum(img[c].astype(np.float64), f, r)).astype(np.int64)
                        q = np.clip(acc >> shift, 0, 255).astype(np.uint8)   # numpy >> on int64 floors
                        np.testing.assert_array_equal(out[c], q, err_msg=str((h, w, r, shift, c)))


def test_k11_u8_config_rgb_sample():
    cfg = synth.rgb_u8(c=3, h=37, w=53)
    out = oracle.filter2d_u8(cfg.image, cfg.filt, cfg.shift)
    for c in range(3):
        acc = np.rint(ndi.correlate(cfg.image[c].astype(np.float64), cfg.filt.astype(np.float64), mode="nearest")).astype(np.int64)
        np.testing.assert_array_equal(out[c], np.clip(acc >> 6, 0, 255).astype(np.uint8))


# ---- K9: separability -----------------------------------------------------

@pytest.mark.parametrize("h,w,r", [(1, 1, 2), (1, 9, 1), (9, 1, 3), (17, 23, 2), (6, 5, 4)])
def test_k9_separable(h, w, r):
    rng = np.random.default_rng(h * 100 + w * 10 + r)
    img = rng.random((h, w), dtype=np.float32)
    fx = rng.standard_normal(2 * r + 1).astype(np.float32)
    fy = rng.standard_normal(2 * r + 1).astype(np.float32)   # fx != fy catches swapped passes
    out = oracle.filter_sep_f32(img, fx, fy).astype(np.float64)
    e = ndi.correlate1d(ndi.correlate1d(img.astype(np.float64), fx.astype(np.float64), axis=1, mode="nearest"),
                        fy.astype(np.float64), axis=0, mode="nearest")
    d = abs_bound(img, np.outer(np.abs(fy).astype(np.float64), np.abs(fx).astype(np.float64)))
    k = 2 * r + 1
    assert np.all(np.abs(out - e) <= (2 * gamma(k) + gamma(k) ** 2) * d + 1e-30)
    # and the 2D oracle on the exact outer product agrees within both bounds
    f2 = np.outer(fy.astype(np.float64), fx.astype(np.float64)).astype(np.float32)
    o2 = oracle.filter2d_f32(img, f2).astype(np.float64)
    assert np.all(np.abs(o2 - out) <= (gamma(k * k) + 2 * gamma(k) + gamma(k) ** 2 + U) * d + 1e-30)


# ---- K10: one-column and one-row images ------------------------------------

def test_k10_degenerate_shapes():
    rng = np.random.default_rng(10)
    r = 2
    f = rng.random((5, 5)).astype(np.float32)
    col = rng.random((9, 1), dtype=np.float32)
    out = oracle.filter2d_f32(col, f).astype(np.float64)
    fr = f.astype(np.float64).sum(axis=1)                    # sum over dx
    idx = np.clip(np.arange(9)[:, None] + np.arange(-r, r + 1)[None, :], 0, 8)
    expect = (fr[None, :] * col[idx, 0].astype(np.float64)).sum(axis=1)
    assert np.allclose(out[:, 0], expect, rtol=gamma(25) * 2, atol=0)
    row = col.T.copy()
    out_r = oracle.filter2d_f32(row, f).astype(np.float64)
    fc = f.astype(np.float64).sum(axis=0)
    expect_r = (fc[None, :] * row[0, idx].astype(np.float64)).sum(axis=1)
    assert np.allclose(out_r[0], expect_r, rtol=gamma(25) * 2, atol=0)
    one = np.array([[0.5]], np.float32)
    assert np.isclose(float(oracle.filter2d_f32(one, f)[0, 0]), 0.5 * float(f.astype(np.float64).sum()), rtol=gamma(25))


# ---- K12: order independence -----------------------------------------------

def test_k12_order_independence():
    rng = np.random.default_rng(12)
    img = rng.random((19, 21), dtype=np.float32)
    f = rng.standard_normal((5, 5)).astype(np.float32)
    ref = oracle.filter2d_f32(img, f)
    n = img.size
    for order in (np.arange(n)[::-1], rng.permutation(n)):
        np.testing.assert_array_equal(oracle.filter2d_f32_permuted(img, f, 2, order), ref)
    for y, x in ((0, 0), (18, 20), (7, 3)):
        assert oracle.filter2d_f32_at(img, f, 2, y, x) == ref[y, x]


# ---- K13: flip symmetry ---------------------------------------------------

def test_k13_flip():
    rng = np.random.default_rng(13)
    img = rng.random((15, 16), dtype=np.float32)
    f = rng.standard_normal((7, 7)).astype(np.float32)
    a = oracle.filter2d_f32(img[:, ::-1], f[:, ::-1])
    b = oracle.filter2d_f32(img, f)[:, ::-1]
    d = abs_bound(img, f)[:, ::-1]
    assert np.all(np.abs(a.astype(np.float64) - b) <= 2 * gamma(49) * d)
    u = rng.integers(0, 256, (1, 15, 16), dtype=np.uint8)
    g = rng.integers(-8, 9, (7, 7)).astype(np.int8)
    np.testing.assert_array_equal(oracle.filter2d_u8(u[:, :, ::-1], g[:, ::-1], 6),
                                  oracle.filter2d_u8(u, g, 6)[:, :, ::-1])


# ---- NaN propagation (IEEE) -----------------------------------------------

def test_nan_propagates():
    img = np.zeros((5, 5), np.float32)
    img[2, 2] = np.nan
    out = oracle.filter2d_f32(img, synth.gaussian_2d(1, 1.0))
    assert np.isnan(out[1:4, 1:4]).all()
    assert not np.isnan(out[0, 0])
