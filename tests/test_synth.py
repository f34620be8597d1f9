"""Seeded input generators: same seed, same bytes; statistics of the
workloads they stand for."""
import numpy as np

import synth


def test_gaussian_weights():
    np.testing.assert_array_equal(synth.gaussian_1d(1, 1.0), np.array([0.27406862, 0.45186275, 0.27406862], np.float32))
    # 8-digit decimals: equal to within one float32 ulp
    np.testing.assert_allclose(synth.gaussian_1d(2, 1.5),
                               np.array([0.12007838, 0.23388076, 0.2920817, 0.23388076, 0.12007838], np.float32),
                               rtol=1.2e-7, atol=0)
    g2 = synth.gaussian_2d(1, 1.0)
    assert g2.dtype == np.float32 and g2.shape == (3, 3)
    assert np.float32(g2.sum(dtype=np.float32)) == np.float32(0.99999994)


def test_determinism():
    a = synth.single_f32(33, 44, 2, 1.5, 9)
    b = synth.single_f32(33, 44, 2, 1.5, 9)
    np.testing.assert_array_equal(a.image, b.image)
    u = synth.rgb_u8(c=3, h=10, w=12)
    v = synth.rgb_u8(c=3, h=10, w=12)
    np.testing.assert_array_equal(u.image, v.image)
    np.testing.assert_array_equal(u.filt, v.filt)
    assert u.filt.min() >= -8 and u.filt.max() <= 8


def test_batch_statistics_seed3():
    b = synth.config_batch(with_pixels=False)
    assert b.n == 512
    assert b.pixels == 155_777_366
    assert np.bincount(b.r, minlength=5).tolist() == [0, 134, 113, 124, 141]
    px = b.h * b.w
    assert px.min() == 4352 and px.max() == 2_859_101
    assert b.w.min() >= 64 and b.w.max() <= 2048 and b.h.min() >= 64 and b.h.max() <= 2048
    assert ((b.sigma >= 0.5) & (b.sigma < 2.0)).all()


def test_arrival_trace():
    t = synth.arrival_trace()
    assert t.n == 120_237
    assert np.all(np.diff(t.t) > 0) and t.t[-1] < 60.0
    assert abs(np.diff(t.t).mean() - 1 / 2000) < 1e-5
    assert t.pool_index.min() >= 0 and t.pool_index.max() < 1024
