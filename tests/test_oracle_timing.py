"""The CPU-baseline timing driver runs the oracle's own functions; its
parallel form (bands of output rows with their halo rows, or one image per
task for batches) must give the oracle's results bit for bit."""
import numpy as np
import pytest

import oracle
import synth


@pytest.mark.parametrize("threads", [1, 3, 8])
@pytest.mark.parametrize("r", [0, 1, 2, 4])
def test_banded_image_equals_oracle(threads, r):
    rng = np.random.default_rng(50 + r)
    for h, w in [(1, 5), (7, 3), (37, 61), (100, 9)]:
        img = rng.random((h, w), dtype=np.float32)
        f2 = rng.standard_normal((2 * r + 1, 2 * r + 1)).astype(np.float32)
        out = np.full_like(img, np.nan)
        oracle.time_image("2d", img, f2, out, threads, reps=1)
        assert np.array_equal(out, oracle.filter2d_f32(img, f2))
        fx = rng.standard_normal(2 * r + 1).astype(np.float32)
        fy = rng.standard_normal(2 * r + 1).astype(np.float32)
        out[:] = np.nan
        oracle.time_image("sep", img, np.concatenate([fx, fy]), out, threads, reps=1)
        assert np.array_equal(out, oracle.filter_sep_f32(img, fx, fy))
        u = rng.integers(0, 256, (3, h, w), dtype=np.uint8)
        fu = rng.integers(-8, 9, (2 * r + 1, 2 * r + 1)).astype(np.int8)
        ou = np.zeros_like(u)
        oracle.time_image("u8", u, fu, ou, threads, reps=1, shift=6)
        assert np.array_equal(ou, oracle.filter2d_u8(u, fu, 6))


def test_batch_timing_equals_oracle():
    b = synth.batch_f32(12, 9, lo=8, hi=90)
    off = np.zeros(b.n, np.int64)
    foff = np.zeros(b.n, np.int64)
    o = fo = 0
    for i in range(b.n):
        off[i], foff[i] = o, fo
        o += int(b.h[i]) * int(b.w[i])
        fo += 2 * (2 * int(b.r[i]) + 1)
    pix = np.concatenate([im.ravel() for im in b.images]).astype(np.float32)
    flt = np.concatenate([np.concatenate([b.fx[i], b.fx[i]]) for i in range(b.n)]).astype(np.float32)
    out = np.full_like(pix, np.nan)
    oracle.time_batch_sep(b.h, b.w, b.r, off, pix, flt, foff, out, threads=4, reps=1)
    for i in range(b.n):
        n = int(b.h[i]) * int(b.w[i])
        ref = oracle.filter_sep_f32(b.images[i], b.fx[i], b.fx[i])
        assert np.array_equal(out[off[i]:off[i] + n].reshape(ref.shape), ref)
