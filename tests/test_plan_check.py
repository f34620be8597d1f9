"""Batch tile tables on the CPU: pf_batch_plan_check builds the tables a
batch plan would upload and replays, with the FP32 strip kernel's own
geometry functions, where each wave tile of the persistent kernel reads
and writes. Every tile must stay inside its image's span of the arena, for
the 512-image benchmark batch under the committed MI355X tune table and
under every legal tile height, and for mixed batches of every radius,
kind and ragged shape. No device is touched."""
import os

import numpy as np
import pytest

import paper_1302_5586_amd as pf
import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TABLE = os.path.join(ROOT, "paper_1302_5586_amd", "tune_mi355x.json")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(pf.LIB_PATH):
        from paper_1302_5586_amd import build as b
        b.build()
    return pf.load()


def _layout(h, w, r, kinds):
    """Offsets the way pack_batch lays images out (64-element alignment)."""
    n = len(h)
    po = np.zeros(n, np.int64)
    off = 0
    for i in range(n):
        po[i] = off
        off = (off + int(h[i]) * int(w[i]) + 63) // 64 * 64
    k = 2 * np.asarray(r, np.int64) + 1
    nf = np.where(np.asarray(kinds) == pf.KIND_2D, k * k, 2 * k)
    fo = np.concatenate([[0], np.cumsum(nf)[:-1]]).astype(np.int64)
    return po, fo, max(off, 1), int(nf.sum())


def _batch_entries(by):
    return [pf.TuneEntry(kind=k, r=r, size_class=sc, variant=(pf.VAR_SEPARABLE if k == pf.KIND_SEP else pf.VAR_DIRECT),
                         rows_per_wave=by, waves_per_group=4, us=0.0, context=pf.TUNE_BATCH)
            for k in (pf.KIND_2D, pf.KIND_SEP) for r in range(pf.PF_R_MAX + 1) for sc in range(3)]


def test_batch512_tiles_inside_images(lib):
    b = synth.config_batch(with_pixels=False)
    kinds = np.full(b.n, pf.KIND_SEP, np.int32)
    po, fo, npix, nfilt = _layout(b.h, b.w, b.r, kinds)
    try:
        pf.tune_load(TABLE)
        got = pf.batch_plan_check(b.h, b.w, b.r, kinds, po, fo, npix, nfilt)
        assert got["violations"] == 0 and got["tiles"] > 10000
        for by in (4, 8, 16, 32, 64, 128):
            pf.tune_set(_batch_entries(by))
            got = pf.batch_plan_check(b.h, b.w, b.r, kinds, po, fo, npix, nfilt)
            assert got["violations"] == 0, by
    finally:
        pf.tune_reset()


def _ragged_widths():
    # around every strip width (256 for r <= 2, 248 for r 3..4, 240 above),
    # the 4-column vector width and its multiples
    out = {1, 2, 3, 4, 5, 7, 8, 9}
    for sw in (240, 248, 256):
        for m in (1, 2, 3):
            for d in (-5, -4, -3, -2, -1, 0, 1, 2, 3, 4, 5):
                out.add(m * sw + d)
    return sorted(v for v in out if v >= 1)


@pytest.mark.parametrize("r", range(0, pf.PF_BATCH_R_MAX + 1))
def test_mixed_shapes_every_radius(lib, r):
    widths = _ragged_widths()
    heights = [1, 2, 3, 5, 17, 33, 64, 65, 129]
    h, w = np.meshgrid(heights, widths, indexing="ij")
    h, w = h.ravel().astype(np.int32), w.ravel().astype(np.int32)
    n = h.size
    rr = np.full(n, r, np.int32)
    kinds = (np.arange(n) % 2).astype(np.int32)
    po, fo, npix, nfilt = _layout(h, w, rr, kinds)
    try:
        for by in (4, 8, 16, 32, 64, 128):
            pf.tune_set(_batch_entries(by))
            got = pf.batch_plan_check(h, w, rr, kinds, po, fo, npix, nfilt)
            assert got["violations"] == 0 and got["tiles"] >= n
    finally:
        pf.tune_reset()


def test_random_mixed_batch(lib):
    rng = np.random.default_rng(8)
    n = 400
    h = rng.integers(1, 700, n).astype(np.int32)
    w = rng.integers(1, 1100, n).astype(np.int32)
    rr = rng.integers(0, pf.PF_BATCH_R_MAX + 1, n).astype(np.int32)
    kinds = rng.integers(0, 2, n).astype(np.int32)
    po, fo, npix, nfilt = _layout(h, w, rr, kinds)
    got = pf.batch_plan_check(h, w, rr, kinds, po, fo, npix, nfilt, no_tune=True)
    assert got["violations"] == 0
    # the same validation as plan creation
    end = int(po[-1]) + int(h[-1]) * int(w[-1])
    with pytest.raises(pf.PFInvalid):
        pf.batch_plan_check(h, w, rr, kinds, po, fo, end - 1, nfilt)
    bad = po.copy()
    bad[1] = bad[0]
    with pytest.raises(pf.PFAlias):
        pf.batch_plan_check(h, w, rr, kinds, bad, fo, npix, nfilt)


def test_batch_radius_limit(lib):
    """Batches take radii 0..PF_BATCH_R_MAX; larger radii are refused
    before anything is built (they run as single-image calls)."""
    h = np.array([9, 9], np.int32)
    w = np.array([9, 9], np.int32)
    kinds = np.array([pf.KIND_2D, pf.KIND_SEP], np.int32)
    for r in (pf.PF_BATCH_R_MAX + 1, pf.PF_R_MAX):
        rr = np.array([1, r], np.int32)
        po, fo, npix, nfilt = _layout(h, w, rr, kinds)
        with pytest.raises(pf.PFUnsupported):
            pf.batch_plan_check(h, w, rr, kinds, po, fo, npix, nfilt)
