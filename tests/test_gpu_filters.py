"""Parity of the HIP single-image filters with the oracle (GPU).

FP32: every element within 1e-5 * sum(|w| |x|) of the oracle (see
gpu_util), and bit-identical to the oracle with the exact flag. uint8:
bit-exact. Shapes span several wave strips (248 columns for r <= 4, 240
above) and several row tiles, with ragged tails, plus the degenerate
shapes (1x1, one row, one column, images smaller than the window).
"""
import numpy as np
import pytest

import oracle
import paper_1302_5586_amd as pf
import synth
from gpu_util import assert_close, device, tolerance_2d, tolerance_sep

pytestmark = pytest.mark.gpu

SHAPES = [(1, 1), (1, 700), (700, 1), (3, 5), (37, 301), (129, 250), (64, 496), (257, 513)]


def _t(a, dev):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def _rand_filter(rng, r):
    return rng.standard_normal((2 * r + 1, 2 * r + 1)).astype(np.float32)


@pytest.mark.parametrize("r", range(0, 9))
def test_2d_all_radii(r):
    dev = device()
    rng = np.random.default_rng(1000 + r)
    f = _rand_filter(rng, r)
    fd = _t(f, dev)
    for h, w in SHAPES:
        img = rng.random((h, w), dtype=np.float32)
        ref = oracle.filter2d_f32(img, f)
        got = pf.filter2d(_t(img, dev), fd).cpu().numpy()
        assert_close(got, ref, tolerance_2d(img, f, r), "2d r=%d %dx%d" % (r, h, w))
        exact = pf.filter2d(_t(img, dev), fd, exact=True).cpu().numpy()
        assert np.array_equal(exact, ref), "exact 2d r=%d %dx%d differs from the oracle" % (r, h, w)


@pytest.mark.parametrize("r", range(0, 9))
def test_separable_all_radii(r):
    dev = device()
    rng = np.random.default_rng(2000 + r)
    fx = rng.standard_normal(2 * r + 1).astype(np.float32)
    fy = rng.standard_normal(2 * r + 1).astype(np.float32)
    for h, w in SHAPES:
        img = rng.random((h, w), dtype=np.float32)
        ref = oracle.filter_sep_f32(img, fx, fy)
        got = pf.filter_sep(_t(img, dev), _t(fx, dev), _t(fy, dev)).cpu().numpy()
        assert_close(got, ref, tolerance_sep(img, fx, fy), "sep r=%d %dx%d" % (r, h, w))
        exact = pf.filter_sep(_t(img, dev), _t(fx, dev), _t(fy, dev), exact=True).cpu().numpy()
        assert np.array_equal(exact, ref), "exact sep r=%d %dx%d differs from the oracle" % (r, h, w)


@pytest.mark.parametrize("r", [0, 1, 2, 4, 5])
def test_separable_as_direct(r):
    dev = device()
    rng = np.random.default_rng(3000 + r)
    fx = rng.random(2 * r + 1).astype(np.float32)
    fy = rng.random(2 * r + 1).astype(np.float32)
    both = _t(np.concatenate([fx, fy]), dev)
    for h, w in SHAPES:
        img = rng.random((h, w), dtype=np.float32)
        ref = oracle.filter_sep_f32(img, fx, fy)
        got = pf.filter_shaped(_t(img, dev), both, r, pf.KIND_SEP, pf.VAR_SEP_DIRECT, 16, 4).cpu().numpy()
        assert_close(got, ref, tolerance_sep(img, fx, fy), "sep-as-2d r=%d %dx%d" % (r, h, w))


@pytest.mark.parametrize("kind,var", [(0, 0), (1, 1), (1, 2)])
def test_launch_shape_does_not_change_results(kind, var):
    dev = device()
    rng = np.random.default_rng(44)
    r = 2
    img = rng.random((300, 777), dtype=np.float32)
    filt = rng.standard_normal(25 if kind == 0 else 10).astype(np.float32)
    x, fd = _t(img, dev), _t(filt, dev)
    outs = [pf.filter_shaped(x, fd, r, kind, var, by, wpg).cpu().numpy()
            for by in (4, 8, 12, 16, 20, 32, 64, 128) for wpg in (1, 2, 4, 8)]
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])


def test_config_small_2d():
    dev = device()
    cfg = synth.config_small()
    ref = oracle.filter2d_f32(cfg.image, cfg.f2d)
    got = pf.filter2d(_t(cfg.image, dev), _t(cfg.f2d, dev)).cpu().numpy()
    err, rel = assert_close(got, ref, tolerance_2d(cfg.image, cfg.f2d, 1), "256x256 r=1")
    print("256x256 r=1: max abs %.3g max rel %.3g" % (err, rel))


def test_config_large_full():
    """4096x4096, 5x5 Gaussian, as full 2D and as fused separable passes:
    every output element against the oracle."""
    dev = device()
    cfg = synth.config_large()
    x = _t(cfg.image, dev)
    ref2 = oracle.filter2d_f32(cfg.image, cfg.f2d)
    got2 = pf.filter2d(x, _t(cfg.f2d, dev)).cpu().numpy()
    err, rel = assert_close(got2, ref2, tolerance_2d(cfg.image, cfg.f2d, 2), "4096^2 2d")
    print("4096^2 2d: max abs %.3g max rel %.3g" % (err, rel))
    refs = oracle.filter_sep_f32(cfg.image, cfg.f1d, cfg.f1d)
    g = _t(cfg.f1d, dev)
    gots = pf.filter_sep(x, g, g).cpu().numpy()
    err, rel = assert_close(gots, refs, tolerance_sep(cfg.image, cfg.f1d, cfg.f1d), "4096^2 sep")
    print("4096^2 sep: max abs %.3g max rel %.3g" % (err, rel))
    # the two forms of the same Gaussian agree within both bounds
    assert_close(gots, ref2, 2 * tolerance_2d(cfg.image, cfg.f2d, 2), "4096^2 sep vs 2d")
    # exact mode: both forms bit for bit equal to the sequential definition
    ex2 = pf.filter2d(x, _t(cfg.f2d, dev), exact=True).cpu().numpy()
    assert np.array_equal(ex2, ref2), "4096^2 exact 2d: %d pixels differ" % int((ex2 != ref2).sum())
    exs = pf.filter_sep(x, g, g, exact=True).cpu().numpy()
    assert np.array_equal(exs, refs), "4096^2 exact sep: %d pixels differ" % int((exs != refs).sum())


@pytest.mark.parametrize("r", range(0, 9))
def test_u8_all_radii(r):
    dev = device()
    rng = np.random.default_rng(4000 + r)
    for (c, h, w) in [(1, 1, 1), (3, 1, 9), (2, 9, 1), (3, 37, 301), (2, 70, 250), (1, 33, 257), (3, 20, 1920)]:
        for shift in (0, 6, 9):
            img = rng.integers(0, 256, (c, h, w), dtype=np.uint8)
            f = rng.integers(-8, 9, (2 * r + 1, 2 * r + 1)).astype(np.int8)
            ref = oracle.filter2d_u8(img, f, shift)
            got = pf.filter2d_u8(_t(img, dev), _t(f, dev), shift).cpu().numpy()
            assert np.array_equal(got, ref), "u8 r=%d c=%d %dx%d shift=%d" % (r, c, h, w, shift)


def _u8_entries(r, var, by, wpg):
    return [pf.TuneEntry(kind=pf.KIND_U8, r=r, size_class=sc, variant=var, rows_per_wave=by, waves_per_group=wpg,
                         us=0.0, context=pf.TUNE_SINGLE) for sc in range(3)]


@pytest.mark.parametrize("r", [4, 8])
@pytest.mark.parametrize("var", [pf.VAR_DIRECT, pf.VAR_MFMA])
def test_u8_extreme_weights(var, r):
    """All-(-128) and all-127 weights (the largest sums of either sign) at
    9x9 and 17x17, on v_dot4 and on the matrix cores."""
    dev = device()
    rng = np.random.default_rng(77)
    try:
        pf.tune_set(_u8_entries(r, var, 16, 4 if var == pf.VAR_MFMA else 1))
        for wv in (-128, 127):
            img = rng.integers(0, 256, (1, 40, 300), dtype=np.uint8)
            f = np.full((2 * r + 1, 2 * r + 1), wv, np.int8)
            for shift in (0, 13, 31):
                ref = oracle.filter2d_u8(img, f, shift)
                got = pf.filter2d_u8(_t(img, dev), _t(f, dev), shift).cpu().numpy()
                assert np.array_equal(got, ref)
    finally:
        pf.tune_reset()


def test_config_rgb_full():
    """1920x1080 planar RGB, 7x7 int8 weights, shift 6: bit-exact, every pixel."""
    dev = device()
    cfg = synth.config_rgb()
    ref = oracle.filter2d_u8(cfg.image, cfg.filt, cfg.shift)
    got = pf.filter2d_u8(_t(cfg.image, dev), _t(cfg.filt, dev), cfg.shift).cpu().numpy()
    assert np.array_equal(got, ref)


def test_determinism_and_nan():
    dev = device()
    rng = np.random.default_rng(5)
    img = rng.random((123, 456), dtype=np.float32)
    img[60, 200] = np.nan
    f = _rand_filter(rng, 2)
    x, fd = _t(img, dev), _t(f, dev)
    a = pf.filter2d(x, fd).cpu().numpy()
    b = pf.filter2d(x, fd).cpu().numpy()
    assert np.array_equal(a, b, equal_nan=True)
    assert np.isnan(a[58:63, 198:203]).all()
    assert not np.isnan(a[0, 0])


def test_calls_on_a_side_stream():
    """The single-image calls run on the stream they are given: inputs copied
    from pinned host memory and scaled on a side stream, then filtered on it
    with nothing synchronising the default stream, match the oracle (FP32 2D
    and separable, uint8 on the matrix cores)."""
    dev = device()
    import torch
    rng = np.random.default_rng(4500)
    img = rng.random((300, 500), dtype=np.float32)
    f = _rand_filter(rng, 2)
    fx = rng.random(5).astype(np.float32)
    fy = rng.random(5).astype(np.float32)
    u = rng.integers(0, 128, (3, 200, 300), dtype=np.uint8)
    f8 = rng.integers(-8, 9, (7, 7)).astype(np.int8)
    hx = torch.from_numpy(img).pin_memory()
    hu = torch.from_numpy(u).pin_memory()
    side = torch.cuda.Stream()
    torch.cuda.synchronize()
    with torch.cuda.stream(side):
        x = hx.to(dev, non_blocking=True) * 2.0
        xu = hu.to(dev, non_blocking=True) * 2
        fd, fxd, fyd, f8d = (torch.from_numpy(a).to(dev, non_blocking=False) for a in (f, fx, fy, f8))
        o2 = pf.filter2d(x, fd, stream=side)
        osep = pf.filter_sep(x, fxd, fyd, stream=side)
        ou = pf.filter2d_u8(xu, f8d, 6, stream=side)
    side.synchronize()
    img2 = img * np.float32(2.0)
    assert_close(o2.cpu().numpy(), oracle.filter2d_f32(img2, f), tolerance_2d(img2, f, 2), "2d on a side stream")
    assert_close(osep.cpu().numpy(), oracle.filter_sep_f32(img2, fx, fy), tolerance_sep(img2, fx, fy),
                 "sep on a side stream")
    assert np.array_equal(ou.cpu().numpy(), oracle.filter2d_u8(u * 2, f8, 6))


def test_u8_graph_replays():
    """The uint8 call captured in a graph (as the benchmark times it) and
    replayed four times, with the input rewritten eagerly between replays:
    every replay's output is bit-exact against the oracle for the input it
    read."""
    dev = device()
    import torch
    rng = np.random.default_rng(4600)
    imgs = [rng.integers(0, 256, (3, 120, 400), dtype=np.uint8) for _ in range(4)]
    f8 = rng.integers(-8, 9, (7, 7)).astype(np.int8)
    x = _t(imgs[0], dev)
    fd = _t(f8, dev)
    out = torch.empty_like(x)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        pf.filter2d_u8(x, fd, 6, out=out)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        pf.filter2d_u8(x, fd, 6, out=out)
    for img in imgs:
        x.copy_(torch.from_numpy(img).to(dev))
        out.zero_()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), oracle.filter2d_u8(img, f8, 6))
    del g


def test_strided_views_rejected():
    dev = device()
    import torch
    x = torch.zeros(16, 16, device=dev)[:, ::2]
    with pytest.raises(ValueError):
        pf.filter2d(x, torch.zeros(3, 3, device=dev))
    y = torch.zeros(16, 16, device=dev)
    with pytest.raises(pf.PFAlias):
        pf.filter2d(y, torch.zeros(3, 3, device=dev), out=y)


@pytest.mark.parametrize("by,wpg", [(12, 1), (20, 2), (24, 4), (48, 1), (4, 8)])
def test_u8_tile_shapes_bit_exact(by, wpg):
    """The uint8 kernel under other tile heights and group sizes (set
    through the tune table): still bit-exact on the 1080p RGB config."""
    dev = device()
    cfg = synth.config_rgb()
    ref = oracle.filter2d_u8(cfg.image, cfg.filt, cfg.shift)
    e = pf.TuneEntry(kind=pf.KIND_U8, r=cfg.r, size_class=2, variant=pf.VAR_DIRECT, rows_per_wave=by,
                     waves_per_group=wpg, us=0.0, context=pf.TUNE_SINGLE)
    try:
        pf.tune_set([e])
        got = pf.filter2d_u8(_t(cfg.image, dev), _t(cfg.filt, dev), cfg.shift).cpu().numpy()
    finally:
        pf.tune_reset()
    assert np.array_equal(got, ref)


# Multi-plane and tall images under workgroups of 2, 4 and 8 waves: groups
# that straddle strip columns and planes, and (wpg 8) waves without a tile.
GROUP_IMAGES = [(3, 1080, 1920), (2, 2000, 1000), (1, 1400, 1000)]


@pytest.mark.parametrize("r", [1, 2, 3, 4])
def test_u8_group_shapes_bit_exact(r):
    dev = device()
    rng = np.random.default_rng(4100 + r)
    for (c, h, w) in GROUP_IMAGES:
        img = rng.integers(0, 256, (c, h, w), dtype=np.uint8)
        f = rng.integers(-8, 9, (2 * r + 1, 2 * r + 1)).astype(np.int8)
        ref = oracle.filter2d_u8(img, f, 6)
        x, fd = _t(img, dev), _t(f, dev)
        for by, wpg in ((16, 2), (16, 4), (12, 8), (24, 4)):
            es = [pf.TuneEntry(kind=pf.KIND_U8, r=r, size_class=sc, variant=pf.VAR_DIRECT, rows_per_wave=by,
                               waves_per_group=wpg, us=0.0, context=pf.TUNE_SINGLE) for sc in range(3)]
            try:
                pf.tune_set(es)
                got = pf.filter2d_u8(x, fd, 6).cpu().numpy()
            finally:
                pf.tune_reset()
            bad = int((got != ref).sum())
            assert bad == 0, "u8 r=%d %dx%dx%d by=%d wpg=%d: %d bytes differ" % (r, c, h, w, by, wpg, bad)


# The matrix-core uint8 kernel: one- to eight-wave workgroups, one to eight
# 16-row wave tiles per wave, up to the 256-row workgroup tile; images
# smaller than a tile, ragged in both directions, with rows that are not
# 4-byte aligned (w not a multiple of 4), with 4-byte aligned rows whose
# width is not a multiple of the 16-byte stores, and with interior tiles
# (staged without column clamps) beside edge tiles.
MFMA_SHAPES = [(16, 1), (16, 4), (32, 2), (48, 4), (32, 8), (128, 2)]
MFMA_IMAGES = [(1, 1, 1), (3, 1, 9), (2, 9, 1), (1, 3, 4), (2, 17, 4), (3, 37, 301), (2, 70, 250), (1, 65, 68),
               (1, 300, 5), (2, 40, 1000), (3, 1080, 1920)]


@pytest.mark.parametrize("r", range(1, pf.PF_U8_MFMA_R_MAX + 1))
def test_u8_mfma_shapes_bit_exact(r):
    dev = device()
    import torch
    rng = np.random.default_rng(4300 + r)
    try:
        for (c, h, w) in MFMA_IMAGES:
            img = rng.integers(0, 256, (c, h, w), dtype=np.uint8)
            f = rng.integers(-128, 128, (2 * r + 1, 2 * r + 1)).astype(np.int8)
            shift = int(rng.integers(0, 14))
            ref = oracle.filter2d_u8(img, f, shift)
            x, fd = _t(img, dev), _t(f, dev)
            for by, wpg in MFMA_SHAPES:
                pf.tune_set(_u8_entries(r, pf.VAR_MFMA, by, wpg))
                got = pf.filter2d_u8(x, fd, shift).cpu().numpy()
                bad = int((got != ref).sum())
                assert bad == 0, "mfma u8 r=%d %dx%dx%d shift=%d by=%d wpg=%d: %d bytes differ" % (
                    r, c, h, w, shift, by, wpg, bad)
            # input and output one and three bytes past 4-byte alignment
            buf = torch.empty(img.size + 1, dtype=torch.uint8, device=dev)
            xu = buf[1:].view(img.shape)
            xu.copy_(x)
            obuf = torch.empty(img.size + 3, dtype=torch.uint8, device=dev)
            ou = obuf[3:].view(img.shape)
            pf.tune_set(_u8_entries(r, pf.VAR_MFMA, 16, 4))
            got = pf.filter2d_u8(xu, fd, shift, out=ou).cpu().numpy()
            assert np.array_equal(got, ref), "mfma u8 unaligned r=%d %dx%dx%d" % (r, c, h, w)
    finally:
        pf.tune_reset()


def test_u8_planes_past_2gib():
    """Nine 16384 x 16384 planes (2.4 GB; the last planes start past 2^31
    bytes): sampled rows of the first, middle and last planes, edge rows
    included, against the oracle, on the matrix cores and on v_dot4. A
    row's reference is the oracle on its 2r+1 clamped input rows, whose
    middle row needs no clamping there and so equals the full image's."""
    dev = device()
    import torch
    c, h, w, r = 9, 16384, 16384, 3
    gen = torch.Generator(device=dev)
    gen.manual_seed(4400)
    x = torch.randint(0, 256, (c, h, w), dtype=torch.uint8, device=dev, generator=gen)
    rng = np.random.default_rng(4401)
    f = rng.integers(-8, 9, (2 * r + 1, 2 * r + 1)).astype(np.int8)
    fd = _t(f, dev)
    out = torch.empty_like(x)
    samples = [(p, y) for p in (0, 4, c - 1) for y in (0, 1, 2, h // 2, h - 2, h - 1)]
    samples += [(int(p), int(y)) for p, y in zip(rng.integers(0, c, 6), rng.integers(0, h, 6))]
    try:
        for var, by, wpg in ((pf.VAR_MFMA, 16, 4), (pf.VAR_DIRECT, 16, 1)):
            pf.tune_set(_u8_entries(r, var, by, wpg))
            out.zero_()
            pf.filter2d_u8(x, fd, 6, out=out)
            for p, y in samples:
                rows = [min(max(y + d, 0), h - 1) for d in range(-r, r + 1)]
                sub = x[p, rows, :].cpu().numpy()[None]
                ref = oracle.filter2d_u8(sub, f, 6)[0, r]
                got = out[p, y].cpu().numpy()
                assert np.array_equal(got, ref), "variant %d plane %d row %d: %d bytes differ" % (
                    var, p, y, int((got != ref).sum()))
    finally:
        pf.tune_reset()
    del x, out
    torch.cuda.empty_cache()


def test_class_autotune_keeps_results(tmp_path):
    """The class tuner changes only launch shapes and variants: after it (and
    after reloading the table it saved), single-image calls of every kind
    still match the oracle, FP32 within the bound and uint8 bit for bit, in
    all three size classes."""
    dev = device()
    path = str(tmp_path / "class.json")
    rng = np.random.default_rng(4242)
    try:
        pf.autotune(r_max=2, reps=2, path=path)
        pf.tune_reset()
        pf.tune_load(path)
        for r in (0, 1, 2):
            for h, w in ((37, 301), (129, 250), (300, 1100), (1100, 1300)):
                img = rng.random((h, w), dtype=np.float32)
                f = _rand_filter(rng, r)
                got = pf.filter2d(_t(img, dev), _t(f, dev)).cpu().numpy()
                assert_close(got, oracle.filter2d_f32(img, f), tolerance_2d(img, f, r),
                             "tuned 2d r=%d %dx%d" % (r, h, w))
                fx = rng.random(2 * r + 1).astype(np.float32)
                fy = rng.random(2 * r + 1).astype(np.float32)
                got = pf.filter_sep(_t(img, dev), _t(fx, dev), _t(fy, dev)).cpu().numpy()
                assert_close(got, oracle.filter_sep_f32(img, fx, fy), tolerance_sep(img, fx, fy),
                             "tuned sep r=%d %dx%d" % (r, h, w))
            for c, h, w in ((3, 40, 300), (1, 700, 500), (3, 600, 800)):
                img = rng.integers(0, 256, (c, h, w), dtype=np.uint8)
                f8 = rng.integers(-8, 9, (2 * r + 1, 2 * r + 1)).astype(np.int8)
                got = pf.filter2d_u8(_t(img, dev), _t(f8, dev), 6).cpu().numpy()
                assert np.array_equal(got, oracle.filter2d_u8(img, f8, 6)), "tuned u8 r=%d %dx%dx%d" % (r, c, h, w)
    finally:
        pf.tune_reset()
