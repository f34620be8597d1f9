"""The C ABI on the CPU: the library loads, exports every function that
include/pf.h declares, and rejects invalid arguments before touching the
device (host-side validation only; no compute call runs here)."""
import ctypes
import glob
import json
import os
import re

import pytest

import paper_1302_5586_amd as pf

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = sorted(glob.glob(os.path.join(ROOT, "include", "*.h")))


def declared_functions():
    names = set()
    for h in HEADERS:
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names |= set(re.findall(r"\b(pf_[a-z0-9_]+)\s*\(", text))
    return sorted(names)


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(pf.LIB_PATH):
        from paper_1302_5586_amd import build as b
        b.build()
    return pf.load()


def test_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert len(names) >= 20
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    # and the binding knows a signature for each of them
    assert set(names) <= set(pf._SIGS), set(names) - set(pf._SIGS)


def test_status_strings(lib):
    assert lib.pf_status_str(pf.PF_OK) == b"PF_OK"
    assert lib.pf_status_str(pf.PF_EALIAS) == b"PF_EALIAS"
    assert lib.pf_status_str(99) == b"PF_UNKNOWN"
    assert b"gfx950" in lib.pf_version()


FAKE = 1 << 40  # a 4-byte aligned address that validation never dereferences


@pytest.mark.parametrize("h,w,r,inp,out,status", [
    (0, 5, 1, FAKE, FAKE + (1 << 20), pf.PF_EINVAL),          # empty image
    (5, -1, 1, FAKE, FAKE + (1 << 20), pf.PF_EINVAL),         # negative width
    (5, 5, 9, FAKE, FAKE + (1 << 20), pf.PF_EINVAL),          # radius above PF_R_MAX
    (5, 5, -1, FAKE, FAKE + (1 << 20), pf.PF_EINVAL),         # negative radius
    (5, 5, 1, 0, FAKE, pf.PF_EINVAL),                         # null input
    (5, 5, 1, FAKE + 2, FAKE + (1 << 20), pf.PF_EINVAL),      # misaligned
    (5, 5, 1, FAKE, FAKE, pf.PF_EALIAS),                      # in place
    (5, 5, 1, FAKE, FAKE + 4 * 24, pf.PF_EALIAS),             # partial overlap
])
def test_filter2d_validation(lib, h, w, r, inp, out, status):
    got = lib.pf_filter2d_f32(h, w, r, inp, FAKE + (1 << 30), out, 0, None)
    assert got == status
    assert lib.pf_last_error() != b""


def test_filter_flags_and_filter_alias(lib):
    assert lib.pf_filter2d_f32(4, 4, 1, FAKE, FAKE + 4096, FAKE + (1 << 20), 0x80, None) == pf.PF_EINVAL
    # filter overlapping the output
    assert lib.pf_filter2d_f32(4, 4, 1, FAKE, FAKE + (1 << 20) + 8, FAKE + (1 << 20), 0, None) == pf.PF_EALIAS
    assert lib.pf_filter_sep_f32(4, 4, 1, FAKE, 0, FAKE + 64, FAKE + (1 << 20), 0, None) == pf.PF_EINVAL
    assert lib.pf_filter_f32_shaped(4, 4, 1, pf.KIND_2D, pf.VAR_SEPARABLE, 16, 4, FAKE, FAKE + 4096,
                                    FAKE + (1 << 20), 0, None) == pf.PF_EINVAL
    assert lib.pf_filter_f32_shaped(4, 4, 1, pf.KIND_2D, pf.VAR_DIRECT, 10, 4, FAKE, FAKE + 4096,
                                    FAKE + (1 << 20), 0, None) == pf.PF_EINVAL
    assert lib.pf_filter_f32_shaped(4, 4, 1, pf.KIND_2D, pf.VAR_DIRECT, 132, 4, FAKE, FAKE + 4096,
                                    FAKE + (1 << 20), 0, None) == pf.PF_EINVAL
    # separable filters run as 2D taps up to radius 5 only
    assert lib.pf_filter_f32_shaped(40, 40, 6, pf.KIND_SEP, pf.VAR_SEP_DIRECT, 16, 4, FAKE, FAKE + 65536,
                                    FAKE + (1 << 20), 0, None) == pf.PF_EUNSUPPORTED


def test_u8_validation(lib):
    ok = dict(c=3, h=4, w=4, r=1, shift=6)
    def call(**kw):
        a = dict(ok, **kw)
        return lib.pf_filter2d_u8(a["c"], a["h"], a["w"], a["r"], a["shift"], a.get("inp", FAKE),
                                  FAKE + 4096, a.get("out", FAKE + (1 << 20)), a.get("flags", 0), None)
    assert call(c=0) == pf.PF_EINVAL
    assert call(shift=32) == pf.PF_EINVAL
    assert call(shift=-1) == pf.PF_EINVAL
    assert call(flags=1) == pf.PF_EINVAL
    assert call(out=FAKE + 10) == pf.PF_EALIAS
    assert call(inp=0) == pf.PF_EINVAL


def test_tune_table_roundtrip(lib, tmp_path):
    pf.tune_reset()
    e = pf.tune_lookup(pf.KIND_SEP, 2, 4096 * 4096)
    assert e.variant == pf.VAR_SEPARABLE and e.size_class == 2 and e.context == pf.TUNE_SINGLE
    new = pf.TuneEntry(kind=pf.KIND_2D, r=1, size_class=0, variant=pf.VAR_DIRECT, rows_per_wave=64,
                       waves_per_group=2, us=1.5, context=pf.TUNE_SINGLE)
    newb = pf.TuneEntry(kind=pf.KIND_SEP, r=3, size_class=1, variant=pf.VAR_SEPARABLE, rows_per_wave=8,
                        waves_per_group=4, us=2.5, context=pf.TUNE_BATCH)
    sepd = pf.TuneEntry(kind=pf.KIND_SEP, r=1, size_class=2, variant=pf.VAR_SEP_DIRECT, rows_per_wave=32,
                        waves_per_group=4, us=3.0, context=pf.TUNE_SINGLE)
    pf.tune_set([new, newb, sepd])
    assert pf.tune_lookup(pf.KIND_2D, 1, 100).rows_per_wave == 64
    # the two contexts are separate keys
    assert pf.tune_lookup(pf.KIND_2D, 1, 100, pf.TUNE_BATCH).rows_per_wave == 16
    assert pf.tune_lookup(pf.KIND_SEP, 3, 600 * 700, pf.TUNE_BATCH).rows_per_wave == 8
    assert pf.tune_lookup(pf.KIND_SEP, 3, 600 * 700).rows_per_wave == 32
    path = str(tmp_path / "tune.json")
    pf.tune_save(path)
    doc = json.load(open(path))
    # single-image entries for 3 kinds, batch entries for the 2 FP32 kinds
    assert len(doc["entries"]) == 3 * 9 * 3 + 2 * 9 * 3
    pf.tune_reset()
    assert pf.tune_lookup(pf.KIND_2D, 1, 100).rows_per_wave != 64
    pf.tune_load(path)
    got = pf.tune_lookup(pf.KIND_2D, 1, 100)
    assert (got.rows_per_wave, got.waves_per_group) == (64, 2)
    assert pf.tune_lookup(pf.KIND_SEP, 3, 600 * 700, pf.TUNE_BATCH).rows_per_wave == 8
    assert pf.tune_lookup(pf.KIND_SEP, 1, 4096 * 4096).variant == pf.VAR_SEP_DIRECT
    # a file written before contexts existed loads as single-image entries
    for d in doc["entries"]:
        d.pop("context")
    old = str(tmp_path / "old.json")
    json.dump({"entries": [d for d in doc["entries"][:3 * 9 * 3]]}, open(old, "w"))
    pf.tune_load(old)
    assert pf.tune_lookup(pf.KIND_2D, 1, 100).rows_per_wave == 64
    with pytest.raises(pf.PFInvalid):   # batches never run separable filters as 2D taps
        pf.tune_set([pf.TuneEntry(kind=pf.KIND_SEP, r=3, size_class=0, variant=pf.VAR_SEP_DIRECT,
                                  rows_per_wave=16, waves_per_group=4, context=pf.TUNE_BATCH)])
    with pytest.raises(pf.PFInvalid):   # 2D taps of a separable filter: radii 0..5
        pf.tune_set([pf.TuneEntry(kind=pf.KIND_SEP, r=6, size_class=0, variant=pf.VAR_SEP_DIRECT,
                                  rows_per_wave=16, waves_per_group=4, context=pf.TUNE_SINGLE)])
    with pytest.raises(pf.PFInvalid):   # batch kernels run four waves per workgroup
        pf.tune_set([pf.TuneEntry(kind=pf.KIND_SEP, r=3, size_class=0, variant=pf.VAR_SEPARABLE,
                                  rows_per_wave=16, waves_per_group=2, context=pf.TUNE_BATCH)])
    with pytest.raises(pf.PFInvalid):
        pf.tune_set([pf.TuneEntry(kind=pf.KIND_U8, r=3, size_class=0, variant=pf.VAR_DIRECT,
                                  rows_per_wave=16, waves_per_group=4, context=pf.TUNE_BATCH)])
    with pytest.raises(pf.PFInvalid):
        pf.tune_set([pf.TuneEntry(kind=pf.KIND_2D, r=1, size_class=0, variant=pf.VAR_DIRECT,
                                  rows_per_wave=14, waves_per_group=4)])
    with pytest.raises(pf.PFInvalid):
        pf.tune_lookup(pf.KIND_U8, 1, 100, pf.TUNE_BATCH)
    pf.tune_reset()


def test_u8_variant_entries(lib):
    """uint8 runs on v_dot4 at every radius, on the matrix cores at radii
    1..8 (the default there) with wave tiles of 16k rows and workgroup tiles
    of at most 256 rows; other variants and shapes are refused."""
    pf.tune_reset()
    for r in range(pf.PF_R_MAX + 1):
        e = pf.tune_lookup(pf.KIND_U8, r, 1080 * 1920 * 3)
        want = pf.VAR_MFMA if 1 <= r <= pf.PF_U8_MFMA_R_MAX else pf.VAR_DIRECT
        assert e.variant == want, (r, e.variant)
        if want == pf.VAR_MFMA:
            assert e.rows_per_wave % 16 == 0 and e.rows_per_wave * e.waves_per_group <= pf.PF_U8_MFMA_TILE_MAX

    def u8(r, var, by, wpg):
        return pf.TuneEntry(kind=pf.KIND_U8, r=r, size_class=2, variant=var, rows_per_wave=by, waves_per_group=wpg,
                            context=pf.TUNE_SINGLE)
    try:
        pf.tune_set([u8(3, pf.VAR_MFMA, 32, 8), u8(1, pf.VAR_MFMA, 128, 2), u8(4, pf.VAR_DIRECT, 12, 8)])
        assert pf.tune_lookup(pf.KIND_U8, 3, 1 << 22).rows_per_wave == 32
        pf.tune_set([u8(8, pf.VAR_MFMA, 16, 8)])
        for bad in (u8(0, pf.VAR_MFMA, 16, 4), u8(8, pf.VAR_MFMA, 40, 2), u8(3, pf.VAR_MFMA, 24, 1),
                    u8(3, pf.VAR_MFMA, 64, 8), u8(3, pf.VAR_MFMA, 128, 4), u8(3, pf.VAR_SEPARABLE, 16, 1),
                    u8(3, pf.VAR_SEP_DIRECT, 16, 1)):
            with pytest.raises(pf.PFInvalid):
                pf.tune_set([bad])
        with pytest.raises(pf.PFInvalid):   # the 2D FP32 kind has no matrix-core variant
            pf.tune_set([pf.TuneEntry(kind=pf.KIND_2D, r=1, size_class=0, variant=pf.VAR_MFMA, rows_per_wave=16,
                                      waves_per_group=4)])
    finally:
        pf.tune_reset()


def _arr(t, vals):
    a = (t * len(vals))(*vals)
    return ctypes.cast(a, ctypes.c_void_p), a


def test_batch_plan_validation(lib):
    P = ctypes.c_void_p()
    def create(h, w, r, kind, po, fo, npix, nfilt, flags=0):
        keep = []
        args = []
        for t, v in ((ctypes.c_int32, h), (ctypes.c_int32, w), (ctypes.c_int32, r), (ctypes.c_int32, kind),
                     (ctypes.c_int64, po), (ctypes.c_int64, fo)):
            p, a = _arr(t, v)
            keep.append(a)
            args.append(p)
        return lib.pf_batch_plan_create(len(h), *args, npix, nfilt, flags, ctypes.byref(P))
    assert create([4], [4], [1], [0], [1], [0], 16, 9) == pf.PF_EINVAL        # image past the arena
    assert create([4], [4], [1], [0], [0], [1], 16, 9) == pf.PF_EINVAL        # filter past the arena
    assert create([4], [4], [1], [5], [0], [0], 16, 9) == pf.PF_EINVAL        # unknown kind
    assert create([4, 4], [4, 4], [1, 1], [0, 0], [0, 8], [0, 0], 64, 9) == pf.PF_EALIAS   # overlapping images
    assert create([4], [4], [1], [0], [0], [0], 16, 9, flags=0x100) == pf.PF_EINVAL
    assert lib.pf_batch_plan_create(0, None, None, None, None, None, None, 1, 1, 0, ctypes.byref(P)) == pf.PF_EINVAL
    assert lib.pf_batch_plan_destroy(None) == pf.PF_OK


def test_server_validation(lib):
    S = ctypes.c_void_p()
    assert lib.pf_server_create(100, 2, 8, 16, 0, ctypes.byref(S)) == pf.PF_EINVAL     # budget too small
    assert lib.pf_server_create(1 << 20, 0, 8, 16, 0, ctypes.byref(S)) == pf.PF_EINVAL  # no streams
    assert lib.pf_server_create(1 << 20, 2, 0, 16, 0, ctypes.byref(S)) == pf.PF_EINVAL  # empty batches
    assert lib.pf_server_create(1 << 20, 2, 8, 0, 0, ctypes.byref(S)) == pf.PF_EINVAL   # no queue
    assert lib.pf_server_destroy(None) == pf.PF_OK


def test_binding_rejects_host_tensors():
    torch = pytest.importorskip("torch")
    x = torch.zeros(4, 4)
    with pytest.raises(ValueError):
        pf.filter2d(x, torch.zeros(3, 3))


def test_tune_batch_blocks_roundtrip(lib, tmp_path):
    pf.tune_reset()
    assert pf.tune_batch_blocks() == 1
    assert pf.tune_batch_blocks(3) == 1
    assert pf.tune_batch_blocks() == 3
    path = str(tmp_path / "tune.json")
    pf.tune_save(path)
    assert json.load(open(path))["batch_blocks_per_cu"] == 3
    pf.tune_reset()
    assert pf.tune_batch_blocks() == 1
    pf.tune_load(path)
    assert pf.tune_batch_blocks() == 3
    with pytest.raises(pf.PFInvalid):
        pf.tune_batch_blocks(9)
    doc = json.load(open(path))
    doc["batch_blocks_per_cu"] = 0
    bad = str(tmp_path / "bad.json")
    json.dump(doc, open(bad, "w"))
    with pytest.raises(pf.PFInvalid):
        pf.tune_load(bad)
    pf.tune_reset()
    assert pf.tune_batch_blocks() == 1


def test_chain_and_border_validation(lib):
    def chain(h=8, w=8, r=1, passes=2, border=pf.BORDER_CLAMP, inp=FAKE, filt=FAKE + 4096, out=FAKE + (1 << 20),
              flags=0):
        return lib.pf_filter_chain_f32(h, w, r, passes, border, inp, filt, out, flags, None)
    assert chain(passes=0) == pf.PF_EINVAL
    assert chain(border=4) == pf.PF_EINVAL
    assert chain(border=-1) == pf.PF_EINVAL
    assert chain(flags=0x2) == pf.PF_EINVAL
    assert chain(filt=0) == pf.PF_EINVAL
    assert chain(h=0) == pf.PF_EINVAL
    assert chain(r=9) == pf.PF_EINVAL
    assert chain(r=4, passes=5) == pf.PF_EUNSUPPORTED      # halo 20 > PF_CHAIN_HALO_MAX
    assert chain(r=1, passes=17) == pf.PF_EUNSUPPORTED
    assert chain(out=FAKE) == pf.PF_EALIAS
    assert chain(filt=FAKE + (1 << 20) + 4) == pf.PF_EALIAS
    assert lib.pf_filter2d_f32_border(8, 8, 1, 7, FAKE, FAKE + 4096, FAKE + (1 << 20), 0, None) == pf.PF_EINVAL
    assert lib.pf_filter2d_f32_border(8, 8, 9, pf.BORDER_ZERO, FAKE, FAKE + 4096, FAKE + (1 << 20), 0,
                                      None) == pf.PF_EINVAL
    assert lib.pf_filter2d_f32_border(8, 8, 1, pf.BORDER_REFLECT, FAKE, FAKE + 4096, FAKE, 0,
                                      None) == pf.PF_EALIAS


def test_reduce_validation(lib):
    import ctypes
    nb = ctypes.c_size_t(0)
    assert lib.pf_sum_workspace(0, ctypes.byref(nb)) == pf.PF_EINVAL
    assert lib.pf_sum_workspace(1 << 41, ctypes.byref(nb)) == pf.PF_EINVAL
    assert lib.pf_sum_workspace(65537, ctypes.byref(nb)) == pf.PF_OK and nb.value == 2 * 8
    assert lib.pf_hist_workspace(1, ctypes.byref(nb)) == pf.PF_OK and nb.value == 256 * 4
    assert lib.pf_hist_workspace(1 << 30, ctypes.byref(nb)) == pf.PF_OK and nb.value == 1024 * 256 * 4
    ws, out = FAKE + (1 << 30), FAKE + (1 << 31)
    assert lib.pf_sum_f32(100, FAKE + 2, out, ws, 8, None) == pf.PF_EINVAL       # misaligned x
    assert lib.pf_sum_f32(100, FAKE, out + 4, ws, 8, None) == pf.PF_EINVAL       # misaligned out
    assert lib.pf_sum_f32(100, FAKE, out, ws, 4, None) == pf.PF_EINVAL           # workspace too small
    assert lib.pf_sum_f32(100, FAKE, FAKE + 8, ws, 8, None) == pf.PF_EALIAS      # out inside x
    assert lib.pf_sum_f32(100, FAKE, out, 0, 8, None) == pf.PF_EINVAL
    assert lib.pf_hist256_u8(0, FAKE, out, ws, 1024, None) == pf.PF_EINVAL
    assert lib.pf_hist256_u8(100, FAKE, out + 4, ws, 1024, None) == pf.PF_EINVAL  # misaligned hist
    assert lib.pf_hist256_u8(100, FAKE, out, ws, 1000, None) == pf.PF_EINVAL      # workspace too small
    assert lib.pf_hist256_u8(100, FAKE, FAKE + 48, ws, 1024, None) == pf.PF_EALIAS


def test_inc_validation(lib):
    import ctypes
    import numpy as np
    h = ctypes.c_void_p()
    bad = np.array([0, 5], np.int32)
    assert lib.pf_inc_plan_create(5, 1, bad.ctypes.data_as(ctypes.c_void_p), ctypes.byref(h)) == pf.PF_EINVAL
    assert lib.pf_inc_plan_create(0, 0, None, ctypes.byref(h)) == pf.PF_EINVAL
    assert lib.pf_inc_plan_create(5, -1, None, ctypes.byref(h)) == pf.PF_EINVAL
    assert lib.pf_inc_plan_create(5, (1 << 30) + 1, bad.ctypes.data_as(ctypes.c_void_p),
                                  ctypes.byref(h)) == pf.PF_EUNSUPPORTED
    assert lib.pf_inc_plan_run(None, 5, 1, FAKE, FAKE + 4096, None) == pf.PF_EINVAL
    assert lib.pf_inc_plan_destroy(None) == pf.PF_OK
    assert lib.pf_edge_inc_atomic_f64(0, 1, FAKE, FAKE + 64, FAKE + 4096, None) == pf.PF_EINVAL
    assert lib.pf_edge_inc_atomic_f64(4, 1, FAKE + 2, FAKE + 64, FAKE + 4096, None) == pf.PF_EINVAL
    assert lib.pf_edge_inc_atomic_f64(4, 2, FAKE, FAKE + 64, FAKE + 8, None) == pf.PF_EALIAS
