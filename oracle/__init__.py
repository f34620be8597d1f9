"""Oracle for the clamp-to-edge 2D image filter (test infrastructure only).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg
may import this package. The product library never loads it, and the two
share no code: this package wraps the plain C99 loops in ``ref_filter.c``
(and the other ``ref_*.c`` files) through ctypes, on numpy arrays.

The C sources follow the paper's framing of a PENCIL function: sequential
semantics, buildable by an ordinary C compiler (Sec. II; Sec. II-A), sizes
first and then ``restrict const static`` VLA array parameters (Sec. II-B.1),
with independent output iterations (Sec. II-B.3).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SOURCES = ["ref_filter.c", "ref_next.c"]
_CFLAGS = ["-std=c99", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared", "-Wall"]

_lib = None


_TIME_LIB_PATH = os.path.join(_HERE, "liboracle_time.so")


def build(verbose: bool = False) -> str:
    """Compile the C oracle into ``oracle/liboracle.so`` with gcc, and its
    OpenMP timing driver (the oracle's sources plus ``time_oracle.c``) into
    ``oracle/liboracle_time.so``."""
    srcs = [os.path.join(_HERE, s) for s in _SOURCES if os.path.exists(os.path.join(_HERE, s))]
    for path, extra, flags in ((_LIB_PATH, [], []),
                               (_TIME_LIB_PATH, [os.path.join(_HERE, "time_oracle.c")], ["-fopenmp"])):
        tmp = path + ".tmp%d" % os.getpid()
        cmd = ["gcc", *_CFLAGS, *flags, "-o", tmp, *srcs, *extra, "-lm"]
        if verbose:
            print(" ".join(cmd))
        subprocess.run(cmd, check=True)
        os.replace(tmp, path)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build()
    lib = ctypes.CDLL(_LIB_PATH)
    P = ctypes.c_void_p
    I = ctypes.c_int
    lib.ref_filter2d_f32.argtypes = [I, I, I, P, P, P]
    lib.ref_filter2d_f32.restype = None
    lib.ref_filter2d_f32_at.argtypes = [I, I, I, P, P, I, I]
    lib.ref_filter2d_f32_at.restype = ctypes.c_float
    lib.ref_filter2d_f32_permuted.argtypes = [I, I, I, P, P, P, P]
    lib.ref_filter2d_f32_permuted.restype = None
    lib.ref_filter_sep_f32.argtypes = [I, I, I, P, P, P, P]
    lib.ref_filter_sep_f32.restype = I
    lib.ref_filter2d_u8.argtypes = [I, I, I, I, I, P, P, P]
    lib.ref_filter2d_u8.restype = None
    if hasattr(lib, "ref_filter2d_f32_border"):
        lib.ref_filter2d_f32_border.argtypes = [I, I, I, I, P, P, P]
        lib.ref_filter2d_f32_border.restype = I
        lib.ref_filter_chain_f32.argtypes = [I, I, I, I, I, P, P, P]
        lib.ref_filter_chain_f32.restype = I
        lib.ref_sum_f32.argtypes = [ctypes.c_int64, P]
        lib.ref_sum_f32.restype = ctypes.c_double
        lib.ref_hist256_u8.argtypes = [ctypes.c_int64, P, P]
        lib.ref_hist256_u8.restype = None
        lib.ref_edge_inc_f64.argtypes = [I, I, P, P, P]
        lib.ref_edge_inc_f64.restype = None
    _lib = lib
    return lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _f32(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float32)


def _check_r(r: int, f: np.ndarray, n: int):
    if r < 0 or f.size != n:
        raise ValueError("filter size %d does not match radius %d" % (f.size, r))


def filter2d_f32(img, f2d, r: int | None = None) -> np.ndarray:
    """out[y][x] = sum over dy, dx in -r..r of f[dy+r][dx+r] * img[clamp(y+dy)][clamp(x+dx)]."""
    img = _f32(img)
    f = _f32(f2d)
    if r is None:
        r = (f.shape[0] - 1) // 2
    _check_r(r, f, (2 * r + 1) ** 2)
    h, w = img.shape
    out = np.empty_like(img)
    _load().ref_filter2d_f32(h, w, r, _p(img), _p(f), _p(out))
    return out


def filter2d_f32_at(img, f2d, r: int, y: int, x: int) -> np.float32:
    """One output element of ``filter2d_f32`` (same arithmetic, same order)."""
    img = _f32(img)
    f = _f32(f2d)
    _check_r(r, f, (2 * r + 1) ** 2)
    h, w = img.shape
    return np.float32(_load().ref_filter2d_f32_at(h, w, r, _p(img), _p(f), int(y), int(x)))


def filter2d_f32_permuted(img, f2d, r: int, order) -> np.ndarray:
    """The 2D filter with output elements visited in ``order`` (linear indices)."""
    img = _f32(img)
    f = _f32(f2d)
    _check_r(r, f, (2 * r + 1) ** 2)
    h, w = img.shape
    order = np.ascontiguousarray(order, dtype=np.int64)
    if order.size != h * w:
        raise ValueError("order must list every output element")
    out = np.full_like(img, np.nan)
    _load().ref_filter2d_f32_permuted(h, w, r, _p(img), _p(f), _p(order), _p(out))
    return out


def filter_sep_f32(img, fx, fy) -> np.ndarray:
    """Row pass with fx into an FP32 temporary, then column pass with fy."""
    img = _f32(img)
    fx = _f32(fx)
    fy = _f32(fy)
    r = (fx.size - 1) // 2
    _check_r(r, fx, 2 * r + 1)
    _check_r(r, fy, 2 * r + 1)
    h, w = img.shape
    out = np.empty_like(img)
    rc = _load().ref_filter_sep_f32(h, w, r, _p(img), _p(fx), _p(fy), _p(out))
    if rc != 0:
        raise MemoryError("oracle could not allocate its temporary")
    return out


def filter2d_u8(img, f, shift: int) -> np.ndarray:
    """Planar uint8 [c][h][w] with int8 weights: int32 accumulate, floor
    shift, saturate to [0, 255]."""
    img = np.ascontiguousarray(img, dtype=np.uint8)
    if img.ndim == 2:
        img = img[None]
    f = np.ascontiguousarray(f, dtype=np.int8)
    r = (f.shape[0] - 1) // 2
    _check_r(r, f, (2 * r + 1) ** 2)
    c, h, w = img.shape
    out = np.empty_like(img)
    _load().ref_filter2d_u8(c, h, w, r, int(shift), _p(img), _p(f), _p(out))
    return out


# Border modes of the extended filter (zero padding and two reflections),
# numbered as the C oracle numbers them.
BORDER_CLAMP = 0
BORDER_ZERO = 1
BORDER_REFLECT = 2   # edge pixel repeated:  d c b a | a b c d | d c b a
BORDER_MIRROR = 3    # edge pixel not repeated:  d c b | a b c d | c b a


def filter2d_f32_border(img, f2d, border: int) -> np.ndarray:
    img = _f32(img)
    f = _f32(f2d)
    r = (f.shape[0] - 1) // 2
    _check_r(r, f, (2 * r + 1) ** 2)
    h, w = img.shape
    out = np.empty_like(img)
    rc = _load().ref_filter2d_f32_border(h, w, r, int(border), _p(img), _p(f), _p(out))
    if rc != 0:
        raise ValueError("bad border mode")
    return out


def filter_chain_f32(img, f2d, passes: int, border: int = BORDER_CLAMP) -> np.ndarray:
    """``passes`` applications of the 2D filter, each reading the previous
    pass's FP32 output."""
    img = _f32(img)
    f = _f32(f2d)
    r = (f.shape[0] - 1) // 2
    _check_r(r, f, (2 * r + 1) ** 2)
    h, w = img.shape
    out = np.empty_like(img)
    rc = _load().ref_filter_chain_f32(h, w, r, int(passes), int(border), _p(img), _p(f), _p(out))
    if rc != 0:
        raise ValueError("bad chain arguments")
    return out


def sum_f32(x) -> float:
    """Sum of FP32 values accumulated in float64, in index order."""
    x = _f32(x).ravel()
    return float(_load().ref_sum_f32(x.size, _p(x)))


def hist256_u8(x) -> np.ndarray:
    """256-bin histogram of uint8 values: hist[v] counts the elements equal to v."""
    x = np.ascontiguousarray(x, dtype=np.uint8).ravel()
    hist = np.zeros(256, dtype=np.int64)
    _load().ref_hist256_u8(x.size, _p(x), _p(hist))
    return hist


def edge_inc_f64(ncells: int, edge_to_cells, edge_data, cell_data) -> np.ndarray:
    """For each edge i in order: cell[e2c[2i+1]] += edge[i], then cell[e2c[2i]] += edge[i]."""
    e2c = np.ascontiguousarray(edge_to_cells, dtype=np.int32).ravel()
    ed = np.ascontiguousarray(edge_data, dtype=np.float64).ravel()
    cells = np.array(cell_data, dtype=np.float64, copy=True).ravel()
    if cells.size != ncells or e2c.size != 2 * ed.size:
        raise ValueError("mesh arrays do not match")
    _load().ref_edge_inc_f64(int(ncells), int(ed.size), _p(e2c), _p(ed), _p(cells))
    return cells


# ---------------------------------------------------------------- timing
# The CPU baseline of the benchmark: the oracle's own functions timed on
# one host thread or on several (OpenMP over bands of output rows, or one
# image per task for batches; see time_oracle.c). Results are written to
# `out` and equal the oracle's bit for bit.

_tlib = None


def _time_lib():
    global _tlib
    if _tlib is not None:
        return _tlib
    if not os.path.exists(_TIME_LIB_PATH):
        build()
    lib = ctypes.CDLL(_TIME_LIB_PATH)
    P, I = ctypes.c_void_p, ctypes.c_int
    lib.time_image.argtypes = [I, I, I, I, I, I, P, P, P, I, I]
    lib.time_image.restype = ctypes.c_double
    lib.time_batch_sep.argtypes = [I, P, P, P, P, P, P, P, P, I, I]
    lib.time_batch_sep.restype = ctypes.c_double
    _tlib = lib
    return lib


def time_image(kind: str, img, filt, out, threads: int, reps: int = 3, shift: int = 6) -> float:
    """Median seconds of the oracle on one image: kind "2d" (filt: 2D taps),
    "sep" (filt: fx then fy) or "u8" ([c, h, w] uint8, int8 taps)."""
    k = {"2d": 0, "sep": 1, "u8": 2}[kind]
    if k == 2:
        img = np.ascontiguousarray(img, dtype=np.uint8)
        c, h, w = img.shape if img.ndim == 3 else (1,) + img.shape
        filt = np.ascontiguousarray(filt, dtype=np.int8)
        r = (filt.shape[0] - 1) // 2
    else:
        img = _f32(img)
        c, (h, w) = 1, img.shape
        filt = _f32(filt).ravel()
        r = ((int(round(filt.size ** 0.5)) - 1) // 2) if k == 0 else (filt.size // 2 - 1) // 2
    t = _time_lib().time_image(k, c, h, w, r, int(shift), _p(img), _p(filt), _p(out), int(threads), int(reps))
    if t < 0:
        raise MemoryError("oracle timing could not allocate")
    return t


def time_batch_sep(h, w, r, off, pixels, filters, foff, out, threads: int, reps: int = 3) -> float:
    """Median seconds of the separable oracle over a packed batch (one image per task)."""
    hh, ww, rr = (np.ascontiguousarray(a, dtype=np.int32) for a in (h, w, r))
    oo, fo = (np.ascontiguousarray(a, dtype=np.int64) for a in (off, foff))
    t = _time_lib().time_batch_sep(hh.size, _p(hh), _p(ww), _p(rr), _p(oo), _p(pixels), _p(filters), _p(fo),
                                   _p(out), int(threads), int(reps))
    if t < 0:
        raise MemoryError("oracle timing could not allocate")
    return t
