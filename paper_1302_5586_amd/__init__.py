"""pencilfilter: clamp-to-edge 2D image filters for MI355X (gfx950).

A thin ctypes binding over ``libpencilfilter.so`` (C ABI in
``include/pf.h``). Every filter step runs in the library's HIP kernels;
this module only checks tensor arguments, allocates outputs with torch and
passes device pointers plus torch's current HIP stream. There is no CPU
fallback: without the built library every call raises.

The calling convention follows the paper's C99 rules for PENCIL functions
(Sec. II-B.1): sizes first, then restrict-qualified input, filter and
output arrays.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# PENCILFILTER_LIB selects another build of the same library (a variant
# built with different compile-time options).
LIB_PATH = os.environ.get("PENCILFILTER_LIB") or os.path.join(_HERE, "libpencilfilter.so")

PF_OK, PF_EINVAL, PF_EALIAS, PF_EUNSUPPORTED, PF_EDEVICE, PF_ENOMEM, PF_EBUDGET, PF_EAGAIN, PF_ETIMEDOUT = range(9)
PF_R_MAX = 8
PF_BATCH_R_MAX = 4
PF_SEP_DIRECT_R_MAX = 5
FLAG_EXACT = 0x1
BATCH_GRAPH = 0x2
BATCH_NO_TUNE = 0x4
KIND_2D, KIND_SEP, KIND_U8 = 0, 1, 2
VAR_DIRECT, VAR_SEPARABLE, VAR_SEP_DIRECT = 0, 1, 2
# uint8 on the int8 matrix cores (radius 1..PF_U8_MFMA_R_MAX, wave tiles of 16k rows).
VAR_MFMA = 3
PF_U8_MFMA_R_MAX = 8
PF_U8_MFMA_TILE_MAX = 256
BORDER_CLAMP, BORDER_ZERO, BORDER_REFLECT, BORDER_MIRROR = 0, 1, 2, 3
OP_SUM_F32, OP_HIST_U8 = 1, 2
CHAIN_HALO_MAX = 16


class PFError(RuntimeError):
    """A pf_* call returned a status other than PF_OK."""

    def __init__(self, status: int, msg: str):
        super().__init__("%s: %s" % (_status_name(status), msg))
        self.status = status


class PFInvalid(PFError, ValueError):
    pass


class PFAlias(PFError, ValueError):
    pass


class PFAgain(PFError):
    pass


class PFTimeout(PFError, TimeoutError):
    pass


class PFBudget(PFError):
    pass


class PFUnsupported(PFError):
    pass


_ERRORS = {PF_EUNSUPPORTED: PFUnsupported, PF_EINVAL: PFInvalid, PF_EALIAS: PFAlias, PF_EAGAIN: PFAgain, PF_ETIMEDOUT: PFTimeout, PF_EBUDGET: PFBudget}


TUNE_SINGLE, TUNE_BATCH = 0, 1


class TuneEntry(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("r", ctypes.c_int32), ("size_class", ctypes.c_int32),
                ("variant", ctypes.c_int32), ("rows_per_wave", ctypes.c_int32),
                ("waves_per_group", ctypes.c_int32), ("us", ctypes.c_float), ("context", ctypes.c_int32)]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("admitted", ctypes.c_int64), ("completed", ctypes.c_int64),
                ("rejected", ctypes.c_int64), ("batches", ctypes.c_int64), ("pixels", ctypes.c_int64),
                ("bytes_high_water", ctypes.c_int64), ("queue_high_water", ctypes.c_int64),
                ("mean_batch", ctypes.c_double), ("p50_us", ctypes.c_double), ("p99_us", ctypes.c_double),
                ("p999_us", ctypes.c_double), ("max_us", ctypes.c_double), ("wall_s", ctypes.c_double),
                ("gpx_per_s", ctypes.c_double)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


# Every exported symbol with its ctypes signature (return type first).
_P = ctypes.c_void_p
_I32 = ctypes.c_int32
_I64 = ctypes.c_int64
_SIGS = {
    "pf_status_str": (ctypes.c_char_p, [_I32]),
    "pf_last_error": (ctypes.c_char_p, []),
    "pf_version": (ctypes.c_char_p, []),
    "pf_filter2d_f32": (_I32, [_I32, _I32, _I32, _P, _P, _P, _I32, _P]),
    "pf_filter_sep_f32": (_I32, [_I32, _I32, _I32, _P, _P, _P, _P, _I32, _P]),
    "pf_filter2d_f32_border": (_I32, [_I32, _I32, _I32, _I32, _P, _P, _P, _I32, _P]),
    "pf_sum_workspace": (_I32, [_I64, _P]),
    "pf_inc_plan_create": (_I32, [_I32, _I32, _P, _P]),
    "pf_inc_plan_run": (_I32, [_P, _I32, _I32, _P, _P, _P]),
    "pf_inc_plan_destroy": (_I32, [_P]),
    "pf_edge_inc_atomic_f64": (_I32, [_I32, _I32, _P, _P, _P, _P]),
    "pf_sum_f32": (_I32, [_I64, _P, _P, _P, ctypes.c_size_t, _P]),
    "pf_sum_f32_noalloc": (_I32, [_I64, _P, _P, _P]),
    "pf_probe_alu": (_I32, [_I32, _I32, _I32, _P, _P]),
    "pf_probe_copy": (_I32, [_I64, _P, _P, _P]),
    "pf_hist_workspace": (_I32, [_I64, _P]),
    "pf_hist256_u8": (_I32, [_I64, _P, _P, _P, ctypes.c_size_t, _P]),
    "pf_filter_chain_f32": (_I32, [_I32, _I32, _I32, _I32, _I32, _P, _P, _P, _I32, _P]),
    "pf_filter2d_u8": (_I32, [_I32, _I32, _I32, _I32, _I32, _P, _P, _P, _I32, _P]),
    "pf_filter_f32_shaped": (_I32, [_I32, _I32, _I32, _I32, _I32, _I32, _I32, _P, _P, _P, _I32, _P]),
    "pf_tune_lookup": (_I32, [_I32, _I32, _I64, _I32, ctypes.POINTER(TuneEntry)]),
    "pf_tune_set": (_I32, [_I32, ctypes.POINTER(TuneEntry)]),
    "pf_tune_reset": (_I32, []),
    "pf_tune_load": (_I32, [ctypes.c_char_p]),
    "pf_tune_save": (_I32, [ctypes.c_char_p]),
    "pf_autotune": (_I32, [_I32, _I32, ctypes.c_char_p]),
    "pf_tune_batch_blocks": (_I32, [_I32, _P]),
    "pf_batch_autotune": (_I32, [_I32, _P, _P, _P, _P, _P, _P, _I64, _I64, _P, _P, _P, _I32, ctypes.c_char_p]),
    "pf_batch_plan_create": (_I32, [_I32, _P, _P, _P, _P, _P, _P, _I64, _I64, _I32, ctypes.POINTER(_P)]),
    "pf_batch_plan_run": (_I32, [_P, _I64, _I64, _P, _P, _P, _P]),
    "pf_batch_plan_variants": (_I32, [_P, _I32, _P]),
    "pf_batch_plan_info": (_I32, [_P, ctypes.POINTER(_I64), ctypes.POINTER(_I32), ctypes.POINTER(_I32)]),
    "pf_batch_plan_destroy": (_I32, [_P]),
    "pf_arena_replay": (_I32, [_I64, _I32, _P, _P, ctypes.POINTER(_I64)]),
    "pf_batch_plan_check": (_I32, [_I32, _P, _P, _P, _P, _P, _P, _I64, _I64, _I32, ctypes.POINTER(_I64),
                                   ctypes.POINTER(_I64)]),
    "pf_server_create": (_I32, [_I64, _I32, _I32, _I32, _I32, ctypes.POINTER(_P)]),
    "pf_server_submit": (_I32, [_P, _I32, _I32, _I32, _I32, _P, _I32, _P, _P, _I64, ctypes.POINTER(_I64)]),
    "pf_server_submit_reduce": (_I32, [_P, _I32, _I64, _P, _I32, _P, _I64, ctypes.POINTER(_I64)]),
    "pf_server_result_reduce": (_I32, [_P, _I64, _I32, _P, _I32]),
    "pf_server_poll": (_I32, [_P, _I64, ctypes.POINTER(_I32)]),
    "pf_server_wait": (_I32, [_P, _I64, _I64]),
    "pf_server_result": (_I32, [_P, _I64, _I32, _I32, _P, _I32]),
    "pf_server_release": (_I32, [_P, _I64]),
    "pf_server_stats_get": (_I32, [_P, ctypes.POINTER(ServerStats)]),
    "pf_server_run_trace": (_I32, [_P, _I32, _P, _P, _P, _P, _P, _P, _I64, _P, _I64, _P]),
    "pf_server_destroy": (_I32, [_P]),
}

_lib = None


def library_path() -> str:
    return LIB_PATH


def load() -> ctypes.CDLL:
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libpencilfilter.so is not built; run `python paper_1302_5586_amd/build.py`")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _status_name(s: int) -> str:
    try:
        return load().pf_status_str(s).decode()
    except Exception:  # noqa: BLE001 - name lookup must not mask the real error
        return "PF_STATUS_%d" % s


def _check(status: int):
    if status != PF_OK:
        msg = load().pf_last_error().decode(errors="replace")
        raise _ERRORS.get(status, PFError)(status, msg)


def version() -> str:
    return load().pf_version().decode()


# ---------------------------------------------------------------- tensors

def _torch():
    import torch  # plumbing only: device memory and streams
    return torch


def _stream_ptr(stream=None) -> int:
    torch = _torch()
    s = torch.cuda.current_stream() if stream is None else stream
    return int(s.cuda_stream)


def _dev_tensor(t, dtype, name, ndim=None):
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        raise TypeError("%s must be a torch tensor on the GPU" % name)
    if t.device.type != "cuda":
        raise ValueError("%s must be on the GPU (got %s)" % (name, t.device))
    if t.dtype != dtype:
        raise TypeError("%s must be %s (got %s)" % (name, dtype, t.dtype))
    if ndim is not None and t.dim() not in ndim:
        raise ValueError("%s must have %s dimensions (got %d)" % (name, ndim, t.dim()))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    return t


def _radius_of(n: int, what: str) -> int:
    if n % 2 != 1:
        raise ValueError("%s must have odd size 2r+1 (got %d)" % (what, n))
    return (n - 1) // 2


def filter2d(x, f, *, exact: bool = False, out=None, stream=None):
    """FP32 clamp-to-edge 2D correlation of ``x`` [H, W] with ``f`` [2r+1, 2r+1]."""
    torch = _torch()
    _dev_tensor(x, torch.float32, "x", (2,))
    _dev_tensor(f, torch.float32, "f", (2,))
    if f.shape[0] != f.shape[1]:
        raise ValueError("filter must be square")
    r = _radius_of(f.shape[0], "filter")
    h, w = x.shape
    if out is None:
        out = torch.empty_like(x)
    _dev_tensor(out, torch.float32, "out", (2,))
    _check(load().pf_filter2d_f32(h, w, r, x.data_ptr(), f.data_ptr(), out.data_ptr(),
                                  FLAG_EXACT if exact else 0, _stream_ptr(stream)))
    return out


def filter2d_border(x, f, border: int, *, exact: bool = False, out=None, stream=None):
    """FP32 2D correlation of ``x`` [H, W] with ``f`` under a border rule (BORDER_*)."""
    torch = _torch()
    _dev_tensor(x, torch.float32, "x", (2,))
    _dev_tensor(f, torch.float32, "f", (2,))
    if f.shape[0] != f.shape[1]:
        raise ValueError("filter must be square")
    r = _radius_of(f.shape[0], "filter")
    h, w = x.shape
    if out is None:
        out = torch.empty_like(x)
    _dev_tensor(out, torch.float32, "out", (2,))
    _check(load().pf_filter2d_f32_border(h, w, r, border, x.data_ptr(), f.data_ptr(), out.data_ptr(),
                                         FLAG_EXACT if exact else 0, _stream_ptr(stream)))
    return out


def filter_chain(x, f, passes: int, border: int = 0, *, exact: bool = False, out=None, stream=None):
    """``passes`` fused applications of the 2D filter ``f`` to ``x`` [H, W] (one kernel)."""
    torch = _torch()
    _dev_tensor(x, torch.float32, "x", (2,))
    _dev_tensor(f, torch.float32, "f", (2,))
    if f.shape[0] != f.shape[1]:
        raise ValueError("filter must be square")
    r = _radius_of(f.shape[0], "filter")
    h, w = x.shape
    if out is None:
        out = torch.empty_like(x)
    _dev_tensor(out, torch.float32, "out", (2,))
    _check(load().pf_filter_chain_f32(h, w, r, passes, border, x.data_ptr(), f.data_ptr(), out.data_ptr(),
                                      FLAG_EXACT if exact else 0, _stream_ptr(stream)))
    return out


def _workspace(fn, n, dev):
    torch = _torch()
    nb = ctypes.c_size_t(0)
    _check(fn(n, ctypes.byref(nb)))
    return torch.empty(max((nb.value + 7) // 8, 1), dtype=torch.float64, device=dev)


def sum_f32(x, *, out=None, workspace=None, stream=None):
    """Reproducible float64 sum and mean of a contiguous FP32 tensor:
    returns a device float64 tensor [sum, mean]."""
    torch = _torch()
    if not x.is_cuda or x.dtype != torch.float32 or not x.is_contiguous():
        raise ValueError("x must be a contiguous CUDA float32 tensor")
    n = x.numel()
    if out is None:
        out = torch.empty(2, dtype=torch.float64, device=x.device)
    if workspace is None:
        workspace = _workspace(load().pf_sum_workspace, n, x.device)
    _check(load().pf_sum_f32(n, x.data_ptr(), out.data_ptr(), workspace.data_ptr(),
                             workspace.numel() * workspace.element_size(), _stream_ptr(stream)))
    return out


def sum_f32_noalloc(x, *, out=None, stream=None):
    """The sum and mean of ``sum_f32`` (same bits) with no workspace: the
    library's static device scratch holds the partials (x up to 2^29
    elements). Calls that overlap in time on one GPU share that scratch and
    must be ordered by the caller."""
    torch = _torch()
    if not x.is_cuda or x.dtype != torch.float32 or not x.is_contiguous():
        raise ValueError("x must be a contiguous CUDA float32 tensor")
    if out is None:
        out = torch.empty(2, dtype=torch.float64, device=x.device)
    _check(load().pf_sum_f32_noalloc(x.numel(), x.data_ptr(), out.data_ptr(), _stream_ptr(stream)))
    return out


PROBE_DOT4 = 0
PROBE_FMA = 1


def probe_alu(op: int, blocks: int, iters: int, out, stream=None) -> int:
    """Launch the ALU-rate probe (``PROBE_DOT4`` or ``PROBE_FMA``) into a
    CUDA int32/float32 tensor of ``blocks * 256`` elements; returns the
    lane-instructions of the launch."""
    if not out.is_cuda or out.numel() < blocks * 256 or out.element_size() != 4:
        raise ValueError("out must be a CUDA tensor of blocks * 256 4-byte values")
    _check(load().pf_probe_alu(op, blocks, iters, out.data_ptr(), _stream_ptr(stream)))
    return blocks * 256 * iters * 128


def probe_copy(x, out, stream=None):
    """The HBM copy probe: out[:] = x (contiguous CUDA float32 tensors)."""
    torch = _torch()
    for t in (x, out):
        if not t.is_cuda or t.dtype != torch.float32 or not t.is_contiguous():
            raise ValueError("x and out must be contiguous CUDA float32 tensors")
    if out.numel() != x.numel():
        raise ValueError("x and out differ in size")
    _check(load().pf_probe_copy(x.numel(), x.data_ptr(), out.data_ptr(), _stream_ptr(stream)))
    return out


def hist256_u8(x, *, out=None, workspace=None, stream=None):
    """256-bin histogram (int64 counts) of a contiguous uint8 tensor."""
    torch = _torch()
    if not x.is_cuda or x.dtype != torch.uint8 or not x.is_contiguous():
        raise ValueError("x must be a contiguous CUDA uint8 tensor")
    n = x.numel()
    if out is None:
        out = torch.empty(256, dtype=torch.int64, device=x.device)
    if workspace is None:
        workspace = _workspace(load().pf_hist_workspace, n, x.device)
    _check(load().pf_hist256_u8(n, x.data_ptr(), out.data_ptr(), workspace.data_ptr(),
                                workspace.numel() * workspace.element_size(), _stream_ptr(stream)))
    return out


class IncPlan:
    """OP2-style edge-to-cell increment plan (see pf_inc_plan_create):
    ``run(edge, cell)`` adds every edge value into its two cells, in the
    sequential loop's order, bit for bit."""

    def __init__(self, ncells: int, edge_to_cells):
        m = _i32(np.asarray(edge_to_cells).reshape(-1))
        if m.size % 2:
            raise ValueError("edge_to_cells needs two cells per edge")
        self.ncells, self.nedges = int(ncells), m.size // 2
        h = ctypes.c_void_p()
        _check(load().pf_inc_plan_create(self.ncells, self.nedges, _np_ptr(m), ctypes.byref(h)))
        self._h = h

    def run(self, edge, cell, stream=None):
        torch = _torch()
        for t, name, n in ((edge, "edge", self.nedges), (cell, "cell", self.ncells)):
            if not t.is_cuda or t.dtype != torch.float64 or not t.is_contiguous() or t.numel() != n:
                raise ValueError("%s must be a contiguous CUDA float64 tensor of %d elements" % (name, n))
        _check(load().pf_inc_plan_run(self._h, self.ncells, self.nedges, edge.data_ptr(), cell.data_ptr(),
                                      _stream_ptr(stream)))
        return cell

    def close(self):
        if getattr(self, "_h", None):
            load().pf_inc_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def edge_inc_atomic(edge_to_cells, edge, cell, stream=None):
    """Edge-to-cell increment with float64 atomics (device map int32 [2 * nedges])."""
    torch = _torch()
    if not edge_to_cells.is_cuda or edge_to_cells.dtype != torch.int32 or not edge_to_cells.is_contiguous():
        raise ValueError("edge_to_cells must be a contiguous CUDA int32 tensor")
    nedges = edge_to_cells.numel() // 2
    for t, name in ((edge, "edge"), (cell, "cell")):
        if not t.is_cuda or t.dtype != torch.float64 or not t.is_contiguous():
            raise ValueError("%s must be a contiguous CUDA float64 tensor" % name)
    if edge.numel() != nedges:
        raise ValueError("edge must have one value per edge")
    _check(load().pf_edge_inc_atomic_f64(cell.numel(), nedges, edge_to_cells.data_ptr(), edge.data_ptr(),
                                         cell.data_ptr(), _stream_ptr(stream)))
    return cell


def filter_sep(x, fx, fy, *, exact: bool = False, out=None, stream=None):
    """FP32 separable filter: row pass with ``fx``, then column pass with ``fy``."""
    torch = _torch()
    _dev_tensor(x, torch.float32, "x", (2,))
    _dev_tensor(fx, torch.float32, "fx", (1,))
    _dev_tensor(fy, torch.float32, "fy", (1,))
    if fx.numel() != fy.numel():
        raise ValueError("fx and fy must have the same length")
    r = _radius_of(fx.numel(), "fx")
    h, w = x.shape
    if out is None:
        out = torch.empty_like(x)
    _dev_tensor(out, torch.float32, "out", (2,))
    _check(load().pf_filter_sep_f32(h, w, r, x.data_ptr(), fx.data_ptr(), fy.data_ptr(), out.data_ptr(),
                                    FLAG_EXACT if exact else 0, _stream_ptr(stream)))
    return out


def filter2d_u8(x, f, shift: int = 6, *, out=None, stream=None):
    """uint8 planar [C, H, W] (or [H, W]) with int8 weights: int32 sum,
    arithmetic shift, saturation to uint8."""
    torch = _torch()
    _dev_tensor(x, torch.uint8, "x", (2, 3))
    _dev_tensor(f, torch.int8, "f", (2,))
    if f.shape[0] != f.shape[1]:
        raise ValueError("filter must be square")
    r = _radius_of(f.shape[0], "filter")
    c, h, w = (1,) + tuple(x.shape) if x.dim() == 2 else tuple(x.shape)
    if out is None:
        out = torch.empty_like(x)
    _dev_tensor(out, torch.uint8, "out", (2, 3))
    _check(load().pf_filter2d_u8(c, h, w, r, int(shift), x.data_ptr(), f.data_ptr(), out.data_ptr(), 0,
                                 _stream_ptr(stream)))
    return out


def filter_shaped(x, filt, r: int, kind: int, variant: int, rows_per_wave: int, waves_per_group: int,
                  *, exact: bool = False, out=None, stream=None):
    """The FP32 filter with a forced variant and launch shape. ``filt`` is
    the flattened 2D taps (kind 2D) or fx followed by fy (kind SEP)."""
    torch = _torch()
    _dev_tensor(x, torch.float32, "x", (2,))
    _dev_tensor(filt, torch.float32, "filt")
    k = 2 * r + 1
    need = k * k if kind == KIND_2D else 2 * k
    if filt.numel() != need:
        raise ValueError("filter has %d weights, kind needs %d" % (filt.numel(), need))
    h, w = x.shape
    if out is None:
        out = torch.empty_like(x)
    _check(load().pf_filter_f32_shaped(h, w, r, kind, variant, rows_per_wave, waves_per_group, x.data_ptr(),
                                       filt.data_ptr(), out.data_ptr(), FLAG_EXACT if exact else 0,
                                       _stream_ptr(stream)))
    return out


# ---------------------------------------------------------------- tuning

def tune_lookup(kind: int, r: int, pixels: int, context: int = TUNE_SINGLE) -> TuneEntry:
    """The tune entry single-image calls (TUNE_SINGLE) or batch plans and
    servers (TUNE_BATCH) use for this key."""
    e = TuneEntry()
    _check(load().pf_tune_lookup(kind, r, pixels, context, ctypes.byref(e)))
    return e


def tune_set(entries: Sequence[TuneEntry]):
    arr = (TuneEntry * len(entries))(*entries)
    _check(load().pf_tune_set(len(entries), arr))


def tune_reset():
    _check(load().pf_tune_reset())


def tune_load(path: str):
    _check(load().pf_tune_load(path.encode()))


def tune_save(path: str):
    _check(load().pf_tune_save(path.encode()))


def autotune(r_max: int = 4, reps: int = 20, path: str | None = None):
    """Time every candidate variant and launch shape on the current GPU and
    install the fastest per (kind, radius, size class)."""
    _check(load().pf_autotune(r_max, reps, path.encode() if path else None))


def tune_batch_blocks(blocks_per_cu: int = 0) -> int:
    """Set workgroups per compute unit of batch launches (0: leave); returns the previous value."""
    prev = ctypes.c_int32(0)
    _check(load().pf_tune_batch_blocks(blocks_per_cu, ctypes.byref(prev)))
    return prev.value


def autotune_batch(h, w, r, kind, pix_off, filt_off, x, filt, out, reps: int = 10, path: str | None = None):
    """Tune the batch-context tile heights of the table on one batch (see pf_batch_autotune)."""
    torch = _torch()
    _dev_tensor(x, torch.float32, "x")
    _dev_tensor(filt, torch.float32, "filt")
    _dev_tensor(out, torch.float32, "out")
    hh, ww, rr, kk = _i32(h), _i32(w), _i32(r), _i32(kind)
    po, fo = _i64(pix_off), _i64(filt_off)
    _check(load().pf_batch_autotune(hh.size, _np_ptr(hh), _np_ptr(ww), _np_ptr(rr), _np_ptr(kk), _np_ptr(po),
                                    _np_ptr(fo), x.numel(), filt.numel(), x.data_ptr(), filt.data_ptr(),
                                    out.data_ptr(), reps, path.encode() if path else None))


# ---------------------------------------------------------------- batches

def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _i64(a):
    return np.ascontiguousarray(a, dtype=np.int64)


def _np_ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


class BatchPlan:
    """Many images in one persistent launch (optionally a graph replay).

    Images live in one pixel arena (input and output arenas share the
    layout) at ``pix_off``; filters in one filter arena at ``filt_off``.
    """

    def __init__(self, h, w, r, kind, pix_off, filt_off, npix: int, nfilt: int, *, graph: bool = True,
                 exact: bool = False, no_tune: bool = False):
        self._h, self._w, self._r, self._k = _i32(h), _i32(w), _i32(r), _i32(kind)
        self._po, self._fo = _i64(pix_off), _i64(filt_off)
        n = self._h.size
        if not all(a.size == n for a in (self._w, self._r, self._k, self._po, self._fo)):
            raise ValueError("descriptor arrays differ in length")
        self.n, self.npix, self.nfilt = n, int(npix), int(nfilt)
        flags = (BATCH_GRAPH if graph else 0) | (FLAG_EXACT if exact else 0) | (BATCH_NO_TUNE if no_tune else 0)
        p = ctypes.c_void_p()
        _check(load().pf_batch_plan_create(n, _np_ptr(self._h), _np_ptr(self._w), _np_ptr(self._r), _np_ptr(self._k),
                                           _np_ptr(self._po), _np_ptr(self._fo), self.npix, self.nfilt, flags,
                                           ctypes.byref(p)))
        self._p = p

    def run(self, x, filt, out, stream=None):
        torch = _torch()
        _dev_tensor(x, torch.float32, "x")
        _dev_tensor(filt, torch.float32, "filt")
        _dev_tensor(out, torch.float32, "out")
        if x.numel() != self.npix or out.numel() != self.npix or filt.numel() != self.nfilt:
            raise ValueError("arena sizes differ from the plan's")
        _check(load().pf_batch_plan_run(self._p, self.npix, self.nfilt, x.data_ptr(), filt.data_ptr(),
                                        out.data_ptr(), _stream_ptr(stream)))
        return out

    def variants(self) -> np.ndarray:
        v = np.zeros(self.n, dtype=np.int32)
        _check(load().pf_batch_plan_variants(self._p, self.n, _np_ptr(v)))
        return v

    def info(self) -> dict:
        t, l, g = _I64(), _I32(), _I32()
        _check(load().pf_batch_plan_info(self._p, ctypes.byref(t), ctypes.byref(l), ctypes.byref(g)))
        return {"tasks": t.value, "launches": l.value, "grid": g.value}

    def close(self):
        if getattr(self, "_p", None):
            load().pf_batch_plan_destroy(self._p)
            self._p = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001 - interpreter shutdown
            pass


def batch_plan_check(h, w, r, kind, pix_off, filt_off, npix: int, nfilt: int, *, exact: bool = False,
                     no_tune: bool = False) -> dict:
    """Host-only replay of a batch plan's tile table (see pf_batch_plan_check):
    returns {"tiles": checked, "violations": found}; raises on a violation."""
    hh, ww, rr, kk = _i32(h), _i32(w), _i32(r), _i32(kind)
    po, fo = _i64(pix_off), _i64(filt_off)
    flags = (FLAG_EXACT if exact else 0) | (BATCH_NO_TUNE if no_tune else 0)
    tiles, bad = _I64(), _I64()
    _check(load().pf_batch_plan_check(hh.size, _np_ptr(hh), _np_ptr(ww), _np_ptr(rr), _np_ptr(kk), _np_ptr(po),
                                      _np_ptr(fo), int(npix), int(nfilt), flags, ctypes.byref(tiles),
                                      ctypes.byref(bad)))
    return {"tiles": tiles.value, "violations": bad.value}


def arena_replay(budget: int, ops) -> tuple:
    """Host-only replay of the server's first-fit arena allocator (see
    pf_arena_replay): returns (per-operation results, bytes in use)."""
    o = _i64(ops)
    res = np.zeros(o.size, np.int64)
    used = _I64()
    _check(load().pf_arena_replay(int(budget), o.size, _np_ptr(o), _np_ptr(res), ctypes.byref(used)))
    return res, used.value


@dataclass
class PackedBatch:
    """Host-side packing of a list of images and filters into arenas."""
    h: np.ndarray
    w: np.ndarray
    r: np.ndarray
    kind: np.ndarray
    pix_off: np.ndarray
    filt_off: np.ndarray
    pixels: np.ndarray      # float32[npix]
    filters: np.ndarray     # float32[nfilt]


def pack_batch(images: Sequence[np.ndarray], filters: Sequence[np.ndarray], kinds: Sequence[int],
               align: int = 64) -> PackedBatch:
    """Pack images at ``align``-element offsets and their weights (2D taps,
    or fx then fy for separable kinds) into one filter arena."""
    n = len(images)
    h = np.array([im.shape[0] for im in images], np.int32)
    w = np.array([im.shape[1] for im in images], np.int32)
    po = np.zeros(n, np.int64)
    off = 0
    for i in range(n):
        po[i] = off
        off += int(h[i]) * int(w[i])
        off = (off + align - 1) // align * align
    npix = max(off, 1)
    pix = np.zeros(npix, np.float32)
    for i, im in enumerate(images):
        pix[po[i]:po[i] + im.size] = np.asarray(im, np.float32).ravel()
    fo = np.zeros(n, np.int64)
    flist, foff, rr = [], 0, np.zeros(n, np.int32)
    for i, (f, k) in enumerate(zip(filters, kinds)):
        f = np.asarray(f, np.float32).ravel()
        if k == KIND_2D:
            rr[i] = _radius_of(int(round(np.sqrt(f.size))), "filter")
        else:
            rr[i] = _radius_of(f.size // 2, "fx")
        fo[i] = foff
        flist.append(f)
        foff += f.size
    return PackedBatch(h, w, rr, np.asarray(kinds, np.int32), po, fo, pix, np.concatenate(flist).astype(np.float32))


# ---------------------------------------------------------------- serving

class Server:
    """Continuous-batching server for filter, sum and histogram requests
    under an HBM budget.

    A GPU tensor submitted as input is read later by the server's own
    streams: the server orders that read after the work queued on the
    current (or given) torch stream at submit, and this object keeps a
    reference to the tensor until its result is fetched or released."""

    def __init__(self, hbm_budget_bytes: int, n_streams: int = 3, max_batch: int = 256, max_queue: int = 1 << 16,
                 flags: int = 0):
        p = ctypes.c_void_p()
        _check(load().pf_server_create(int(hbm_budget_bytes), n_streams, max_batch, max_queue, flags,
                                       ctypes.byref(p)))
        self._s = p
        self._inputs = {}

    def submit(self, x, r: int, kind: int, filt: np.ndarray, arrival_ns: int = 0, stream=None) -> int:
        """Submit one FP32 image: a GPU tensor (read in place) or a host numpy
        array (copied into the server's arena)."""
        f = np.ascontiguousarray(filt, dtype=np.float32).ravel()
        t = _I64()
        if isinstance(x, np.ndarray):
            a = np.ascontiguousarray(x, dtype=np.float32)
            h, w = a.shape
            _check(load().pf_server_submit(self._s, h, w, r, kind, _np_ptr(a), 1, _np_ptr(f), None, int(arrival_ns),
                                           ctypes.byref(t)))
        else:
            torch = _torch()
            _dev_tensor(x, torch.float32, "x", (2,))
            h, w = x.shape
            _check(load().pf_server_submit(self._s, h, w, r, kind, x.data_ptr(), 0, _np_ptr(f), _stream_ptr(stream),
                                           int(arrival_ns), ctypes.byref(t)))
            self._inputs[t.value] = x
        return t.value

    def _submit_reduce(self, op: int, x, dtype, np_dtype, stream, arrival_ns) -> int:
        t = _I64()
        if isinstance(x, np.ndarray):
            a = np.ascontiguousarray(x, dtype=np_dtype).ravel()
            _check(load().pf_server_submit_reduce(self._s, op, a.size, _np_ptr(a), 1, None, int(arrival_ns),
                                                  ctypes.byref(t)))
        else:
            torch = _torch()
            _dev_tensor(x, getattr(torch, dtype), "x")
            _check(load().pf_server_submit_reduce(self._s, op, x.numel(), x.data_ptr(), 0, _stream_ptr(stream),
                                                  int(arrival_ns), ctypes.byref(t)))
            self._inputs[t.value] = x
        return t.value

    def submit_sum(self, x, arrival_ns: int = 0, stream=None) -> int:
        """Submit the float64 sum and mean of an FP32 array (GPU tensor or numpy)."""
        return self._submit_reduce(OP_SUM_F32, x, "float32", np.float32, stream, arrival_ns)

    def submit_hist(self, x, arrival_ns: int = 0, stream=None) -> int:
        """Submit the 256-bin histogram of a uint8 array (GPU tensor or numpy)."""
        return self._submit_reduce(OP_HIST_U8, x, "uint8", np.uint8, stream, arrival_ns)

    def poll(self, ticket: int) -> bool:
        d = _I32()
        _check(load().pf_server_poll(self._s, ticket, ctypes.byref(d)))
        return bool(d.value)

    def wait(self, ticket: int, timeout_s: float | None = None):
        _check(load().pf_server_wait(self._s, ticket, -1 if timeout_s is None else int(timeout_s * 1e9)))

    def result(self, ticket: int, h: int, w: int, out=None):
        """Copy the output to ``out`` (GPU tensor) or to a new numpy array."""
        if out is None:
            a = np.empty((h, w), np.float32)
            _check(load().pf_server_result(self._s, ticket, h, w, _np_ptr(a), 1))
            self._inputs.pop(ticket, None)
            return a
        torch = _torch()
        _dev_tensor(out, torch.float32, "out", (2,))
        _check(load().pf_server_result(self._s, ticket, h, w, out.data_ptr(), 0))
        self._inputs.pop(ticket, None)
        return out

    def result_sum(self, ticket: int) -> np.ndarray:
        """[sum, mean] (float64) of a finished sum request."""
        a = np.empty(2, np.float64)
        _check(load().pf_server_result_reduce(self._s, ticket, OP_SUM_F32, _np_ptr(a), 1))
        self._inputs.pop(ticket, None)
        return a

    def result_hist(self, ticket: int) -> np.ndarray:
        """The 256 int64 counts of a finished histogram request."""
        a = np.empty(256, np.int64)
        _check(load().pf_server_result_reduce(self._s, ticket, OP_HIST_U8, _np_ptr(a), 1))
        self._inputs.pop(ticket, None)
        return a

    def release(self, ticket: int):
        _check(load().pf_server_release(self._s, ticket))
        self._inputs.pop(ticket, None)

    def stats(self) -> dict:
        st = ServerStats()
        _check(load().pf_server_stats_get(self._s, ctypes.byref(st)))
        return st.as_dict()

    def run_trace(self, arrival_ns, h, w, r, pix_off, filt_off, pool, filters: np.ndarray) -> dict:
        """Replay an open-loop arrival schedule against a device-resident
        image pool (GPU tensor) with host filter weights (fx then fy)."""
        torch = _torch()
        _dev_tensor(pool, torch.float32, "pool")
        torch.cuda.current_stream().synchronize()  # the pool must be complete before the call
        a, hh, ww, rr = _i64(arrival_ns), _i32(h), _i32(w), _i32(r)
        po, fo = _i64(pix_off), _i64(filt_off)
        fl = np.ascontiguousarray(filters, dtype=np.float32).ravel()
        _check(load().pf_server_run_trace(self._s, a.size, _np_ptr(a), _np_ptr(hh), _np_ptr(ww), _np_ptr(rr),
                                          _np_ptr(po), _np_ptr(fo), pool.numel(), pool.data_ptr(), fl.size,
                                          _np_ptr(fl)))
        return self.stats()

    def close(self):
        if getattr(self, "_s", None):
            _check(load().pf_server_destroy(self._s))
            self._s = None
            self._inputs = {}

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001 - interpreter shutdown
            pass
