"""Helpers shared by the GPU tests: device setup and the FP32 tolerance.

FP32 tolerance (per element, applied to every FP32 comparison with the
oracle): |gpu - oracle| <= 1e-5 * D, where D = sum over the window of
|w| * |x| (the scale of the inner-product error bound). For the
non-negative weights and pixels of the Gaussian workloads D equals |out|,
so this is the 1e-5 relative contract. Two recursive FP32 sums of n = 81
products (r = 4) differ by at most 2 * gamma_81 * D, about 9.7e-6 * D, so the
bound holds for every radius up to 4; for larger radii the bound used is
2 * gamma_n * D + 2^-24 * D, the proven worst case.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle

U = 2.0 ** -24


def gamma(n: int) -> float:
    return n * U / (1.0 - n * U)


def device():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1302_5586_amd as pf
    pf.load()  # raises if the HIP library is not built: no fallback
    return torch.device("cuda:0")


def tolerance_2d(img: np.ndarray, f2d: np.ndarray, r: int) -> np.ndarray:
    """Per-element allowed error for a 2D filter of radius r."""
    d = oracle.filter2d_f32(np.abs(img), np.abs(f2d)).astype(np.float64) * (1 + 1e-6)
    n = (2 * r + 1) ** 2
    rel = 1e-5 if r <= 4 else 2 * gamma(n) + U
    return rel * d + 1e-30


def tolerance_sep(img: np.ndarray, fx: np.ndarray, fy: np.ndarray) -> np.ndarray:
    """Per-element allowed error for a separable filter: D is the separable
    oracle over |x| with |fx| and |fy|, which equals sum |fy[a] fx[b]| |x|
    over the window up to its own rounding (below 1e-6 relative)."""
    r = (fx.size - 1) // 2
    d = oracle.filter_sep_f32(np.abs(img), np.abs(fx), np.abs(fy)).astype(np.float64) * (1 + 1e-6)
    n = (2 * r + 1) ** 2
    rel = 1e-5 if r <= 4 else 2 * gamma(n) + U
    return rel * d + 1e-30


def assert_close(got: np.ndarray, ref: np.ndarray, tol: np.ndarray, what: str = ""):
    g = got.astype(np.float64)
    o = ref.astype(np.float64)
    err = np.abs(g - o)
    bad = ~(err <= tol)
    # NaN in both is agreement
    both_nan = np.isnan(g) & np.isnan(o)
    bad &= ~both_nan
    if bad.any():
        idx = np.argwhere(bad)[0]
        raise AssertionError("%s: %d elements outside tolerance; first at %s: gpu %r oracle %r tol %r; max abs %g"
                             % (what, int(bad.sum()), tuple(idx), g[tuple(idx)], o[tuple(idx)], tol[tuple(idx)],
                                np.nanmax(err)))
    denom = np.maximum(np.abs(o), 1e-30)
    return float(np.nanmax(err)) if err.size else 0.0, float(np.nanmax(err / denom)) if err.size else 0.0
