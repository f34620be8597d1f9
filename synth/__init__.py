"""Seeded synthetic inputs for the clamp-to-edge image filter.

This module only draws numbers: images, filter weights, batch lists and
arrival traces. It holds none of the filter's arithmetic, so both the
oracle side and the device side can take their inputs from here without
sharing any part of the computation.

Every generator uses numpy's PCG64 (``numpy.random.default_rng``) with a
fixed seed and a fixed draw order, so the same seed always gives the same
bytes.

Workloads (sizes and value distributions):

* ``single_f32``: one grayscale FP32 image, pixels uniform on [0, 1).
  256x256 with a 3x3 Gaussian (sigma 1.0, seed 0) and 4096x4096 with a
  5x5 Gaussian (sigma 1.5, seed 1).
* ``rgb_u8``: three planar uint8 planes of 1080 rows by 1920 columns,
  pixels uniform on {0..255}, and a 7x7 int8 filter with weights uniform
  on {-8..8}; pixels are drawn before weights from one generator (seed 2).
* ``batch_f32``: 512 images; widths, then heights, each log-uniform on
  [64, 2048] and rounded to the nearest integer; radius uniform on
  {1, 2, 3, 4}; Gaussian sigma uniform on [0.5, 2.0); then the pixels of
  each image in index order (seed 3).
* ``arrival_trace``: open-loop Poisson arrivals (exponential gaps, mean
  1/rate) until the duration is reached, then per request a pool index,
  a radius and a sigma (seed 4); the pool itself is a ``batch_f32`` list
  of 1024 images drawn with seed 40.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# Gaussian filters are inputs here: the filter applies whatever weights it
# is given. The sampled, window-normalised Gaussian is the usual
# image-processing smoothing kernel; weights are formed in float64 and
# rounded once to float32.


def gaussian_1d(r: int, sigma: float) -> np.ndarray:
    """Sampled Gaussian over the taps -r..r, normalised over the truncated
    window in float64, then rounded to float32."""
    i = np.arange(-r, r + 1, dtype=np.float64)
    g = np.exp(-(i * i) / (2.0 * sigma * sigma))
    g = g / g.sum()
    return g.astype(np.float32)


def outer_2d(fy: np.ndarray, fx: np.ndarray) -> np.ndarray:
    """2D weights f[i][j] = fy[i] * fx[j], product formed in float64 and
    rounded once to float32 (row index i is the vertical tap)."""
    return (fy.astype(np.float64)[:, None] * fx.astype(np.float64)[None, :]).astype(np.float32)


def gaussian_2d(r: int, sigma: float) -> np.ndarray:
    g = gaussian_1d(r, sigma)
    return outer_2d(g, g)


def image_f32(rng: np.random.Generator, h: int, w: int) -> np.ndarray:
    return rng.random((h, w), dtype=np.float32)


@dataclass
class SingleF32:
    h: int
    w: int
    r: int
    sigma: float
    seed: int
    image: np.ndarray
    f1d: np.ndarray
    f2d: np.ndarray


def single_f32(h: int, w: int, r: int, sigma: float, seed: int) -> SingleF32:
    rng = np.random.default_rng(seed)
    img = image_f32(rng, h, w)
    g = gaussian_1d(r, sigma)
    return SingleF32(h, w, r, sigma, seed, img, g, outer_2d(g, g))


def config_small() -> SingleF32:
    """256x256 FP32 image, 3x3 Gaussian with sigma 1.0, seed 0."""
    return single_f32(256, 256, 1, 1.0, 0)


def config_large() -> SingleF32:
    """4096x4096 FP32 image, 5x5 Gaussian with sigma 1.5, seed 1."""
    return single_f32(4096, 4096, 2, 1.5, 1)


@dataclass
class RgbU8:
    c: int
    h: int
    w: int
    r: int
    shift: int
    image: np.ndarray
    filt: np.ndarray


def rgb_u8(c: int = 3, h: int = 1080, w: int = 1920, r: int = 3, shift: int = 6,
           seed: int = 2, wlo: int = -8, whi: int = 8) -> RgbU8:
    """Planar uint8 image and an int8 (2r+1)x(2r+1) filter; pixels are
    drawn first, then weights, from one generator."""
    rng = np.random.default_rng(seed)
    img = rng.integers(0, 256, size=(c, h, w), dtype=np.uint8)
    k = 2 * r + 1
    filt = rng.integers(wlo, whi + 1, size=(k, k)).astype(np.int8)
    return RgbU8(c, h, w, r, shift, img, filt)


def config_rgb() -> RgbU8:
    """1080p planar RGB, 7x7 int8 weights on {-8..8}, shift 6, seed 2."""
    return rgb_u8()


def log_uniform_sizes(rng: np.random.Generator, n: int, lo: int = 64, hi: int = 2048) -> np.ndarray:
    v = np.exp(rng.uniform(math.log(lo), math.log(hi), n))
    return np.clip(np.rint(v), lo, hi).astype(np.int64)


@dataclass
class BatchF32:
    n: int
    h: np.ndarray          # int64[n]
    w: np.ndarray          # int64[n]
    r: np.ndarray          # int64[n]
    sigma: np.ndarray      # float64[n]
    images: list = field(repr=False, default_factory=list)   # float32[h_i, w_i]
    fx: list = field(repr=False, default_factory=list)       # float32[2r_i+1]
    f2d: list = field(repr=False, default_factory=list)      # float32[2r_i+1, 2r_i+1]

    @property
    def pixels(self) -> int:
        return int((self.h * self.w).sum())


def batch_f32(n: int = 512, seed: int = 3, lo: int = 64, hi: int = 2048,
              rmax: int = 4, with_pixels: bool = True) -> BatchF32:
    """n images: widths, heights, radii, sigmas, then pixels per image."""
    rng = np.random.default_rng(seed)
    w = log_uniform_sizes(rng, n, lo, hi)
    h = log_uniform_sizes(rng, n, lo, hi)
    r = rng.integers(1, rmax + 1, n).astype(np.int64)
    sigma = rng.uniform(0.5, 2.0, n)
    b = BatchF32(n, h, w, r, sigma)
    for i in range(n):
        g = gaussian_1d(int(r[i]), float(sigma[i]))
        b.fx.append(g)
        b.f2d.append(outer_2d(g, g))
        if with_pixels:
            b.images.append(image_f32(rng, int(h[i]), int(w[i])))
    return b


def config_batch(with_pixels: bool = True) -> BatchF32:
    """512 FP32 images of log-uniform sizes in [64, 2048], r in 1..4,
    sigma in [0.5, 2.0), seed 3."""
    return batch_f32(512, 3, with_pixels=with_pixels)


@dataclass
class ArrivalTrace:
    rate: float
    duration: float
    t: np.ndarray          # float64[n] scheduled arrival times (s)
    pool_index: np.ndarray  # int64[n]
    r: np.ndarray          # int64[n]
    sigma: np.ndarray      # float64[n]

    @property
    def n(self) -> int:
        return int(self.t.shape[0])


def arrival_trace(rate: float = 2000.0, duration: float = 60.0, seed: int = 4,
                  pool_size: int = 1024, rmax: int = 4) -> ArrivalTrace:
    """Open-loop Poisson arrivals: exponential gaps drawn one at a time
    until ``duration``; then, per request, a pool index, radius and sigma."""
    rng = np.random.default_rng(seed)
    ts = []
    t = 0.0
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration:
            break
        ts.append(t)
    n = len(ts)
    pool_index = rng.integers(0, pool_size, n).astype(np.int64)
    r = rng.integers(1, rmax + 1, n).astype(np.int64)
    sigma = rng.uniform(0.5, 2.0, n)
    return ArrivalTrace(rate, duration, np.asarray(ts, dtype=np.float64), pool_index, r, sigma)


def serve_pool(n: int = 1024, seed: int = 40, with_pixels: bool = True) -> BatchF32:
    """Device-resident image pool for the served stream (sizes as the batch)."""
    return batch_f32(n, seed, with_pixels=with_pixels)


@dataclass
class QuadMesh:
    """An unstructured-looking mesh: the cells of an nx x ny grid of quads,
    numbered by a random permutation, and one edge per pair of cells that
    share a face, listed in random order with its two cells in random
    order. Edge values are float64 draws."""
    ncells: int
    nedges: int
    edge_to_cells: np.ndarray  # int32 [nedges, 2]
    edge: np.ndarray           # float64 [nedges]
    cell: np.ndarray           # float64 [ncells], initial cell values


def quad_mesh(nx: int, ny: int, seed: int) -> QuadMesh:
    rng = np.random.default_rng(seed)
    perm = rng.permutation(nx * ny).astype(np.int64)
    ids = perm.reshape(ny, nx)
    horiz = np.stack([ids[:, :-1].reshape(-1), ids[:, 1:].reshape(-1)], axis=1)
    vert = np.stack([ids[:-1, :].reshape(-1), ids[1:, :].reshape(-1)], axis=1)
    e2c = np.concatenate([horiz, vert])
    e2c = e2c[rng.permutation(len(e2c))]
    flip = rng.random(len(e2c)) < 0.5
    e2c[flip] = e2c[flip][:, ::-1]
    edge = rng.standard_normal(len(e2c))
    cell = rng.standard_normal(nx * ny)
    return QuadMesh(nx * ny, len(e2c), np.ascontiguousarray(e2c, dtype=np.int32), edge, cell)


def config_mesh() -> QuadMesh:
    """2048 x 2048 quads: 4,194,304 cells and 8,384,512 edges, seed 6."""
    return quad_mesh(2048, 2048, 6)
