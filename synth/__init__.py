"""Seeded synthetic inputs shared by the tests, the smoke check and the
benchmark.

This module holds no arithmetic of the transform: only random draws and the
shapes, value distributions and size mixes of the workloads.  It stands in
for the paper's image bank (45 natural 512x512 8-bit grayscale images,
Section 3.1) and video set (CIF sequences coded by an HEVC encoder,
Section 3.2), neither of which is available: the first-order Markov field is
the image model the DCT is designed for (Section 1), and Laplacian residuals
are the usual model of motion-compensated prediction residuals.

All generators use numpy's PCG64 ``default_rng(seed)``.
"""
from __future__ import annotations

import numpy as np
from scipy.signal import lfilter

RHO = 0.95
SIGMA = 40.0
MEAN = 127.5

# Seed bases per workload.
SEED_SINGLE = 1
SEED_BATCH = 2_000_000
SEED_VIDEO = 3_000_000
SEED_UNEVEN_SIZES = 4_000_000
SEED_UNEVEN_CONTENT = 4_000_001
SEED_ARRIVALS = 5_000_000
SEED_REQ_SIZES = 5_000_001
SEED_REQ_CONTENT = 5_100_000


def _ar1_axis(w: np.ndarray, axis: int, rho: float) -> np.ndarray:
    """a_0 = w_0, a_j = rho a_{j-1} + sqrt(1 - rho^2) w_j along ``axis``."""
    c = np.sqrt(1.0 - rho * rho)
    w = np.array(w, dtype=np.float64, copy=True)
    idx = [slice(None)] * w.ndim
    idx[axis] = 0
    w[tuple(idx)] /= c
    return lfilter([c], [1.0, -rho], w, axis=axis)


def ar1_field(rng: np.random.Generator, h: int, w: int, rho: float = RHO) -> np.ndarray:
    """Unit-variance separable first-order Markov (AR(1)) field, float64."""
    z = rng.standard_normal((h, w))
    return _ar1_axis(_ar1_axis(z, 1, rho), 0, rho)


def ar1_image(seed: int, h: int, w: int, rho: float = RHO) -> np.ndarray:
    """uint8 image: clip(rint(127.5 + 40 * field), 0, 255)."""
    f = ar1_field(np.random.default_rng(seed), h, w, rho)
    return np.clip(np.rint(MEAN + SIGMA * f), 0, 255).astype(np.uint8)


def ar1_batch(n: int, h: int, w: int, seed_base: int = SEED_BATCH) -> np.ndarray:
    """n images stacked as one (n*h) x w plane; image i uses seed_base + i."""
    out = np.empty((n * h, w), dtype=np.uint8)
    for i in range(n):
        out[i * h:(i + 1) * h] = ar1_image(seed_base + i, h, w)
    return out


def laplacian_residual(seed: int, h: int, w: int, scale: float = 8.0) -> np.ndarray:
    """int16 residual plane: clip(rint(Laplace(0, scale)), -255, 255)."""
    rng = np.random.default_rng(seed)
    x = rng.laplace(0.0, scale, size=(h, w))
    return np.clip(np.rint(x), -255, 255).astype(np.int16)


def video_frame_planes(frame: int, width: int = 1920, height: int = 1088):
    """One 4:2:0 frame of residual planes (Y, U, V), each int16."""
    seed = SEED_VIDEO + frame
    y = laplacian_residual(seed * 3 + 0, height, width)
    u = laplacian_residual(seed * 3 + 1, height // 2, width // 2)
    v = laplacian_residual(seed * 3 + 2, height // 2, width // 2)
    return y, u, v


def uneven_sizes(n: int, lo: int = 64, hi: int = 2048, seed: int = SEED_UNEVEN_SIZES):
    """(h, w) pairs, each side uniform over the multiples of 16 in [lo, hi]."""
    rng = np.random.default_rng(seed)
    hw = 16 * rng.integers(lo // 16, hi // 16 + 1, size=(n, 2))
    return [(int(h), int(w)) for h, w in hw]


def crop_pool(n_pool: int = 16, side: int = 2048, seed: int = SEED_UNEVEN_CONTENT) -> np.ndarray:
    """A pool of AR(1) images from which uneven images are cropped, so that a
    multi-gigabyte batch is generated in seconds with the same statistics."""
    return np.stack([ar1_image(seed + i, side, side) for i in range(n_pool)])


def crop_from_pool(pool: np.ndarray, k: int, h: int, w: int, seed: int = SEED_UNEVEN_CONTENT) -> np.ndarray:
    """Image k of an uneven batch: an h x w crop of a seeded pool member."""
    rng = np.random.default_rng(seed + 1_000_000 + k)
    p = int(rng.integers(0, pool.shape[0]))
    y = int(rng.integers(0, pool.shape[1] - h + 1))
    x = int(rng.integers(0, pool.shape[2] - w + 1))
    return pool[p, y:y + h, x:x + w]


def poisson_arrivals(rate: float, n: int, seed: int = SEED_ARRIVALS) -> np.ndarray:
    """Arrival times (seconds, from 0) of a Poisson process of the given rate."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=n))


def request_sides(n: int, lo: int = 256, hi: int = 4096, seed: int = SEED_REQ_SIZES) -> np.ndarray:
    """Square request sides, log-uniform in [lo, hi], rounded to multiples of 16."""
    rng = np.random.default_rng(seed)
    u = rng.uniform(np.log(lo), np.log(hi), size=n)
    return (16 * np.clip(np.round(np.exp(u) / 16), lo // 16, hi // 16)).astype(np.int64)


def structured_tiles() -> np.ndarray:
    """Edge-case 16x16 uint8 tiles: constant 0 and 255, checkerboards and
    stripes of periods 1, 2, 4, 8 in both phases, and a ramp."""
    i = np.arange(16)
    out = [np.zeros((16, 16)), np.full((16, 16), 255)]
    for p in (1, 2, 4, 8):
        cb = ((i[:, None] // p + i[None, :] // p) % 2) * 255
        hs = ((i[:, None] // p) % 2) * 255 + 0 * i[None, :]
        vs = ((i[None, :] // p) % 2) * 255 + 0 * i[:, None]
        for t in (cb, hs, vs):
            out.append(t)
            out.append(255 - t)
    out.append(np.add.outer(i, i) * 8)
    return np.array(out).astype(np.uint8)


def random_binary_tiles(n: int, seed: int = 7, lo: int = 0, hi: int = 255) -> np.ndarray:
    """n tiles whose samples are each lo or hi at random (range extremes)."""
    rng = np.random.default_rng(seed)
    return np.where(rng.integers(0, 2, size=(n, 16, 16)) == 1, hi, lo)


def tiles_to_plane(tiles: np.ndarray, tiles_per_row: int) -> np.ndarray:
    """Lay out a stack of 16x16 tiles in raster order into a plane."""
    n = tiles.shape[0]
    rows = -(-n // tiles_per_row)
    pad = rows * tiles_per_row - n
    if pad:
        tiles = np.concatenate([tiles, np.zeros((pad, 16, 16), tiles.dtype)])
    return tiles.reshape(rows, tiles_per_row, 16, 16).transpose(0, 2, 1, 3).reshape(rows * 16, tiles_per_row * 16)
