"""Plain CPU oracle for mixed 8/16-point coding: the second scenario of the
paper's video experiment (Section 3.2), in which both the 8-point and the
16-point transforms of the codec are the approximations (T8 and T).

TEST INFRASTRUCTURE ONLY: nothing in the product path imports this module.

Reading.  The paper runs the scenario inside an HEVC encoder and does not
describe how that encoder chooses the transform size of a block.  Here the
choice is made per 16x16 region, by the Lagrangian rule such encoders use:

* the region is coded twice at the same QP: once as one 16x16 block with T
  (the codec of ``adct_oracle.quant_reconstruct``) and once as four 8x8
  blocks with T8 (the codec of ``t8.quant_reconstruct8``);
* each coding has a distortion D, the region's sum of squared errors after
  reconstruction, and a rate proxy R, its number of nonzero levels;
* the 8x8 coding is kept when D8 + lam R8 < D16 + lam R16 for the caller's
  integer lam >= 0; ties keep the 16x16 coding (one block, less side
  information).  Everything is integer, so the choice has one exact answer.

Outputs, per region k (block-major over the plane, like the 16-point levels):
split[k] (1 = four 8x8 blocks), the chosen levels in a 16x16 array, and the
reconstruction.  An 8x8 sub-block (a, b) of a split region (a the vertical
and b the horizontal index) puts its element (i, j) at [8a + i][8b + j].
"""
from __future__ import annotations

import numpy as np

from . import adct_oracle as O
from . import t8 as E8

N = O.N
ADDITIONS_16 = 44  # one 1D 16-point transform (Table 1)
ADDITIONS_8 = 14   # one 1D 8-point transform T8 (Section 2.1)


def _region_of_8x8_levels(q8: np.ndarray, H: int, W: int) -> np.ndarray:
    """8x8 block-major levels of a plane regrouped into 16x16 regions: the
    sub-block (a, b) of region (by, bx) is 8x8 block (2 by + a, 2 bx + b)."""
    b8 = q8.reshape(H // 8, W // 8, 8, 8)
    nby, nbx = H // N, W // N
    out = np.empty((nby * nbx, N, N), dtype=q8.dtype)
    for by in range(nby):
        for bx in range(nbx):
            k = by * nbx + bx
            for a in range(2):
                for b in range(2):
                    out[k, 8 * a:8 * a + 8, 8 * b:8 * b + 8] = b8[2 * by + a, 2 * bx + b]
    return out


def region_costs(plane: np.ndarray, qp: int, lo: int, hi: int) -> dict:
    """Both codings of every region: levels, reconstruction, D and R."""
    plane = np.asarray(plane)
    H, W = plane.shape
    x = plane.astype(np.int64)
    q16, _, out16 = O.quant_reconstruct(x, qp, lo, hi)
    q8, out8 = E8.quant_reconstruct8(x, qp, lo, hi)
    d16 = O.to_tiles((out16 - x) ** 2).sum(axis=(1, 2))
    d8 = O.to_tiles((out8 - x) ** 2).sum(axis=(1, 2))
    q8r = _region_of_8x8_levels(q8, H, W)
    return {
        "q16": q16, "out16": out16, "D16": d16, "R16": (q16 != 0).sum(axis=(1, 2)),
        "q8": q8r, "out8": out8, "D8": d8, "R8": (q8r != 0).sum(axis=(1, 2)),
    }


def keep_8x8(j16: np.ndarray, j8: np.ndarray) -> np.ndarray:
    """The decision: the 8x8 coding only when strictly cheaper."""
    return j8 < j16


def mixed_encode(plane: np.ndarray, qp: int, lam: int, lo: int = -255, hi: int = 255):
    """Returns (split uint8 [nreg], levels int64 [nreg, 16, 16], output plane
    int64 [H, W])."""
    if lam < 0:
        raise ValueError("lam must be >= 0")
    H, W = np.asarray(plane).shape
    c = region_costs(plane, qp, lo, hi)
    j16 = c["D16"] + lam * c["R16"]
    j8 = c["D8"] + lam * c["R8"]
    split = keep_8x8(j16, j8).astype(np.uint8)
    levels = np.where(split[:, None, None] == 1, c["q8"], c["q16"])
    t16 = O.to_tiles(c["out16"])
    t8 = O.to_tiles(c["out8"])
    out = O.from_tiles(np.where(split[:, None, None] == 1, t8, t16), H, W)
    return split, levels, out


def mixed_decode(split: np.ndarray, levels: np.ndarray, qp: int, H: int, W: int,
                 lo: int = -255, hi: int = 255) -> np.ndarray:
    """The decoder side: dequantise and invert each region with the transform
    its flag names (for the 8x8 case, each sub-block on its own)."""
    out = np.empty((H, W), dtype=np.int64)
    nbx = W // N
    for k in range(len(split)):
        by, bx = divmod(k, nbx)
        if split[k]:
            blk = np.empty((N, N), dtype=np.int64)
            for a in range(2):
                for b in range(2):
                    q = levels[k, 8 * a:8 * a + 8, 8 * b:8 * b + 8][None]
                    R = E8.inv2d8(E8.dequantise8(q, qp))
                    blk[8 * a:8 * a + 8, 8 * b:8 * b + 8] = E8.round_clamp8(R, lo, hi)[0]
        else:
            R = O.reconstruct_fixed(O.dequantise(levels[k][None], qp))
            blk = O.round_clamp(R, lo, hi)[0]
        out[N * by:N * by + N, N * bx:N * bx + N] = blk
    return out


def sse_per_image(out: np.ndarray, plane: np.ndarray, image_height: int) -> np.ndarray:
    d = (np.asarray(out, dtype=np.int64) - np.asarray(plane, dtype=np.int64)) ** 2
    return d.reshape(-1, image_height, d.shape[1]).sum(axis=(1, 2))


def decoder_additions(split: np.ndarray) -> int:
    """Additions of the decoder's 2D inverse transforms: 2 x 16 x 44 for a
    16x16 region, 4 x 2 x 8 x 14 for a split one."""
    s = np.asarray(split, dtype=np.int64)
    return int(((1 - s) * 2 * N * ADDITIONS_16 + s * 4 * 2 * 8 * ADDITIONS_8).sum())
