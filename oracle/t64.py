"""Plain CPU oracle for a 64-point extension of the approximation and its
blockwise 64x64 codec.

TEST INFRASTRUCTURE ONLY: nothing in the product path imports this module.

Reading.  The conclusion (Section 5) names 32- and 64-point extensions by
the scaled construction of its reference [Jridi2015]; Section 2.1 builds T
from two instances of the 8-point approximation joined by the outer
butterfly M1 of Section 2.2.  The paper prints no 64-point matrix, so this
module repeats the construction once more on the 32-point extension of
oracle/t32.py:

  T64 = P64 . diag(T32, T32) . B64

- B64: output j (j < 32) is the folded sum x_j + x_{63-j}, output 32 + j the
  folded difference x_j - x_{63-j}.
- Each half goes through T32 (120 additions each).
- P64 interleaves the halves: coefficient 2k is row k of T32 on the sums,
  2k + 1 row k of T32 on the differences.

Every entry is 0 or +-1; T64 T64^T = 2 diag(d32_0, d32_0, d32_1, d32_1, ...)
with d32 the diagonal of T32 T32^T, so its entries are 16, 32 or 64 and S64
= diag(T64 T64^T)^(-1/2) orthogonalises T64; the fast algorithm costs
64 + 2 x 120 = 304 additions.

The codec mirrors the 32-point one with 64 in place of 32: W64 = 4096 /
(d_u d_v) is a power of two in {1, 2, 4, 8, 16}, reconstructions carry 12
fractional bits, clamp(floor((R + 2048) / 4096)).  Quantiser tables qs =
fp32(s_u s_v / Delta) and dqs = fp32(4096 Delta s_u s_v), rounding half away
from zero; levels saturated to int16 before they are stored or dequantised
(that acts only for int16 samples beyond +-255: |Y s_u s_v| <= 64 * 255 =
16320 and 1 / Delta < 1.6 keep residual and uint8 levels inside int16).

Parity unpinned for quality figures: the paper prints no PSNR or Table 2
measures for a 64-point transform.
"""
from __future__ import annotations

import numpy as np

from . import adct_oracle as O
from . import t32 as T32

N64 = 64
FRAC64 = 4096  # 2^12: fixed-point scale of the 64-point reconstruction


def butterfly_64() -> np.ndarray:
    """B64: folded sums x_j + x_{63-j} (rows 0..31), then folded differences
    x_j - x_{63-j} (rows 32..63)."""
    B = np.zeros((N64, N64), dtype=np.int64)
    for j in range(32):
        B[j, j], B[j, 63 - j] = 1, 1
        B[32 + j, j], B[32 + j, 63 - j] = 1, -1
    return B


def interleave_64() -> np.ndarray:
    """P64: output 2k takes input k (sum path), output 2k + 1 takes input
    32 + k (difference path)."""
    P = np.zeros((N64, N64), dtype=np.int64)
    for k in range(32):
        P[2 * k, k] = 1
        P[2 * k + 1, 32 + k] = 1
    return P


def transform_matrix_64() -> np.ndarray:
    """T64 = P64 diag(T32, T32) B64 (int64 64x64)."""
    t = T32.transform_matrix_32()
    return interleave_64() @ O._block_diag(t, t) @ butterfly_64()


def gram_diagonal_64() -> np.ndarray:
    t = transform_matrix_64()
    return np.diag(t @ t.T).astype(np.int64)


def scaling_vector_64() -> np.ndarray:
    return 1.0 / np.sqrt(gram_diagonal_64().astype(np.float64))


def orthogonal_approximation_64() -> np.ndarray:
    """C-hat_64 = S64 T64 (float64)."""
    return scaling_vector_64()[:, None] * transform_matrix_64().astype(np.float64)


def fast_forward_1d_64(x):
    """T64 x by the construction's steps: the butterfly B64 (64 additions),
    the 32-point fast algorithm on each half (120 each), the interleave.
    Returns (X, additions performed)."""
    v = np.asarray(x, dtype=np.int64)
    a, adds = O._apply_sparse(butterfly_64(), v)
    lo, n_lo = T32.fast_forward_1d_32(a[:32])
    hi, n_hi = T32.fast_forward_1d_32(a[32:])
    out = np.empty(N64, dtype=np.int64)
    out[0::2], out[1::2] = lo, hi
    return out, adds + n_lo + n_hi


def fast_inverse_1d_64(X):
    """T64^T X = B64^T diag(T32^T, T32^T) P64^T X, right to left.  Returns
    (x, additions performed)."""
    X = np.asarray(X, dtype=np.int64)
    lo, n_lo = T32.fast_inverse_1d_32(X[0::2])
    hi, n_hi = T32.fast_inverse_1d_32(X[1::2])
    x, adds = O._apply_sparse(butterfly_64().T, np.concatenate([lo, hi]))
    return x, adds + n_lo + n_hi


# ---- blockwise 2D on disjoint 64x64 blocks (Section 3.1 with 64 for 16) ----
def to_tiles64(img: np.ndarray) -> np.ndarray:
    H, W = img.shape
    if H % N64 or W % N64:
        raise ValueError("plane sides must be multiples of 64")
    return img.reshape(H // N64, N64, W // N64, N64).transpose(0, 2, 1, 3).reshape(-1, N64, N64)


def from_tiles64(tiles: np.ndarray, H: int, W: int) -> np.ndarray:
    return tiles.reshape(H // N64, W // N64, N64, N64).transpose(0, 2, 1, 3).reshape(H, W)


def fwd2d_64(img: np.ndarray) -> np.ndarray:
    """Y_k = T64 A_k T64^T per 64x64 block, exact int64, block-major."""
    T = transform_matrix_64()
    A = to_tiles64(np.asarray(img).astype(np.int64))
    return np.einsum("ui,kij,vj->kuv", T, A, T, optimize=True)


def inv2d_64(coef: np.ndarray) -> np.ndarray:
    """T64^T Y_k T64 per block (un-normalised, like the 16-point inv2d)."""
    T = transform_matrix_64()
    Y = np.asarray(coef).astype(np.int64)
    return np.einsum("ui,kuv,vj->kij", T, Y, T, optimize=True)


def zonal_weights_64() -> np.ndarray:
    d = gram_diagonal_64()
    W = FRAC64 // (d[:, None] * d[None, :])
    assert np.all(W * d[:, None] * d[None, :] == FRAC64)
    return W.astype(np.int64)


def zonal_mask_64(r: int) -> np.ndarray:
    k = np.arange(N64)
    return ((k[:, None] < r) & (k[None, :] < r)).astype(np.int64)


def zonal_64(coef: np.ndarray, r: int) -> np.ndarray:
    """Z' = (Y . mask_r) . W64 (12 fractional bits)."""
    return np.asarray(coef).astype(np.int64) * (zonal_mask_64(r) * zonal_weights_64())[None]


def round_clamp_64(R: np.ndarray, lo: int, hi: int) -> np.ndarray:
    """clamp(floor((R + 2048) / 4096), lo, hi)."""
    return np.clip(np.floor_divide(np.asarray(R, dtype=np.int64) + FRAC64 // 2, FRAC64), lo, hi)


def quant_tables_64(qp: int):
    """(qs, dqs) float32 64x64: fp32(s_u s_v / Delta), fp32(4096 Delta s_u s_v),
    computed in float64 and rounded once."""
    d = gram_diagonal_64().astype(np.float64)
    ss = 1.0 / np.sqrt(d[:, None] * d[None, :])
    delta = O.quant_step(qp)
    return (ss / delta).astype(np.float32), (float(FRAC64) * delta * ss).astype(np.float32)


def quantise_64(coef: np.ndarray, qp: int) -> np.ndarray:
    """Levels: fp32(Y) * qs in float32, rounded half away from zero, then
    saturated to int16 (the stored type)."""
    qs, _ = quant_tables_64(qp)
    v = np.asarray(coef).astype(np.float32) * qs[None]
    return np.clip(O.round_half_away(v.astype(np.float64)), -32768, 32767)


def dequantise_64(q: np.ndarray, qp: int) -> np.ndarray:
    """Z' = rnd(fp32(q) * dqs): 12 fractional bits."""
    _, dqs = quant_tables_64(qp)
    v = np.asarray(q).astype(np.float32) * dqs[None]
    return O.round_half_away(v.astype(np.float64))


def zonal_reconstruct_64(img: np.ndarray, r: int, lo: int = 0, hi: int = 255) -> np.ndarray:
    H, W = img.shape
    R = inv2d_64(zonal_64(fwd2d_64(img), r))
    return from_tiles64(round_clamp_64(R, lo, hi), H, W)


def quant_reconstruct_64(plane: np.ndarray, qp: int, lo: int = -255, hi: int = 255):
    """(levels, Z', output plane) of the quantising 64x64 codec."""
    H, W = plane.shape
    q = quantise_64(fwd2d_64(plane), qp)
    z = dequantise_64(q, qp)
    return q, z, from_tiles64(round_clamp_64(inv2d_64(z), lo, hi), H, W)
