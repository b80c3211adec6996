"""Plain CPU oracle for a 32-point extension of the approximation and its
blockwise 32x32 codec.

TEST INFRASTRUCTURE ONLY: nothing in the product path imports this module.

Reading.  The conclusion (Section 5) says the 16-point approach extends to 32
points by the scaled construction of its reference [Jridi2015], and Section
2.1 builds T itself from two instances of the 8-point approximation joined
by the outer butterfly M1 of Section 2.2.  The paper prints no 32-point
matrix, so this module takes the same construction one level up:

  T32 = P32 . diag(T, T) . B32

- B32 is the even/odd butterfly of length 32: output j (j < 16) is the
  folded sum x_j + x_{31-j}, output 16 + j the folded difference
  x_j - x_{31-j}.
- Each half goes through the 16-point T of Section 2.1 (44 additions each,
  by the factorisation of Section 2.2).
- P32 interleaves the halves: coefficient 2k is row k of T on the sums,
  coefficient 2k + 1 row k of T on the differences.  On the sums this is
  exactly the exact DCT's even/odd split (the even DCT-32 coefficients are
  the 16-point DCT of the folded sums); on the differences T stands in for
  the 16-point DCT-IV of the exact split, the same substitution of one
  approximation for both halves that Section 2.1 makes with T8.

Every entry is 0 or +-1, T32 T32^T = 2 diag(d_0, d_0, d_1, d_1, ...) with d
the diagonal of T T^T (so S32 = diag(T32 T32^T)^(-1/2) orthogonalises it as
S does T), and the fast algorithm costs 32 + 2 x 44 = 120 additions.

The codec mirrors the 16-point one with 32 in place of 16: the diagonal
entries are 8, 16 or 32, so W32 = 1024 / (d_u d_v) is a power of two in
{1, 2, 4, 8, 16} and reconstructions carry 10 fractional bits:
clamp(floor((R + 512) / 1024)).  Quantiser tables qs = fp32(s_u s_v / Delta)
and dqs = fp32(1024 Delta s_u s_v), rounding half away from zero as in the
16-point oracle.  Levels are the codec's stored type, int16: a level is
saturated to [-32768, 32767] before it is stored or dequantised.  For
uint8 samples or residuals within [-255, 255] that never acts (|Y s_u s_v|
<= 32 * 255 = 8160 and 1 / Delta < 1.6); for int16 samples up to 2047 it
can, below QP 10.

Parity unpinned for quality figures: the paper prints no PSNR or Table 2
measures for a 32-point transform.
"""
from __future__ import annotations

import numpy as np

from . import adct_oracle as O

N32 = 32
FRAC32 = 1024  # 2^10: fixed-point scale of the 32-point reconstruction


def butterfly_32() -> np.ndarray:
    """B32: folded sums x_j + x_{31-j} (rows 0..15), then folded differences
    x_j - x_{31-j} (rows 16..31)."""
    B = np.zeros((N32, N32), dtype=np.int64)
    for j in range(16):
        B[j, j], B[j, 31 - j] = 1, 1
        B[16 + j, j], B[16 + j, 31 - j] = 1, -1
    return B


def interleave_32() -> np.ndarray:
    """P32: output 2k takes input k (sum path), output 2k + 1 takes input
    16 + k (difference path)."""
    P = np.zeros((N32, N32), dtype=np.int64)
    for k in range(16):
        P[2 * k, k] = 1
        P[2 * k + 1, 16 + k] = 1
    return P


def transform_matrix_32() -> np.ndarray:
    """T32 = P32 diag(T, T) B32 (int64 32x32)."""
    T = O.transform_matrix()
    return interleave_32() @ O._block_diag(T, T) @ butterfly_32()


def gram_diagonal_32() -> np.ndarray:
    T32 = transform_matrix_32()
    return np.diag(T32 @ T32.T).astype(np.int64)


def scaling_vector_32() -> np.ndarray:
    return 1.0 / np.sqrt(gram_diagonal_32().astype(np.float64))


def orthogonal_approximation_32() -> np.ndarray:
    """C-hat_32 = S32 T32 (float64)."""
    return scaling_vector_32()[:, None] * transform_matrix_32().astype(np.float64)


def fast_forward_1d_32(x):
    """T32 x by the construction's steps: the butterfly B32 (32 additions),
    the Section 2.2 fast algorithm on each half (44 each), the interleave.
    Returns (X, additions performed)."""
    v = np.asarray(x, dtype=np.int64)
    a, adds = O._apply_sparse(butterfly_32(), v)
    lo, n_lo = O.fast_forward_1d(a[:16])
    hi, n_hi = O.fast_forward_1d(a[16:])
    out = np.empty(N32, dtype=np.int64)
    out[0::2], out[1::2] = lo, hi
    return out, adds + n_lo + n_hi


def fast_inverse_1d_32(X):
    """T32^T X = B32^T diag(T^T, T^T) P32^T X, right to left.  Returns
    (x, additions performed)."""
    X = np.asarray(X, dtype=np.int64)
    lo, n_lo = O.fast_inverse_1d(X[0::2])
    hi, n_hi = O.fast_inverse_1d(X[1::2])
    x, adds = O._apply_sparse(butterfly_32().T, np.concatenate([lo, hi]))
    return x, adds + n_lo + n_hi


# ---- blockwise 2D on disjoint 32x32 blocks (Section 3.1 with 32 for 16) ----
def to_tiles32(img: np.ndarray) -> np.ndarray:
    H, W = img.shape
    if H % N32 or W % N32:
        raise ValueError("plane sides must be multiples of 32")
    return img.reshape(H // N32, N32, W // N32, N32).transpose(0, 2, 1, 3).reshape(-1, N32, N32)


def from_tiles32(tiles: np.ndarray, H: int, W: int) -> np.ndarray:
    return tiles.reshape(H // N32, W // N32, N32, N32).transpose(0, 2, 1, 3).reshape(H, W)


def fwd2d_32(img: np.ndarray) -> np.ndarray:
    """Y_k = T32 A_k T32^T per 32x32 block, exact int64, block-major."""
    T = transform_matrix_32()
    A = to_tiles32(np.asarray(img).astype(np.int64))
    return np.einsum("ui,kij,vj->kuv", T, A, T, optimize=True)


def inv2d_32(coef: np.ndarray) -> np.ndarray:
    """T32^T Y_k T32 per block (un-normalised, like the 16-point inv2d)."""
    T = transform_matrix_32()
    Y = np.asarray(coef).astype(np.int64)
    return np.einsum("ui,kuv,vj->kij", T, Y, T, optimize=True)


def zonal_weights_32() -> np.ndarray:
    d = gram_diagonal_32()
    W = FRAC32 // (d[:, None] * d[None, :])
    assert np.all(W * d[:, None] * d[None, :] == FRAC32)
    return W.astype(np.int64)


def zonal_mask_32(r: int) -> np.ndarray:
    k = np.arange(N32)
    return ((k[:, None] < r) & (k[None, :] < r)).astype(np.int64)


def zonal_32(coef: np.ndarray, r: int) -> np.ndarray:
    """Z' = (Y . mask_r) . W32 (10 fractional bits)."""
    return np.asarray(coef).astype(np.int64) * (zonal_mask_32(r) * zonal_weights_32())[None]


def round_clamp_32(R: np.ndarray, lo: int, hi: int) -> np.ndarray:
    """clamp(floor((R + 512) / 1024), lo, hi)."""
    return np.clip(np.floor_divide(np.asarray(R, dtype=np.int64) + FRAC32 // 2, FRAC32), lo, hi)


def quant_tables_32(qp: int):
    """(qs, dqs) float32 32x32: fp32(s_u s_v / Delta), fp32(1024 Delta s_u s_v),
    computed in float64 and rounded once."""
    d = gram_diagonal_32().astype(np.float64)
    ss = 1.0 / np.sqrt(d[:, None] * d[None, :])
    delta = O.quant_step(qp)
    return (ss / delta).astype(np.float32), (float(FRAC32) * delta * ss).astype(np.float32)


def quantise_32(coef: np.ndarray, qp: int) -> np.ndarray:
    """Levels: fp32(Y) * qs in float32, rounded half away from zero, then
    saturated to int16 (the stored type)."""
    qs, _ = quant_tables_32(qp)
    v = np.asarray(coef).astype(np.float32) * qs[None]
    return np.clip(O.round_half_away(v.astype(np.float64)), -32768, 32767)


def dequantise_32(q: np.ndarray, qp: int) -> np.ndarray:
    """Z' = rnd(fp32(q) * dqs): 10 fractional bits."""
    _, dqs = quant_tables_32(qp)
    v = np.asarray(q).astype(np.float32) * dqs[None]
    return O.round_half_away(v.astype(np.float64))


def zonal_reconstruct_32(img: np.ndarray, r: int, lo: int = 0, hi: int = 255) -> np.ndarray:
    H, W = img.shape
    R = inv2d_32(zonal_32(fwd2d_32(img), r))
    return from_tiles32(round_clamp_32(R, lo, hi), H, W)


def quant_reconstruct_32(plane: np.ndarray, qp: int, lo: int = -255, hi: int = 255):
    """(levels, Z', output plane) of the quantising 32x32 codec."""
    H, W = plane.shape
    q = quantise_32(fwd2d_32(plane), qp)
    z = dequantise_32(q, qp)
    return q, z, from_tiles32(round_clamp_32(inv2d_32(z), lo, hi), H, W)
