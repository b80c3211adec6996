"""Plain CPU oracle for the 8-point approximate DCT T8 and its blockwise 8x8
codec (the 8-point half of the paper's second video scenario, Section 3.2).

TEST INFRASTRUCTURE ONLY: nothing in the product path imports this module.

Reading.  The paper builds T from two instances of the 8-point approximation
T8 (Section 2.1) but prints T only.  The even-indexed rows of T are symmetric
(T[2k, j] = T[2k, 15 - j]), so they act on the folded sums x_j + x_{15-j}
alone, and in the factorisation of Section 2.2 the even outputs of
P2 M4 M3 M2 P1 depend only on the first half of M1's output.  That block is
the sum-path instance of T8:  T8[k, j] = T[2k, j], j < 8.  Its fast
algorithm is the top-left 8x8 blocks of M2, M3 and M4 (8 + 4 + 2 = 14
additions, the count the paper gives for T8), followed by the even rows of
P2.

Everything else mirrors the 16-point codec with 8 in place of 16: S8 =
diag(T8 T8^T)^(-1/2); zonal weights W8 = 64 / (d_u d_v) (6 fractional
bits, since max d_u d_v = 64); quantiser tables qs = fp32(s_u s_v / Delta),
dqs = fp32(64 Delta s_u s_v); reconstruction clamp(floor((R + 32) / 64)).
"""
from __future__ import annotations

import numpy as np

from . import adct_oracle as O

N8 = 8
FRAC8 = 64  # 2^6: fixed-point scale of the 8-point reconstruction


def transform_matrix_8() -> np.ndarray:
    """T8: the left halves of the even-indexed rows of T (int64 8x8)."""
    return O.transform_matrix()[0::2, :N8].copy()


def gram_diagonal_8() -> np.ndarray:
    T8 = transform_matrix_8()
    return np.diag(T8 @ T8.T).astype(np.int64)


def scaling_vector_8() -> np.ndarray:
    return 1.0 / np.sqrt(gram_diagonal_8().astype(np.float64))


def orthogonal_approximation_8() -> np.ndarray:
    return scaling_vector_8()[:, None] * transform_matrix_8().astype(np.float64)


def even_path_stages():
    """The 8-point stages of Section 2.2's factorisation in application
    order: top-left blocks of M2, M3, M4, then the reordering that P2 applies
    to the even outputs."""
    st = dict(O.factorisation_stages())
    P2 = st["P2"]
    # row k of the reordering takes the even output 2k of P2
    R = np.zeros((N8, N8), dtype=np.int64)
    for k in range(N8):
        src = int(np.argmax(P2[2 * k]))
        R[k, src] = 1
    return [("M2", st["M2"][:N8, :N8]), ("M3", st["M3"][:N8, :N8]), ("M4", st["M4"][:N8, :N8]), ("P2even", R)]


def fast_forward_1d_8(x):
    """T8 x through the even-path stages."""
    v = np.asarray(x, dtype=np.int64)
    for _, M in even_path_stages():
        v = M @ v
    return v


def to_tiles8(img: np.ndarray) -> np.ndarray:
    H, W = img.shape
    if H % N8 or W % N8:
        raise ValueError("plane sides must be multiples of 8")
    return img.reshape(H // N8, N8, W // N8, N8).transpose(0, 2, 1, 3).reshape(-1, N8, N8)


def from_tiles8(tiles: np.ndarray, H: int, W: int) -> np.ndarray:
    return tiles.reshape(H // N8, W // N8, N8, N8).transpose(0, 2, 1, 3).reshape(H, W)


def fwd2d8(img: np.ndarray) -> np.ndarray:
    """Y_k = T8 A_k T8^T for every 8x8 block, exact int64, block-major."""
    T8 = transform_matrix_8()
    A = to_tiles8(np.asarray(img).astype(np.int64))
    return np.einsum("ui,kij,vj->kuv", T8, A, T8, optimize=True)


def inv2d8(coef: np.ndarray) -> np.ndarray:
    """T8^T Y_k T8 for every block."""
    T8 = transform_matrix_8()
    Y = np.asarray(coef).astype(np.int64)
    return np.einsum("ui,kuv,vj->kij", T8, Y, T8, optimize=True)


def zonal_mask_8(r: int) -> np.ndarray:
    k = np.arange(N8)
    return ((k[:, None] < r) & (k[None, :] < r)).astype(np.int64)


def zonal_weights_8() -> np.ndarray:
    d = gram_diagonal_8()
    W = FRAC8 // (d[:, None] * d[None, :])
    assert np.all(W * d[:, None] * d[None, :] == FRAC8)
    return W.astype(np.int64)


def zonal8(coef: np.ndarray, r: int) -> np.ndarray:
    """Z' = (Y . mask_r) . W8, 6 fractional bits."""
    return np.asarray(coef).astype(np.int64) * (zonal_mask_8(r) * zonal_weights_8())[None]


def round_clamp8(R: np.ndarray, lo: int, hi: int) -> np.ndarray:
    """clamp(floor((R + 32) / 64), lo, hi)."""
    return np.clip(np.floor_divide(np.asarray(R, dtype=np.int64) + FRAC8 // 2, FRAC8), lo, hi)


def zonal_reconstruct8(img: np.ndarray, r: int, lo: int = 0, hi: int = 255) -> np.ndarray:
    H, W = img.shape
    out = from_tiles8(round_clamp8(inv2d8(zonal8(fwd2d8(img), r)), lo, hi), H, W)
    return out.astype(np.uint8) if np.asarray(img).dtype == np.uint8 else out


def quant_tables_8(qp: int):
    """(qs, dqs) float32 8x8: fp32(s_u s_v / Delta), fp32(64 Delta s_u s_v)."""
    d = gram_diagonal_8().astype(np.float64)
    ss = 1.0 / np.sqrt(d[:, None] * d[None, :])
    delta = O.quant_step(qp)
    return (ss / delta).astype(np.float32), (FRAC8 * delta * ss).astype(np.float32)


def quantise8(coef: np.ndarray, qp: int) -> np.ndarray:
    """Levels with the decision in fp32 (as the 16-point quantiser)."""
    qs, _ = quant_tables_8(qp)
    v = np.asarray(coef).astype(np.float32) * qs[None]
    return O.round_half_away(v.astype(np.float64))


def dequantise8(q: np.ndarray, qp: int) -> np.ndarray:
    _, dqs = quant_tables_8(qp)
    v = np.asarray(q).astype(np.float32) * dqs[None]
    return O.round_half_away(v.astype(np.float64))


def quant_reconstruct8(plane: np.ndarray, qp: int, lo: int = -255, hi: int = 255):
    """Forward, quantise, dequantise, inverse, round/clamp of one plane with
    8x8 blocks.  Returns (levels, output plane)."""
    H, W = plane.shape
    q = quantise8(fwd2d8(plane), qp)
    out = from_tiles8(round_clamp8(inv2d8(dequantise8(q, qp)), lo, hi), H, W)
    return q, out
