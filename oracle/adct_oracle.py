"""Plain CPU oracle: the 16-point approximate DCT and its blockwise 2D codec.

TEST INFRASTRUCTURE ONLY -- see the package docstring.  Nothing in the
product path imports this module.

Every function states the passage of the paper it follows.  The integer
transforms are written as their plain definition (dense matrix products in
exact int64); the fast algorithm of Section 2.2 is written as the sequence of
sparse stage matrices applied in the paper's order, so that both can be
checked against each other and against the paper by eye.

Readings of the paper that this module fixes (where the text is silent or
ambiguous) are listed in the module-level constants' comments and in the
function docstrings that use them.
"""
from __future__ import annotations

import math

import numpy as np

N = 16  # transform length (Section 2.1)

# --------------------------------------------------------------------------
# Section 2.1: the transformation matrix T, entries in {0, +1, -1}.
# Transcribed row by row from the displayed matrix.
# --------------------------------------------------------------------------
_T_ROWS = (
    "+ + + + + + + + + + + + + + + +",
    "+ + + + + + + + - - - - - - - -",
    "+ 0 0 0 0 0 0 - - 0 0 0 0 0 0 +",
    "+ + 0 0 0 0 - - + + 0 0 0 0 - -",
    "+ 0 0 - - 0 0 + + 0 0 - - 0 0 +",
    "+ + - - - - + + - - + + + + - -",
    "0 0 - 0 0 + 0 0 0 0 + 0 0 - 0 0",
    "0 0 0 0 0 0 - + - + 0 0 0 0 0 0",
    "+ - - + + - - + + - - + + - - +",
    "0 0 - + 0 0 0 0 0 0 0 0 - + 0 0",
    "0 - 0 0 0 0 + 0 0 + 0 0 0 0 - 0",
    "0 0 + + - - 0 0 0 0 + + - - 0 0",
    "0 - + 0 0 + - 0 0 - + 0 0 + - 0",
    "+ - 0 0 0 0 0 0 0 0 0 0 0 0 + -",
    "0 0 0 - + 0 0 0 0 0 0 + - 0 0 0",
    "0 0 0 0 - + 0 0 0 0 - + 0 0 0 0",
)
_SYM = {"+": 1, "-": -1, "0": 0}


def transform_matrix() -> np.ndarray:
    """T of Section 2.1 as an int64 16x16 array (rows = output frequency)."""
    return np.array([[_SYM[c] for c in row.split()] for row in _T_ROWS], dtype=np.int64)


# Section 2.1: the printed orthogonalising diagonal,
#   S = 1/4 * diag(1, 1, 2, sqrt2, sqrt2, 1, 2, 2, 1, 2, 2, sqrt2, sqrt2, 2, 2, 2).
# Encoded as (factor, uses_sqrt2) so that the printed values are kept apart
# from anything computed from T.
_S_PRINTED = (
    (1, False), (1, False), (2, False), (1, True), (1, True), (1, False),
    (2, False), (2, False), (1, False), (2, False), (2, False), (1, True),
    (1, True), (2, False), (2, False), (2, False),
)


def printed_scaling() -> np.ndarray:
    """The diagonal of S exactly as printed in Section 2.1 (float64)."""
    return np.array([f * (math.sqrt(2.0) if r2 else 1.0) / 4.0 for f, r2 in _S_PRINTED])


def gram_diagonal() -> np.ndarray:
    """d = diag(T T^T) as int64 (Section 2.1: S = sqrt((T T^T)^-1))."""
    T = transform_matrix()
    return np.diag(T @ T.T).copy()


def scaling_vector() -> np.ndarray:
    """s_k = 1/sqrt(d_k), the diagonal of S computed from T (Section 2.1)."""
    return 1.0 / np.sqrt(gram_diagonal().astype(np.float64))


def orthogonal_approximation() -> np.ndarray:
    """C-hat = S T, the orthonormal approximate DCT (Section 2.1)."""
    return scaling_vector()[:, None] * transform_matrix().astype(np.float64)


# --------------------------------------------------------------------------
# Section 2.2: sparse factorisation  T = P2 M4 M3 M2 P1 M1.
# --------------------------------------------------------------------------
def counter_identity(n: int) -> np.ndarray:
    """The order-n counter-identity (ones on the anti-diagonal), Section 2.2."""
    return np.fliplr(np.eye(n, dtype=np.int64))


def _butterfly(n: int) -> np.ndarray:
    """The block [[I_{n/2}, J_{n/2}], [J_{n/2}, -I_{n/2}]] used by M1, M2, M3."""
    h = n // 2
    I, J = np.eye(h, dtype=np.int64), counter_identity(h)
    return np.block([[I, J], [J, -I]])


def _block_diag(*blocks: np.ndarray) -> np.ndarray:
    n = sum(b.shape[0] for b in blocks)
    out = np.zeros((n, n), dtype=np.int64)
    k = 0
    for b in blocks:
        m = b.shape[0]
        out[k:k + m, k:k + m] = b
        k += m
    return out


def stage_M1() -> np.ndarray:
    return _butterfly(16)


def stage_M2() -> np.ndarray:
    return _block_diag(_butterfly(8), _butterfly(8))


def stage_M3() -> np.ndarray:
    mI4 = -np.eye(4, dtype=np.int64)
    return _block_diag(_butterfly(4), mI4, _butterfly(4), mI4)


def stage_M4() -> np.ndarray:
    a = np.array([[1, 1, 0], [1, -1, 0], [0, 0, -1]], dtype=np.int64)
    b = np.array([[-1, 0, 0], [0, 1, 1], [0, 1, -1]], dtype=np.int64)
    c = np.array([[1, 0], [0, -1]], dtype=np.int64)
    return _block_diag(a, np.eye(4, dtype=np.int64), b, -np.eye(4, dtype=np.int64), c)


# Cycle notation of Section 2.2, 1-based.  The paper closes each cycle by
# repeating its first element ("(10 12 16 10)"); that repetition is dropped.
P1_CYCLES = ((10, 12, 16), (11, 13, 15))
P2_CYCLES = ((2, 9), (3, 8, 16, 15, 5, 4, 12, 11, 7, 6, 10, 14, 13))


def permutation_from_cycles(cycles, n: int = N, convention: str = "row_takes_successor") -> np.ndarray:
    """Permutation matrix for cycles given in 1-based notation.

    Reading (the paper gives only the cycles): row i of P has its one in
    column sigma(i), sigma mapping each element to its successor in its
    cycle, so (P v)_i = v_sigma(i).  The other conventions are available for
    the test that shows this is the only one under which the factorisation
    reproduces T.
    """
    sigma = list(range(n))
    for cyc in cycles:
        for k, a in enumerate(cyc):
            sigma[a - 1] = cyc[(k + 1) % len(cyc)] - 1
    P = np.zeros((n, n), dtype=np.int64)
    for i in range(n):
        if convention == "row_takes_successor":
            P[i, sigma[i]] = 1
        elif convention == "successor_takes_row":
            P[sigma[i], i] = 1
        else:
            raise ValueError(convention)
    return P


def factorisation_stages(p_convention: str = "row_takes_successor"):
    """The stages in application order: M1, P1, M2, M3, M4, P2 (Section 2.2)."""
    P1 = permutation_from_cycles(P1_CYCLES, convention=p_convention)
    P2 = permutation_from_cycles(P2_CYCLES, convention=p_convention)
    return [("M1", stage_M1()), ("P1", P1), ("M2", stage_M2()),
            ("M3", stage_M3()), ("M4", stage_M4()), ("P2", P2)]


def factorised_product(p_convention: str = "row_takes_successor") -> np.ndarray:
    """P2 M4 M3 M2 P1 M1 multiplied out (Section 2.2)."""
    out = np.eye(N, dtype=np.int64)
    for _, M in factorisation_stages(p_convention):
        out = M @ out
    return out


def addition_count(M: np.ndarray) -> int:
    """Two-input additions needed to apply M directly: each output row that
    combines k > 1 non-zero {+-1} terms costs k-1 additions/subtractions; sign
    changes alone cost none (Section 2.2: 112 for T, 44 for the factors)."""
    nnz = np.count_nonzero(M, axis=1)
    return int(np.sum(np.maximum(nnz - 1, 0)))


def _apply_sparse(M: np.ndarray, v: np.ndarray):
    """Apply one {0,+-1} stage matrix to v by explicit signed accumulation,
    counting the two-input additions actually performed."""
    out = np.zeros_like(v)
    adds = 0
    for i in range(M.shape[0]):
        terms = [(int(M[i, j]), v[j]) for j in range(M.shape[1]) if M[i, j] != 0]
        acc = terms[0][0] * terms[0][1]
        for sgn, val in terms[1:]:
            acc = acc + sgn * val
            adds += 1
        out[i] = acc
    return out, adds


def fast_forward_1d(x):
    """X = T x by the Section 2.2 fast algorithm: the sparse stages applied in
    the order M1, P1, M2, M3, M4, P2.  Returns (X, additions performed)."""
    v = np.asarray(x, dtype=np.int64).copy()
    total = 0
    for _, M in factorisation_stages():
        v, a = _apply_sparse(M, v)
        total += a
    return v, total


def fast_inverse_1d(X):
    """x = T^T X through the transposed factorisation
    T^T = M1^T P1^T M2^T M3^T M4^T P2^T, applied right to left (Section 2.2,
    every M_i is symmetric).  Returns (x, additions performed)."""
    v = np.asarray(X, dtype=np.int64).copy()
    total = 0
    for _, M in reversed(factorisation_stages()):
        v, a = _apply_sparse(M.T, v)
        total += a
    return v, total


# --------------------------------------------------------------------------
# Section 3.1: blockwise 2D application on disjoint 16x16 blocks.
# Coefficient arrays are block-major [tile][u][v], tiles in raster order
# (tile = by * (W/16) + bx), u = vertical and v = horizontal frequency.
# --------------------------------------------------------------------------
def to_tiles(img: np.ndarray) -> np.ndarray:
    """Split an HxW plane into its disjoint 16x16 blocks, raster order."""
    H, W = img.shape
    if H % N or W % N:
        raise ValueError("plane sides must be multiples of 16")
    return img.reshape(H // N, N, W // N, N).transpose(0, 2, 1, 3).reshape(-1, N, N)


def from_tiles(tiles: np.ndarray, H: int, W: int) -> np.ndarray:
    """Inverse of to_tiles: reassemble raster-ordered blocks into a plane."""
    return tiles.reshape(H // N, W // N, N, N).transpose(0, 2, 1, 3).reshape(H, W)


def fwd2d(img: np.ndarray) -> np.ndarray:
    """Y_k = T A_k T^T for every block A_k (Section 3.1 with C-tilde = T).
    Exact int64, block-major output."""
    T = transform_matrix()
    A = to_tiles(np.asarray(img).astype(np.int64))
    return np.einsum("ui,kij,vj->kuv", T, A, T, optimize=True)


def inv2d(coef: np.ndarray) -> np.ndarray:
    """T^T Y_k T for every block (the un-normalised inverse of Section 3.1).
    Note T^T T is not diagonal, so this is not the inverse of fwd2d."""
    T = transform_matrix()
    Y = np.asarray(coef).astype(np.int64)
    return np.einsum("ui,kuv,vj->kij", T, Y, T, optimize=True)


def scale(coef: np.ndarray) -> np.ndarray:
    """B = S Y S, i.e. B_uv = Y_uv s_u s_v in float64: the coefficients of the
    orthonormal approximation C-hat A C-hat^T (Section 2.1)."""
    s = scaling_vector()
    return np.asarray(coef).astype(np.float64) * (s[:, None] * s[None, :])


def orthonormal_fwd2d(img: np.ndarray) -> np.ndarray:
    """C-hat A_k C-hat^T computed directly in float64 (Section 3.1)."""
    C = orthogonal_approximation()
    A = to_tiles(np.asarray(img).astype(np.float64))
    return np.einsum("ui,kij,vj->kuv", C, A, C, optimize=True)


# --------------------------------------------------------------------------
# Quantisation with S merged in (Section 2.1: S folds into the codec's
# quantisation step; Section 3.2: HEVC-style quantisation).
# Readings: uniform quantiser with step Delta = 2^((QP-4)/6), round half away
# from zero, no dead zone.  Tables are computed in float64 and rounded once
# to float32:  qs_uv = fp32(s_u s_v / Delta),  dqs_uv = fp32(256 Delta s_u s_v).
# --------------------------------------------------------------------------
def quant_step(qp: int) -> float:
    return float(np.exp2((qp - 4) / 6.0))


def quant_tables(qp: int):
    """(qs, dqs) as float32 16x16 arrays."""
    d = gram_diagonal().astype(np.float64)
    ss = 1.0 / np.sqrt(d[:, None] * d[None, :])  # s_u s_v
    delta = quant_step(qp)
    qs = (ss / delta).astype(np.float32)
    dqs = (256.0 * delta * ss).astype(np.float32)
    return qs, dqs


def round_half_away(v: np.ndarray) -> np.ndarray:
    """sgn(v) floor(|v| + 1/2), evaluated in float64 (exact for |v| < 2^52)."""
    v = np.asarray(v, dtype=np.float64)
    return (np.sign(v) * np.floor(np.abs(v) + 0.5)).astype(np.int64)


def quantise(coef: np.ndarray, qp: int) -> np.ndarray:
    """Quantisation levels with the decision taken in fp32: the product
    fp32(Y) * qs is formed in float32, then rounded half away from zero
    (exactly, in float64)."""
    qs, _ = quant_tables(qp)
    v = np.asarray(coef).astype(np.float32) * qs[None]
    return round_half_away(v.astype(np.float64))


def quantise_fp64(coef: np.ndarray, qp: int) -> tuple[np.ndarray, np.ndarray]:
    """Real-valued reference: v = Y s_u s_v / Delta in float64, rounded half
    away from zero.  Also returns v so tests can find near-ties."""
    s = scaling_vector()
    v = np.asarray(coef).astype(np.float64) * (s[:, None] * s[None, :]) / quant_step(qp)
    return round_half_away(v), v


def dequantise(q: np.ndarray, qp: int) -> np.ndarray:
    """Fixed-point dequantised coefficients Z' = rnd(fp32(q) * dqs) (int),
    with 8 fractional bits: Z' approximates 256 s_u s_v q Delta, so that
    T^T Z' T approximates 256 C-hat^T (q Delta) C-hat."""
    _, dqs = quant_tables(qp)
    v = np.asarray(q).astype(np.float32) * dqs[None]
    return round_half_away(v.astype(np.float64))


def dequantise_fp64(q: np.ndarray, qp: int) -> np.ndarray:
    """Real-valued dequantisation B-hat = q Delta (float64)."""
    return np.asarray(q).astype(np.float64) * quant_step(qp)


# --------------------------------------------------------------------------
# Section 3.1: zonal retention and reconstruction.
# Reading: the benchmark keeps the top-left r x r block of coefficients
# (u < r and v < r).  With C-tilde = C-hat = S T and S^2 = D^-1,
#   256 C-hat^T (mask . C-hat A C-hat^T) C-hat = T^T (mask . Y . W) T
# exactly, with W_uv = 256 / (d_u d_v) in {1, 2, 4, 8, 16}.
# --------------------------------------------------------------------------
def zonal_mask(r: int) -> np.ndarray:
    k = np.arange(N)
    return ((k[:, None] < r) & (k[None, :] < r)).astype(np.int64)


def zonal_weights() -> np.ndarray:
    d = gram_diagonal()
    W = 256 // (d[:, None] * d[None, :])
    assert np.all(W * d[:, None] * d[None, :] == 256)
    return W.astype(np.int64)


def zonal(coef: np.ndarray, r: int) -> np.ndarray:
    """Z' = (Y . mask_r) . W: fixed-point coefficients (8 fractional bits)."""
    return np.asarray(coef).astype(np.int64) * (zonal_mask(r) * zonal_weights())[None]


def reconstruct_fixed(zfix: np.ndarray) -> np.ndarray:
    """R = T^T Z' T (int64), 256 times the reconstructed block."""
    return inv2d(zfix)


def round_clamp(R: np.ndarray, lo: int, hi: int) -> np.ndarray:
    """Output = clamp(floor((R + 128) / 256), lo, hi): the real value R/256
    rounded half up, then clipped to the sample range."""
    return np.clip(np.floor_divide(np.asarray(R, dtype=np.int64) + 128, 256), lo, hi)


def zonal_reconstruct(img: np.ndarray, r: int) -> np.ndarray:
    """The JPEG-like experiment of Section 3.1 on one uint8 plane with the
    r x r zonal mask: forward, keep, inverse, round, reassemble."""
    H, W = img.shape
    R = reconstruct_fixed(zonal(fwd2d(img), r))
    return from_tiles(round_clamp(R, 0, 255), H, W).astype(np.uint8)


def zonal_reconstruct_real(img: np.ndarray, r: int) -> np.ndarray:
    """Real-valued reconstruction C-hat^T (mask . C-hat A C-hat^T) C-hat,
    unrounded, float64 (Section 3.1 with C-tilde = C-hat)."""
    C = orthogonal_approximation()
    B = orthonormal_fwd2d(img) * zonal_mask(r)[None]
    H, W = img.shape
    return from_tiles(np.einsum("ui,kuv,vj->kij", C, B, C, optimize=True), H, W)


def quant_reconstruct(plane: np.ndarray, qp: int, lo: int = -255, hi: int = 255):
    """Forward, quantise, dequantise (fixed point), inverse, round/clamp of one
    plane.  Returns (levels, Z', output plane)."""
    H, W = plane.shape
    q = quantise(fwd2d(plane), qp)
    z = dequantise(q, qp)
    out = from_tiles(round_clamp(reconstruct_fixed(z), lo, hi), H, W)
    return q, z, out


# --------------------------------------------------------------------------
# Quality measures (Section 3.1 PSNR; Section 3.2 per-plane PSNR).
# --------------------------------------------------------------------------
def sse(a: np.ndarray, b: np.ndarray) -> int:
    """Exact integer sum of squared differences."""
    d = np.asarray(a).astype(np.int64) - np.asarray(b).astype(np.int64)
    return int(np.sum(d * d))


def psnr(sse_value, npix, peak: float = 255.0) -> float:
    """10 log10(peak^2 npix / SSE); +inf when SSE is 0."""
    if sse_value == 0:
        return math.inf
    return 10.0 * math.log10(peak * peak * npix / float(sse_value))


def psnr_real(a_real: np.ndarray, ref: np.ndarray, peak: float = 255.0) -> float:
    """PSNR of a real-valued reconstruction against the reference plane."""
    mse = float(np.mean((np.asarray(a_real, np.float64) - np.asarray(ref, np.float64)) ** 2))
    return math.inf if mse == 0.0 else 10.0 * math.log10(peak * peak / mse)
