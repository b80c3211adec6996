"""Exact DCT and the similarity / coding measures of Section 2.3 (Table 2).

TEST INFRASTRUCTURE ONLY -- see the package docstring.

The paper names the measures and their sources but prints no formulas.  The
definitions below are the standard ones from the transform-coding
literature; with them the "Proposed approx." row of Table 2 is reproduced to
every printed digit (the test-suite checks this), as are the Chen DCT and WHT
rows.

    d2   DCT distortion: 1 - ||diag(C A^T)||^2 / ||C A^T||_F^2
    eps  total error energy: pi * ||C - A||_F^2
    MSE  (1/N) tr((C - A) R (C - A)^T), R the Markov(rho) correlation matrix
    Cg   coding gain: 10 log10[(tr R / N) / prod_k (Rhat_kk ||g_k||^2)^(1/N)],
         Rhat = A R A^T and g_k the k-th column of A^-1
    eta  transform efficiency: 100 sum_k |Rhat_kk| / sum_kl |Rhat_kl|
"""
from __future__ import annotations

import numpy as np


def dct_matrix(n: int = 16) -> np.ndarray:
    """Orthonormal DCT-II: C_kj = a_k cos(pi (2j + 1) k / (2n)), a_0 = sqrt(1/n),
    a_k = sqrt(2/n) (the exact DCT the approximation targets, Section 1)."""
    k = np.arange(n)[:, None]
    j = np.arange(n)[None, :]
    C = np.sqrt(2.0 / n) * np.cos(np.pi * (2 * j + 1) * k / (2 * n))
    C[0, :] = np.sqrt(1.0 / n)
    return C


def markov_correlation(n: int = 16, rho: float = 0.95) -> np.ndarray:
    """First-order Markov correlation matrix R_ij = rho^|i-j| (Section 2.3)."""
    i = np.arange(n)
    return rho ** np.abs(i[:, None] - i[None, :]).astype(np.float64)


def dct_distortion(A: np.ndarray) -> float:
    M = dct_matrix(A.shape[0]) @ A.T
    return float(1.0 - np.sum(np.diag(M) ** 2) / np.sum(M ** 2))


def total_error_energy(A: np.ndarray) -> float:
    return float(np.pi * np.sum((dct_matrix(A.shape[0]) - A) ** 2))


def mse(A: np.ndarray, rho: float = 0.95) -> float:
    n = A.shape[0]
    E = dct_matrix(n) - A
    return float(np.trace(E @ markov_correlation(n, rho) @ E.T) / n)


def coding_gain(A: np.ndarray, rho: float = 0.95) -> float:
    n = A.shape[0]
    R = markov_correlation(n, rho)
    Rh = A @ R @ A.T
    g2 = np.sum(np.linalg.inv(A) ** 2, axis=0)
    geo = np.exp(np.mean(np.log(np.diag(Rh) * g2)))
    return float(10.0 * np.log10((np.trace(R) / n) / geo))


def transform_efficiency(A: np.ndarray, rho: float = 0.95) -> float:
    n = A.shape[0]
    Rh = A @ markov_correlation(n, rho) @ A.T
    return float(100.0 * np.sum(np.abs(np.diag(Rh))) / np.sum(np.abs(Rh)))


def table2_row(A: np.ndarray) -> dict:
    """The five Table 2 measures of a 16-point transform matrix A."""
    return {"d2": dct_distortion(A), "eps": total_error_energy(A), "mse": mse(A),
            "cg": coding_gain(A), "eta": transform_efficiency(A)}


def exact_dct2d_tiles(tiles: np.ndarray) -> np.ndarray:
    """C A_k C^T for every 16x16 block, float64 (the FP64 exact-DCT reference)."""
    C = dct_matrix(16)
    return np.einsum("ui,kij,vj->kuv", C, np.asarray(tiles, np.float64), C, optimize=True)


def coefficient_psnr(B: np.ndarray, B_ref: np.ndarray, peak: float = 255.0) -> float:
    """10 log10(peak^2 / mean((B - B_ref)^2)): PSNR of orthonormal coefficients
    against a reference set of coefficients.  With both transforms orthonormal
    this equals the pixel PSNR of decoding B with the reference inverse."""
    m = float(np.mean((np.asarray(B, np.float64) - np.asarray(B_ref, np.float64)) ** 2))
    return float("inf") if m == 0.0 else float(10.0 * np.log10(peak * peak / m))
