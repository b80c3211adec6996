"""Plain CPU oracle for the comparison transforms of Tables 1 and 2 run
through the codec of Section 3.1: the Walsh-Hadamard transform in natural
order (the WHT row of Table 2) and the exact DCT-II (the reference the
approximation targets), each with zonal (r x r) or zig-zag (first r)
retention.

TEST INFRASTRUCTURE ONLY: nothing in the product path imports this module.

* WHT: H16 with H[k][j] = (-1)^popcount(k & j) (Sylvester's natural order).
  H H^T = 16 I, so its orthonormal form is H / 4 and the weights that fold
  the normalisation into retention are all 1:  H^T (H X H^T) H = 256 X.
  The integer reconstruction is then floor((R + 128) / 256), R = H^T Z' H,
  exactly as for the proposed transform.  Its fast algorithm has four
  butterfly stages of 16 additions (64 in all).
* Exact DCT: C the orthonormal DCT-II; coefficients B = C A C^T, retention,
  X = C^T B C in float64, output clamp(floor(X + 1/2)) (the rounding of the
  integer paths, round half up).
"""
from __future__ import annotations

import numpy as np

from . import adct_oracle as O
from . import image_experiment as E
from . import metrics as M

N = O.N
ZONAL, ZIGZAG = 0, 1
ADDITIONS_WHT = 64


def wht_matrix() -> np.ndarray:
    """Natural-order Walsh-Hadamard matrix of order 16 (int64)."""
    k = np.arange(N)
    bits = np.vectorize(lambda v: bin(v).count("1"))(k[:, None] & k[None, :])
    return np.where(bits % 2 == 0, 1, -1).astype(np.int64)


def wht_stages() -> list[np.ndarray]:
    """The fast algorithm: butterflies (a + b, a - b) at strides 8, 4, 2, 1."""
    stages = []
    for s in (8, 4, 2, 1):
        B = np.zeros((N, N), dtype=np.int64)
        for i in range(N):
            if i & s:
                B[i, i - s], B[i, i] = 1, -1
            else:
                B[i, i], B[i, i + s] = 1, 1
        stages.append(B)
    return stages


def retention_mask(kind: int, r: int) -> np.ndarray:
    return O.zonal_mask(r) if kind == ZONAL else E.zigzag_mask(r)


def wht_fwd2d(img: np.ndarray) -> np.ndarray:
    H = wht_matrix()
    A = O.to_tiles(np.asarray(img).astype(np.int64))
    return np.einsum("ui,kij,vj->kuv", H, A, H, optimize=True)


def wht_reconstruct(img: np.ndarray, kind: int, r: int, lo: int = 0, hi: int = 255) -> np.ndarray:
    """Forward WHT, retention (weights 1), inverse, round/clamp."""
    H = wht_matrix()
    Z = wht_fwd2d(img) * retention_mask(kind, r)[None]
    R = np.einsum("ui,kuv,vj->kij", H, Z, H, optimize=True)
    out = O.from_tiles(O.round_clamp(R, lo, hi), *img.shape)
    return out.astype(np.uint8) if np.asarray(img).dtype == np.uint8 else out


def dct_reconstruct_real(img: np.ndarray, kind: int, r: int) -> np.ndarray:
    """C^T (mask . C A C^T) C per block, float64, unrounded."""
    C = M.dct_matrix(N)
    B = M.exact_dct2d_tiles(O.to_tiles(img)) * retention_mask(kind, r)[None]
    return O.from_tiles(np.einsum("ui,kuv,vj->kij", C, B, C, optimize=True), *img.shape)


def dct_reconstruct(img: np.ndarray, kind: int, r: int, lo: int = 0, hi: int = 255) -> np.ndarray:
    """The exact-DCT codec: real reconstruction rounded half up and clamped."""
    out = np.clip(np.floor(dct_reconstruct_real(img, kind, r) + 0.5), lo, hi).astype(np.int64)
    return out.astype(np.uint8) if np.asarray(img).dtype == np.uint8 else out
