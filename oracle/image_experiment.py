"""Plain CPU oracle for the image experiment of Section 3.1 as the paper runs
it: zig-zag retention of the first r coefficients of every 16x16 block, and
the SSIM quality index the paper reports beside PSNR.

TEST INFRASTRUCTURE ONLY: nothing in the product path imports this module.

Readings (the paper names the zig-zag sequence and SSIM by citation only):

* Zig-zag order for 16x16 blocks: the JPEG order extended to 16x16.  Positions
  (u, v), u the vertical and v the horizontal frequency, are visited by
  anti-diagonal s = u + v; on odd s the row index u increases, on even s it
  decreases, so the order starts (0,0), (0,1), (1,0), (2,0), (1,1), (0,2) ...
  and restricted to u, v < 8 it is the 8x8 JPEG order.
* SSIM: the index of Wang, Bovik, Sheikh and Simoncelli (2004) with that
  paper's parameters: an 11x11 circular-symmetric Gaussian window with
  standard deviation 1.5 samples (normalised to unit sum), K1 = 0.01,
  K2 = 0.03, dynamic range L = 255, local statistics over every window that
  lies entirely inside the image, and the mean of the SSIM map as the index
  of the image (no downsampling step).
* "Per additive cost": the quality value divided by the additions of one
  16-point transform (44 for the proposed transform, Table 1).
"""
from __future__ import annotations

import numpy as np

from . import adct_oracle as O

N = O.N

SSIM_WINDOW = 11
SSIM_SIGMA = 1.5
SSIM_K1, SSIM_K2, SSIM_L = 0.01, 0.03, 255.0
ADDITIONS_PROPOSED = 44  # Table 1: additions of the proposed 16-point transform


# --------------------------------------------------------------------------
# Zig-zag retention (Section 3.1: "only the first r elements ... are retained")
# --------------------------------------------------------------------------
def zigzag_order(n: int = N) -> list[tuple[int, int]]:
    """Positions (u, v) of an n x n block in zig-zag order."""
    order = []
    for s in range(2 * n - 1):
        us = range(max(0, s - n + 1), min(s, n - 1) + 1)
        if s % 2 == 0:
            us = reversed(us)
        order.extend((u, s - u) for u in us)
    return order


def zigzag_index(n: int = N) -> np.ndarray:
    """n x n int64 array: the zig-zag rank of every position."""
    idx = np.empty((n, n), dtype=np.int64)
    for k, (u, v) in enumerate(zigzag_order(n)):
        idx[u, v] = k
    return idx


def zigzag_mask(r: int) -> np.ndarray:
    """1 on the first r positions of the zig-zag order (0 <= r <= 256)."""
    return (zigzag_index() < r).astype(np.int64)


def zigzag(coef: np.ndarray, r: int) -> np.ndarray:
    """Z' = (Y . zigzag_mask_r) . W: fixed-point coefficients with S folded in
    (the weights of the zonal reading, Section 3.1)."""
    return np.asarray(coef).astype(np.int64) * (zigzag_mask(r) * O.zonal_weights())[None]


def zigzag_reconstruct(img: np.ndarray, r: int, lo: int = 0, hi: int = 255) -> np.ndarray:
    """Forward, keep the first r zig-zag coefficients, inverse, round/clamp."""
    H, W = img.shape
    R = O.reconstruct_fixed(zigzag(O.fwd2d(img), r))
    out = O.from_tiles(O.round_clamp(R, lo, hi), H, W)
    return out.astype(np.uint8) if np.asarray(img).dtype == np.uint8 else out


def zigzag_reconstruct_real(img: np.ndarray, r: int) -> np.ndarray:
    """Real-valued C-hat^T (mask . C-hat A C-hat^T) C-hat, float64."""
    C = O.orthogonal_approximation()
    B = O.orthonormal_fwd2d(img) * zigzag_mask(r)[None]
    H, W = img.shape
    return O.from_tiles(np.einsum("ui,kuv,vj->kij", C, B, C, optimize=True), H, W)


# --------------------------------------------------------------------------
# SSIM (Wang et al. 2004), float64
# --------------------------------------------------------------------------
def ssim_window() -> np.ndarray:
    """The 11 x 11 Gaussian weights (standard deviation 1.5), unit sum."""
    k = np.arange(SSIM_WINDOW) - (SSIM_WINDOW - 1) / 2.0
    g = np.exp(-(k[:, None] ** 2 + k[None, :] ** 2) / (2.0 * SSIM_SIGMA ** 2))
    return g / g.sum()


def _local_mean(img: np.ndarray, w: np.ndarray) -> np.ndarray:
    """Weighted mean over every window entirely inside the image."""
    win = np.lib.stride_tricks.sliding_window_view(img, w.shape)
    return np.einsum("ijkl,kl->ij", win, w)


def ssim_map(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """SSIM at every window position: luminance, contrast and structure
    comparisons of the local Gaussian-weighted statistics."""
    x = np.asarray(a, dtype=np.float64)
    y = np.asarray(b, dtype=np.float64)
    w = ssim_window()
    c1 = (SSIM_K1 * SSIM_L) ** 2
    c2 = (SSIM_K2 * SSIM_L) ** 2
    mx, my = _local_mean(x, w), _local_mean(y, w)
    sxx = _local_mean(x * x, w) - mx * mx
    syy = _local_mean(y * y, w) - my * my
    sxy = _local_mean(x * y, w) - mx * my
    return ((2 * mx * my + c1) * (2 * sxy + c2)) / ((mx * mx + my * my + c1) * (sxx + syy + c2))


def ssim(a: np.ndarray, b: np.ndarray) -> float:
    """Mean SSIM of one image pair (the index of the image)."""
    return float(np.mean(ssim_map(a, b)))


def ssim_per_image(a: np.ndarray, b: np.ndarray, image_height: int) -> np.ndarray:
    """Mean SSIM of every image of two stacked planes."""
    n = a.shape[0] // image_height
    return np.array([ssim(a[i * image_height:(i + 1) * image_height], b[i * image_height:(i + 1) * image_height])
                     for i in range(n)])


def per_additive_cost(value: float, additions: int = ADDITIONS_PROPOSED) -> float:
    """A quality value per unit of additive cost (Section 3.1, Fig. 2)."""
    return value / additions
