"""Pins of the comparison-transform oracle (WHT and exact DCT codecs)."""
import numpy as np
import pytest
import scipy.fft
import scipy.linalg

from oracle import adct_oracle as O
from oracle import comparison as CMP
from oracle import metrics as M
import synth


def test_wht_is_the_natural_order_hadamard():
    H = CMP.wht_matrix()
    assert np.array_equal(H, scipy.linalg.hadamard(16))
    assert np.array_equal(H @ H.T, 16 * np.eye(16, dtype=np.int64))


def test_wht_fast_algorithm_has_64_additions():
    P = np.eye(16, dtype=np.int64)
    for B in CMP.wht_stages():
        P = B @ P
    assert np.array_equal(P, CMP.wht_matrix())
    assert sum(O.addition_count(B) for B in CMP.wht_stages()) == CMP.ADDITIONS_WHT == 64


def test_wht_roundtrip_is_256X_and_full_keep_is_lossless():
    rng = np.random.default_rng(9)
    X = rng.integers(0, 256, size=(32, 48)).astype(np.uint8)
    H = CMP.wht_matrix()
    Y = CMP.wht_fwd2d(X)
    R = np.einsum("ui,kuv,vj->kij", H, Y, H)
    assert np.array_equal(R, 256 * O.to_tiles(X.astype(np.int64)))
    assert np.array_equal(CMP.wht_reconstruct(X, CMP.ZONAL, 16), X)
    assert np.array_equal(CMP.wht_reconstruct(X, CMP.ZIGZAG, 256), X)


def test_wht_dc_only_is_the_rounded_mean():
    img = synth.ar1_image(90, 32, 32)
    t = O.to_tiles(img).astype(np.int64)
    means = np.floor_divide(t.sum(axis=(1, 2)) + 128, 256)
    got = O.to_tiles(CMP.wht_reconstruct(img, CMP.ZONAL, 1)).astype(np.int64)
    assert np.all(got == means[:, None, None])


def test_dct_coefficients_against_scipy():
    img = synth.ar1_image(91, 48, 32).astype(np.float64)
    B = M.exact_dct2d_tiles(O.to_tiles(img))
    want = np.stack([scipy.fft.dctn(t, norm="ortho") for t in O.to_tiles(img)])
    assert np.allclose(B, want, atol=1e-9)


def test_dct_reconstruction_special_cases():
    img = synth.ar1_image(92, 32, 48)
    assert np.array_equal(CMP.dct_reconstruct(img, CMP.ZONAL, 16), img)
    t = O.to_tiles(img).astype(np.float64)
    means = np.clip(np.floor(t.mean(axis=(1, 2)) + 0.5), 0, 255)
    got = O.to_tiles(CMP.dct_reconstruct(img, CMP.ZIGZAG, 1)).astype(np.float64)
    assert np.all(got == means[:, None, None])


def test_quality_order_dct_beats_proposed_beats_wht():
    # the exact DCT compacts energy best, the WHT worst (Table 2's coding gain order)
    img = synth.ar1_batch(4, 64, 64)
    for kind, r in ((CMP.ZONAL, 4), (CMP.ZIGZAG, 21)):
        e_dct = O.sse(CMP.dct_reconstruct(img, kind, r), img)
        e_wht = O.sse(CMP.wht_reconstruct(img, kind, r), img)
        from oracle import image_experiment as E
        e_t = O.sse(O.zonal_reconstruct(img, r) if kind == CMP.ZONAL else E.zigzag_reconstruct(img, r), img)
        assert e_dct < e_t < e_wht, (kind, e_dct, e_t, e_wht)
