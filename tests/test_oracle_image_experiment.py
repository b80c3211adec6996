"""Pins of the zig-zag retention and SSIM oracle (Section 3.1's experiment).

The zig-zag order is pinned to the JPEG table (tests/golden/jpeg_zigzag_8x8.json)
and to the properties that define a zig-zag scan; SSIM is pinned to closed
forms, to an independent filtering routine (scipy), and to brute force.
"""
import json
import os

import numpy as np
import pytest
import scipy.signal

from oracle import adct_oracle as O
from oracle import image_experiment as E
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _jpeg():
    with open(os.path.join(GOLDEN, "jpeg_zigzag_8x8.json")) as f:
        return np.array(json.load(f)["index"])


# ---------------------------------------------------------------- zig-zag order
def test_8x8_order_is_the_jpeg_table():
    assert np.array_equal(E.zigzag_index(8), _jpeg())


def test_16x16_order_starts_as_jpeg():
    # diagonals u + v <= 7 are complete in both block sizes
    idx, jp = E.zigzag_index(16), _jpeg()
    for u in range(8):
        for v in range(8 - u):
            assert idx[u, v] == jp[u, v]


@pytest.mark.parametrize("n", [8, 16])
def test_order_is_a_scan(n):
    order = E.zigzag_order(n)
    assert sorted(order) == [(u, v) for u in range(n) for v in range(n)]
    for (u0, v0), (u1, v1) in zip(order, order[1:]):
        assert max(abs(u1 - u0), abs(v1 - v0)) == 1      # each step moves to a neighbour
        assert u1 + v1 >= u0 + v0                        # anti-diagonals in order
    idx = E.zigzag_index(n)
    assert np.all(idx + idx[::-1, ::-1] == n * n - 1)    # point symmetry of the scan


def test_masks():
    assert E.zigzag_mask(0).sum() == 0 and E.zigzag_mask(256).sum() == 256
    for r in (1, 3, 10, 100, 150, 255):
        assert E.zigzag_mask(r).sum() == r
    m3 = E.zigzag_mask(3)
    assert m3[0, 0] == m3[0, 1] == m3[1, 0] == 1 and m3.sum() == 3
    assert np.array_equal(E.zigzag_mask(1), O.zonal_mask(1))
    # the first k(k+1)/2 positions are the full triangle u + v < k
    for k in (1, 4, 9, 16):
        u, v = np.indices((16, 16))
        assert np.array_equal(E.zigzag_mask(k * (k + 1) // 2), ((u + v) < k).astype(np.int64))


def test_zigzag_reconstruction_special_cases():
    img = synth.ar1_image(41, 64, 80)
    assert np.array_equal(E.zigzag_reconstruct(img, 256), img)
    assert np.array_equal(E.zigzag_reconstruct(img, 1), O.zonal_reconstruct(img, 1))
    t = O.to_tiles(img).astype(np.int64)
    means = np.floor_divide(t.sum(axis=(1, 2)) + 128, 256)   # rounded block mean
    got = O.to_tiles(E.zigzag_reconstruct(img, 1)).astype(np.int64)
    assert np.all(got == means[:, None, None])


@pytest.mark.parametrize("r", [2, 6, 21, 50, 150])
def test_fixed_point_path_equals_real_valued_reconstruction(r):
    # 256 C-hat^T (mask . C-hat A C-hat^T) C-hat == T^T (mask . Y . W) T exactly
    img = synth.ar1_image(42 + r, 48, 64)
    R = O.from_tiles(O.reconstruct_fixed(E.zigzag(O.fwd2d(img), r)), 48, 64)
    real = E.zigzag_reconstruct_real(img, r)
    assert np.max(np.abs(R / 256.0 - real)) < 1e-9


def test_zigzag_prefix_never_beats_the_full_set():
    img = synth.ar1_image(43, 64, 64)
    errs = [O.sse(E.zigzag_reconstruct(img, r), img) for r in (1, 3, 10, 36, 136, 256)]
    assert errs[-1] == 0
    assert all(e > 0 for e in errs[:-1])


# ---------------------------------------------------------------- SSIM
def test_window():
    w = E.ssim_window()
    assert w.shape == (11, 11)
    assert abs(w.sum() - 1.0) < 1e-15
    assert np.allclose(w, w.T) and np.allclose(w, w[::-1, ::-1])
    g = w.sum(axis=1)
    assert np.allclose(np.outer(g, g), w, rtol=0, atol=1e-17)   # separable
    # a sampled Gaussian of standard deviation 1.5: g(k+1)/g(k) = exp(-(2k+1)/(2 sigma^2))
    for k in range(5, 10):
        assert abs(np.log(g[k] / g[k + 1]) - (2 * (k - 5) + 1) / (2 * 1.5 ** 2)) < 1e-12


def test_ssim_of_an_image_with_itself_is_one():
    img = synth.ar1_image(44, 40, 52)
    assert np.all(np.abs(E.ssim_map(img, img) - 1.0) < 1e-14)


def test_ssim_constant_images_closed_form():
    c1 = (0.01 * 255) ** 2
    for a, b in ((100, 120), (0, 255), (17, 17)):
        x = np.full((20, 24), a, np.uint8)
        y = np.full((20, 24), b, np.uint8)
        want = (2 * a * b + c1) / (a * a + b * b + c1)
        m = E.ssim_map(x, y)
        assert m.shape == (10, 14)
        assert np.allclose(m, want, rtol=1e-12, atol=0)


def test_ssim_scaled_image_closed_form():
    # y = k x: mu_y = k mu_x, s_yy = k^2 s_xx, s_xy = k s_xx in every window
    c1, c2 = (0.01 * 255) ** 2, (0.03 * 255) ** 2
    x = synth.ar1_image(45, 36, 40).astype(np.float64) / 2
    w = E.ssim_window()
    mx = scipy.signal.correlate2d(x, w, mode="valid")
    sxx = scipy.signal.correlate2d(x * x, w, mode="valid") - mx * mx
    for k in (0.5, 1.5, 2.0):
        want = ((2 * k * mx * mx + c1) * (2 * k * sxx + c2)) / (((1 + k * k) * mx * mx + c1) * ((1 + k * k) * sxx + c2))
        assert np.allclose(E.ssim_map(x, k * x), want, rtol=1e-10, atol=1e-12)


def test_ssim_map_against_scipy_filtering():
    a = synth.ar1_image(46, 30, 33).astype(np.float64)
    b = E.zigzag_reconstruct(synth.ar1_image(46, 32, 48), 10)[:30, :33].astype(np.float64)
    w = E.ssim_window()
    f = lambda z: scipy.signal.correlate2d(z, w, mode="valid")
    c1, c2 = (0.01 * 255) ** 2, (0.03 * 255) ** 2
    ma, mb = f(a), f(b)
    saa, sbb, sab = f(a * a) - ma * ma, f(b * b) - mb * mb, f(a * b) - ma * mb
    want = ((2 * ma * mb + c1) * (2 * sab + c2)) / ((ma * ma + mb * mb + c1) * (saa + sbb + c2))
    assert np.allclose(E.ssim_map(a, b), want, rtol=1e-10, atol=1e-12)


def test_ssim_brute_force_tiny():
    rng = np.random.default_rng(47)
    a = rng.integers(0, 256, (13, 12)).astype(np.float64)
    b = np.clip(a + rng.normal(0, 20, a.shape), 0, 255)
    w = E.ssim_window()
    c1, c2 = (0.01 * 255) ** 2, (0.03 * 255) ** 2
    got = E.ssim_map(a, b)
    assert got.shape == (3, 2)
    for i in range(3):
        for j in range(2):
            pa, pb = a[i:i + 11, j:j + 11], b[i:i + 11, j:j + 11]
            ma, mb = (w * pa).sum(), (w * pb).sum()
            va = (w * (pa - ma) ** 2).sum()
            vb = (w * (pb - mb) ** 2).sum()
            cab = (w * (pa - ma) * (pb - mb)).sum()
            want = (2 * ma * mb + c1) * (2 * cab + c2) / ((ma ** 2 + mb ** 2 + c1) * (va + vb + c2))
            assert abs(got[i, j] - want) < 1e-12


def test_ssim_symmetric_bounded_and_monotone_in_r():
    img = synth.ar1_image(48, 64, 64)
    rec = [E.zigzag_reconstruct(img, r) for r in (1, 6, 28, 120)]
    vals = [E.ssim(img, x) for x in rec]
    assert all(-1 <= v < 1 for v in vals)
    assert vals == sorted(vals)                          # more coefficients, more similar
    assert abs(E.ssim(img, rec[1]) - E.ssim(rec[1], img)) < 1e-15


def test_per_image_and_per_cost():
    a = np.concatenate([synth.ar1_image(49 + i, 32, 32) for i in range(3)])
    b = E.zigzag_reconstruct(a, 6)
    per = E.ssim_per_image(a, b, 32)
    assert per.shape == (3,)
    assert per[1] == E.ssim(a[32:64], b[32:64])
    assert E.ADDITIONS_PROPOSED == O.addition_count(O.stage_M1()) + O.addition_count(O.stage_M2()) + \
        O.addition_count(O.stage_M3()) + O.addition_count(O.stage_M4())
    assert E.per_additive_cost(22.0) == 22.0 / 44
