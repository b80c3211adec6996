"""Planted mistakes in the oracle must each fail at least one pin.

Each case patches one plausible error into the oracle (on the CPU only) and
runs the pins that should catch it.
"""
import numpy as np
import pytest

from oracle import adct_oracle as O
import tests.test_oracle_pins as P


def _fails(fn, *args):
    try:
        fn(*args)
    except (AssertionError, ValueError):
        return True
    return False


@pytest.fixture
def orig_T():
    return O.transform_matrix()


def test_wrong_sign_in_T_is_caught(monkeypatch, orig_T, golden_dir):
    bad = orig_T.copy()
    bad[6, 5] = -bad[6, 5]
    monkeypatch.setattr(O, "transform_matrix", lambda: bad.copy())
    assert _fails(P.test_factorisation_equals_T) or _fails(P.test_scaling_matches_printed_S, golden_dir)
    assert _fails(P.test_fast_algorithm_basis_vectors)


def test_swapped_rows_of_T_are_caught(monkeypatch, orig_T, golden_dir):
    bad = orig_T[[0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12, 14, 13, 15]].copy()
    monkeypatch.setattr(O, "transform_matrix", lambda: bad.copy())
    assert _fails(P.test_factorisation_equals_T)
    assert _fails(P.test_table2_rows, golden_dir) or _fails(P.test_scaling_matches_printed_S, golden_dir)


def test_transposed_operand_in_fwd2d_is_caught(monkeypatch):
    def bad_fwd2d(img):
        T = O.transform_matrix()
        A = O.to_tiles(np.asarray(img).astype(np.int64))
        return np.einsum("ui,kji,vj->kuv", T, A, T)  # A transposed
    monkeypatch.setattr(O, "fwd2d", bad_fwd2d)
    assert _fails(P.test_fwd2d_basis_tiles_brute_force)


def test_wrong_zonal_weight_is_caught(monkeypatch):
    W = O.zonal_weights()
    bad = W.copy()
    bad[3, 3] *= 2
    monkeypatch.setattr(O, "zonal_weights", lambda: bad.copy())
    assert _fails(P.test_zonal_full_keep_is_lossless)
    assert _fails(P.test_identity_weighted_roundtrip_is_256X)


def test_round_half_even_is_caught(monkeypatch):
    monkeypatch.setattr(O, "round_half_away", lambda v: np.rint(np.asarray(v, np.float64)).astype(np.int64))
    assert _fails(P.test_quant_small_values_are_zero)


def test_dropped_rounding_offset_is_caught(monkeypatch):
    monkeypatch.setattr(O, "round_clamp", lambda R, lo, hi: np.clip(np.floor_divide(R, 256), lo, hi))
    assert _fails(P.test_zonal_r1_is_rounded_block_mean)


def test_wrong_quant_step_is_caught(monkeypatch):
    monkeypatch.setattr(O, "quant_step", lambda qp: float(np.exp2((qp - 4) / 5.0)))
    assert _fails(P.test_quant_step_closed_form)


def test_psnr_missing_pixel_count_is_caught(monkeypatch):
    import math
    monkeypatch.setattr(O, "psnr", lambda s, n, peak=255.0: math.inf if s == 0 else 10 * math.log10(peak * peak / s))
    assert _fails(P.test_psnr_closed_forms)


def test_wrong_stage_block_is_caught(monkeypatch):
    good = O.stage_M4()
    bad = good.copy()
    bad[1, 1] = 1  # [[1,1],[1,-1]] -> [[1,1],[1,1]]
    monkeypatch.setattr(O, "stage_M4", lambda: bad.copy())
    assert _fails(P.test_factorisation_equals_T)
    assert _fails(P.test_fast_algorithm_basis_vectors)


def test_dropped_permutation_is_caught(monkeypatch):
    monkeypatch.setattr(O, "P1_CYCLES", ())
    assert _fails(P.test_factorisation_equals_T)


# ---- zig-zag retention and SSIM (image_experiment) ----
from oracle import image_experiment as E  # noqa: E402
import tests.test_oracle_image_experiment as PE  # noqa: E402


def test_zigzag_wrong_direction_is_caught(monkeypatch):
    def bad_order(n=16):
        order = []
        for s in range(2 * n - 1):
            us = range(max(0, s - n + 1), min(s, n - 1) + 1)
            if s % 2 == 1:  # directions swapped
                us = reversed(us)
            order.extend((u, s - u) for u in us)
        return order
    monkeypatch.setattr(E, "zigzag_order", bad_order)
    assert _fails(PE.test_8x8_order_is_the_jpeg_table)
    assert _fails(PE.test_16x16_order_starts_as_jpeg)


def test_zigzag_row_major_scan_is_caught(monkeypatch):
    monkeypatch.setattr(E, "zigzag_order", lambda n=16: [(u, v) for u in range(n) for v in range(n)])
    assert _fails(PE.test_order_is_a_scan, 16)


def test_ssim_wrong_sigma_is_caught(monkeypatch):
    def bad_window():
        k = np.arange(11) - 5.0
        g = np.exp(-(k[:, None] ** 2 + k[None, :] ** 2) / (2.0 * 1.0 ** 2))
        return g / g.sum()
    monkeypatch.setattr(E, "ssim_window", bad_window)
    assert _fails(PE.test_window)


def test_ssim_swapped_constants_are_caught(monkeypatch):
    monkeypatch.setattr(E, "SSIM_K1", 0.03)
    monkeypatch.setattr(E, "SSIM_K2", 0.01)
    assert _fails(PE.test_ssim_constant_images_closed_form)
    assert _fails(PE.test_ssim_scaled_image_closed_form)


def test_ssim_covariance_without_mean_product_is_caught(monkeypatch):
    real_local_mean = E._local_mean

    def bad_map(a, b):
        x, y = np.asarray(a, np.float64), np.asarray(b, np.float64)
        w = E.ssim_window()
        c1, c2 = (E.SSIM_K1 * E.SSIM_L) ** 2, (E.SSIM_K2 * E.SSIM_L) ** 2
        mx, my = real_local_mean(x, w), real_local_mean(y, w)
        sxx = real_local_mean(x * x, w) - mx * mx
        syy = real_local_mean(y * y, w) - my * my
        sxy = real_local_mean(x * y, w)  # dropped the mean product
        return ((2 * mx * my + c1) * (2 * sxy + c2)) / ((mx * mx + my * my + c1) * (sxx + syy + c2))
    monkeypatch.setattr(E, "ssim_map", bad_map)
    assert _fails(PE.test_ssim_of_an_image_with_itself_is_one)
    assert _fails(PE.test_ssim_brute_force_tiny)


# ---- 8-point oracle (t8) ----
from oracle import t8 as E8  # noqa: E402
import tests.test_oracle_t8 as P8  # noqa: E402


def test_t8_taken_from_odd_rows_is_caught(monkeypatch):
    monkeypatch.setattr(E8, "transform_matrix_8", lambda: O.transform_matrix()[1::2, :8].copy())
    assert _fails(P8.test_even_rows_of_T_are_symmetric_and_form_T8)
    assert _fails(P8.test_factorisation_even_path_is_T8_with_14_additions)


def test_t8_wrong_weight_is_caught(monkeypatch):
    W = E8.zonal_weights_8()
    bad = W.copy()
    bad[1, 2] *= 2
    monkeypatch.setattr(E8, "zonal_weights_8", lambda: bad.copy())
    assert _fails(P8.test_weighted_roundtrip_is_64X)
    assert _fails(P8.test_zonal8_special_cases)


def test_t8_wrong_rounding_offset_is_caught(monkeypatch):
    monkeypatch.setattr(E8, "round_clamp8",
                        lambda R, lo, hi: np.clip(np.floor_divide(np.asarray(R, np.int64), 64), lo, hi))
    assert _fails(P8.test_zonal8_special_cases)


# ---- comparison transforms ----
from oracle import comparison as CMP  # noqa: E402
import tests.test_oracle_comparison as PC  # noqa: E402


def test_wht_sequency_order_is_caught(monkeypatch):
    H = CMP.wht_matrix()
    seq = np.argsort([np.count_nonzero(np.diff(row)) for row in H])  # rows by sign changes
    monkeypatch.setattr(CMP, "wht_matrix", lambda: H[seq].copy())
    assert _fails(PC.test_wht_is_the_natural_order_hadamard)
    assert _fails(PC.test_wht_fast_algorithm_has_64_additions)


def test_dct_rounding_down_is_caught(monkeypatch):
    real = CMP.dct_reconstruct_real
    monkeypatch.setattr(CMP, "dct_reconstruct",
                        lambda img, kind, r, lo=0, hi=255: np.clip(np.floor(real(img, kind, r)), lo, hi)
                        .astype(np.uint8))
    assert _fails(PC.test_dct_reconstruction_special_cases)


def test_mixed_decision_reversed_is_caught(monkeypatch):
    from oracle import mixed as X
    import tests.test_oracle_mixed as PM
    monkeypatch.setattr(X, "keep_8x8", lambda j16, j8: j8 > j16)
    assert _fails(PM.test_choice_minimises_the_lagrangian_cost, 27, 5)


def test_mixed_tie_to_8x8_is_caught(monkeypatch):
    from oracle import mixed as X
    import tests.test_oracle_mixed as PM
    monkeypatch.setattr(X, "keep_8x8", lambda j16, j8: j8 <= j16)
    assert _fails(PM.test_constant_quadrants_choose_8x8)


def test_mixed_sub_blocks_transposed_is_caught(monkeypatch):
    from oracle import mixed as X
    import tests.test_oracle_mixed as PM
    good = X._region_of_8x8_levels

    def bad(q8, H, W):
        r = good(q8, H, W).copy()
        r[:, :8, 8:], r[:, 8:, :8] = r[:, 8:, :8].copy(), r[:, :8, 8:].copy()
        return r
    monkeypatch.setattr(X, "_region_of_8x8_levels", bad)
    assert _fails(PM.test_decoding_the_levels_reproduces_the_output, 32, 30, "i16")
    assert _fails(PM.test_sub_block_placement)


def test_mixed_rate_of_one_sub_block_is_caught(monkeypatch):
    from oracle import mixed as X
    import tests.test_oracle_mixed as PM
    good = X.region_costs

    def bad(plane, qp, lo, hi):
        c = good(plane, qp, lo, hi)
        c["R8"] = (c["q8"][:, :8, :8] != 0).sum(axis=(1, 2))
        return c
    monkeypatch.setattr(X, "region_costs", bad)
    assert _fails(PM.test_choice_minimises_the_lagrangian_cost, 37, 200)
