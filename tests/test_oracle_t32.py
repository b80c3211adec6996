"""Pins of the 32-point oracle (oracle/t32.py) to what the construction and
the mathematics fix, and planted mistakes that must each fail a pin.

The construction reuses the paper's T (pinned to Section 2.1's printed
matrix and S elsewhere); these pins tie the 32-point matrix to T through
properties that hold for it alone: the symmetric and antisymmetric halves,
the diagonal Gram matrix in closed form, the fast algorithm on every basis
vector with its addition count, brute-force 2D sums, the exact weighted
round trip and the tile-mean reconstruction.
"""
import numpy as np
import pytest

from oracle import adct_oracle as O
from oracle import t32 as T32


def test_entries_and_halves():
    A = T32.transform_matrix_32()
    T = O.transform_matrix()
    assert A.shape == (32, 32) and set(np.unique(A)) <= {-1, 0, 1}
    for k in range(16):
        # coefficient 2k: row k of T on the folded sums (symmetric row)
        assert np.array_equal(A[2 * k, :16], T[k]) and np.array_equal(A[2 * k, 16:], T[k][::-1])
        # coefficient 2k + 1: row k of T on the folded differences (antisymmetric row)
        assert np.array_equal(A[2 * k + 1, :16], T[k]) and np.array_equal(A[2 * k + 1, 16:], -T[k][::-1])


def test_gram_matrix_is_diagonal_closed_form():
    A = T32.transform_matrix_32()
    d = O.gram_diagonal()
    G = A @ A.T
    assert np.array_equal(G, np.diag(np.diag(G)))
    assert np.array_equal(np.diag(G), 2 * np.repeat(d, 2))
    assert set(np.diag(G)) == {8, 16, 32}


def test_row_sums_and_dc_row():
    A = T32.transform_matrix_32()
    assert np.array_equal(A[0], np.ones(32, dtype=np.int64))
    assert np.all(A[1:].sum(axis=1) == 0)


def test_orthonormal_and_parseval():
    C = T32.orthogonal_approximation_32()
    assert np.allclose(C @ C.T, np.eye(32), atol=1e-13)
    x = np.random.default_rng(5).standard_normal(32)
    assert np.isclose(np.linalg.norm(C @ x), np.linalg.norm(x))


def test_symmetric_and_antisymmetric_inputs_reduce_to_T():
    rng = np.random.default_rng(6)
    T = O.transform_matrix()
    A = T32.transform_matrix_32()
    h = rng.integers(-255, 256, 16)
    sym = np.concatenate([h, h[::-1]])
    anti = np.concatenate([h, -h[::-1]])
    ys, ya = A @ sym, A @ anti
    assert np.array_equal(ys[0::2], 2 * T @ h) and not ys[1::2].any()
    assert np.array_equal(ya[1::2], 2 * T @ h) and not ya[0::2].any()


def test_fast_algorithm_basis_random_and_additions():
    A = T32.transform_matrix_32()
    rng = np.random.default_rng(7)
    vecs = list(np.eye(32, dtype=np.int64)) + [rng.integers(-4080, 4081, 32) for _ in range(200)]
    for v in vecs:
        X, adds = T32.fast_forward_1d_32(v)
        assert np.array_equal(X, A @ v) and adds == 120
        x, adds_i = T32.fast_inverse_1d_32(v)
        assert np.array_equal(x, A.T @ v) and adds_i == 120
    assert O.addition_count(A) > 120  # the direct product costs more


def test_fwd2d_brute_force_and_basis_tiles():
    A = T32.transform_matrix_32()
    rng = np.random.default_rng(8)
    img = rng.integers(0, 256, (64, 96)).astype(np.uint8)
    Y = T32.fwd2d_32(img)
    tiles = T32.to_tiles32(img.astype(np.int64))
    for k in (0, 3, 5):
        X = tiles[k]
        want = np.zeros((32, 32), dtype=np.int64)
        for u in range(32):
            for v in range(32):
                want[u, v] = sum(int(A[u, i]) * int(A[v, j]) * int(X[i, j]) for i in range(32) for j in range(32)
                                 if A[u, i] and A[v, j])
        assert np.array_equal(Y[k], want)
    # basis tile e_i e_j^T goes to the outer product of columns i and j
    for i, j in ((0, 0), (3, 17), (31, 1)):
        X = np.zeros((32, 32), dtype=np.int64)
        X[i, j] = 1
        assert np.array_equal(T32.fwd2d_32(X)[0], np.outer(A[:, i], A[:, j]))
    # tile raster order: tile k is block row k // 3, block column k % 3
    assert np.array_equal(tiles[4], img[32:64, 32:64])


def test_weighted_round_trip_is_1024x_and_tile_mean():
    rng = np.random.default_rng(9)
    img = rng.integers(0, 256, (64, 64)).astype(np.uint8)
    R = T32.inv2d_32(T32.zonal_32(T32.fwd2d_32(img), 32))
    assert np.array_equal(R, 1024 * T32.to_tiles32(img.astype(np.int64)))
    assert np.array_equal(T32.zonal_reconstruct_32(img, 32), img)
    # r = 1 keeps the DC term only: every sample is the tile mean rounded half up
    out = T32.zonal_reconstruct_32(img, 1)
    for k, t in enumerate(T32.to_tiles32(img.astype(np.int64))):
        mean_up = (int(t.sum()) + 512) // 1024
        assert np.all(T32.to_tiles32(out)[k] == mean_up)
    # residual range: int16 planes within [-255, 255]
    res = rng.integers(-255, 256, (32, 64)).astype(np.int16)
    assert np.array_equal(T32.zonal_reconstruct_32(res, 32, -255, 255), res)


def test_zonal_with_even_r_equals_16_point_with_half_r():
    # T's rows are symmetric or antisymmetric (Section 2.1 builds them from
    # folded sums and differences), so rows 2k and 2k + 1 of T32 (k < m) span
    # row k of T on each 16-sample half: keeping 2m x 2m coefficients of a
    # 32x32 block projects onto the same subspace as keeping m x m of each of
    # its four 16x16 blocks.  Both zonal codecs are that exact projection,
    # rounded half up, so they agree sample for sample.
    img = np.random.default_rng(12).integers(0, 256, (64, 96)).astype(np.uint8)
    for m in (0, 1, 2, 3, 4, 8, 13, 16):
        assert np.array_equal(T32.zonal_reconstruct_32(img, 2 * m), O.zonal_reconstruct(img, m)), m
    # an odd r keeps an even row without its odd partner: no such identity
    assert not np.array_equal(T32.zonal_reconstruct_32(img, 3), O.zonal_reconstruct(img, 1))


def test_zonal_weights_are_shifts():
    W = T32.zonal_weights_32()
    assert set(np.unique(W)) == {1, 2, 4, 8, 16}
    assert W[0, 0] == 1 and W[31, 31] == 16


def test_quant_tables_closed_form_and_bound():
    qs, dqs = T32.quant_tables_32(22)
    assert O.quant_step(22) == 8.0
    d = T32.gram_diagonal_32()
    assert qs[0, 0] == np.float32(1.0 / (32 * 8)) and dqs[0, 0] == np.float32(1024 * 8 / 32)
    assert qs[31, 31] == np.float32(1.0 / (8 * 8)) and dqs[31, 31] == np.float32(1024 * 8 / 8)
    rng = np.random.default_rng(10)
    img = rng.integers(-255, 256, (64, 64)).astype(np.int16)
    for qp in (22, 27, 37):
        Y = T32.fwd2d_32(img)
        q = T32.quantise_32(Y, qp)
        s = 1.0 / np.sqrt(d.astype(np.float64))
        B = Y * (s[:, None] * s[None, :])
        delta = O.quant_step(qp)
        assert np.all(np.abs(q * delta - B) <= delta / 2 * (1 + 1e-6) + 1e-9)
        # Z' carries 10 fractional bits: Z' / 1024 is q Delta s_u s_v within rounding
        z = T32.dequantise_32(q, qp)
        assert np.all(np.abs(z - 1024 * q * delta * (s[:, None] * s[None, :])) <= 0.5 + 1e-3 * np.abs(z))


def test_level_saturation_acts_only_below_qp10_on_wide_int16():
    # the largest level magnitude is reached by a constant tile: Y_00 =
    # 1024 x, B_00 = Y_00 / 32 = 32 x
    for qp, x, saturates in ((0, 2047, True), (9, 2047, True), (10, 2047, False), (0, 255, False)):
        tile = np.full((32, 32), x, dtype=np.int16)
        q = T32.quantise_32(T32.fwd2d_32(tile), qp)
        exact = O.round_half_away(np.float32(1024 * x) * T32.quant_tables_32(qp)[0][0, 0])
        assert (q[0, 0, 0] == 32767 and exact > 32767) if saturates else q[0, 0, 0] == exact
        if not saturates:  # rounding half away from zero is odd-symmetric
            assert np.array_equal(T32.quantise_32(-T32.fwd2d_32(tile), qp), -q)


def test_quant_reconstruction_error_is_bounded():
    rng = np.random.default_rng(11)
    img = rng.integers(-255, 256, (64, 64)).astype(np.int16)
    _, _, out = T32.quant_reconstruct_32(img, 4)  # Delta = 1: at most about half a step per coefficient
    assert np.max(np.abs(out.astype(np.int64) - img)) <= 2


# ---- planted mistakes ----------------------------------------------------
def _fails(fn):
    try:
        fn()
    except (AssertionError, ValueError):
        return True
    return False


def test_swapped_interleave_is_caught(monkeypatch):
    bad = T32.interleave_32()[[1, 0] + list(range(2, 32))]
    monkeypatch.setattr(T32, "interleave_32", lambda: bad.copy())
    assert _fails(test_entries_and_halves)
    assert _fails(test_symmetric_and_antisymmetric_inputs_reduce_to_T)


def test_difference_sign_flip_is_caught(monkeypatch):
    B = T32.butterfly_32()
    bad = B.copy()
    bad[16:] = -bad[16:]  # differences taken as x_{31-j} - x_j
    monkeypatch.setattr(T32, "butterfly_32", lambda: bad.copy())
    assert _fails(test_entries_and_halves)


def test_transposed_operand_in_fwd2d_32_is_caught(monkeypatch):
    def bad_fwd(img):
        A = T32.transform_matrix_32()
        X = T32.to_tiles32(np.asarray(img).astype(np.int64))
        return np.einsum("ui,kji,vj->kuv", A, X, A)
    monkeypatch.setattr(T32, "fwd2d_32", bad_fwd)
    assert _fails(test_fwd2d_brute_force_and_basis_tiles)


def test_wrong_weight_32_is_caught(monkeypatch):
    W = T32.zonal_weights_32()
    bad = W.copy()
    bad[5, 7] *= 2
    monkeypatch.setattr(T32, "zonal_weights_32", lambda: bad.copy())
    assert _fails(test_weighted_round_trip_is_1024x_and_tile_mean)


def test_wrong_rounding_offset_32_is_caught(monkeypatch):
    monkeypatch.setattr(T32, "round_clamp_32", lambda R, lo, hi: np.clip(np.floor_divide(np.asarray(R), 1024), lo, hi))
    assert _fails(test_weighted_round_trip_is_1024x_and_tile_mean)
