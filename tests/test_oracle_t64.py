"""Pins of the 64-point oracle (oracle/t64.py) to what the construction and
the mathematics fix, and planted mistakes that must each fail a pin.

The construction reuses the 32-point extension (itself pinned to the
paper's T in tests/test_oracle_t32.py); these pins tie the 64-point matrix
to it through properties that hold for it alone: the symmetric and
antisymmetric halves, the diagonal Gram matrix in closed form, the fast
algorithm on every basis vector with its addition count, row-by-row 2D
sums, the exact weighted round trip, the tile-mean reconstruction and the
quantiser's closed forms.
"""
import numpy as np

from oracle import adct_oracle as O
from oracle import t32 as T32
from oracle import t64 as T64


def test_entries_and_halves():
    A = T64.transform_matrix_64()
    t = T32.transform_matrix_32()
    assert A.shape == (64, 64) and set(np.unique(A)) <= {-1, 0, 1}
    for k in range(32):
        # coefficient 2k: row k of T32 on the folded sums (symmetric row)
        assert np.array_equal(A[2 * k, :32], t[k]) and np.array_equal(A[2 * k, 32:], t[k][::-1])
        # coefficient 2k + 1: row k of T32 on the folded differences (antisymmetric row)
        assert np.array_equal(A[2 * k + 1, :32], t[k]) and np.array_equal(A[2 * k + 1, 32:], -t[k][::-1])


def test_gram_matrix_is_diagonal_closed_form():
    A = T64.transform_matrix_64()
    d32 = T32.gram_diagonal_32()
    G = A @ A.T
    assert np.array_equal(G, np.diag(np.diag(G)))
    assert np.array_equal(np.diag(G), 2 * np.repeat(d32, 2))
    # and four times the 16-point diagonal: d64_u = 4 d_{u // 4}
    assert np.array_equal(np.diag(G), 4 * np.repeat(O.gram_diagonal(), 4))
    assert set(np.diag(G)) == {16, 32, 64}


def test_row_sums_and_dc_row():
    A = T64.transform_matrix_64()
    assert np.array_equal(A[0], np.ones(64, dtype=np.int64))
    assert np.all(A[1:].sum(axis=1) == 0)


def test_orthonormal_and_parseval():
    C = T64.orthogonal_approximation_64()
    assert np.allclose(C @ C.T, np.eye(64), atol=1e-13)
    x = np.random.default_rng(15).standard_normal(64)
    assert np.isclose(np.linalg.norm(C @ x), np.linalg.norm(x))


def test_symmetric_and_antisymmetric_inputs_reduce_to_T32():
    rng = np.random.default_rng(16)
    t = T32.transform_matrix_32()
    A = T64.transform_matrix_64()
    h = rng.integers(-255, 256, 32)
    sym = np.concatenate([h, h[::-1]])
    anti = np.concatenate([h, -h[::-1]])
    ys, ya = A @ sym, A @ anti
    assert np.array_equal(ys[0::2], 2 * t @ h) and not ys[1::2].any()
    assert np.array_equal(ya[1::2], 2 * t @ h) and not ya[0::2].any()


def test_fast_algorithm_basis_random_and_additions():
    A = T64.transform_matrix_64()
    rng = np.random.default_rng(17)
    vecs = list(np.eye(64, dtype=np.int64)) + [rng.integers(-8160, 8161, 64) for _ in range(100)]
    for v in vecs:
        X, adds = T64.fast_forward_1d_64(v)
        assert np.array_equal(X, A @ v) and adds == 304
        x, adds_i = T64.fast_inverse_1d_64(v)
        assert np.array_equal(x, A.T @ v) and adds_i == 304
    assert O.addition_count(A) > 304  # the direct product costs more


def test_fwd2d_row_by_row_and_basis_tiles():
    A = T64.transform_matrix_64()
    rng = np.random.default_rng(18)
    img = rng.integers(0, 256, (128, 192)).astype(np.uint8)
    Y = T64.fwd2d_64(img)
    tiles = T64.to_tiles64(img.astype(np.int64))
    for k in (0, 4):
        X = tiles[k]
        want = np.zeros((64, 64), dtype=np.int64)
        for u in range(64):
            row = (A[u][:, None] * X).sum(axis=0)  # sum over i of A[u, i] X[i, :]
            for v in range(64):
                want[u, v] = int((row * A[v]).sum())
        assert np.array_equal(Y[k], want)
    for i, j in ((0, 0), (5, 40), (63, 1)):
        X = np.zeros((64, 64), dtype=np.int64)
        X[i, j] = 1
        assert np.array_equal(T64.fwd2d_64(X)[0], np.outer(A[:, i], A[:, j]))
    # tile raster order: tile k is block row k // 3, block column k % 3
    assert np.array_equal(tiles[4], img[64:128, 64:128])


def test_weighted_round_trip_is_4096x_and_tile_mean():
    rng = np.random.default_rng(19)
    img = rng.integers(0, 256, (64, 128)).astype(np.uint8)
    R = T64.inv2d_64(T64.zonal_64(T64.fwd2d_64(img), 64))
    assert np.array_equal(R, 4096 * T64.to_tiles64(img.astype(np.int64)))
    assert np.array_equal(T64.zonal_reconstruct_64(img, 64), img)
    # r = 1 keeps the DC term only: every sample is the tile mean rounded half
    # up; the second tile's mean is exactly 10.5 (2048 samples of 10, 2048 of 11)
    img[:, 64:] = 10
    img[::2, 64:] = 11
    out = T64.zonal_reconstruct_64(img, 1)
    for k, t in enumerate(T64.to_tiles64(img.astype(np.int64))):
        mean_up = (int(t.sum()) + 2048) // 4096
        assert np.all(T64.to_tiles64(out)[k] == mean_up)
    assert np.all(T64.to_tiles64(out)[1] == 11)
    res = rng.integers(-255, 256, (64, 64)).astype(np.int16)
    assert np.array_equal(T64.zonal_reconstruct_64(res, 64, -255, 255), res)


def test_zonal_with_even_r_equals_32_point_with_half_r():
    # T32's rows are symmetric (even k) or antisymmetric (odd k), so rows 2k
    # and 2k + 1 of T64 (k < m) span row k of T32 on each 32-sample half:
    # keeping 2m x 2m coefficients of a 64x64 block projects onto the same
    # subspace as keeping m x m of each of its four 32x32 blocks.  Both zonal
    # codecs are that exact projection, rounded half up, so they agree sample
    # for sample, on samples and on residuals.
    rng = np.random.default_rng(22)
    img = rng.integers(0, 256, (128, 192)).astype(np.uint8)
    res = rng.integers(-255, 256, (64, 128)).astype(np.int16)
    for m in (0, 1, 2, 5, 8, 16, 27, 32):
        assert np.array_equal(T64.zonal_reconstruct_64(img, 2 * m), T32.zonal_reconstruct_32(img, m)), m
        assert np.array_equal(T64.zonal_reconstruct_64(res, 2 * m, -255, 255),
                              T32.zonal_reconstruct_32(res, m, -255, 255)), m
    assert not np.array_equal(T64.zonal_reconstruct_64(img, 5), T32.zonal_reconstruct_32(img, 2))


def test_zonal_weights_are_shifts():
    W = T64.zonal_weights_64()
    assert set(np.unique(W)) == {1, 2, 4, 8, 16}
    assert W[0, 0] == 1 and W[63, 63] == 16


def test_quant_tables_closed_form_and_bound():
    qs, dqs = T64.quant_tables_64(22)
    assert O.quant_step(22) == 8.0
    d = T64.gram_diagonal_64()
    assert d[0] == 64 and d[63] == 16
    assert qs[0, 0] == np.float32(1.0 / (64 * 8)) and dqs[0, 0] == np.float32(4096 * 8 / 64)
    assert qs[63, 63] == np.float32(1.0 / (16 * 8)) and dqs[63, 63] == np.float32(4096 * 8 / 16)
    rng = np.random.default_rng(20)
    img = rng.integers(-255, 256, (64, 128)).astype(np.int16)
    s = 1.0 / np.sqrt(d.astype(np.float64))
    for qp in (22, 27, 37):
        Y = T64.fwd2d_64(img)
        q = T64.quantise_64(Y, qp)
        B = Y * (s[:, None] * s[None, :])
        delta = O.quant_step(qp)
        assert np.all(np.abs(q * delta - B) <= delta / 2 * (1 + 1e-6) + 1e-9)
        # Z' carries 12 fractional bits: Z' / 4096 is q Delta s_u s_v within rounding
        z = T64.dequantise_64(q, qp)
        assert np.all(np.abs(z - 4096 * q * delta * (s[:, None] * s[None, :])) <= 0.5 + 1e-3 * np.abs(z))


def test_level_saturation_acts_only_below_qp16_on_wide_int16():
    # a constant tile has Y_00 = 4096 x and B_00 = Y_00 / 64 = 64 x; with
    # x = 2047 the level leaves int16 while Delta < 4, that is below QP 16
    for qp, x, saturates in ((0, 2047, True), (15, 2047, True), (16, 2047, False), (0, 255, False)):
        tile = np.full((64, 64), x, dtype=np.int16)
        q = T64.quantise_64(T64.fwd2d_64(tile), qp)
        exact = O.round_half_away(np.float32(4096 * x) * T64.quant_tables_64(qp)[0][0, 0])
        assert (q[0, 0, 0] == 32767 and exact > 32767) if saturates else q[0, 0, 0] == exact
        if not saturates:  # rounding half away from zero is odd-symmetric
            assert np.array_equal(T64.quantise_64(-T64.fwd2d_64(tile), qp), -q)


def test_quant_reconstruction_error_rms_bound():
    # S64 T64 is orthonormal, so the reconstruction error's energy is the
    # coefficient error's: each scaled coefficient is off by at most Delta / 2
    # (plus the 2^-12 rounding of Z'), and the final rounding adds at most 1/2
    # per sample; with Delta = 1 the RMS error stays below 1/2 + 1/2
    rng = np.random.default_rng(21)
    img = rng.integers(-255, 256, (128, 128)).astype(np.int16)
    _, _, out = T64.quant_reconstruct_64(img, 4)
    err = out.astype(np.float64) - img
    assert np.sqrt(np.mean(err ** 2)) <= 1.0


# ---- planted mistakes ----------------------------------------------------
def _fails(fn):
    try:
        fn()
    except (AssertionError, ValueError):
        return True
    return False


def test_swapped_interleave_is_caught(monkeypatch):
    bad = T64.interleave_64()[[1, 0] + list(range(2, 64))]
    monkeypatch.setattr(T64, "interleave_64", lambda: bad.copy())
    assert _fails(test_entries_and_halves)
    assert _fails(test_symmetric_and_antisymmetric_inputs_reduce_to_T32)


def test_difference_sign_flip_is_caught(monkeypatch):
    bad = T64.butterfly_64().copy()
    bad[32:] = -bad[32:]  # differences taken as x_{63-j} - x_j
    monkeypatch.setattr(T64, "butterfly_64", lambda: bad.copy())
    assert _fails(test_entries_and_halves)


def test_transposed_operand_in_fwd2d_64_is_caught(monkeypatch):
    def bad_fwd(img):
        A = T64.transform_matrix_64()
        X = T64.to_tiles64(np.asarray(img).astype(np.int64))
        return np.einsum("ui,kji,vj->kuv", A, X, A)
    monkeypatch.setattr(T64, "fwd2d_64", bad_fwd)
    assert _fails(test_fwd2d_row_by_row_and_basis_tiles)


def test_wrong_weight_64_is_caught(monkeypatch):
    bad = T64.zonal_weights_64().copy()
    bad[9, 40] *= 2
    monkeypatch.setattr(T64, "zonal_weights_64", lambda: bad.copy())
    assert _fails(test_weighted_round_trip_is_4096x_and_tile_mean)


def test_wrong_rounding_offset_64_is_caught(monkeypatch):
    monkeypatch.setattr(T64, "round_clamp_64", lambda R, lo, hi: np.clip(np.floor_divide(np.asarray(R), 4096), lo, hi))
    assert _fails(test_weighted_round_trip_is_4096x_and_tile_mean)


def test_wrong_scale_in_dequantiser_is_caught(monkeypatch):
    real = T64.quant_tables_64
    monkeypatch.setattr(T64, "quant_tables_64", lambda qp: (real(qp)[0], real(qp)[1] / np.float32(2)))
    assert _fails(test_quant_tables_closed_form_and_bound)
