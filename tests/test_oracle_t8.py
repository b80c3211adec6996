"""Pins of the 8-point oracle (T8 recovered from T, and the 8x8 codec).

T8 is pinned to the structure of Section 2.2's factorisation (the even path
of P2 M4 M3 M2 P1 M1 is T8 on the folded sums, with 14 additions), to
orthogonality, to the sign pattern of the exact 8-point DCT-II, and the 2D
codec to brute force and exact identities.
"""
import numpy as np
import pytest
import scipy.fft

from oracle import adct_oracle as O
from oracle import t8 as E8
import synth


def test_even_rows_of_T_are_symmetric_and_form_T8():
    T = O.transform_matrix()
    assert np.array_equal(T[0::2, :8], T[0::2, 8:][:, ::-1])
    assert np.array_equal(E8.transform_matrix_8(), T[0::2, :8])
    # T x on even outputs = T8 (x_j + x_{15-j})
    rng = np.random.default_rng(8)
    for x in rng.integers(-1000, 1000, size=(200, 16)):
        assert np.array_equal((T @ x)[0::2], E8.transform_matrix_8() @ (x[:8] + x[::-1][:8]))


def test_factorisation_even_path_is_T8_with_14_additions():
    st = dict(O.factorisation_stages())
    G = st["P2"] @ st["M4"] @ st["M3"] @ st["M2"] @ st["P1"]
    assert not G[0::2, 8:].any()                      # even outputs ignore the difference half
    assert np.array_equal(G[0::2, :8], E8.transform_matrix_8())
    counts = [O.addition_count(M) for _, M in E8.even_path_stages()]
    assert counts == [8, 4, 2, 0] and sum(counts) == 14


def test_fast_algorithm_8():
    T8 = E8.transform_matrix_8()
    for k in range(8):
        e = np.zeros(8, np.int64)
        e[k] = 1
        assert np.array_equal(E8.fast_forward_1d_8(e), T8[:, k])
    rng = np.random.default_rng(88)
    for x in rng.integers(-(1 << 20), 1 << 20, size=(10000, 8)):
        assert np.array_equal(E8.fast_forward_1d_8(x), T8 @ x)


def test_T8_orthogonality_and_scaling():
    T8 = E8.transform_matrix_8()
    assert set(np.unique(T8)) <= {-1, 0, 1}
    G = T8 @ T8.T
    assert np.array_equal(G, np.diag(np.diag(G)))
    assert E8.gram_diagonal_8().tolist() == [8, 2, 4, 2, 8, 2, 4, 2]
    C = E8.orthogonal_approximation_8()
    assert np.allclose(C @ C.T, np.eye(8), atol=1e-15)
    assert np.all(T8[0] == 1)


def test_T8_signs_follow_the_dct():
    C8 = scipy.fft.dct(np.eye(8), norm="ortho", axis=0)
    T8 = E8.transform_matrix_8()
    nz = T8 != 0
    assert np.all(np.sign(T8[nz]) == np.sign(C8[nz]))


def test_fwd2d8_basis_tiles_brute_force():
    T8 = E8.transform_matrix_8()
    for i in range(8):
        for j in range(8):
            img = np.zeros((8, 8), np.int64)
            img[i, j] = 1
            want = np.outer(T8[:, i], T8[:, j])
            assert np.array_equal(E8.fwd2d8(img)[0], want)
            assert np.array_equal(E8.inv2d8(want[None])[0], T8.T @ want @ T8)


def test_weighted_roundtrip_is_64X():
    rng = np.random.default_rng(808)
    X = rng.integers(-255, 256, size=(5, 8, 8))
    Y = np.einsum("ui,kij,vj->kuv", E8.transform_matrix_8(), X, E8.transform_matrix_8())
    R = E8.inv2d8(Y * E8.zonal_weights_8()[None])
    assert np.array_equal(R, 64 * X)


def test_zonal8_special_cases():
    img = synth.ar1_image(80, 32, 48)
    assert np.array_equal(E8.zonal_reconstruct8(img, 8), img)
    t = E8.to_tiles8(img).astype(np.int64)
    means = np.floor_divide(t.sum(axis=(1, 2)) + 32, 64)
    got = E8.to_tiles8(E8.zonal_reconstruct8(img, 1)).astype(np.int64)
    assert np.all(got == means[:, None, None])


@pytest.mark.parametrize("r", [2, 4, 6])
def test_zonal8_fixed_point_equals_real_valued(r):
    img = synth.ar1_image(81 + r, 24, 40)
    C = E8.orthogonal_approximation_8()
    B = np.einsum("ui,kij,vj->kuv", C, E8.to_tiles8(img.astype(np.float64)), C) * E8.zonal_mask_8(r)[None]
    real = np.einsum("ui,kuv,vj->kij", C, B, C)
    R = E8.inv2d8(E8.zonal8(E8.fwd2d8(img), r))
    assert np.max(np.abs(R / 64.0 - real)) < 1e-9


@pytest.mark.parametrize("qp", [4, 22, 27, 32, 37])
def test_quantiser8_error_bound(qp):
    res = synth.laplacian_residual(82 + qp, 32, 32)
    Y = E8.fwd2d8(res)
    s = E8.scaling_vector_8()
    B = Y * (s[:, None] * s[None, :])[None]
    q = E8.quantise8(Y, qp)
    delta = O.quant_step(qp)
    assert np.all(np.abs(q * delta - B) <= delta / 2 * (1 + 1e-6))
    if qp == 4:
        # Delta = 1: the levels are B rounded, except at exact ties, where the
        # float64 product s_u s_v may land either side of k + 1/2
        tie = np.abs(np.abs(B) - np.floor(np.abs(B)) - 0.5) < 1e-9
        assert np.array_equal(q[~tie], O.round_half_away(B)[~tie])
        assert np.all(np.abs(q[tie]) == np.floor(np.abs(B[tie])) + 1)  # half away from zero
    # dequantised fixed point approximates 64 s_u s_v q Delta
    z = E8.dequantise8(q, qp)
    assert np.all(np.abs(z - 64 * delta * q * (s[:, None] * s[None, :])[None]) <= 0.5 + 1e-6 * np.abs(z))


def test_quant_reconstruct8_identity_at_fine_step():
    # QP 4 (Delta = 1) on a smooth plane: the reconstruction error stays small
    img = synth.ar1_image(83, 32, 32).astype(np.int64)
    _, out = E8.quant_reconstruct8(img, 4, 0, 255)
    assert np.max(np.abs(out - img)) <= 2
