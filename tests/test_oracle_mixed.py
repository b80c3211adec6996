"""Pins of the mixed 8/16-point coding oracle (Section 3.2, second scenario).

The decision is pinned to its defining property (each region keeps the
coding of lower Lagrangian cost, recomputed here from the two standalone
codecs and from the returned output itself), the stored levels to the
decoder (decoding them reproduces the encoder's reconstruction), and the
behaviour to image content whose best coding is known: 8x8 quadrants of
constant value are coded exactly by four 8x8 DC levels, and a constant
region by a single 16x16 DC level.
"""
import numpy as np
import pytest

from oracle import adct_oracle as O
from oracle import mixed as X
from oracle import t8 as E8
import synth


def _costs_from_outputs(plane, split, levels, out):
    d = O.to_tiles((np.asarray(out, np.int64) - np.asarray(plane, np.int64)) ** 2).sum(axis=(1, 2))
    return d, (levels != 0).sum(axis=(1, 2))


@pytest.mark.parametrize("qp,lam", [(22, 0), (27, 5), (32, 40), (37, 200)])
def test_choice_minimises_the_lagrangian_cost(qp, lam):
    plane = synth.laplacian_residual(900 + qp, 64, 80)
    split, levels, out = X.mixed_encode(plane, qp, lam)
    d, r = _costs_from_outputs(plane, split, levels, out)
    # the two codings of every region, from the standalone codecs
    x = plane.astype(np.int64)
    q16, _, o16 = O.quant_reconstruct(x, qp)
    q8, o8 = E8.quant_reconstruct8(x, qp)
    d16 = O.to_tiles((o16 - x) ** 2).sum(axis=(1, 2))
    d8 = O.to_tiles((o8 - x) ** 2).sum(axis=(1, 2))
    r16 = (q16 != 0).sum(axis=(1, 2))
    # nonzero levels of the four 8x8 blocks of each region
    nz8 = (q8 != 0).sum(axis=(1, 2)).reshape(64 // 8, 80 // 8)
    r8 = nz8.reshape(4, 2, 5, 2).sum(axis=(1, 3)).reshape(-1)
    j16, j8 = d16 + lam * r16, d8 + lam * r8
    assert np.array_equal(split, (j8 < j16).astype(np.uint8))
    assert np.all(d + lam * r == np.minimum(j16, j8))
    # both codings are used somewhere on this content
    assert 0 < split.sum() < len(split)


@pytest.mark.parametrize("qp,lam", [(22, 3), (32, 30)])
@pytest.mark.parametrize("dtype", ["u8", "i16"])
def test_decoding_the_levels_reproduces_the_output(qp, lam, dtype):
    if dtype == "u8":
        plane, lo = synth.ar1_image(910 + qp, 48, 64), 0
    else:
        plane, lo = synth.laplacian_residual(920 + qp, 48, 64), -255
    split, levels, out = X.mixed_encode(plane, qp, lam, lo, 255)
    assert 0 < split.sum() < len(split) or lam > 0
    dec = X.mixed_decode(split, levels, qp, 48, 64, lo, 255)
    assert np.array_equal(dec, out)


def test_constant_quadrants_choose_8x8():
    # each 8x8 quadrant of each region is constant.  At QP 22 (Delta = 8) the
    # 8x8 DC level of a quadrant of value c is 8c / 8 = c exactly, so the 8x8
    # coding is lossless with at most four levels; T codes the same pattern
    # with four levels too (its rows 0 and 1 are constant on each half), but
    # quantised with error, so the 8x8 coding wins wherever that error is not
    # zero and the tie keeps the 16x16 coding elsewhere.
    rng = np.random.default_rng(930)
    quad = rng.integers(20, 236, size=(6, 8))
    plane = np.kron(quad, np.ones((8, 8), np.int64)).astype(np.uint8)
    c = X.region_costs(plane, 22, 0, 255)
    assert not c["D8"].any() and np.all(c["R8"] <= 4) and np.all(c["R16"] <= 4)
    split, levels, out = X.mixed_encode(plane, 22, 1, 0, 255)
    assert np.array_equal(split, (c["D16"] > 0).astype(np.uint8))
    assert split.sum() >= len(split) // 2
    assert np.array_equal(out, plane)


def test_constant_regions_choose_16x16():
    rng = np.random.default_rng(931)
    vals = rng.integers(0, 256, size=(3, 4))
    plane = np.kron(vals, np.ones((16, 16), np.int64)).astype(np.uint8)
    split, levels, out = X.mixed_encode(plane, 22, 1, 0, 255)
    assert np.all(split == 0)
    assert np.all((levels != 0).sum(axis=(1, 2)) <= 1)


def test_zero_plane_and_extreme_lambdas():
    split, levels, out = X.mixed_encode(np.zeros((32, 48), np.int16), 27, 7)
    assert not split.any() and not levels.any() and not out.any()
    plane = synth.laplacian_residual(932, 64, 64)
    c = X.region_costs(plane, 27, -255, 255)
    s0, _, _ = X.mixed_encode(plane, 27, 0)
    assert np.array_equal(s0, (c["D8"] < c["D16"]).astype(np.uint8))
    big = 1 << 40  # the rate term decides unless the rates are equal
    sb, _, _ = X.mixed_encode(plane, 27, big)
    want = np.where(c["R8"] != c["R16"], c["R8"] < c["R16"], c["D8"] < c["D16"])
    assert np.array_equal(sb, want.astype(np.uint8))


def test_sub_block_placement():
    # a split region's level array holds 8x8 block (2 by + a, 2 bx + b) at
    # rows 8a.., columns 8b..
    plane = synth.laplacian_residual(933, 32, 32)
    q8, _ = E8.quant_reconstruct8(plane.astype(np.int64), 27)
    c = X.region_costs(plane, 27, -255, 255)
    b8 = q8.reshape(4, 4, 8, 8)
    for by in range(2):
        for bx in range(2):
            k = by * 2 + bx
            assert np.array_equal(c["q8"][k, :8, 8:], b8[2 * by, 2 * bx + 1])
            assert np.array_equal(c["q8"][k, 8:, :8], b8[2 * by + 1, 2 * bx])


def test_sse_and_addition_counts():
    plane = synth.laplacian_residual(934, 64, 48)
    split, _, out = X.mixed_encode(plane, 27, 10)
    s = X.sse_per_image(out, plane, 32)
    assert s.shape == (2,)
    assert int(s.sum()) == int(((out - plane.astype(np.int64)) ** 2).sum())
    # a 16x16 region's 2D inverse is 32 one-dimensional 16-point passes, a
    # split region's is 4 blocks of 16 eight-point passes
    assert X.decoder_additions(np.zeros(3, np.uint8)) == 3 * 32 * 44
    assert X.decoder_additions(np.ones(2, np.uint8)) == 2 * 64 * 14
    with pytest.raises(ValueError):
        X.mixed_encode(plane, 27, -1)
