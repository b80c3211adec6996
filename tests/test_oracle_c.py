"""The C oracle (timed CPU baseline) agrees with the pinned numpy oracle."""
import numpy as np
import pytest

from oracle import adct_oracle as O
import synth
from tests import oracle_c


def test_c_oracle_fwd2d_matches():
    img = synth.ar1_batch(2, 64, 80, seed_base=900)
    assert np.array_equal(oracle_c.fwd2d_u8(img), O.fwd2d(img))


@pytest.mark.parametrize("r", [1, 2, 4, 8, 12, 16])
def test_c_oracle_zonal_recon_matches(r):
    img = synth.ar1_batch(3, 48, 64, seed_base=910)
    coef = oracle_c.fwd2d_u8(img)
    out, sse = oracle_c.zonal_recon_u8(coef, 144, 64, r, img, 48)
    want = O.zonal_reconstruct(img, r)
    assert np.array_equal(out, want)
    for i in range(3):
        assert sse[i] == O.sse(want[i * 48:(i + 1) * 48], img[i * 48:(i + 1) * 48])


def test_c_oracle_threads():
    assert oracle_c.threads() >= 1
