"""The seeded generators: determinism, shapes, ranges and statistics."""
import numpy as np

import synth


def test_ar1_deterministic_and_range():
    a = synth.ar1_image(1, 256, 256)
    b = synth.ar1_image(1, 256, 256)
    assert a.dtype == np.uint8 and a.shape == (256, 256)
    assert np.array_equal(a, b)
    assert not np.array_equal(a, synth.ar1_image(2, 256, 256))


def test_ar1_statistics():
    rng = np.random.default_rng(3)
    f = synth.ar1_field(rng, 512, 512)
    assert abs(f.std() - 1.0) < 0.15
    h = np.corrcoef(f[:, :-1].ravel(), f[:, 1:].ravel())[0, 1]
    v = np.corrcoef(f[:-1].ravel(), f[1:].ravel())[0, 1]
    assert abs(h - 0.95) < 0.02 and abs(v - 0.95) < 0.02


def test_batch_layout():
    b = synth.ar1_batch(3, 32, 48, seed_base=10)
    assert b.shape == (96, 48)
    assert np.array_equal(b[32:64], synth.ar1_image(11, 32, 48))


def test_laplacian_residual():
    r = synth.laplacian_residual(5, 544, 960)
    assert r.dtype == np.int16 and r.min() >= -255 and r.max() <= 255
    assert abs(np.mean(np.abs(r.astype(float))) - 8.0) < 0.3


def test_uneven_sizes():
    s = synth.uneven_sizes(4096)
    hs = np.array(s)
    assert hs.min() >= 64 and hs.max() <= 2048 and np.all(hs % 16 == 0)
    tiles = np.sum(hs[:, 0] // 16 * (hs[:, 1] // 16))
    assert 16e6 < tiles < 20e6  # E ~ 4096 * 66^2


def test_request_sides_and_arrivals():
    s = synth.request_sides(2000)
    assert s.min() >= 256 and s.max() <= 4096 and np.all(s % 16 == 0)
    t = synth.poisson_arrivals(1000.0, 2000)
    assert np.all(np.diff(t) > 0)
    assert abs(np.mean(np.diff(t)) - 1e-3) < 1e-4


def test_structured_tiles():
    t = synth.structured_tiles()
    assert t.dtype == np.uint8 and t.shape[1:] == (16, 16)
    assert (t == 0).all(axis=(1, 2)).any() and (t == 255).all(axis=(1, 2)).any()
