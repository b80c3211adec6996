"""GPU parity of the 8-point calls (8x8 blocks) against the oracle: bit-exact
coefficients, levels, reconstructions and per-image SSE."""
import numpy as np
import pytest

from oracle import adct_oracle as O
from oracle import t8 as E8
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1606_07414_amd import adct  # noqa: E402


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


# shapes with ragged waves and workgroups (block counts not multiples of 64 or 256)
SHAPES = [(8, 8), (24, 40), (72, 136), (512, 512), (1088, 1920)]


@pytest.mark.parametrize("shape", SHAPES)
def test_t8_fwd2d_u8(shape):
    img = synth.ar1_image(2000 + shape[1], *shape)
    assert np.array_equal(host(adct.t8_fwd2d(dev(img))), E8.fwd2d8(img))


def test_t8_fwd2d_extremes_and_i16():
    z = np.zeros((16, 24), np.uint8)
    z[:8, :8] = 255
    z[8:, 8:16] = np.indices((8, 8)).sum(axis=0) * 17 % 256
    assert np.array_equal(host(adct.t8_fwd2d(dev(z))), E8.fwd2d8(z))
    res = synth.laplacian_residual(2001, 72, 96)
    res[0, :8] = 255
    res[1, :8] = -255
    assert np.array_equal(host(adct.t8_fwd2d(dev(res))), E8.fwd2d8(res))


def test_t8_inv2d():
    rng = np.random.default_rng(2002)
    Y = rng.integers(-20000, 20000, size=(301, 8, 8)).astype(np.int32)
    assert np.array_equal(host(adct.t8_inv2d(dev(Y))), E8.inv2d8(Y))


@pytest.mark.parametrize("r", [0, 1, 2, 3, 4, 6, 8])
@pytest.mark.parametrize("store", [True, False])
@pytest.mark.parametrize("shape,image_h", [((72, 136), 72), ((96, 40), 24), ((512, 256), 128), ((16, 8), 8)])
def test_t8_encode_zonal(r, store, shape, image_h):
    img = synth.ar1_batch(shape[0] // image_h, image_h, shape[1], seed_base=2100 + r)
    x = dev(img)
    out = torch.empty_like(x)
    coef = torch.full((x.numel() // 64, 8, 8), -9, dtype=torch.int32, device="cuda")
    s = host(adct.t8_encode_zonal(x, r, out, coef=coef if store else None, image_height=image_h))
    want = E8.zonal_reconstruct8(img, r)
    assert np.array_equal(host(out), want)
    if store:
        assert np.array_equal(host(coef), E8.fwd2d8(img))
    else:
        assert np.all(host(coef) == -9)
    for i in range(shape[0] // image_h):
        assert s[i] == O.sse(want[i * image_h:(i + 1) * image_h], img[i * image_h:(i + 1) * image_h]), i


@pytest.mark.parametrize("qp", [4, 22, 27, 32, 37, 51])
@pytest.mark.parametrize("kind", ["u8", "i16"])
def test_t8_encode_quant(qp, kind):
    if kind == "u8":
        src = synth.ar1_batch(2, 64, 104, seed_base=2200 + qp)
        lo, hi = 0, 255
    else:
        src = synth.laplacian_residual(2200 + qp, 128, 104)
        lo, hi = -255, 255
    x = dev(src)
    out = torch.empty_like(x)
    q = torch.zeros((x.numel() // 64, 8, 8), dtype=torch.int16, device="cuda")
    s = host(adct.t8_encode_quant(x, qp, out, q=q, image_height=64))
    qw, want = E8.quant_reconstruct8(src, qp, lo, hi)
    assert np.array_equal(host(q), qw)
    assert np.array_equal(host(out), want)
    for i in range(src.shape[0] // 64):
        assert s[i] == O.sse(want[i * 64:(i + 1) * 64], src[i * 64:(i + 1) * 64]), i


def test_t8_pitched_planes_and_lossless():
    img = synth.ar1_image(2300, 40, 48)
    wide = torch.zeros((40, 96), dtype=torch.uint8, device="cuda")
    wide[:, 16:64] = dev(img)
    out = torch.full((40, 80), 7, dtype=torch.uint8, device="cuda")
    s = host(adct.t8_encode_zonal(wide[:, 16:64], 8, out[:, 16:64]))
    assert np.array_equal(host(out[:, 16:64]), img) and s[0] == 0
    assert np.all(host(out[:, :16]) == 7) and np.all(host(out[:, 64:]) == 7)


def test_t8_video_frames_full_size():
    # the residual planes of one 1920x1088 4:2:0 frame at every QP of the video workload
    for qp in (22, 27, 32, 37):
        for plane in synth.video_frame_planes(5):
            x = dev(plane)
            out = torch.empty_like(x)
            s = host(adct.t8_encode_quant(x, qp, out))
            _, want = E8.quant_reconstruct8(plane, qp)
            assert np.array_equal(host(out), want), qp
            assert s[0] == O.sse(want, plane)


@pytest.mark.parametrize("op", ["zonal", "quant"])
def test_t8_sse_over_large_images_spread_and_split(op):
    # 544 x 960 images: 8160 blocks each, so workgroups of 256 blocks cross
    # image boundaries and the launch interleaves its workgroups
    n, h, w = 5, 544, 960
    if op == "zonal":
        src = synth.ar1_batch(n, h, w, seed_base=2400)
    else:
        src = np.concatenate([synth.laplacian_residual(2400 + i, h, w) for i in range(n)])
    x = dev(src)
    out = torch.empty_like(x)
    if op == "zonal":
        s = host(adct.t8_encode_zonal(x, 3, out, image_height=h))
        want = E8.zonal_reconstruct8(src, 3)
    else:
        s = host(adct.t8_encode_quant(x, 32, out, image_height=h))
        _, want = E8.quant_reconstruct8(src, 32)
    assert np.array_equal(host(out), want)
    for i in range(n):
        assert s[i] == O.sse(want[i * h:(i + 1) * h], src[i * h:(i + 1) * h]), i
