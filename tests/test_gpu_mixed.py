"""GPU parity of the mixed 8/16-point codec against the oracle: bit-exact
split flags, levels, reconstructions and per-image SSE, on ragged shapes,
both sample types, the QPs of the video workload and beyond, lambdas from 0
(distortion only) to the largest accepted (rate first), and full-size video
planes."""
import numpy as np
import pytest

from oracle import adct_oracle as O
from oracle import mixed as X
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1606_07414_amd import adct  # noqa: E402


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def run(src, qp, lam, image_height=None):
    x = dev(src)
    out = torch.full_like(x, 77)
    nreg = (src.shape[0] // 16) * (src.shape[1] // 16)
    q = torch.full((nreg, 16, 16), -7, dtype=torch.int16, device="cuda")
    split = torch.full((nreg,), 9, dtype=torch.uint8, device="cuda")
    s = adct.mixed_encode(x, qp, lam, out, q=q, split=split, image_height=image_height)
    return host(split), host(q), host(out), host(s)


def check(src, qp, lam, image_height=None):
    lo = 0 if src.dtype == np.uint8 else -255
    ih = image_height or src.shape[0]
    split, q, out, s = run(src, qp, lam, ih)
    ws, wq, wout = X.mixed_encode(src, qp, lam, lo, 255)
    assert np.array_equal(split, ws), (qp, lam)
    assert np.array_equal(q, wq), (qp, lam)
    assert np.array_equal(out, wout), (qp, lam)
    assert np.array_equal(s, X.sse_per_image(wout, src, ih)), (qp, lam)
    return ws


@pytest.mark.parametrize("qp", [0, 3, 4, 22, 27, 32, 37, 51])
@pytest.mark.parametrize("lam", [0, 6, 58, 1 << 40])
def test_mixed_i16_residuals(qp, lam):
    # 7 regions per block row: a wave's four regions straddle block rows
    src = synth.laplacian_residual(3000 + qp, 96, 112)
    check(src, qp, lam, image_height=32)


@pytest.mark.parametrize("qp", [4, 22, 32, 51])
@pytest.mark.parametrize("lam", [0, 18])
def test_mixed_u8_images(qp, lam):
    src = synth.ar1_batch(3, 48, 80, seed_base=3100 + qp)
    split = check(src, qp, lam, image_height=48)
    if lam == 18 and qp == 22:
        assert 0 < split.sum() < len(split)


@pytest.mark.parametrize("shape", [(16, 16), (16, 48), (32, 16), (80, 80), (272, 400)])
def test_mixed_ragged_shapes(shape):
    src = synth.laplacian_residual(3200 + shape[1], *shape)
    check(src, 27, 18)


def test_mixed_extremes():
    # saturated and structured content: +-255 residuals, constant regions,
    # 8x8 quadrants of different constants, a checkerboard
    a = np.zeros((64, 64), np.int16)
    a[:16, :16] = 255
    a[:16, 16:32] = -255
    a[16:32, :32] = np.kron(np.array([[200, -200, 7, 9], [-100, 50, -3, 0]]), np.ones((8, 8), np.int64))
    a[32:48, :] = (np.indices((16, 64)).sum(axis=0) % 2) * 510 - 255
    for qp in (0, 4, 22, 37, 63):
        for lam in (0, 1, 1000):
            check(a, qp, lam)
    u = np.clip(a + 128, 0, 255).astype(np.uint8)
    for qp in (0, 22, 51):
        check(u, qp, 3)


def test_mixed_optional_outputs_and_pitch():
    src = synth.laplacian_residual(3300, 64, 96)
    wide = torch.zeros((64, 160), dtype=torch.int16, device="cuda")
    wide[:, 32:128] = dev(src)
    out = torch.full((64, 160), 5, dtype=torch.int16, device="cuda")
    s = adct.mixed_encode(wide[:, 32:128], 32, 40, out[:, 32:128], image_height=32)
    ws, wq, wout = X.mixed_encode(src, 32, 40)
    o = host(out)
    assert np.array_equal(o[:, 32:128], wout)
    assert np.all(o[:, :32] == 5) and np.all(o[:, 128:] == 5)
    assert np.array_equal(host(s), X.sse_per_image(wout, src, 32))
    # no SSE, levels only
    q = torch.zeros((24, 16, 16), dtype=torch.int16, device="cuda")
    adct.mixed_encode(wide[:, 32:128], 32, 40, out[:, 32:128], q=q, want_sse=False)
    assert np.array_equal(host(q), wq)


@pytest.mark.parametrize("qp", [0, 3, 4, 27])
def test_mixed_regions_equal_the_standalone_codecs(qp):
    # each region's levels and reconstruction are those of the codec it
    # chose, coded alone by adct_encode_quant (16x16) or adct_t8_encode_quant
    # (8x8), level saturation included: constant +-2047 regions give 16x16
    # DC levels of 32752 / Delta, saturated to int16 below QP 4
    i = np.arange(16)
    chk = np.where((i[:, None] + i[None, :]) % 2 == 0, 2047, -2047)
    quad = np.kron(np.array([[2047, -2047], [-1000, 600]]), np.ones((8, 8), np.int64))
    top = np.concatenate([np.full((16, 16), 2047), np.full((16, 16), -2047), chk, quad,
                          synth.laplacian_residual(3600 + qp, 16, 16)], axis=1)
    src = np.concatenate([top, synth.laplacian_residual(3700 + qp, 16, 80)]).astype(np.int16)
    x = dev(src)
    o16, o8 = torch.empty_like(x), torch.empty_like(x)
    q16 = torch.empty((10, 16, 16), dtype=torch.int16, device="cuda")
    q8 = torch.empty((40, 8, 8), dtype=torch.int16, device="cuda")
    adct.encode_quant(x, qp, o16, q=q16, want_sse=False)
    adct.t8_encode_quant(x, qp, o8, q=q8, want_sse=False)
    h16, h8, p16, p8 = host(q16), host(q8), host(o16), host(o8)
    if qp < 4:
        assert h16[0, 0, 0] == 32767 and h16[1, 0, 0] == -32768
    for lam in (0, 18, 1 << 40):
        split, q, out, s = run(src, qp, lam, image_height=32)
        for k in range(10):
            by, bx = divmod(k, 5)
            rows, cols = slice(16 * by, 16 * by + 16), slice(16 * bx, 16 * bx + 16)
            if split[k]:
                for a in range(2):
                    for b in range(2):
                        blk = h8[(2 * by + a) * 10 + 2 * bx + b]
                        assert np.array_equal(q[k, 8 * a:8 * a + 8, 8 * b:8 * b + 8], blk), (lam, k, a, b)
                assert np.array_equal(out[rows, cols], p8[rows, cols]), (lam, k)
            else:
                assert np.array_equal(q[k], h16[k]), (lam, k)
                assert np.array_equal(out[rows, cols], p16[rows, cols]), (lam, k)
        d = out.astype(np.int64) - src
        assert s[0] == (d * d).sum()


def test_mixed_sse_over_many_waves_and_images():
    # 5 images of 544 x 960 (2040 regions each): many waves per image, and
    # wave ranges that cross image boundaries
    n, h, w = 5, 544, 960
    src = np.concatenate([synth.laplacian_residual(3400 + i, h, w) for i in range(n)])
    check(src, 27, 18, image_height=h)


def test_mixed_video_frame_full_size():
    # one 1920x1088 4:2:0 frame of residual planes at the QPs of the video workload
    for qp in (22, 27, 32, 37):
        lam = int(round(0.57 * 2 ** ((qp - 12) / 3)))
        for plane in synth.video_frame_planes(7):
            check(plane, qp, lam)


def test_mixed_decodes_with_the_oracle_decoder():
    src = synth.laplacian_residual(3500, 64, 64)
    split, q, out, _ = run(src, 32, 30)
    assert np.array_equal(X.mixed_decode(split, q.astype(np.int64), 32, 64, 64), out)
