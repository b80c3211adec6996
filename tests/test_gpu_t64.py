"""GPU parity of the 64-point calls (64x64 blocks) against the oracle
(oracle/t64.py): bit-exact coefficients, levels, reconstructions and
per-image SSE, on ragged workgroups (odd tile counts), pitched planes,
images straddling workgroups, interleaved launches (large images) and the
benchmark's full size."""
import numpy as np
import pytest

from oracle import adct_oracle as O
from oracle import t64 as T64
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1606_07414_amd import adct  # noqa: E402


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


# tile counts 1, 15 (ragged workgroup), 64, 63 (ragged), 510 (video Y plane)
SHAPES = [(64, 64), (192, 320), (512, 512), (448, 576), (1088, 1920)]


@pytest.mark.parametrize("shape", SHAPES)
def test_t64_fwd2d_u8(shape):
    print(f"[t64] fwd2d u8 {shape}", flush=True)
    img = synth.ar1_image(6400 + shape[1], *shape)
    assert np.array_equal(host(adct.t64_fwd2d(dev(img))), T64.fwd2d_64(img))


def test_t64_fwd2d_extremes_and_i16():
    z = np.zeros((128, 192), np.uint8)
    z[:64, :64] = 255
    z[64:, 64:128] = np.indices((64, 64)).sum(axis=0) * 17 % 256
    assert np.array_equal(host(adct.t64_fwd2d(dev(z))), T64.fwd2d_64(z))
    res = synth.laplacian_residual(6401, 128, 128)
    res[0, :64] = 255
    res[1, :64] = -255
    assert np.array_equal(host(adct.t64_fwd2d(dev(res))), T64.fwd2d_64(res))
    wide = np.full((64, 128), 2047, np.int16)
    wide[:, 64:] = -2047
    assert np.array_equal(host(adct.t64_fwd2d(dev(wide))), T64.fwd2d_64(wide))


@pytest.mark.parametrize("n", [1, 2, 3, 101])
def test_t64_inv2d(n):
    rng = np.random.default_rng(6402 + n)
    Y = rng.integers(-100000, 100000, size=(n, 64, 64)).astype(np.int32)
    assert np.array_equal(host(adct.t64_inv2d(dev(Y))), T64.inv2d_64(Y))


def test_t64_pitched_plane():
    img = synth.ar1_image(6403, 128, 192)
    buf = torch.zeros((128, 320), dtype=torch.uint8, device="cuda")
    buf[:, 64:256] = dev(img)
    view = buf[:, 64:256]
    assert np.array_equal(host(adct.t64_fwd2d(view)), T64.fwd2d_64(img))
    out_buf = torch.full((128, 384), 7, dtype=torch.uint8, device="cuda")
    out = out_buf[:, 128:320]
    s = host(adct.t64_encode_zonal(view, 8, out))
    want = T64.zonal_reconstruct_64(img, 8)
    assert np.array_equal(host(out), want)
    assert s[0] == O.sse(want, img)
    assert int((out_buf[:, :128] != 7).sum().item()) == 0 and int((out_buf[:, 320:] != 7).sum().item()) == 0


# a zonal launch takes a compile-time bound on r (8, 16, 32 or 64): both
# ends of every class are here
@pytest.mark.parametrize("r", [0, 1, 2, 5, 8, 9, 16, 17, 32, 33, 63, 64])
@pytest.mark.parametrize("store", [True, False])
@pytest.mark.parametrize("shape,image_h", [((192, 320), 192), ((384, 128), 128), ((512, 256), 64), ((64, 64), 64)])
def test_t64_encode_zonal(r, store, shape, image_h):
    img = synth.ar1_batch(shape[0] // image_h, image_h, shape[1], seed_base=6500 + r)
    x = dev(img)
    out = torch.empty_like(x)
    coef = torch.full((x.numel() // 4096, 64, 64), -9, dtype=torch.int32, device="cuda")
    s = host(adct.t64_encode_zonal(x, r, out, coef=coef if store else None, image_height=image_h))
    want = T64.zonal_reconstruct_64(img, r)
    assert np.array_equal(host(out), want)
    if store:
        assert np.array_equal(host(coef), T64.fwd2d_64(img))
    else:
        assert int((coef != -9).sum().item()) == 0
    for k in range(shape[0] // image_h):
        assert s[k] == O.sse(want[k * image_h:(k + 1) * image_h], img[k * image_h:(k + 1) * image_h])


@pytest.mark.parametrize("qp", [0, 4, 15, 16, 22, 27, 37, 51, 63])
@pytest.mark.parametrize("kind", ["u8", "i16"])
def test_t64_encode_quant(qp, kind):
    print(f"[t64] encode_quant qp={qp} {kind}", flush=True)
    if kind == "u8":
        img, lo = synth.ar1_batch(3, 128, 192, seed_base=6600 + qp), 0
    else:
        img, lo = np.concatenate([synth.laplacian_residual(6600 + qp + k, 128, 192) for k in range(3)]), -255
    x = dev(img)
    out = torch.empty_like(x)
    q = torch.full((x.numel() // 4096, 64, 64), 99, dtype=torch.int16, device="cuda")
    s = host(adct.t64_encode_quant(x, qp, out, q=q, image_height=128))
    wq, _, want = T64.quant_reconstruct_64(img, qp, lo=lo, hi=255)
    assert np.array_equal(host(q), wq)
    assert np.array_equal(host(out), want)
    for k in range(3):
        assert s[k] == O.sse(want[k * 128:(k + 1) * 128], img[k * 128:(k + 1) * 128])


@pytest.mark.parametrize("qp", [0, 15, 16])
def test_t64_level_saturation_on_wide_int16(qp):
    # constant tiles of +-2047 (the int16 sample bound): the DC level leaves
    # int16 below QP 16 and is saturated on both sides; a random residual
    # tile of the same range beside them
    img = np.full((128, 128), 2047, np.int16)
    img[64:, :64] = -2047
    img[:64, 64:] = np.random.default_rng(6700).integers(-2047, 2048, (64, 64))
    x = dev(img)
    out = torch.empty_like(x)
    q = torch.empty((4, 64, 64), dtype=torch.int16, device="cuda")
    adct.t64_encode_quant(x, qp, out, q=q, want_sse=False)
    wq, _, want = T64.quant_reconstruct_64(img, qp, lo=-255, hi=255)
    assert np.array_equal(host(q), wq)
    assert np.array_equal(host(out), want)


def test_t64_images_straddling_workgroups_and_interleaved_launch():
    # 5 images of 64 x 192 (3 tiles each): groups of 2 tiles straddle images
    img = synth.ar1_batch(5, 64, 192, seed_base=6800)
    x = dev(img)
    out = torch.empty_like(x)
    s = host(adct.t64_encode_quant(x, 27, out, image_height=64))
    _, _, want = T64.quant_reconstruct_64(img, 27, lo=0, hi=255)
    assert np.array_equal(host(out), want)
    for k in range(5):
        assert s[k] == O.sse(want[64 * k:64 * (k + 1)], img[64 * k:64 * (k + 1)])
    # 3 images of 1024 x 1024 (256 tiles, 128 groups each): the launch
    # interleaves its workgroups over the images
    big = synth.ar1_batch(3, 1024, 1024, seed_base=6801)
    xb = dev(big)
    ob = torch.empty_like(xb)
    sb = host(adct.t64_encode_zonal(xb, 12, ob, image_height=1024))
    wantb = T64.zonal_reconstruct_64(big, 12)
    assert np.array_equal(host(ob), wantb)
    for k in range(3):
        assert sb[k] == O.sse(wantb[1024 * k:1024 * (k + 1)], big[1024 * k:1024 * (k + 1)])


def test_t64_full_size_sampled():
    # the 64x64 codec on the benchmark's batch: 1024 images of 512 x 512
    # (65536 tiles); every output against the oracle on a sample of images,
    # and the identity T64^T (W . T64 X T64^T) T64 = 4096 X on the whole batch
    print("[t64] full size 1024 x 512 x 512", flush=True)
    img = synth.ar1_batch(1024, 512, 512)
    x = dev(img)
    out = torch.empty_like(x)
    coef = torch.empty((x.numel() // 4096, 64, 64), dtype=torch.int32, device="cuda")
    s = host(adct.t64_encode_zonal(x, 64, out, coef=coef, image_height=512))
    assert torch.equal(out, x) and not s.any()  # r = 64 keeps everything: lossless
    s = host(adct.t64_encode_zonal(x, 16, out, coef=coef, image_height=512))
    # on every image: keeping 16 x 16 of each 64x64 block is the same
    # projection as keeping 8 x 8 of each 32x32 block (the construction's
    # rows pair up into the 32-point rows on each half), bit for bit
    out32 = torch.empty_like(x)
    s32 = host(adct.t32_encode_zonal(x, 8, out32, image_height=512))
    assert torch.equal(out, out32) and np.array_equal(s, s32)
    del out32
    for k in (0, 511, 1023):
        sub = img[512 * k:512 * (k + 1)]
        want = T64.zonal_reconstruct_64(sub, 16)
        assert np.array_equal(host(out[512 * k:512 * (k + 1)]), want), k
        assert np.array_equal(host(coef[64 * k:64 * (k + 1)]), T64.fwd2d_64(sub)), k
        assert s[k] == O.sse(want, sub), k
    q = torch.empty((x.numel() // 4096, 64, 64), dtype=torch.int16, device="cuda")
    s = host(adct.t64_encode_quant(x, 27, out, q=q, image_height=512))
    for k in (3, 700):
        sub = img[512 * k:512 * (k + 1)]
        wq, _, want = T64.quant_reconstruct_64(sub, 27, lo=0, hi=255)
        assert np.array_equal(host(q[64 * k:64 * (k + 1)]), wq), k
        assert np.array_equal(host(out[512 * k:512 * (k + 1)]), want), k
        assert s[k] == O.sse(want, sub), k


def test_t64_errors_and_empty():
    x = torch.zeros((96, 128), dtype=torch.uint8, device="cuda")  # 96 is not a multiple of 64
    with pytest.raises(adct.AdctError) as e:
        adct.t64_fwd2d(x, coef=torch.empty((2, 64, 64), dtype=torch.int32, device="cuda"))
    assert e.value.code == adct.E_SHAPE
    y = torch.zeros((128, 128), dtype=torch.uint8, device="cuda")
    with pytest.raises(adct.AdctError) as e:
        adct.t64_encode_zonal(y, 65, torch.empty_like(y))
    assert e.value.code == adct.E_ARG
    with pytest.raises(adct.AdctError) as e:
        adct.t64_encode_quant(y, 64, torch.empty_like(y))
    assert e.value.code == adct.E_ARG
    with pytest.raises(adct.AdctError) as e:
        adct.t64_encode_zonal(y, 4, torch.empty_like(y), image_height=96)
    assert e.value.code == adct.E_SHAPE
    empty = torch.empty((0, 64, 64), dtype=torch.int32, device="cuda")
    assert adct.t64_inv2d(empty).numel() == 0
