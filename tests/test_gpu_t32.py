"""GPU parity of the 32-point calls (32x32 blocks) against the oracle
(oracle/t32.py): bit-exact coefficients, levels, reconstructions and
per-image SSE, on ragged workgroups (tile counts not multiples of 8),
pitched planes, images straddling workgroups, interleaved launches (large
images) and the benchmark's full size."""
import numpy as np
import pytest

from oracle import adct_oracle as O
from oracle import t32 as T32
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1606_07414_amd import adct  # noqa: E402


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


# tile counts 1, 15 (ragged group), 64, 255 (ragged), 2040 (video Y plane)
SHAPES = [(32, 32), (96, 160), (256, 256), (480, 544), (1088, 1920)]


@pytest.mark.parametrize("shape", SHAPES)
def test_t32_fwd2d_u8(shape):
    print(f"[t32] fwd2d u8 {shape}", flush=True)
    img = synth.ar1_image(3200 + shape[1], *shape)
    assert np.array_equal(host(adct.t32_fwd2d(dev(img))), T32.fwd2d_32(img))


def test_t32_fwd2d_extremes_and_i16():
    z = np.zeros((64, 96), np.uint8)
    z[:32, :32] = 255
    z[32:, 32:64] = np.indices((32, 32)).sum(axis=0) * 17 % 256
    assert np.array_equal(host(adct.t32_fwd2d(dev(z))), T32.fwd2d_32(z))
    res = synth.laplacian_residual(3201, 96, 128)
    res[0, :32] = 255
    res[1, :32] = -255
    assert np.array_equal(host(adct.t32_fwd2d(dev(res))), T32.fwd2d_32(res))
    wide = np.full((32, 64), 2047, np.int16)
    wide[:, 32:] = -2047
    assert np.array_equal(host(adct.t32_fwd2d(dev(wide))), T32.fwd2d_32(wide))


@pytest.mark.parametrize("n", [1, 7, 8, 301])
def test_t32_inv2d(n):
    rng = np.random.default_rng(3202 + n)
    Y = rng.integers(-200000, 200000, size=(n, 32, 32)).astype(np.int32)
    assert np.array_equal(host(adct.t32_inv2d(dev(Y))), T32.inv2d_32(Y))


def test_t32_pitched_plane():
    img = synth.ar1_image(3203, 64, 96)
    buf = torch.zeros((64, 160), dtype=torch.uint8, device="cuda")
    buf[:, 32:128] = dev(img)
    view = buf[:, 32:128]
    assert np.array_equal(host(adct.t32_fwd2d(view)), T32.fwd2d_32(img))
    out_buf = torch.full((64, 192), 7, dtype=torch.uint8, device="cuda")
    out = out_buf[:, 64:160]
    s = host(adct.t32_encode_zonal(view, 8, out))
    want = T32.zonal_reconstruct_32(img, 8)
    assert np.array_equal(host(out), want)
    assert s[0] == O.sse(want, img)
    assert int((out_buf[:, :64] != 7).sum().item()) == 0 and int((out_buf[:, 160:] != 7).sum().item()) == 0


# a zonal launch takes a compile-time bound on r (8, 16 or 32): both ends of
# every class are here
@pytest.mark.parametrize("r", [0, 1, 2, 5, 8, 9, 16, 17, 31, 32])
@pytest.mark.parametrize("store", [True, False])
@pytest.mark.parametrize("shape,image_h", [((96, 160), 96), ((192, 96), 64), ((512, 256), 128), ((32, 32), 32)])
def test_t32_encode_zonal(r, store, shape, image_h):
    img = synth.ar1_batch(shape[0] // image_h, image_h, shape[1], seed_base=3300 + r)
    x = dev(img)
    out = torch.empty_like(x)
    coef = torch.full((x.numel() // 1024, 32, 32), -9, dtype=torch.int32, device="cuda")
    s = host(adct.t32_encode_zonal(x, r, out, coef=coef if store else None, image_height=image_h))
    want = T32.zonal_reconstruct_32(img, r)
    assert np.array_equal(host(out), want)
    if store:
        assert np.array_equal(host(coef), T32.fwd2d_32(img))
    else:
        assert int((coef != -9).sum().item()) == 0
    for k in range(shape[0] // image_h):
        assert s[k] == O.sse(want[k * image_h:(k + 1) * image_h], img[k * image_h:(k + 1) * image_h])


@pytest.mark.parametrize("qp", [0, 4, 22, 27, 32, 37, 51, 63])
@pytest.mark.parametrize("kind", ["u8", "i16"])
def test_t32_encode_quant(qp, kind):
    print(f"[t32] encode_quant qp={qp} {kind}", flush=True)
    if kind == "u8":
        img, lo = synth.ar1_batch(3, 96, 160, seed_base=3400 + qp), 0
    else:
        img, lo = np.concatenate([synth.laplacian_residual(3400 + qp + k, 96, 160) for k in range(3)]), -255
    x = dev(img)
    out = torch.empty_like(x)
    q = torch.full((x.numel() // 1024, 32, 32), 99, dtype=torch.int16, device="cuda")
    s = host(adct.t32_encode_quant(x, qp, out, q=q, image_height=96))
    wq, _, want = T32.quant_reconstruct_32(img, qp, lo=lo, hi=255)
    assert np.array_equal(host(q), wq)
    assert np.array_equal(host(out), want)
    for k in range(3):
        assert s[k] == O.sse(want[k * 96:(k + 1) * 96], img[k * 96:(k + 1) * 96])


@pytest.mark.parametrize("qp", [0, 9, 10])
def test_t32_level_saturation_on_wide_int16(qp):
    # constant tiles of +-2047 (the int16 sample bound): the DC level leaves
    # int16 below QP 10 and is saturated on both sides
    img = np.full((64, 64), 2047, np.int16)
    img[32:, :32] = -2047
    img[:32, 32:] = synth.laplacian_residual(3500, 32, 32)
    x = dev(img)
    out = torch.empty_like(x)
    q = torch.empty((4, 32, 32), dtype=torch.int16, device="cuda")
    adct.t32_encode_quant(x, qp, out, q=q, want_sse=False)
    wq, _, want = T32.quant_reconstruct_32(img, qp, lo=-255, hi=255)
    assert np.array_equal(host(q), wq)
    assert np.array_equal(host(out), want)


def test_t32_images_straddling_workgroups_and_interleaved_launch():
    # 5 images of 32 x 96 (3 tiles each): groups of 8 tiles straddle images
    img = synth.ar1_batch(5, 32, 96, seed_base=3600)
    x = dev(img)
    out = torch.empty_like(x)
    s = host(adct.t32_encode_quant(x, 27, out, image_height=32))
    _, _, want = T32.quant_reconstruct_32(img, 27, lo=0, hi=255)
    assert np.array_equal(host(out), want)
    for k in range(5):
        assert s[k] == O.sse(want[32 * k:32 * (k + 1)], img[32 * k:32 * (k + 1)])
    # 3 images of 1024 x 1024 (1024 tiles, 128 groups each): the launch
    # interleaves its workgroups over the images
    big = synth.ar1_batch(3, 1024, 1024, seed_base=3601)
    xb = dev(big)
    ob = torch.empty_like(xb)
    sb = host(adct.t32_encode_zonal(xb, 12, ob, image_height=1024))
    wantb = T32.zonal_reconstruct_32(big, 12)
    assert np.array_equal(host(ob), wantb)
    for k in range(3):
        assert sb[k] == O.sse(wantb[1024 * k:1024 * (k + 1)], big[1024 * k:1024 * (k + 1)])


def test_t32_full_size_sampled():
    # the 32x32 codec on the benchmark's batch: 1024 images of 512 x 512
    # (262144 tiles); every output against the oracle on a sample of images,
    # and the identity T32^T (W . T32 X T32^T) T32 = 1024 X on the whole batch
    print("[t32] full size 1024 x 512 x 512", flush=True)
    img = synth.ar1_batch(1024, 512, 512)
    x = dev(img)
    out = torch.empty_like(x)
    coef = torch.empty((x.numel() // 1024, 32, 32), dtype=torch.int32, device="cuda")
    s = host(adct.t32_encode_zonal(x, 32, out, coef=coef, image_height=512))
    assert torch.equal(out, x) and not s.any()  # r = 32 keeps everything: lossless
    s = host(adct.t32_encode_zonal(x, 8, out, coef=coef, image_height=512))
    for k in (0, 511, 1023):
        sub = img[512 * k:512 * (k + 1)]
        want = T32.zonal_reconstruct_32(sub, 8)
        assert np.array_equal(host(out[512 * k:512 * (k + 1)]), want), k
        assert np.array_equal(host(coef[256 * k:256 * (k + 1)]), T32.fwd2d_32(sub)), k
        assert s[k] == O.sse(want, sub), k
    q = torch.empty((x.numel() // 1024, 32, 32), dtype=torch.int16, device="cuda")
    s = host(adct.t32_encode_quant(x, 27, out, q=q, image_height=512))
    for k in (3, 700):
        sub = img[512 * k:512 * (k + 1)]
        wq, _, want = T32.quant_reconstruct_32(sub, 27, lo=0, hi=255)
        assert np.array_equal(host(q[256 * k:256 * (k + 1)]), wq), k
        assert np.array_equal(host(out[512 * k:512 * (k + 1)]), want), k
        assert s[k] == O.sse(want, sub), k


def test_t32_errors_and_empty():
    x = torch.zeros((48, 64), dtype=torch.uint8, device="cuda")  # 48 is not a multiple of 32
    with pytest.raises(adct.AdctError) as e:
        adct.t32_fwd2d(x, coef=torch.empty((2, 32, 32), dtype=torch.int32, device="cuda"))
    assert e.value.code == adct.E_SHAPE
    y = torch.zeros((64, 64), dtype=torch.uint8, device="cuda")
    with pytest.raises(adct.AdctError) as e:
        adct.t32_encode_zonal(y, 33, torch.empty_like(y))
    assert e.value.code == adct.E_ARG
    with pytest.raises(adct.AdctError) as e:
        adct.t32_encode_quant(y, 64, torch.empty_like(y))
    assert e.value.code == adct.E_ARG
    with pytest.raises(adct.AdctError) as e:
        adct.t32_encode_zonal(y, 4, torch.empty_like(y), image_height=48)
    assert e.value.code == adct.E_SHAPE
    empty = torch.empty((0, 32, 32), dtype=torch.int32, device="cuda")
    assert adct.t32_inv2d(empty).numel() == 0
