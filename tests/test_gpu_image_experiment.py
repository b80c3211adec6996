"""GPU parity for Section 3.1's experiment as the paper runs it: zig-zag
retention of the first r coefficients (bit-exact against the oracle) and the
SSIM index (float64 on both sides, within 1e-9 relative); and, at the
experiment's full size (1024 images of 512x512 in one call), the zig-zag
encoder and the comparison codecs."""
import numpy as np
import pytest

from oracle import adct_oracle as O
from oracle import image_experiment as E
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1606_07414_amd import adct  # noqa: E402

SSIM_RTOL = 1e-9


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.mark.parametrize("r", [0, 1, 3, 10, 36, 100, 136, 150, 200, 256])
def test_zigzag_elementwise(r):
    coef = O.fwd2d(synth.ar1_image(1000 + r, 48, 80))
    got = host(adct.zigzag(dev(coef.astype(np.int32)), r))
    assert np.array_equal(got, E.zigzag(coef, r))


@pytest.mark.parametrize("r", [0, 1, 2, 6, 15, 21, 64, 136, 150, 256])
@pytest.mark.parametrize("shape,image_h", [((272, 528), 272), ((96, 48), 32), ((1024, 512), 512)])
def test_zigzag_recon_with_sse(r, shape, image_h):
    img = synth.ar1_batch(shape[0] // image_h, image_h, shape[1], seed_base=1100 + r)
    x = dev(img)
    coef = adct.fwd2d(x)
    out = torch.empty_like(x)
    s = host(adct.zigzag_recon(coef, r, out, ref=x, image_height=image_h))
    want = E.zigzag_reconstruct(img, r)
    assert np.array_equal(host(out), want)
    for i in range(shape[0] // image_h):
        assert s[i] == O.sse(want[i * image_h:(i + 1) * image_h], img[i * image_h:(i + 1) * image_h]), i


@pytest.mark.parametrize("r", [1, 5, 28, 150])
@pytest.mark.parametrize("store", [True, False])
def test_encode_zigzag_u8(r, store):
    img = synth.ar1_batch(3, 144, 208, seed_base=1200 + r)
    x = dev(img)
    out = torch.empty_like(x)
    coef = torch.full((x.numel() // 256, 16, 16), -3, dtype=torch.int32, device="cuda")
    s = host(adct.encode_zigzag(x, r, out, coef=coef if store else None, image_height=144))
    want = E.zigzag_reconstruct(img, r)
    assert np.array_equal(host(out), want)
    if store:
        assert np.array_equal(host(coef), O.fwd2d(img))
    else:
        assert np.all(host(coef) == -3)
    for i in range(3):
        assert s[i] == O.sse(want[i * 144:(i + 1) * 144], img[i * 144:(i + 1) * 144])
    # the two-pass path gives the same bytes
    out2 = torch.empty_like(x)
    s2 = host(adct.zigzag_recon(adct.fwd2d(x), r, out2, ref=x, image_height=144))
    assert torch.equal(out, out2) and np.array_equal(s, s2)


@pytest.mark.parametrize("r", [3, 45, 150])
def test_encode_zigzag_i16_residual(r):
    res = synth.laplacian_residual(1300 + r, 128, 160)
    x = dev(res)
    out = torch.empty_like(x)
    s = host(adct.encode_zigzag(x, r, out, image_height=128))
    want = E.zigzag_reconstruct(res, r, lo=-255, hi=255)
    assert np.array_equal(host(out), want)
    assert s[0] == O.sse(want, res)


def test_zigzag_special_cases_on_gpu():
    img = synth.ar1_image(1400, 64, 96)
    x = dev(img)
    out = torch.empty_like(x)
    s = host(adct.encode_zigzag(x, 256, out))
    assert torch.equal(out, x) and s[0] == 0
    o1, o2 = torch.empty_like(x), torch.empty_like(x)
    adct.encode_zigzag(x, 1, o1)
    adct.encode_zonal(x, 1, o2)
    assert torch.equal(o1, o2)


def test_batch_zigzag_matches_single_image():
    sizes = synth.uneven_sizes(17, 16, 320, seed=1500)
    imgs = [synth.ar1_image(1500 + k, h, w) for k, (h, w) in enumerate(sizes)]
    xs = [dev(i) for i in imgs]
    dsts = [torch.empty_like(x) for x in xs]
    coefs = [torch.empty((x.numel() // 256, 16, 16), dtype=torch.int32, device="cuda") for x in xs]
    sses = [torch.empty(1, dtype=torch.int64, device="cuda") for _ in xs]
    b = adct.Batch(xs, dsts, adct.OP_ZIGZAG, 66, coefs=coefs, sses=sses)
    b.submit()
    torch.cuda.synchronize()
    for k, x in enumerate(xs):
        out = torch.empty_like(x)
        c = torch.empty_like(coefs[k])
        s = adct.encode_zigzag(x, 66, out, coef=c)
        torch.cuda.synchronize()
        assert torch.equal(dsts[k], out) and torch.equal(coefs[k], c) and torch.equal(sses[k], s), k
    for k in (0, 16):
        assert np.array_equal(host(dsts[k]), E.zigzag_reconstruct(imgs[k], 66))
    b.close()


# ---------------------------------------------------------------- SSIM
@pytest.mark.parametrize("r", [1, 6, 45, 150])
def test_ssim_matches_oracle(r):
    img = synth.ar1_batch(3, 96, 112, seed_base=1600 + r)
    x = dev(img)
    out = torch.empty_like(x)
    adct.encode_zigzag(x, r, out, want_sse=False)
    got = host(adct.ssim(x, out, image_height=96))
    want = E.ssim_per_image(img, host(out), 96)
    assert np.allclose(got, want, rtol=SSIM_RTOL, atol=0), (got, want)


def test_ssim_identity_constant_and_pitched():
    img = synth.ar1_image(1700, 64, 80)
    x = dev(img)
    assert abs(host(adct.ssim(x, x))[0] - 1.0) < 1e-12
    a = torch.full((32, 48), 100, dtype=torch.uint8, device="cuda")
    b = torch.full((32, 48), 120, dtype=torch.uint8, device="cuda")
    c1 = (0.01 * 255) ** 2
    assert host(adct.ssim(a, b))[0] == pytest.approx((2 * 100 * 120 + c1) / (100 ** 2 + 120 ** 2 + c1), rel=1e-12)
    # pitched views (rows 16 bytes apart are not contiguous)
    wide = torch.zeros((64, 128), dtype=torch.uint8, device="cuda")
    wide[:, 16:96] = x
    y = dev(E.zigzag_reconstruct(img, 10))
    wide2 = torch.zeros((64, 112), dtype=torch.uint8, device="cuda")
    wide2[:, 32:112] = y
    got = host(adct.ssim(wide[:, 16:96], wide2[:, 32:112]))[0]
    assert got == pytest.approx(E.ssim(img, host(y)), rel=SSIM_RTOL)


def test_ssim_full_size_batch_sampled():
    # the launch shape of the image-experiment benchmark: 1024 images of 512x512
    img = synth.ar1_batch(1024, 512, 512)
    x = dev(img)
    out = torch.empty_like(x)
    adct.encode_zigzag(x, 21, out, want_sse=False)
    got = host(adct.ssim(x, out, image_height=512))
    o = host(out)
    for k in (0, 517, 1023):
        want = E.ssim(img[k * 512:(k + 1) * 512], o[k * 512:(k + 1) * 512])
        assert got[k] == pytest.approx(want, rel=SSIM_RTOL), k
    assert np.all((got > 0.3) & (got < 1.0))


@pytest.fixture(scope="module")
def full_batch():
    img = synth.ar1_batch(1024, 512, 512)
    return img, dev(img)


@pytest.mark.parametrize("codec,kind,r", [("zigzag", None, 21), ("zigzag", None, 150), ("wht", "zigzag", 21),
                                          ("wht", "zonal", 4), ("dct", "zonal", 4), ("dct", "zigzag", 105)])
def test_image_experiment_codecs_full_size(full_batch, codec, kind, r):
    # the launch shape of the image-experiment benchmark (1024 images of
    # 512x512, one call): every image's SSE against the squared error of the
    # returned reconstruction; images 0, 517 and 1023 against the oracle
    from oracle import comparison as CMP
    img, x = full_batch
    out = torch.full_like(x, 5)
    sse = torch.full((1024,), -1, dtype=torch.int64, device="cuda")
    coef = None
    if codec == "zigzag":
        coef = torch.full((x.numel() // 256, 16, 16), -3, dtype=torch.int32, device="cuda")
        adct.encode_zigzag(x, r, out, coef=coef, image_height=512, sse=sse)
    else:
        xf = adct.XF_WHT if codec == "wht" else adct.XF_DCT
        keep = adct.KEEP_ZIGZAG if kind == "zigzag" else adct.KEEP_ZONAL
        adct.compare_encode(x, xf, keep, r, out, image_height=512, sse=sse)
    got, s = host(out).astype(np.int64), host(sse)
    d = got - img.astype(np.int64)
    assert np.array_equal(s, (d * d).reshape(1024, -1).sum(axis=1))
    ckind = CMP.ZIGZAG if kind == "zigzag" else CMP.ZONAL
    for k in (0, 517, 1023):
        sl = slice(k * 512, (k + 1) * 512)
        if codec == "zigzag":
            assert np.array_equal(got[sl], E.zigzag_reconstruct(img[sl], r)), k
            assert np.array_equal(host(coef[k * 1024:(k + 1) * 1024]), O.fwd2d(img[sl])), k
        elif codec == "wht":
            assert np.array_equal(got[sl], CMP.wht_reconstruct(img[sl], ckind, r)), k
        else:
            # fp32 on the matrix cores against float64: equal away from
            # rounding ties, within one step at them
            real = CMP.dct_reconstruct_real(img[sl], ckind, r)
            want = CMP.dct_reconstruct(img[sl], ckind, r).astype(np.int64)
            near = np.abs(real - np.floor(real) - 0.5) < 1e-3
            assert np.array_equal(got[sl][~near], want[~near]), k
            assert np.all(np.abs(got[sl] - want) <= 1), k
