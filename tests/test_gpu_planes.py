"""GPU parity of adct_encode_quant_planes: several planes coded in one launch
must give exactly what the per-plane encoder of the same block size
(adct_encode_quant, adct_t8_encode_quant, adct_t32_encode_quant) gives on
each plane alone (levels, reconstruction, per-image SSE), and a sample the
oracle's values; each job writes only its own outputs; bad job sets are
refused before any launch."""
import numpy as np
import pytest

from oracle import adct_oracle as O
from oracle import t8 as T8
from oracle import t32 as T32
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1606_07414_amd import adct  # noqa: E402


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


ALONE = {16: adct.encode_quant, 8: adct.t8_encode_quant, 32: adct.t32_encode_quant}


def _levels(x, block, fill=None):
    shape = (x.numel() // (block * block), block, block)
    if fill is None:
        return torch.empty(shape, dtype=torch.int16, device="cuda")
    return torch.full(shape, fill, dtype=torch.int16, device="cuda")


def _alone(x, qp, ih, store, want_sse, block):
    out = torch.empty_like(x)
    q = _levels(x, block) if store else None
    s = ALONE[block](x, qp, out, q=q, image_height=ih, want_sse=want_sse)
    torch.cuda.synchronize()
    return out, q, s


def _run_and_compare(xs, ihs, qp, store=True, want_sse=True, block=16):
    jobs, outs, qs = [], [], []
    for x, ih in zip(xs, ihs):
        o = torch.full_like(x, 77)
        q = _levels(x, block, -5) if store else None
        jobs.append((x, o, q, ih))
        outs.append(o)
        qs.append(q)
    sses = adct.encode_quant_planes(jobs, qp, block=block, want_sse=want_sse)
    torch.cuda.synchronize()
    for k, (x, ih) in enumerate(zip(xs, ihs)):
        o1, q1, s1 = _alone(x, qp, ih, store, want_sse, block)
        assert torch.equal(outs[k], o1), k
        if store:
            assert torch.equal(qs[k], q1), k
        if want_sse:
            assert torch.equal(sses[k], s1), k
        else:
            assert sses[k] is None
    return outs, qs, sses


def _frames(n, w=1920, h=1088):
    planes = [[], [], []]
    for f in range(n):
        for i, p in enumerate(synth.video_frame_planes(f, w, h)):
            planes[i].append(p)
    return [np.concatenate(p) for p in planes]


@pytest.mark.parametrize("qp", [0, 3, 4, 22, 27, 37, 51])
def test_video_frame_planes_match_single_calls(qp):
    # 3 frames of 4:2:0 int16 residuals (Y 1088 x 1920: 8160 tiles per frame,
    # interleaved SSE order; U and V 544 x 960: plain order) in one launch;
    # QP 0-3 take the saturating quantiser
    print(f"[planes] video qp={qp}", flush=True)
    ys = _frames(3)
    xs = [dev(p) for p in ys]
    outs, qs, sses = _run_and_compare(xs, [1088, 544, 544], qp)
    # the oracle on the second frame's V plane
    v = ys[2][544:1088]
    wq, _, want = O.quant_reconstruct(v, qp, lo=-255, hi=255)
    assert np.array_equal(outs[2][544:1088].cpu().numpy(), want)
    assert np.array_equal(qs[2][2040:4080].cpu().numpy(), wq)
    assert int(sses[2][1].item()) == O.sse(want, v)


@pytest.mark.parametrize("qp", [0, 27, 51])
@pytest.mark.parametrize("block", [8, 32])
def test_video_frame_planes_other_blocks(block, qp):
    # the same frame stacks with T8 on 8x8 and T32 on 32x32 blocks (every
    # plane side is a multiple of 32); the oracle on the first frame's U plane
    print(f"[planes] video block={block} qp={qp}", flush=True)
    ys = _frames(3)
    xs = [dev(p) for p in ys]
    outs, qs, sses = _run_and_compare(xs, [1088, 544, 544], qp, block=block)
    u = ys[1][:544]
    if block == 8:
        wq, want = T8.quant_reconstruct8(u, qp, lo=-255, hi=255)
    else:
        wq, _, want = T32.quant_reconstruct_32(u, qp, lo=-255, hi=255)
    nb = u.size // (block * block)
    assert np.array_equal(outs[1][:544].cpu().numpy(), want)
    assert np.array_equal(qs[1][:nb].cpu().numpy(), wq)
    assert int(sses[1][0].item()) == O.sse(want, u)


@pytest.mark.parametrize("block", [8, 32])
@pytest.mark.parametrize("kind", ["u8", "i16"])
def test_mixed_plane_sizes_other_blocks(kind, block):
    # 8 planes of block-multiple sides: ragged workgroups, one block, images
    # straddling workgroups, interleaved and plain SSE orders side by side
    b = block
    shapes = [((3 * b, 5 * b), 3 * b), ((b, b), b), ((6 * b, 10 * b), 2 * b), ((1024, 1024), 512), ((4 * b, 3 * b), b),
              ((2048, 2048), 2048), ((17 * b, 4 * b), 17 * b), ((32 * b, 9 * b), 8 * b)]
    xs = []
    for k, ((h, w), ih) in enumerate(shapes):
        if kind == "u8":
            xs.append(dev(synth.ar1_batch(h // ih, ih, w, seed_base=32_000 + 10 * k)))
        else:
            xs.append(dev(synth.laplacian_residual(32_000 + k, h, w)))
    _run_and_compare(xs, [ih for _, ih in shapes], 22, True, True, block)
    _run_and_compare(xs, [ih for _, ih in shapes], 37, False, False, block)


@pytest.mark.parametrize("store,want_sse", [(True, True), (True, False), (False, True), (False, False)])
@pytest.mark.parametrize("kind", ["u8", "i16"])
def test_mixed_plane_sizes(kind, store, want_sse):
    # 8 planes: ragged tile counts (not multiples of the 16-tile group),
    # one tile, images straddling workgroups, and planes large enough for the
    # interleaved SSE order beside small ones
    shapes = [((48, 80), 48), ((16, 16), 16), ((96, 160), 32), ((1024, 1024), 512), ((64, 48), 16),
              ((2048, 2048), 2048), ((272, 64), 272), ((512, 144), 128)]
    xs = []
    for k, ((h, w), ih) in enumerate(shapes):
        if kind == "u8":
            xs.append(dev(synth.ar1_batch(h // ih, ih, w, seed_base=31_000 + 10 * k)))
        else:
            xs.append(dev(synth.laplacian_residual(31_000 + k, h, w)))
    _run_and_compare(xs, [ih for _, ih in shapes], 27, store, want_sse)


def test_pitched_planes_and_untouched_margins():
    img = synth.ar1_image(31_500, 64, 96)
    buf = torch.zeros((64, 160), dtype=torch.uint8, device="cuda")
    buf[:, 32:128] = dev(img)
    out_buf = torch.full((64, 192), 9, dtype=torch.uint8, device="cuda")
    x2 = dev(synth.ar1_image(31_501, 32, 32))
    o2 = torch.empty_like(x2)
    sses = adct.encode_quant_planes([(buf[:, 32:128], out_buf[:, 64:160], None, 64), (x2, o2)], 32)
    _, _, want = O.quant_reconstruct(img, 32, lo=0, hi=255)
    assert np.array_equal(out_buf[:, 64:160].cpu().numpy(), want)
    assert int((out_buf[:, :64] != 9).sum().item()) == 0 and int((out_buf[:, 160:] != 9).sum().item()) == 0
    assert int(sses[0][0].item()) == O.sse(want, img)
    _, _, want2 = O.quant_reconstruct(x2.cpu().numpy(), 32, lo=0, hi=255)
    assert np.array_equal(o2.cpu().numpy(), want2)


def test_bad_job_sets():
    a = torch.zeros((32, 32), dtype=torch.uint8, device="cuda")
    b = torch.zeros((32, 32), dtype=torch.int16, device="cuda")
    q = torch.empty((4, 16, 16), dtype=torch.int16, device="cuda")
    cases = [
        ([], adct.E_ARG),                                                  # no jobs
        ([(a, torch.empty_like(a))] * 9, adct.E_ARG),                      # more than ADCT_MAX_PLANES
        ([(a, torch.empty_like(a)), (b, torch.empty_like(b))], adct.E_ARG),  # mixed dtypes
        ([(a, torch.empty_like(a), q), (a.clone(), torch.empty_like(a))], adct.E_ARG),  # q on some jobs only
        ([(a, torch.empty_like(a), None, 48, torch.empty(1, dtype=torch.int64, device="cuda"))],
         adct.E_SHAPE),                                                    # image height not dividing
        ([(a, torch.empty((32, 48), dtype=torch.uint8, device="cuda"))], adct.E_SHAPE),  # shapes differ
    ]
    for jobs, code in cases:
        with pytest.raises(adct.AdctError) as e:
            adct.encode_quant_planes(jobs, 27)
        assert e.value.code == code, jobs
    with pytest.raises(adct.AdctError) as e:
        adct.encode_quant_planes([(a, torch.empty_like(a))], 64)
    assert e.value.code == adct.E_ARG
    with pytest.raises(adct.AdctError) as e:
        adct.encode_quant_planes([(a, torch.empty_like(a))], 27, block=4)
    assert e.value.code == adct.E_ARG
    # a 32-point job whose sides are not multiples of 32, an 8-point job
    # whose image height is not a multiple of 8
    c = torch.zeros((48, 64), dtype=torch.uint8, device="cuda")
    with pytest.raises(adct.AdctError) as e:
        adct.encode_quant_planes([(c, torch.empty_like(c))], 27, block=32)
    assert e.value.code == adct.E_SHAPE
    with pytest.raises(adct.AdctError) as e:
        adct.encode_quant_planes([(c, torch.empty_like(c), None, 12, torch.empty(4, dtype=torch.int64, device="cuda"))],
                                 27, block=8)
    assert e.value.code == adct.E_SHAPE
