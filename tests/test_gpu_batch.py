"""Uneven batches in one persistent, graph-captured launch.

Per image the batch must be bit-identical to the single-image encoder (and
through it to the oracle), for every tuning (schedule invariance), across
graph replays with eager work in between, and at the full uneven-batch size
(4096 images with sides drawn from the multiples of 16 in [64, 2048]).
"""
import os

import numpy as np
import pytest

from oracle import adct_oracle as O
import synth
from tests import oracle_c

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1606_07414_amd import adct  # noqa: E402


def _images(n, lo, hi, seed, dtype="u8"):
    sizes = synth.uneven_sizes(n, lo, hi, seed=seed)
    if dtype == "u8":
        imgs = [synth.ar1_image(seed + 1 + k, h, w) for k, (h, w) in enumerate(sizes)]
    else:
        imgs = [synth.laplacian_residual(seed + 1 + k, h, w) for k, (h, w) in enumerate(sizes)]
    return imgs, [torch.from_numpy(i).cuda() for i in imgs]


def _outputs(xs, op):
    dsts = [torch.full_like(x, 3) for x in xs]
    cdt = torch.int32 if op == adct.OP_ZONAL else torch.int16
    coefs = [torch.zeros((x.shape[0] // 16 * (x.shape[1] // 16), 16, 16), dtype=cdt, device="cuda") for x in xs]
    sses = [torch.full((1,), -1, dtype=torch.int64, device="cuda") for _ in xs]
    return dsts, coefs, sses


def _single(x, op, param):
    out = torch.empty_like(x)
    if op == adct.OP_ZONAL:
        c = torch.empty((x.shape[0] // 16 * (x.shape[1] // 16), 16, 16), dtype=torch.int32, device="cuda")
        s = adct.encode_zonal(x, param, out, coef=c)
    else:
        c = torch.empty((x.shape[0] // 16 * (x.shape[1] // 16), 16, 16), dtype=torch.int16, device="cuda")
        s = adct.encode_quant(x, param, out, q=c)
    return out, c, s


@pytest.mark.parametrize("op,param,kind", [(adct.OP_ZONAL, 2, "u8"), (adct.OP_ZONAL, 8, "u8"),
                                           (adct.OP_ZONAL, 5, "u8"), (adct.OP_ZONAL, 16, "u8"),
                                           (adct.OP_ZONAL, 8, "i16"), (adct.OP_QUANT, 27, "u8"),
                                           (adct.OP_QUANT, 22, "i16")])
def test_batch_matches_single_image_path(op, param, kind):
    imgs, xs = _images(37, 16, 384, seed=11_000 + param, dtype=kind)
    dsts, coefs, sses = _outputs(xs, op)
    b = adct.Batch(xs, dsts, op, param, coefs=coefs, sses=sses)
    b.submit()
    torch.cuda.synchronize()
    info = b.info()
    assert info["tiles"] == sum(x.numel() // 256 for x in xs)
    for k, x in enumerate(xs):
        out, c, s = _single(x, op, param)
        torch.cuda.synchronize()
        assert torch.equal(dsts[k], out), k
        assert torch.equal(coefs[k], c), k
        assert torch.equal(sses[k], s), k
    # and the oracle on a few images
    lo, hi = (0, 255) if kind == "u8" else (-255, 255)
    for k in (0, 17, 36):
        img = imgs[k]
        if op == adct.OP_ZONAL:
            Y = O.fwd2d(img)
            want = O.from_tiles(O.round_clamp(O.reconstruct_fixed(O.zonal(Y, param)), lo, hi), *img.shape)
        else:
            Y = O.quantise(O.fwd2d(img), param)
            want = O.from_tiles(O.round_clamp(O.reconstruct_fixed(O.dequantise(Y, param)), lo, hi), *img.shape)
        assert np.array_equal(dsts[k].cpu().numpy(), want)
        assert np.array_equal(coefs[k].cpu().numpy(), Y)
        assert sses[k].item() == O.sse(want, img)
    b.close()


@pytest.mark.parametrize("tpg", [8, 16, 32])
@pytest.mark.parametrize("gpi,wpc", [(1, 1), (64, 16), (3, 5)])
def test_every_tuning_gives_the_same_bytes(tpg, gpi, wpc):
    imgs, xs = _images(23, 16, 512, seed=12_000)
    ref_d, ref_c, ref_s = _outputs(xs, adct.OP_ZONAL)
    adct.Batch(xs, ref_d, adct.OP_ZONAL, 8, coefs=ref_c, sses=ref_s, tune=adct.make_tune(16, 4, 8)).submit()
    dsts, coefs, sses = _outputs(xs, adct.OP_ZONAL)
    b = adct.Batch(xs, dsts, adct.OP_ZONAL, 8, coefs=coefs, sses=sses, tune=adct.make_tune(tpg, gpi, wpc))
    b.submit()
    torch.cuda.synchronize()
    for k in range(len(xs)):
        assert torch.equal(dsts[k], ref_d[k]) and torch.equal(coefs[k], ref_c[k]) and torch.equal(sses[k], ref_s[k])


def test_graph_replays_with_eager_work_between():
    imgs, xs = _images(19, 32, 256, seed=13_000)
    dsts, coefs, sses = _outputs(xs, adct.OP_ZONAL)
    b = adct.Batch(xs, dsts, adct.OP_ZONAL, 4, coefs=coefs, sses=sses)
    want = [_single(x, adct.OP_ZONAL, 4) for x in xs]
    for rep in range(4):
        for d, c, s in zip(dsts, coefs, sses):   # eager work between replays
            d.zero_()
            c.fill_(rep)
            s.fill_(12345)
        torch.cuda.synchronize()
        b.submit()
        torch.cuda.synchronize()
        for k in range(len(xs)):
            assert torch.equal(dsts[k], want[k][0]), (rep, k)
            assert torch.equal(coefs[k], want[k][1]), (rep, k)
            assert torch.equal(sses[k], want[k][2]), (rep, k)


def test_optional_outputs():
    imgs, xs = _images(9, 16, 128, seed=14_000)
    dsts = [torch.empty_like(x) for x in xs]
    b = adct.Batch(xs, dsts, adct.OP_ZONAL, 8)  # no coefficients, no SSE
    b.submit()
    torch.cuda.synchronize()
    for k, x in enumerate(xs):
        assert torch.equal(dsts[k], _single(x, adct.OP_ZONAL, 8)[0])


# Items of several groups with neither coefficients nor SSE requested: the
# first group of an item must not overwrite LDS that the last group of the
# previous item is still reading (no SSE flush orders them then).
@pytest.mark.parametrize("op,param", [(adct.OP_ZONAL, 8), (adct.OP_QUANT, 27)])
@pytest.mark.parametrize("tpg,gpi,wpc", [(16, 2, 2), (8, 3, 4), (32, 2, 8), (16, 64, 1), (8, 64, 16)])
def test_multi_group_items_without_optional_outputs(op, param, tpg, gpi, wpc):
    imgs, xs = _images(41, 64, 768, seed=14_500)
    dsts = [torch.full_like(x, 7) for x in xs]
    b = adct.Batch(xs, dsts, op, param, tune=adct.make_tune(tpg, gpi, wpc))
    for _ in range(2):
        b.submit()
    torch.cuda.synchronize()
    for k, x in enumerate(xs):
        assert torch.equal(dsts[k], _single(x, op, param)[0]), k
    for k in (0, 20, 40):
        img = imgs[k]
        if op == adct.OP_ZONAL:
            want = O.zonal_reconstruct(img, param)
        else:
            want = O.quant_reconstruct(img, param, 0, 255)[2]
        assert np.array_equal(dsts[k].cpu().numpy(), want), k
    b.close()


def test_autotune_and_cache(tmp_path):
    imgs, xs = _images(64, 64, 512, seed=15_000)
    dsts, coefs, sses = _outputs(xs, adct.OP_ZONAL)
    cache = str(tmp_path / "tune.jsonl")
    t, ms = adct.autotune(xs, dsts, adct.OP_ZONAL, 8, coefs=coefs, sses=sses, cache_path=cache, reps=2)
    assert t.tiles_per_group in (8, 16, 32) and ms > 0
    t2, ms2 = adct.autotune(xs, dsts, adct.OP_ZONAL, 8, coefs=coefs, sses=sses, cache_path=cache, reps=2)
    assert ms2 == -1.0 and t2.as_dict() == t.as_dict()
    assert len(open(cache).read().strip().splitlines()) == 1
    # the tuned batch is still exact
    b = adct.Batch(xs, dsts, adct.OP_ZONAL, 8, coefs=coefs, sses=sses, tune=t)
    b.submit()
    torch.cuda.synchronize()
    for k in (0, 63):
        out, c, s = _single(xs[k], adct.OP_ZONAL, 8)
        assert torch.equal(dsts[k], out) and torch.equal(coefs[k], c) and torch.equal(sses[k], s)


@pytest.fixture(scope="module")
def uneven_full():
    # 4096 images, sides uniform over the multiples of 16 in [64, 2048]
    sizes = synth.uneven_sizes(4096)
    pool = synth.crop_pool()
    imgs = [np.ascontiguousarray(synth.crop_from_pool(pool, k, h, w)) for k, (h, w) in enumerate(sizes)]
    return sizes, imgs, [torch.from_numpy(i).cuda() for i in imgs]


# the default tuning, and the tunings the autotuner picks on MI355X for the
# two benchmark legs (zonal r = 8; quantised at QP 27)
@pytest.mark.parametrize("op,param,tune", [(adct.OP_ZONAL, 8, None), (adct.OP_ZONAL, 8, (32, 1, 4)),
                                           (adct.OP_QUANT, 27, (32, 2, 8))])
def test_full_size_uneven_batch(uneven_full, op, param, tune):
    sizes, imgs, xs = uneven_full
    zonal = op == adct.OP_ZONAL
    dsts = [torch.empty_like(x) for x in xs]
    cdt = torch.int32 if zonal else torch.int16
    coefs = [torch.empty((x.numel() // 256, 16, 16), dtype=cdt, device="cuda") for x in xs]
    sse = torch.empty(4096, dtype=torch.int64, device="cuda")
    sses = [sse[k:k + 1] for k in range(4096)]
    b = adct.Batch(xs, dsts, op, param, coefs=coefs, sses=sses, tune=adct.make_tune(*tune) if tune else None)
    b.submit()
    b.submit()
    torch.cuda.synchronize()
    assert b.info()["tiles"] == sum(h * w // 256 for h, w in sizes)
    got = sse.cpu().numpy()
    rng = np.random.default_rng(0)
    for k in sorted(set(rng.integers(0, 4096, size=48).tolist()) | {0, 4095}):
        img = imgs[k]
        if zonal:
            c_coef = oracle_c.fwd2d_u8(img)
            want_out, c_sse = oracle_c.zonal_recon_u8(c_coef, img.shape[0], img.shape[1], 8, img, img.shape[0])
            want_sse, want_c = c_sse[0], c_coef.astype(np.int32)
        else:
            want_c, _, want_out = O.quant_reconstruct(img, param, 0, 255)
            want_sse = O.sse(want_out, img)
        assert got[k] == want_sse, k
        assert np.array_equal(dsts[k].cpu().numpy(), want_out), k
        assert np.array_equal(coefs[k].cpu().numpy(), want_c), k
    # every image's SSE equals the single-image encoder's
    for k in range(0, 4096, 7):
        assert int(got[k]) == int(_single(xs[k], op, param)[2].item()), k
    b.close()
