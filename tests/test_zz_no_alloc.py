"""The batch entry point that allocates nothing (adct_batch_run_noalloc):
its job table and work queue live in the library's fixed device array.

Checked against the allocating entry point (adct_batch_create + submit) bit
for bit, and through it against the oracle, on two calls in a row whose
second is smaller (the array keeps the first call's contents), and its
rejection of batches whose table and queue exceed the array.
"""
import numpy as np
import pytest

from oracle import adct_oracle as O
from oracle import image_experiment as IE
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1606_07414_amd import adct  # noqa: E402


def _images(n, lo, hi, seed, kind):
    sizes = synth.uneven_sizes(n, lo, hi, seed=seed)
    gen = synth.ar1_image if kind == "u8" else synth.laplacian_residual
    imgs = [gen(seed + 1 + k, h, w) for k, (h, w) in enumerate(sizes)]
    return imgs, [torch.from_numpy(i).cuda() for i in imgs]


def _outputs(xs, op, fill):
    dsts = [torch.full_like(x, fill) for x in xs]
    cdt = torch.int32 if op != adct.OP_QUANT else torch.int16
    coefs = [torch.full((x.numel() // 256, 16, 16), fill, dtype=cdt, device="cuda") for x in xs]
    sses = [torch.full((1,), -fill, dtype=torch.int64, device="cuda") for _ in xs]
    return dsts, coefs, sses


def _oracle(img, op, param, kind):
    lo, hi = (0, 255) if kind == "u8" else (-255, 255)
    if op == adct.OP_ZONAL:
        Y = O.fwd2d(img)
        Z = O.zonal(Y, param)
    elif op == adct.OP_ZIGZAG:
        Y = O.fwd2d(img)
        Z = IE.zigzag(Y, param)
    else:
        Y = O.quantise(O.fwd2d(img), param)
        Z = O.dequantise(Y, param)
    rec = O.from_tiles(O.round_clamp(O.reconstruct_fixed(Z), lo, hi), *img.shape)
    return Y, rec, O.sse(rec, img)


@pytest.mark.parametrize("op,param,kind,tune", [
    (adct.OP_ZONAL, 8, "u8", None),
    (adct.OP_ZONAL, 8, "u8", (16, 3, 2)),
    (adct.OP_QUANT, 27, "u8", (32, 2, 4)),
    (adct.OP_QUANT, 22, "i16", (8, 64, 1)),
    (adct.OP_ZIGZAG, 45, "u8", (16, 1, 8)),
])
def test_noalloc_matches_batch_on_two_calls(op, param, kind, tune):
    t = adct.Tune(*tune, 0) if tune else None
    first = _images(41, 16, 512, seed=71_000 + param, kind=kind)
    second = _images(9, 16, 160, seed=72_000 + param, kind=kind)
    assert sum(x.numel() for x in second[1]) < sum(x.numel() for x in first[1])
    for call, (imgs, xs) in enumerate((first, second)):
        print(f"[noalloc] op={op} param={param} kind={kind} tune={tune} call={call} images={len(xs)}", flush=True)
        dsts, coefs, sses = _outputs(xs, op, 5)
        adct.batch_run_noalloc(xs, dsts, op, param, coefs=coefs, sses=sses, tune=t)
        rd, rc, rs = _outputs(xs, op, 7)
        b = adct.Batch(xs, rd, op, param, coefs=rc, sses=rs, tune=t)
        b.submit()
        torch.cuda.synchronize()
        b.close()
        for k in range(len(xs)):
            assert torch.equal(dsts[k], rd[k]), (call, k)
            assert torch.equal(coefs[k], rc[k]), (call, k)
            assert torch.equal(sses[k], rs[k]), (call, k)
        for k in (0, len(xs) - 1):
            Y, rec, e = _oracle(imgs[k], op, param, kind)
            assert np.array_equal(coefs[k].cpu().numpy(), Y), (call, k)
            assert np.array_equal(dsts[k].cpu().numpy(), rec), (call, k)
            assert int(sses[k].item()) == e, (call, k)


def test_noalloc_without_optional_outputs_then_with():
    imgs, xs = _images(23, 16, 384, seed=73_000, kind="u8")
    dsts = [torch.full_like(x, 9) for x in xs]
    adct.batch_run_noalloc(xs, dsts, adct.OP_QUANT, 32, tune=adct.Tune(16, 2, 2, 0))
    torch.cuda.synchronize()
    for k in (0, 11, 22):
        _, rec, _ = _oracle(imgs[k], adct.OP_QUANT, 32, "u8")
        assert np.array_equal(dsts[k].cpu().numpy(), rec), k
    # the next call on a smaller batch, with SSE slots, finds them cleared
    sub = xs[:5]
    sd = [torch.empty_like(x) for x in sub]
    ss = [torch.full((1,), 123456789, dtype=torch.int64, device="cuda") for _ in sub]
    adct.batch_run_noalloc(sub, sd, adct.OP_QUANT, 32, sses=ss, tune=adct.Tune(16, 2, 2, 0))
    torch.cuda.synchronize()
    for k in range(5):
        _, rec, e = _oracle(imgs[k], adct.OP_QUANT, 32, "u8")
        assert np.array_equal(sd[k].cpu().numpy(), rec), k
        assert int(ss[k].item()) == e, k


def test_noalloc_rejects_queue_beyond_the_array():
    # 8-tile items of one 4096x4096 image would need 16384 items x 12 bytes
    # (fits); 200 such images need 3.3 M items (39 MB): rejected before any
    # launch.  All jobs share one source and one destination (never launched).
    x = torch.zeros((4096, 4096), dtype=torch.uint8, device="cuda")
    d = torch.full_like(x, 77)
    with pytest.raises(adct.AdctError) as e:
        adct.batch_run_noalloc([x] * 200, [d] * 200, adct.OP_ZONAL, 8, tune=adct.Tune(8, 1, 2, 0))
    assert e.value.code == adct.E_TOO_LARGE
    torch.cuda.synchronize()
    assert int((d != 77).sum().item()) == 0
    # the same jobs in larger items fit: 200 x 4096 items of 512 tiles
    adct.batch_run_noalloc([x] * 1, [d] * 1, adct.OP_ZONAL, 8, tune=adct.Tune(32, 16, 2, 0))
    torch.cuda.synchronize()
    assert int((d != 0).sum().item()) == 0
