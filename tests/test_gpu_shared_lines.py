"""uint8 outputs whose rows share 128-byte lines between neighbouring tile
groups (a row length, pitch or base address that is not a multiple of 128
bytes): plain launches then hand each XCD one contiguous region of the plane
instead of dealing the tile groups round-robin.  Every tile group must still
be coded exactly once, so the outputs equal the oracle's on planes of many
chunks, with a last region only partly filled, and the margins of a pitched
destination stay untouched."""
import numpy as np
import pytest

from oracle import adct_oracle as O
from oracle import image_experiment as E
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1606_07414_amd import adct  # noqa: E402

SENTINEL = 77


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def dst_view(h, w, lead, trail):
    """A uint8 destination of h x w inside rows of lead + w + trail bytes
    filled with a sentinel; the view starts `lead` bytes into each row."""
    buf = torch.full((h, lead + w + trail), SENTINEL, dtype=torch.uint8, device="cuda")
    return buf, buf[:, lead:lead + w]


def margins_untouched(buf, lead, w):
    b = host(buf)
    return np.all(b[:, :lead] == SENTINEL) and np.all(b[:, lead + w:] == SENTINEL)


# (images, side, lead, trail): 1008-byte rows (63 tiles: every group of 16
# tiles but the first of a row starts inside a line); a 16-byte base offset
# on 1024-byte rows; a 64-byte tail making the pitch 1072
GEOMS = [(8, 1008, 0, 0), (6, 1024, 16, 0), (5, 1008, 0, 64)]


@pytest.mark.parametrize("geom", GEOMS, ids=["rows1008", "base+16", "pitch1072"])
@pytest.mark.parametrize("r", [2, 8, 16])
def test_encode_zonal_shared_lines(geom, r):
    n, side, lead, trail = geom
    img = synth.ar1_batch(n, side, side, seed_base=5100 + side + lead)
    x = dev(img)
    buf, out = dst_view(n * side, side, lead, trail)
    ntile = n * (side // 16) ** 2
    coef = torch.empty((ntile, 16, 16), dtype=torch.int32, device="cuda")
    s = host(adct.encode_zonal(x, r, out, coef=coef, image_height=side))
    want = O.zonal_reconstruct(img, r)
    assert np.array_equal(host(out), want)
    assert np.array_equal(host(coef), O.fwd2d(img))
    for i in range(n):
        assert s[i] == O.sse(want[i * side:(i + 1) * side], img[i * side:(i + 1) * side]), i
    assert margins_untouched(buf, lead, side)


@pytest.mark.parametrize("geom", GEOMS[:2], ids=["rows1008", "base+16"])
def test_encode_quant_shared_lines(geom):
    n, side, lead, trail = geom
    img = synth.ar1_batch(n, side, side, seed_base=5200 + side)
    x = dev(img)
    buf, out = dst_view(n * side, side, lead, trail)
    ntile = n * (side // 16) ** 2
    q = torch.empty((ntile, 16, 16), dtype=torch.int16, device="cuda")
    s = host(adct.encode_quant(x, 27, out, q=q, image_height=side))
    qw = O.quantise(O.fwd2d(img), 27)
    want = O.from_tiles(O.round_clamp(O.reconstruct_fixed(O.dequantise(qw, 27)), 0, 255), *img.shape)
    assert np.array_equal(host(q), qw)
    assert np.array_equal(host(out), want)
    for i in range(n):
        assert s[i] == O.sse(want[i * side:(i + 1) * side], img[i * side:(i + 1) * side]), i
    assert margins_untouched(buf, lead, side)


def test_recon_kernels_shared_lines():
    # the second kernel of the codec form and the zig-zag encoder write the
    # same kind of rows
    n, side = 6, 1008
    img = synth.ar1_batch(n, side, side, seed_base=5300)
    x = dev(img)
    coef = adct.fwd2d(x)
    buf, out = dst_view(n * side, side, 0, 32)
    s = host(adct.zonal_recon(coef, 4, out, ref=x, image_height=side))
    want = O.zonal_reconstruct(img, 4)
    assert np.array_equal(host(out), want)
    for i in range(n):
        assert s[i] == O.sse(want[i * side:(i + 1) * side], img[i * side:(i + 1) * side]), i
    assert margins_untouched(buf, 0, side)
    buf, out = dst_view(n * side, side, 0, 32)
    s = host(adct.encode_zigzag(x, 45, out, image_height=side))
    want = E.zigzag_reconstruct(img, 45)
    assert np.array_equal(host(out), want)
    for i in range(n):
        assert s[i] == O.sse(want[i * side:(i + 1) * side], img[i * side:(i + 1) * side]), i
    assert margins_untouched(buf, 0, side)
