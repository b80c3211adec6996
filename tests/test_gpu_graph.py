"""Plain calls captured in a graph: the SSE accumulators are cleared by a
fill kernel (no memset node), so every replay must reproduce the eager
result, with eager work on the same buffers between replays."""
import numpy as np
import pytest

from oracle import adct_oracle as O
from oracle import image_experiment as E
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1606_07414_amd import adct  # noqa: E402


def test_captured_encoders_replay_like_eager():
    img = synth.ar1_batch(4, 128, 160, seed_base=4000)
    x = torch.from_numpy(img).cuda()
    out_z, out_q, out_g = (torch.empty_like(x) for _ in range(3))
    coef = torch.empty((x.numel() // 256, 16, 16), dtype=torch.int32, device="cuda")
    q = torch.empty((x.numel() // 256, 16, 16), dtype=torch.int16, device="cuda")
    s_z, s_q, s_g = (torch.empty(4, dtype=torch.int64, device="cuda") for _ in range(3))
    ss = torch.empty(4, dtype=torch.float64, device="cuda")
    # several planes in one launch (one clear of both SSE arrays), and the
    # 32x32 and 64x64 codecs, on planes whose sides are multiples of 64
    y = torch.from_numpy(synth.ar1_batch(2, 128, 192, seed_base=4010)).cuda()
    u = torch.from_numpy(synth.ar1_batch(2, 64, 128, seed_base=4020)).cuda()
    out_y, out_u, out_32, out_64 = (torch.empty_like(t) for t in (y, u, y, y))
    q_y = torch.empty((y.numel() // 256, 16, 16), dtype=torch.int16, device="cuda")
    q_u = torch.empty((u.numel() // 256, 16, 16), dtype=torch.int16, device="cuda")
    s_y, s_u, s_32, s_64 = (torch.empty(2, dtype=torch.int64, device="cuda") for _ in range(4))
    side = torch.cuda.Stream()

    def work(stream):
        adct.encode_zonal(x, 8, out_z, coef=coef, image_height=128, sse=s_z, stream=stream)
        adct.encode_quant(x, 27, out_q, q=q, image_height=128, sse=s_q, stream=stream)
        adct.encode_zigzag(x, 45, out_g, image_height=128, sse=s_g, stream=stream)
        adct.ssim(x, out_g, image_height=128, out=ss, stream=stream)
        adct.encode_quant_planes([(y, out_y, q_y, 128, s_y), (u, out_u, q_u, 64, s_u)], 32, stream=stream)
        adct.t32_encode_quant(y, 22, out_32, image_height=128, sse=s_32, stream=stream)
        adct.t64_encode_zonal(y, 12, out_64, image_height=128, sse=s_64, stream=stream)

    # eager reference
    work(torch.cuda.current_stream())
    torch.cuda.synchronize()
    extra = (out_y, out_u, q_y, q_u, s_y, s_u, out_32, s_32, out_64, s_64)
    want = [t.clone() for t in (out_z, out_q, out_g, coef, q, s_z, s_q, s_g) + extra + (ss,)]
    assert np.array_equal(want[0].cpu().numpy(), O.zonal_reconstruct(img, 8))
    assert np.array_equal(want[2].cpu().numpy(), E.zigzag_reconstruct(img, 45))

    g = torch.cuda.CUDAGraph()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        with torch.cuda.graph(g, stream=side):
            work(side)
    torch.cuda.synchronize()
    for rep in range(4):
        for t in (out_z, out_q, out_g, coef, q, s_z, s_q, s_g, ss) + extra:  # eager work between replays
            t.fill_(rep + 1)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got = (out_z, out_q, out_g, coef, q, s_z, s_q, s_g) + extra
        for k, (a, b) in enumerate(zip(got, want)):
            assert torch.equal(a, b), (rep, k)
        # SSIM sums in an order that is not fixed: equal to rounding
        assert torch.allclose(ss, want[-1], rtol=1e-13, atol=0), rep
