"""Serving: the continuous-batching server and its plain baseline.

Each request's levels, reconstruction and SSE must be bit-identical to the
same image coded alone by adct_encode_quant (and, for a sample, to the
oracle), whatever else is in flight; admission must respect the pool; stop,
cancel, the loop's idle exit and relaunch, and auto-release must behave as
documented.
"""
import time

import numpy as np
import pytest

from oracle import adct_oracle as O
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1606_07414_amd import adct  # noqa: E402

QP = 27


def _requests(n, lo=256, hi=1024, seed=21_000):
    sides = synth.request_sides(n, lo, hi, seed=seed)
    imgs = [synth.ar1_image(seed + 1 + k, int(s), int(s)) for k, s in enumerate(sides)]
    return imgs, [torch.from_numpy(i).pin_memory() for i in imgs]


def _alone(img):
    x = torch.from_numpy(img).cuda()
    out = torch.empty_like(x)
    q = torch.empty((x.numel() // 256, 16, 16), dtype=torch.int16, device="cuda")
    s = adct.encode_quant(x, QP, out, q=q)
    torch.cuda.synchronize()
    return out, q, int(s.item())


def _result_tensors(res):
    dst = adct.device_view(res.dst, (res.height, res.width), torch.uint8)
    q = adct.device_view(res.q, (res.height * res.width // 256, 16, 16), torch.int16)
    return dst, q


def _check_all(srv, tickets, imgs, oracle_every=0):
    for k, (t, img) in enumerate(zip(tickets, imgs)):
        rc, res = srv.poll(t)
        assert rc == adct.OK, (k, rc)
        dst, q = _result_tensors(res)
        out, q_alone, s_alone = _alone(img)
        assert torch.equal(dst, out), k
        assert torch.equal(q, q_alone), k
        assert res.sse == s_alone, k
        if oracle_every and k % oracle_every == 0:
            qw, _, want = O.quant_reconstruct(img, QP, lo=0, hi=255)
            assert np.array_equal(dst.cpu().numpy(), want), k
            assert res.sse == O.sse(want, img), k
        srv.release(t)


@pytest.mark.parametrize("mode", [adct.SERVE_PERSISTENT, adct.SERVE_PLAIN])
def test_burst_matches_alone(mode):
    imgs, pins = _requests(40)
    srv = adct.Server(pool_bytes=1 << 30, qp=QP, mode=mode, max_inflight=64, max_requests=64)
    tickets = [srv.submit(p) for p in pins]
    srv.wait_all(60)
    _check_all(srv, tickets, imgs, oracle_every=13)
    st = srv.stats()
    assert st["completed"] == 40 and st["cancelled"] == 0
    assert st["tiles_completed"] == sum(i.size // 256 for i in imgs)
    srv.close()


def test_poisson_mix_matches_alone():
    imgs, pins = _requests(120, seed=22_000)
    arr = synth.poisson_arrivals(2000.0, len(pins), seed=22_001)
    # results are held until released and max_inflight counts held requests
    srv = adct.Server(pool_bytes=1 << 30, qp=QP, max_inflight=256, max_requests=256)
    t0 = adct.now_ns() + 2_000_000
    tickets = [srv.submit(p, t0 + int(a * 1e9)) for p, a in zip(pins, arr)]
    srv.wait_all(60)
    st = srv.stats()
    assert st["completed"] == 120
    assert st["latency_p50_ms"] > 0 and st["latency_p99_ms"] >= st["latency_p50_ms"]
    # arrivals were honoured: nothing was admitted before it arrived
    for t in tickets:
        rc, res = srv.poll(t)
        assert res.t_admit_ns >= res.t_arrival_ns and res.t_done_ns >= res.t_admit_ns
    _check_all(srv, tickets, imgs)
    srv.close()


def test_small_pool_queues_and_respects_capacity():
    imgs, pins = _requests(24, 512, 512, seed=23_000)
    need = 4 * 512 * 512
    srv = adct.Server(pool_bytes=2 * need + 4096, qp=QP, max_inflight=64, max_requests=64)
    tickets = [srv.submit(p) for p in pins]
    # results are held until released, so at most two fit at a time
    done = []
    deadline = time.time() + 60
    while len(done) < len(tickets) and time.time() < deadline:
        for t in tickets:
            if t in done:
                continue
            rc, res = srv.poll(t)
            if rc == adct.OK:
                st = srv.stats()
                assert st["pool_high_water"] <= 2 * need + 4096
                srv.release(t)
                done.append(t)
        time.sleep(0.001)
    assert len(done) == len(tickets)
    st = srv.stats()
    assert st["completed"] == 24 and st["queue_p99_ms"] > 0
    srv.close()


def test_oversize_and_bad_requests():
    srv = adct.Server(pool_bytes=1 << 20, qp=QP, max_requests=4)
    big = torch.zeros((1024, 1024), dtype=torch.uint8).pin_memory()
    with pytest.raises(adct.AdctError) as e:
        srv.submit(big)
    assert e.value.code == adct.E_TOO_LARGE
    with pytest.raises(adct.AdctError) as e:
        srv.submit(torch.zeros((24, 16), dtype=torch.uint8))
    assert e.value.code == adct.E_SHAPE
    rc, _ = srv.poll(99)
    assert rc == adct.E_NOTFOUND
    srv.close()


def test_stop_without_drain_cancels_unadmitted():
    imgs, pins = _requests(6, 256, 256, seed=24_000)
    srv = adct.Server(pool_bytes=1 << 28, qp=QP, max_requests=16)
    first = srv.submit(pins[0])
    later = [srv.submit(p, adct.now_ns() + 10_000_000_000) for p in pins[1:]]  # 10 s ahead
    deadline = time.time() + 30
    while srv.poll(first)[0] != adct.OK and time.time() < deadline:
        time.sleep(0.001)
    srv.stop(drain=False)
    assert srv.poll(first)[0] == adct.OK
    for t in later:
        assert srv.poll(t)[0] == adct.E_STOPPED
    assert srv.stats()["cancelled"] == 5
    with pytest.raises(adct.AdctError):
        srv.submit(pins[0])
    srv.close()


def test_idle_loop_exits_and_is_relaunched():
    imgs, pins = _requests(3, 256, 512, seed=25_000)
    srv = adct.Server(pool_bytes=1 << 28, qp=QP, max_requests=8, idle_polls=200)  # ~1 ms idle
    t1 = srv.submit(pins[0])
    srv.wait_all(30)
    time.sleep(0.2)  # the loop goes idle and exits
    t2 = srv.submit(pins[1])
    t3 = srv.submit(pins[2])
    srv.wait_all(30)
    assert srv.stats()["loop_launches"] >= 2
    _check_all(srv, [t1, t2, t3], imgs)
    srv.close()


def test_auto_release_returns_memory():
    imgs, pins = _requests(10, 256, 768, seed=26_000)
    srv = adct.Server(pool_bytes=1 << 28, qp=QP, max_requests=16, auto_release=True)
    tickets = [srv.submit(p) for p in pins]
    srv.wait_all(30)
    for t, img in zip(tickets, imgs):
        rc, res = srv.poll(t)
        assert rc == adct.OK and res.dst is None
        assert res.sse == _alone(img)[2]
    st = srv.stats()
    assert st["in_flight"] == 0
    srv.close()


def test_max_inflight_counts_held_results():
    imgs, pins = _requests(6, 256, 256, seed=27_000)
    srv = adct.Server(pool_bytes=1 << 28, qp=QP, max_inflight=2, max_requests=8)
    tickets = [srv.submit(p) for p in pins]
    time.sleep(0.3)
    st = srv.stats()
    assert st["admitted"] == 2 and st["completed"] == 2  # the rest wait for releases
    for t in tickets:
        deadline = time.time() + 30
        while srv.poll(t)[0] == adct.PENDING and time.time() < deadline:
            time.sleep(0.001)
        assert srv.poll(t)[0] == adct.OK
        srv.release(t)
    assert srv.stats()["completed"] == 6
    srv.close()


def test_persistent_reads_pinned_memory_in_place_only():
    srv = adct.Server(pool_bytes=1 << 26, qp=QP, max_requests=8)
    pageable = np.zeros((64, 64), dtype=np.uint8)
    with pytest.raises(adct.AdctError) as e:
        srv.submit(pageable)
    assert e.value.code == adct.E_ARG
    pinned = torch.zeros((64, 80), dtype=torch.uint8).pin_memory()
    with pytest.raises(adct.AdctError) as e:
        srv.submit(pinned[:, 8:72])  # rows start 8 bytes into the buffer
    assert e.value.code == adct.E_ALIGN
    srv.close()


def test_pitched_pinned_request_and_plain_pageable():
    img = synth.ar1_image(28_000, 256, 320)
    wide = torch.zeros((256, 384), dtype=torch.uint8).pin_memory()
    wide[:, 16:336] = torch.from_numpy(img)
    srv = adct.Server(pool_bytes=1 << 26, qp=QP, max_requests=8)
    t = srv.submit(wide[:, 16:336])  # pitch 384 bytes, rows 16-byte aligned
    srv.wait_all(30)
    _check_all(srv, [t], [img], oracle_every=1)
    srv.close()
    plain = adct.Server(pool_bytes=1 << 26, qp=QP, mode=adct.SERVE_PLAIN, max_requests=8)
    t = plain.submit(np.ascontiguousarray(img))  # pageable host memory is copied
    plain.wait_all(30)
    _check_all(plain, [t], [img])
    plain.close()


@pytest.mark.parametrize("mode", [adct.SERVE_PERSISTENT, adct.SERVE_PLAIN])
def test_benchmark_configuration_full_size_requests(mode):
    # the serving benchmark's server and request mix: sides log-uniform in
    # [256, 4096] with the largest and smallest sides forced in, requests of
    # equal side sharing one pinned crop, Poisson arrivals at 2000 req/s, a
    # 16 GiB pool, 512 in flight, work items sized per request and two loop
    # workgroups per CU; results are held (not auto-released) to be checked
    n = 48
    sides = [int(s) for s in synth.request_sides(n - 2, seed=24_000)] + [4096, 256]
    rng = np.random.default_rng(24_001)
    pool = [synth.ar1_image(24_100 + i, 4096, 4096) for i in range(2)]
    bufs = {}
    for s in sorted(set(sides)):
        p, y, x = int(rng.integers(0, 2)), int(rng.integers(0, 4096 - s + 1)), int(rng.integers(0, 4096 - s + 1))
        bufs[s] = torch.from_numpy(np.ascontiguousarray(pool[p][y:y + s, x:x + s])).pin_memory()
    views = [bufs[s] for s in sides]
    arr = synth.poisson_arrivals(2000.0, n, seed=24_002)
    srv = adct.Server(pool_bytes=16 << 30, qp=QP, mode=mode, max_inflight=512, max_requests=n, tiles_per_item=0,
                      wgs_per_cu=2)
    t0 = adct.now_ns() + 5_000_000
    tickets = [srv.submit(v, t0 + int(a * 1e9)) for v, a in zip(views, arr)]
    srv.wait_all(120)
    st = srv.stats()
    assert st["completed"] == n and st["cancelled"] == 0
    assert st["tiles_completed"] == sum(s * s // 256 for s in sides)
    # every result against the same image coded alone; requests 0, 23 and
    # 46 (the 4096 x 4096 one) against the oracle as well
    _check_all(srv, tickets, [v.numpy() for v in views], oracle_every=23)
    srv.close()


@pytest.mark.parametrize("dma_min,policy", [(1, adct.SERVE_DMA_BY_SIZE), (512 * 512, adct.SERVE_DMA_BY_SIZE),
                                            (-1, adct.SERVE_DMA_ADAPTIVE), (512 * 512, adct.SERVE_DMA_ADAPTIVE),
                                            (1, adct.SERVE_DMA_ADAPTIVE)])
def test_dma_copied_requests_match_alone(dma_min, policy):
    # by size, dma_min_pixels = 1: every request is copied into the pool by
    # the DMA engine and published afterwards; 512 x 512: a mix of DMA-copied
    # and loop-staged requests in one stream of arrivals; -1: none is copied;
    # adaptive: the routing depends on what is in flight at each admission
    imgs, pins = _requests(60, 256, 1024, seed=29_000)
    arr = synth.poisson_arrivals(3000.0, len(pins), seed=29_001)
    srv = adct.Server(pool_bytes=1 << 30, qp=QP, max_inflight=64, max_requests=64, dma_min_pixels=dma_min,
                      dma_policy=policy)
    t0 = adct.now_ns() + 2_000_000
    tickets = [srv.submit(p, t0 + int(a * 1e9)) for p, a in zip(pins, arr)]
    srv.wait_all(60)
    st = srv.stats()
    assert st["completed"] == 60 and st["cancelled"] == 0
    if dma_min == 1 and policy == adct.SERVE_DMA_BY_SIZE:
        assert st["dma_copies"] == 60
    if dma_min == -1:
        assert st["dma_copies"] == 0
    _check_all(srv, tickets, imgs, oracle_every=29)
    srv.close()


def test_adaptive_routing():
    # dma_min_pixels = 512^2, adaptive.  A large request alone is staged by
    # the loop.  Requests arriving together are admitted in one pass: the
    # first large one finds nothing in flight (staged), the next large one
    # finds it in flight (DMA), and the small ones find a large one being
    # staged (DMA).  Then a small request alone is staged.
    big = [synth.ar1_image(29_900 + k, 768, 768) for k in range(2)]
    small = [synth.ar1_image(29_910 + k, 256, 256) for k in range(3)]
    srv = adct.Server(pool_bytes=1 << 30, qp=QP, max_inflight=64, max_requests=16, dma_min_pixels=512 * 512)
    pins = [torch.from_numpy(i).pin_memory() for i in big + small]
    t = srv.submit(pins[0])
    srv.wait_all(30)
    assert srv.stats()["dma_copies"] == 0
    t0 = adct.now_ns() + 50_000_000
    tickets = [srv.submit(p, t0) for p in (pins[0], pins[2], pins[1], pins[3], pins[4])]
    srv.wait_all(30)
    assert srv.stats()["dma_copies"] == 4
    t_last = srv.submit(pins[2])
    srv.wait_all(30)
    assert srv.stats()["dma_copies"] == 4
    imgs = [big[0], big[0], small[0], big[1], small[1], small[2], small[0]]
    _check_all(srv, [t] + tickets + [t_last], imgs, oracle_every=3)
    srv.close()


def test_dma_copied_pitched_request_and_pool_reuse():
    # a pitched pinned request through the DMA path, then requests that reuse
    # its pool block (the block's old contents must not be read back)
    img = synth.ar1_image(29_500, 256, 320)
    wide = torch.zeros((256, 384), dtype=torch.uint8).pin_memory()
    wide[:, 16:336] = torch.from_numpy(img)
    srv = adct.Server(pool_bytes=1 << 20, qp=QP, max_inflight=1, max_requests=8, dma_min_pixels=1,
                      dma_policy=adct.SERVE_DMA_BY_SIZE)
    t = srv.submit(wide[:, 16:336])
    srv.wait_all(30)
    _check_all(srv, [t], [img], oracle_every=1)
    imgs, pins = _requests(4, 256, 320, seed=29_600)
    tickets = [srv.submit(p) for p in pins]
    for k, tk in enumerate(tickets):
        while srv.poll(tk)[0] == adct.PENDING:
            time.sleep(0.001)
        _check_all(srv, [tk], [imgs[k]])
    assert srv.stats()["dma_copies"] == 5
    srv.close()


def test_server_rejects_bad_dma_threshold_and_policy():
    with pytest.raises(adct.AdctError) as e:
        adct.Server(pool_bytes=1 << 20, qp=QP, max_requests=4, dma_min_pixels=-2)
    assert e.value.code == adct.E_ARG
    with pytest.raises(adct.AdctError) as e:
        adct.Server(pool_bytes=1 << 20, qp=QP, max_requests=4, dma_policy=2)
    assert e.value.code == adct.E_ARG
