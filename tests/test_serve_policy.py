"""The server's host policy without a GPU: pool allocator, admission order
under a fake clock, and the latency percentile, each against an
independent Python model."""
import math

import numpy as np
import pytest

from paper_1606_07414_amd import adct


class FirstFit:
    """Reference first-fit allocator over 256-byte granules."""

    def __init__(self, cap):
        self.cap = cap // 256 * 256
        self.blocks = {}  # off -> size

    def alloc(self, n):
        need = (max(n, 1) + 255) // 256 * 256
        pos = 0
        for off in sorted(self.blocks):
            if off - pos >= need:
                break
            pos = off + self.blocks[off]
        if pos + need > self.cap:
            return -1
        self.blocks[pos] = need
        return pos

    def free(self, off):
        del self.blocks[off]


def test_pool_first_fit_and_coalescing():
    rng = np.random.default_rng(1)
    ops, live, ref = [], [], FirstFit(1 << 20)
    want = []
    for i in range(2000):
        if live and rng.random() < 0.45:
            j = live.pop(int(rng.integers(0, len(live))))
            ops.append(-j)
            ref.free(want[j])
            want.append(0)
        else:
            n = int(rng.integers(1, 120000))
            ops.append(n)
            off = ref.alloc(n)
            want.append(off)
            if off >= 0:
                live.append(i)
    got, hw = adct.pool_simulate(1 << 20, ops)
    assert got.tolist() == want
    assert 0 < hw <= 1 << 20


def test_pool_exact_fill_and_reuse():
    got, hw = adct.pool_simulate(1024, [256, 256, 512, 1, -1, 256, -0, -2, 512])
    # the 256 bytes freed at 0 cannot hold 512: first fit places it at 512
    assert got.tolist() == [0, 256, 512, -1, 0, 256, 0, 0, 512]
    assert hw == 1024


def test_pool_rejects_bad_free():
    with pytest.raises(adct.AdctError):
        adct.pool_simulate(1024, [256, -5])


def admission_model(cap, max_inflight, arrival, nbytes, hold):
    """Event-driven reference: strict submission order, head of line blocks."""
    n = len(arrival)
    admit = [None] * n
    live = []  # (end, off)
    pool = FirstFit(cap)
    head, now = 0, arrival[0]
    while head < n:
        while head < n and arrival[head] <= now and len(live) < max_inflight:
            off = pool.alloc(nbytes[head])
            if off < 0:
                break
            admit[head] = now
            live.append((now + hold[head], off))
            head += 1
        if head >= n:
            break
        cands = [e for e, _ in live if e > now]
        if arrival[head] > now:
            cands.append(arrival[head])
        now = min(cands) if cands else now
        for e, off in list(live):
            if e <= now:
                pool.free(off)
                live.remove((e, off))
    return admit


@pytest.mark.parametrize("seed,max_inflight", [(1, 64), (2, 3), (3, 1)])
def test_admission_matches_model(seed, max_inflight):
    rng = np.random.default_rng(seed)
    n = 300
    arrival = np.cumsum(rng.exponential(1000.0, size=n)).astype(np.int64)
    nbytes = rng.integers(1000, 400000, size=n)
    hold = rng.integers(0, 20000, size=n)
    got = adct.admission_simulate(1 << 20, max_inflight, arrival, nbytes, hold)
    want = admission_model(1 << 20, max_inflight, arrival.tolist(), nbytes.tolist(), hold.tolist())
    assert got.tolist() == want
    assert np.all(got >= arrival)
    assert np.all(np.diff(got) >= 0)  # admission keeps submission order


def test_admission_rejects_oversize():
    with pytest.raises(adct.AdctError):
        adct.admission_simulate(4096, 4, [0], [8192], [1])


def test_percentile_nearest_rank():
    v = np.arange(1, 101, dtype=np.float64)[::-1]
    assert adct.percentile(v, 50) == 50.0
    assert adct.percentile(v, 99) == 99.0
    assert adct.percentile(v, 100) == 100.0
    assert adct.percentile(v, 0) == 1.0
    rng = np.random.default_rng(0)
    x = rng.random(777)
    for p in (1, 25, 50, 90, 99):
        k = max(1, math.ceil(p / 100 * len(x)))
        assert adct.percentile(x, p) == np.sort(x)[k - 1]
