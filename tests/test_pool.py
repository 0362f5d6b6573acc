"""CPU tests of the buddy allocator behind the serving pool (pure host code
in the library: no GPU needed)."""
import numpy as np
import pytest

from paper_1704_00605_amd import _lib
from paper_1704_00605_amd.pool import BuddyPool


def test_basic_alloc_free_merge():
    p = BuddyPool(1 << 20, 256)
    assert p.free_bytes() == 1 << 20
    a = p.try_alloc(100)      # 256
    b = p.try_alloc(300)      # 512
    c = p.try_alloc(1 << 19)  # half the pool
    assert a == 0 and b == 512 and c == 1 << 19
    assert p.free_bytes() == (1 << 20) - 256 - 512 - (1 << 19)
    assert p.try_alloc(1 << 19) is None
    p.free(c)
    p.free(a)
    p.free(b)
    assert p.free_bytes() == 1 << 20
    # everything merged back: the whole pool is one block again
    assert p.try_alloc(1 << 20) == 0


def test_blocks_are_aligned_and_disjoint():
    rng = np.random.default_rng(0)
    p = BuddyPool(64 << 20, 256)
    live = {}
    for _ in range(5000):
        if live and rng.uniform() < 0.45:
            off = list(live)[int(rng.integers(0, len(live)))]
            p.free(off)
            del live[off]
            continue
        n = int(rng.integers(1, 1 << 20))
        off = p.try_alloc(n)
        if off is None:
            continue
        size = 256
        while size < n:
            size *= 2
        assert off % size == 0
        live[off] = size
    spans = sorted(live.items())
    for (o1, s1), (o2, _) in zip(spans, spans[1:]):
        assert o1 + s1 <= o2
    assert p.free_bytes() == (64 << 20) - sum(live.values())
    for off in list(live):
        p.free(off)
    assert p.free_bytes() == 64 << 20
    assert p.try_alloc(64 << 20) == 0


def test_non_power_of_two_capacity():
    cap = (8 << 20) + (1 << 20) + 4096
    p = BuddyPool(cap, 256)
    a = p.try_alloc(8 << 20)
    b = p.try_alloc(1 << 20)
    c = p.try_alloc(4096)
    assert (a, b, c) == (0, 8 << 20, 9 << 20)
    assert p.try_alloc(1) is None
    for o in (b, a, c):
        p.free(o)
    assert p.free_bytes() == cap


def test_errors():
    p = BuddyPool(1 << 16, 256)
    with pytest.raises(_lib.B64Error):
        p.free(12345)
    assert p.try_alloc((1 << 16) + 1) is None
    with pytest.raises(_lib.B64Error):
        BuddyPool(100, 256)
    with pytest.raises(_lib.B64Error):
        BuddyPool(1 << 16, 300)


def test_eight_gib_pool_peak_tracking():
    p = BuddyPool(8 << 30, 256)
    offs = [p.try_alloc(1 << 20) for _ in range(1000)]
    assert None not in offs
    assert p.peak_bytes() == 1000 << 20
    for o in offs:
        p.free(o)
    assert p.free_bytes() == 8 << 30


class _ModelBuddy:
    """Plain buddy allocator with sorted free lists: the lowest free block of
    the smallest size that has one, split keeping the lower half, merged with
    a free buddy inside its top block on release."""

    def __init__(self, capacity, minb):
        self.minb = minb
        units = capacity // minb
        self.maxk = units.bit_length() - 1
        self.free = {k: set() for k in range(self.maxk + 1)}
        self.live = {}
        self.tops = []
        off = 0
        for k in range(self.maxk, -1, -1):
            if units & (1 << k):
                self.tops.append((off, k))
                self.free[k].add(off)
                off += minb << k

    def alloc(self, n):
        n = max(n, 1)
        k = 0
        while (self.minb << k) < n:
            k += 1
        if k > self.maxk:
            return None
        j = next((j for j in range(k, self.maxk + 1) if self.free[j]), None)
        if j is None:
            return None
        off = min(self.free[j])
        self.free[j].remove(off)
        while j > k:
            j -= 1
            self.free[j].add(off + (self.minb << j))
        self.live[off] = k
        return off

    def release(self, off):
        k = self.live.pop(off)
        topk = next(t for o, t in self.tops if o <= off < o + (self.minb << t))
        while k < topk:
            buddy = off ^ (self.minb << k)
            if buddy not in self.free[k]:
                break
            self.free[k].remove(buddy)
            off = min(off, buddy)
            k += 1
        self.free[k].add(off)


@pytest.mark.parametrize("capacity,minb", [((64 << 20) + (3 << 16) + 768, 256), (1 << 24, 4096)])
def test_same_offsets_as_a_plain_buddy_model(capacity, minb):
    """20,000 random allocations and releases (sizes log-uniform from 1 byte
    to the pool's capacity): every returned offset, every refusal and the
    free byte count equal those of a plain model of the same policy."""
    rng = np.random.default_rng(7)
    p = BuddyPool(capacity, minb)
    m = _ModelBuddy(capacity, minb)
    live = []
    for _ in range(20000):
        if live and rng.uniform() < 0.48:
            off = live.pop(int(rng.integers(0, len(live))))
            p.free(off)
            m.release(off)
        else:
            n = int(np.exp(rng.uniform(0, np.log(capacity))))
            got, want = p.try_alloc(n), m.alloc(n)
            assert got == want, n
            if got is not None:
                live.append(got)
        assert p.free_bytes() == capacity // minb * minb - sum(minb << k for k in m.live.values())
    for off in live:
        p.free(off)
    assert p.free_bytes() == capacity // minb * minb
