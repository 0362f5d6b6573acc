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
