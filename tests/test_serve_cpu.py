"""Host logic of the server that needs no GPU: the ring arena."""
import numpy as np
import pytest

from paper_1401_5245_amd.serve import RingArena, _runs


def test_ring_fifo_never_overlaps():
    rng = np.random.default_rng(0)
    ring = RingArena(1000, align=2)
    live = []
    for step in range(5000):
        if live and (rng.random() < 0.45 or ring.used > 900):
            off, n = ring.free_oldest()
            assert (off, n) == live.pop(0)
        else:
            n = int(rng.integers(1, 300))
            off = ring.alloc(n)
            if off is None:
                assert live, "an empty ring must accept any block that fits"
                continue
            n = -(-n // 2) * 2
            assert off % 2 == 0 and 0 <= off and off + n <= 1000
            for o, m in live:
                assert off + n <= o or o + m <= off, "blocks overlap"
            live.append((off, n))
        assert ring.used == sum(m for _, m in live)


def test_ring_rejects_oversize_and_waits_when_full():
    ring = RingArena(100, align=1)
    with pytest.raises(ValueError):
        ring.alloc(101)
    with pytest.raises(ValueError):
        ring.alloc(0)
    assert ring.alloc(60) == 0
    assert ring.alloc(50) is None           # must wait for space
    assert ring.alloc(40) == 60
    ring.free_oldest()
    assert ring.alloc(50) == 0              # wraps to the freed front
    assert ring.alloc(11) is None
    assert ring.alloc(10) == 50


def test_runs_merge_contiguous_copies():
    assert _runs([0, 10, 30], [100, 110, 200], [10, 20, 5]) == [[0, 100, 30], [30, 200, 5]]
    assert _runs([], [], []) == []
