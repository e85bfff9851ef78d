"""Host logic of the serving loop: the arena allocator and job footprints
(no GPU needed)."""
import numpy as np
import pytest

from paper_1509_08267_amd.serve import ArenaAllocator, job_words


def test_first_fit_and_coalescing():
    a = ArenaAllocator(100)
    x = a.alloc(30)
    y = a.alloc(30)
    z = a.alloc(30)
    assert (x, y, z) == (0, 30, 60)
    assert a.alloc(20) is None and a.alloc(10) == 90
    a.release(y, 30)
    assert a.free_blocks() == [(30, 30)]
    assert a.alloc(40) is None            # fragmented: 30 free in one block
    a.release(x, 30)
    assert a.free_blocks() == [(0, 60)]   # merged with the following block
    a.release(z, 30)
    assert a.free_blocks() == [(0, 90)]
    assert a.used == 10
    a.release(90, 10)
    assert a.free_blocks() == [(0, 100)] and a.used == 0


def test_double_free_is_rejected():
    a = ArenaAllocator(64)
    x = a.alloc(16)
    a.release(x, 16)
    with pytest.raises(ValueError):
        a.release(x, 16)
    with pytest.raises(ValueError):
        a.alloc(0)


def test_random_alloc_release_keeps_invariants():
    rng = np.random.default_rng(0)
    a = ArenaAllocator(10_000)
    live = {}
    for _ in range(3000):
        if live and rng.random() < 0.45:
            k = list(live)[int(rng.integers(len(live)))]
            a.release(k, live.pop(k))
        else:
            s = int(rng.integers(1, 400))
            off = a.alloc(s)
            if off is not None:
                for o, w in live.items():
                    assert off + s <= o or o + w <= off   # no overlap
                live[off] = s
        assert a.used == sum(live.values())
        blocks = a.free_blocks()
        assert sum(w for _, w in blocks) + a.used == a.capacity
        for (s1, w1), (s2, _) in zip(blocks, blocks[1:]):
            assert s1 + w1 < s2                           # coalesced, sorted


def test_job_words():
    assert job_words(0, 0) == 64 + 64 + 64
    assert job_words(100, 1000) == 128 + 1024 + 128
