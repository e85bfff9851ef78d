"""Host logic of the serving loop: the arena allocator and job footprints
(no GPU needed)."""
import numpy as np
import pytest

from paper_1509_08267_amd.serve import ArenaAllocator, job_words


def test_fit_and_coalescing():
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
        assert a.largest_free() == max((w for _, w in blocks), default=0)


def test_best_fit_takes_the_smallest_block_that_holds_the_request():
    a = ArenaAllocator(1000)
    offs = [a.alloc(100) for _ in range(10)]             # 0, 100, ..., 900
    a.release(offs[1], 100)                               # hole of 100 at 100
    a.release(offs[4], 100)
    a.release(offs[5], 100)                               # hole of 200 at 400
    a.release(offs[8], 100)                               # hole of 100 at 800
    assert a.alloc(150) == 400                            # only the 200 hole holds it
    assert a.alloc(50) == 550                             # its 50 left over beats the 100s
    assert a.alloc(100) == 100                            # equal sizes: the lowest start
    assert a.alloc(100) == 800 and a.alloc(1) is None


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_release_many_equals_one_at_a_time(seed):
    rng = np.random.default_rng(seed)
    a, b = ArenaAllocator(200_000), ArenaAllocator(200_000)
    live = []
    for step in range(40):
        for _ in range(int(rng.integers(20, 200))):
            s = int(rng.integers(1, 900))
            x, y = a.alloc(s), b.alloc(s)
            assert x == y
            if x is not None:
                live.append((x, s))
        rng.shuffle(live)
        k = int(rng.integers(0, len(live) + 1))
        gone, live = live[:k], live[k:]
        for x, s in gone:
            a.release(x, s)
        b.release_many([x for x, _ in gone], [s for _, s in gone])
        assert a.free_blocks() == b.free_blocks() and a.used == b.used
        assert b._by_size == sorted((w, x) for x, w in b.free_blocks())
    with pytest.raises(ValueError):   # a block released twice in one call
        b.release_many([live[0][0]] * 40, [live[0][1]] * 40)


def test_many_fragments_stay_fast():
    # thousands of free fragments below one large free tail: each request
    # still costs a search, not a walk over the fragments
    import time
    a = ArenaAllocator(10_000_000)
    offs = [a.alloc(64) for _ in range(20_000)]
    for o in offs[::2]:
        a.release(o, 64)
    t0 = time.perf_counter()
    for _ in range(5_000):
        assert a.alloc(1_000) is not None
    assert time.perf_counter() - t0 < 1.0


def test_job_words():
    assert job_words(0, 0) == 64 + 64 + 64
    assert job_words(100, 1000) == 128 + 1024 + 128
