"""GPU: Algorithm 1 with p blocks (GC_ALGO_BLOCKS) against the oracle's
literal reading, bit for bit: colours, round count and per-round sizes, for
several p on the named graphs, random graphs, unsorted rows, int64 row
pointers, a power-law graph and the 1M-vertex ER workload; the round cap;
switching algorithms on one handle.  Integer work: exact equality."""
import json
import os

import numpy as np
import pytest

import graphgen
import oracle
from conftest import ROOT

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
GOLDEN = json.load(open(os.path.join(ROOT, "tests", "golden", "workloads.json")))


@pytest.fixture(scope="module")
def gc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1509_08267_amd import gc as gcmod
    gcmod.load()
    return gcmod


def _dev(g, rp64=False):
    rp = torch.from_numpy(g.rowptr.astype(np.int64 if rp64 else np.int32)).cuda()
    ci = torch.from_numpy(g.colidx if g.nnz else np.zeros(0, np.int32)).cuda()
    return rp, ci


def assert_blocks(gc, g, p, *, rp64=False, rows_sorted=True, calls=2):
    want, R, rec = oracle.blocks(g.rowptr, g.colidx, p)
    sizes = [int((rec >= r - 1).sum()) for r in range(1, R + 1)]
    rp, ci = _dev(g, rp64)
    with gc.Graph(rp, ci, validate=True, rows_sorted=rows_sorted, algorithm="blocks",
                  partitions=p) as G:
        assert G.get(gc.GC_OPT_ALGORITHM) == gc.GC_ALGO_BLOCKS
        assert G.get(gc.GC_OPT_PARTITIONS) == p
        for _ in range(calls):
            out = G.color()
            rounds, ncol = G.stats()
            assert rounds == R, (rounds, R, p)
            assert np.array_equal(out.cpu().numpy(), want), p
            assert ncol == (int(want.max()) + 1 if g.n else 0)
        assert list(G.round_sizes()[:R]) == sizes


def _named():
    return [
        ("K1", graphgen.complete(1)), ("K2", graphgen.complete(2)), ("K40", graphgen.complete(40)),
        ("path3", graphgen.path(3)), ("path257", graphgen.path(257)), ("C9", graphgen.cycle(9)),
        ("star_lo", graphgen.star(300, 0)), ("star_hi", graphgen.star(300, 300)),
        ("crown8", graphgen.crown(8)), ("empty7", graphgen.empty(7)),
        ("er_small", graphgen.er(3000, 24000, 11)),
    ]


@pytest.mark.parametrize("p", [1, 2, 7, 64, 100000])
def test_blocks_named_graphs(gc, p):
    for name, g in _named():
        print(f"[case] blocks {name} p={p}", flush=True)
        assert_blocks(gc, g, p)


def test_blocks_every_vertex_its_own_block(gc):
    for name, g in _named():
        if g.n:
            print(f"[case] blocks {name} p=n", flush=True)
            assert_blocks(gc, g, g.n)


def test_blocks_random_graphs(gc):
    rng = np.random.default_rng(8)
    for i in range(40):
        n = int(rng.integers(1, 400))
        m = int(rng.integers(0, min(n * (n - 1) // 2, 4000) + 1))
        g = graphgen.er(n, m, 500 + i)
        for p in (1, 3, int(rng.integers(1, n + 2))):
            assert_blocks(gc, g, p, calls=1)


def test_blocks_unsorted_rows_int64_and_power_law(gc):
    g = graphgen.er(6000, 70000, 41)
    u = graphgen.shuffle_rows(g, np.random.default_rng(5))
    for p in (16, 1024):
        print(f"[case] blocks unsorted/int64 p={p}", flush=True)
        assert_blocks(gc, u, p, rows_sorted=False)
        assert_blocks(gc, g, p, rp64=True)
    r = graphgen.rmat(13, 16, seed=2)
    for p in (4, 256):
        print(f"[case] blocks rmat13 p={p}", flush=True)
        assert_blocks(gc, r, p, rp64=True)


def test_blocks_default_partitions_and_round_cap(gc):
    g = graphgen.er(20000, 200000, 9)
    rp, ci = _dev(g)
    with gc.Graph(rp, ci, algorithm="blocks") as G:
        p = G.get(gc.GC_OPT_PARTITIONS)
        assert p == 64 * torch.cuda.get_device_properties(0).multi_processor_count
        want, R, _ = oracle.blocks(g.rowptr, g.colidx, p)
        out = G.color()
        assert G.stats()[0] == R and np.array_equal(out.cpu().numpy(), want)
        if R > 1:
            G.set("max_rounds", 1)
            G.color()
            with pytest.raises(gc.GCError) as e:
                G.stats()
            assert e.value.code == gc.GC_EROUNDS
            G.set("max_rounds", 0)
            out = G.color()
            assert G.stats()[0] == R and np.array_equal(out.cpu().numpy(), want)


def test_switching_between_blocks_and_speculation(gc):
    g = graphgen.er(20000, 200000, 5)
    rsc = oracle.rsc(g.rowptr, g.colidx)
    blk, R, _ = oracle.blocks(g.rowptr, g.colidx, 512)
    rp, ci = _dev(g)
    with gc.Graph(rp, ci) as G:
        for algo, want, rounds in [("push", rsc.colors, rsc.rounds), ("blocks", blk, R),
                                   ("push", rsc.colors, rsc.rounds), ("blocks", blk, R)]:
            G.set("algorithm", algo)
            G.set("partitions", 512)
            for _ in range(2):
                out = G.color()
                r, _ = G.stats()
                assert r == rounds and np.array_equal(out.cpu().numpy(), want), algo


def test_blocks_workload_er_1m(gc):
    g = graphgen.workload("er_1m_16m")
    assert g.sha256() == GOLDEN["er_1m_16m"]["input_sha256"]
    assert_blocks(gc, g, 16384, calls=1)
