"""GPU: the id-priority schedule (GC_ALGO_SEQ) reproduces the sequential
First-Fit colouring of the oracle bit for bit, in exactly the oracle's
number of rounds (the longest id-increasing path), on every round driver,
lane width, degree-class path, row layout and state width, and on the
full-size workloads.  Integer work: exact equality."""
import json
import os

import numpy as np
import pytest

import graphgen
import oracle
from conftest import ROOT

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

MODES = ["host", "chunked", "graph", "persistent"]
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


def assert_seq(gc, g, *, rp64=False, rows_sorted=True, calls=2, **opts):
    want = oracle.seq(g.rowptr, g.colidx)
    R, ro = oracle.seq_rounds(g.rowptr, g.colidx)
    sizes = [int((ro >= r).sum()) for r in range(1, R + 1)]
    rp, ci = _dev(g, rp64)
    with gc.Graph(rp, ci, validate=True, rows_sorted=rows_sorted, algorithm="seq", **opts) as G:
        assert G.get(gc.GC_OPT_ALGORITHM) == gc.GC_ALGO_SEQ
        for _ in range(calls):  # the second call runs with R known
            out = G.color()
            rounds, ncol = G.stats()
            assert rounds == R, (rounds, R, opts)
            assert np.array_equal(out.cpu().numpy(), want), opts
            assert ncol == (int(want.max()) + 1 if g.n else 0)
        assert list(G.round_sizes()[:R]) == sizes


def _named():
    return [
        ("K1", graphgen.complete(1)), ("K2", graphgen.complete(2)), ("K65", graphgen.complete(65)),
        ("path1001", graphgen.path(1001)), ("C5", graphgen.cycle(5)), ("C10", graphgen.cycle(10)),
        ("star_lo", graphgen.star(300, 0)), ("star_hi", graphgen.star(300, 300)),
        ("crown8", graphgen.crown(8)), ("empty7", graphgen.empty(7)),
        ("er_small", graphgen.er(3000, 24000, 11)),
    ]


@pytest.mark.parametrize("mode", MODES)
def test_seq_named_graphs_every_mode(gc, mode):
    for name, g in _named():
        print(f"[case] seq {name} mode={mode}", flush=True)
        assert_seq(gc, g, mode=mode)


@pytest.mark.parametrize("lanes", [2, 8, 64])
def test_seq_lane_widths(gc, lanes):
    g = graphgen.er(5000, 60000, 31)
    for mode in ("graph", "persistent"):
        print(f"[case] seq er lanes={lanes} mode={mode}", flush=True)
        assert_seq(gc, g, lanes=lanes, mode=mode)


def test_seq_medium_and_heavy_paths(gc):
    g = graphgen.er(4000, 80000, 21)
    for medium, heavy in [(4, 30), (1, 2), (64, 100000)]:
        print(f"[case] seq classes medium={medium} heavy={heavy}", flush=True)
        assert_seq(gc, g, mode="host", medium_degree=medium, heavy_degree=heavy)
    # a genuine hub, on the workgroup path by default
    assert_seq(gc, graphgen.star(40000, 7), mode="graph")


def test_seq_unsorted_rows_and_int64_rowptr(gc):
    g = graphgen.er(6000, 70000, 41)
    u = graphgen.shuffle_rows(g, np.random.default_rng(3))
    for rp64 in (False, True):
        print(f"[case] seq sorted rp64={rp64}", flush=True)
        assert_seq(gc, g, rp64=rp64, mode="graph")
        print(f"[case] seq unsorted rp64={rp64}", flush=True)
        assert_seq(gc, u, rp64=rp64, rows_sorted=False, mode="graph")


def test_seq_state_width_boundaries(gc):
    # the smallest state value marks "waiting": K_127 (max degree 126) still
    # fits one byte with colour 126 in use, K_128 takes two
    for g, width in [(graphgen.complete(127), 1), (graphgen.complete(128), 2),
                     (graphgen.star(40000, 0), 4)]:
        rp, ci = _dev(g)
        with gc.Graph(rp, ci) as G:
            assert G.get(gc.GC_OPT_STATE_BYTES) == width
        assert_seq(gc, g, mode="graph")


def test_switching_algorithms_on_one_handle(gc):
    g = graphgen.er(20000, 200000, 5)
    rsc = oracle.rsc(g.rowptr, g.colidx)
    seq = oracle.seq(g.rowptr, g.colidx)
    R, _ = oracle.seq_rounds(g.rowptr, g.colidx)
    rp, ci = _dev(g)
    with gc.Graph(rp, ci) as G:
        for algo, want, rounds in [("push", rsc.colors, rsc.rounds), ("seq", seq, R),
                                   ("pull", rsc.colors, rsc.rounds), ("seq", seq, R),
                                   ("push", rsc.colors, rsc.rounds)]:
            G.set("algorithm", algo)
            for _ in range(2):
                out = G.color()
                r, _ = G.stats()
                assert r == rounds and np.array_equal(out.cpu().numpy(), want), algo


@pytest.mark.parametrize("name", ["er_1m_16m", "stencil27_160", "rmat22_ef16"])
def test_seq_workloads(gc, name):
    g = graphgen.workload(name)
    assert g.sha256() == GOLDEN[name]["input_sha256"]
    print(f"[case] seq workload {name}", flush=True)
    assert_seq(gc, g, rp64=name.startswith("rmat"), mode="graph")
