"""GPU parity: the HIP colouring through the C ABI, bit for bit against the
CPU oracle (colours and round count), on every round driver, every lane
width, forced degree-class paths, sorted and unsorted rows, int32 and int64
row pointers, the degenerate graphs, and the full-size workloads.

Integer work: the bar is exact equality (no tolerance)."""
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
ALGOS = ["pull", "push"]
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


def gpu_color(gc, g, *, mode="persistent", rp64=False, rows_sorted=True, validate=True, **opts):
    rp, ci = _dev(g, rp64)
    with gc.Graph(rp, ci, validate=validate, rows_sorted=rows_sorted, mode=mode, **opts) as G:
        out = G.color()
        rounds, ncol = G.stats()
        sizes = G.round_sizes()
    return out.cpu().numpy(), rounds, ncol, sizes


def assert_parity(gc, g, ref=None, **kw):
    ref = ref or oracle.rsc(g.rowptr, g.colidx)
    col, rounds, ncol, sizes = gpu_color(gc, g, **kw)
    assert rounds == ref.rounds, (rounds, ref.rounds, kw)
    assert np.array_equal(col, ref.colors), kw
    assert ncol == ref.num_colors
    assert np.array_equal(sizes[: ref.rounds], ref.trace[:, 0]), kw
    return col


def _named_cases():
    return [
        ("K1", graphgen.complete(1)), ("K2", graphgen.complete(2)), ("K65", graphgen.complete(65)),
        ("K130", graphgen.complete(130)), ("path1", graphgen.path(1)), ("path2", graphgen.path(2)),
        ("path1001", graphgen.path(1001)), ("C5", graphgen.cycle(5)), ("C9", graphgen.cycle(9)),
        ("C10", graphgen.cycle(10)),
        ("P6", graphgen.from_edges(6, [(0, 1), (1, 2), (2, 3), (3, 5), (4, 5)])),
        ("star_lo", graphgen.star(300, 0)), ("star_hi", graphgen.star(300, 300)),
        ("crown8", graphgen.crown(8)), ("empty7", graphgen.empty(7)),
        ("er_small", graphgen.er(3000, 24000, 11)),
    ]


@pytest.mark.parametrize("algorithm", ALGOS)
@pytest.mark.parametrize("mode", MODES)
def test_named_graphs_every_mode(gc, mode, algorithm):
    for name, g in _named_cases():
        print(f"[case] {name} mode={mode} algorithm={algorithm}", flush=True)
        assert_parity(gc, g, mode=mode, algorithm=algorithm)


def test_no_vertices(gc):
    g = graphgen.CSR(np.zeros(1, np.int64), np.zeros(0, np.int32))
    for mode in MODES:
        col, rounds, ncol, _ = gpu_color(gc, g, mode=mode)
        assert col.size == 0 and rounds == 0 and ncol == 0


@pytest.mark.parametrize("lanes", [2, 4, 8, 16, 32, 64])
def test_every_lane_width(gc, lanes):
    for seed, (n, m) in enumerate([(5000, 60000), (777, 20000)]):
        g = graphgen.er(n, m, 100 + seed)
        print(f"[case] er n={n} m={m} lanes={lanes}", flush=True)
        for algo in ALGOS:
            assert_parity(gc, g, lanes=lanes, mode="persistent", algorithm=algo)
            assert_parity(gc, g, lanes=lanes, mode="chunked", algorithm=algo)


def test_forced_medium_and_heavy_paths(gc):
    # thresholds low enough that ordinary vertices take the wavefront and
    # workgroup paths
    g = graphgen.er(4000, 80000, 21)
    ref = oracle.rsc(g.rowptr, g.colidx)
    for medium, heavy in [(4, 30), (0, 1), (1, 2), (16, 40), (64, 100000)]:
        for mode in ("persistent", "host"):
            for algo in ALGOS:
                print(f"[case] classes medium={medium} heavy={heavy} mode={mode} {algo}", flush=True)
                assert_parity(gc, g, ref, mode=mode, medium_degree=medium or 1, heavy_degree=heavy,
                              algorithm=algo)


@pytest.mark.parametrize("k", [300, 600])
def test_hub_lists_and_their_pushes(gc, k):
    # The hub commits in round 2 while its k lower neighbours are all still
    # uncoloured: its conflict scan lists every one of them, and its pushes
    # to them come from that list (queued for the grid-wide push pass when
    # longer than a row the detect pass pushes itself, pushed inline by the
    # persistent kernel).  A lost push would let them take the hub's colour.
    g = graphgen.hub_over_losers(k)
    ref = oracle.rsc(g.rowptr, g.colidx)
    for medium, heavy in [(16, 100000), (16, 200)]:  # hub: wavefront class, then workgroup class
        for mode in ("host", "graph", "persistent"):
            print(f"[case] hub k={k} medium={medium} heavy={heavy} mode={mode}", flush=True)
            assert_parity(gc, g, ref, mode=mode, medium_degree=medium, heavy_degree=heavy,
                          algorithm="push")


def test_multiword_colour_windows(gc):
    # K_n needs colours up to n-1: beyond 64 (light/medium window) and with
    # heavy_degree small, beyond nothing; K_4200 would exceed the 4096-bit
    # heavy window but is large, so use a dense graph with heavy_degree low
    # (with pushed masks, colours >= 64 take the row-scan fallback)
    g = graphgen.complete(300)
    for medium, heavy in [(0, 100000), (1, 100000), (1, 2)]:
        for algo in ALGOS:
            print(f"[case] K300 medium={medium} heavy={heavy} {algo}", flush=True)
            assert_parity(gc, g, mode="persistent", medium_degree=medium or 400, heavy_degree=heavy,
                          algorithm=algo)


def test_unsorted_rows_and_int64_rowptr(gc):
    rng = np.random.default_rng(5)
    for g in (graphgen.er(3000, 30000, 7), graphgen.rmat(11, 8, .57, .19, .19, 2)):
        ref = oracle.rsc(g.rowptr, g.colidx)
        gs = graphgen.shuffle_rows(g, rng)
        for rp64 in (False, True):
            for sorted_rows, gg in ((True, g), (False, gs)):
                for algo in ALGOS:
                    print(f"[case] n={g.n} rp64={rp64} sorted={sorted_rows} {algo}", flush=True)
                    assert_parity(gc, gg, ref, rp64=rp64, rows_sorted=sorted_rows,
                                  mode="persistent", algorithm=algo)
                    assert_parity(gc, gg, ref, rp64=rp64, rows_sorted=sorted_rows, mode="host",
                                  medium_degree=8, heavy_degree=64, algorithm=algo)


def test_random_small_graphs(gc):
    rng = np.random.default_rng(42)
    for i in range(120):
        n = int(rng.integers(1, 60))
        g = graphgen.random_small(n, float(rng.choice([0.05, 0.2, 0.6])), rng)
        mode = MODES[i % len(MODES)]
        assert_parity(gc, g, mode=mode, lanes=int(rng.choice([2, 4, 16, 64])),
                      algorithm=ALGOS[(i // len(MODES)) % 2])


def test_validation_rejects_malformed_graphs(gc):
    def create(rp, ci, n, m, flags):
        return gc.gc_create(torch.tensor(rp, dtype=torch.int32).cuda(),
                            torch.tensor(ci, dtype=torch.int32).cuda(), n, m, flags)

    V = gc.GC_VALIDATE | gc.GC_ROWS_SORTED
    bad = {
        "self-loop": ([0, 1, 2], [0, 0], 2, 2),
        "range": ([0, 1, 2], [1, 5], 2, 2),
        "asymmetric": ([0, 1, 1], [1, 0], 2, 1),
        "duplicate": ([0, 2, 4], [1, 1, 0, 0], 2, 4),
        "unsorted": ([0, 2, 3, 4], [2, 1, 0, 0], 3, 4),
        "rowptr": ([0, 2, 1], [1, 0], 2, 2),
        "total": ([0, 1, 2], [1, 0], 2, 3),
    }
    for name, (rp, ci, n, m) in bad.items():
        with pytest.raises(gc.GCError) as ei:
            create(rp, ci, n, m, V)
        assert ei.value.code == gc.GC_EINVAL, name
    h = create([0, 1, 2], [1, 0], 2, 2, V)   # a single edge is fine
    gc.gc_destroy(h)


def test_validation_of_unsorted_rows(gc):
    """Rows not given as ascending are checked on a sorted copy: every
    malformed case names its check, valid unsorted graphs pass, and a hub of
    300,000 entries is checked in well under a second of device time."""
    import time

    def create(rp, ci, n, m):
        return gc.gc_create(torch.as_tensor(np.asarray(rp, np.int32)).cuda(),
                            torch.as_tensor(np.asarray(ci, np.int32)).cuda(), n, m, gc.GC_VALIDATE)

    bad = [  # (rowptr, colidx, n, m, the check named)
        ([0, 1, 2], [0, 0], 2, 2, "self-loop"),
        ([0, 1, 2], [1, 5], 2, 2, "out of range"),
        ([0, 1, 2], [1, -3], 2, 2, "out of range"),
        ([0, 1, 1], [1, 0], 2, 1, "one direction only"),
        ([0, 3, 5, 6], [1, 2, 1, 0, 0, 0], 3, 6, "duplicate"),
        ([0, 3, 2], [1, 0], 2, 2, "rowptr decreases"),
        ([0, 1, 2], [1, 0], 2, 3, "rowptr[0] != 0"),
    ]
    for rp, ci, n, m, what in bad:
        with pytest.raises(gc.GCError) as ei:
            create(rp, ci, n, m)
        assert ei.value.code == gc.GC_EINVAL, what
        assert what in str(ei.value), (what, str(ei.value))
    # a descending row is fine without GC_ROWS_SORTED
    gc.gc_destroy(create([0, 2, 3, 4], [2, 1, 0, 0], 3, 4))

    rng = np.random.default_rng(7)
    leaves = 300000
    g = graphgen.shuffle_rows(graphgen.star(leaves, centre=leaves // 2), rng)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    gc.gc_destroy(create(g.rowptr, g.colidx, g.n, g.nnz))
    assert time.perf_counter() - t0 < 5.0
    # the same hub with one repeated leaf, and with one leaf missing its reverse edge
    ci = g.colidx.copy()
    hub = slice(int(g.rowptr[leaves // 2]), int(g.rowptr[leaves // 2 + 1]))
    row = ci[hub]
    j = int(np.nonzero(row == 17)[0][0])
    k = int(np.nonzero(row == leaves - 3)[0][0])
    row2 = row.copy()
    row2[k] = 17
    ci[hub] = row2
    with pytest.raises(gc.GCError) as ei:
        create(g.rowptr, ci, g.n, g.nnz)
    assert "duplicate" in str(ei.value) and j != k
    # a shuffled ER graph passes; without one entry of its longest row it
    # stores that edge in one direction only
    e = graphgen.shuffle_rows(graphgen.er(5000, 40000, 3), rng)
    gc.gc_destroy(create(e.rowptr, e.colidx, e.n, e.nnz))
    rp = e.rowptr.copy()
    ci = e.colidx.copy()
    v = int(np.argmax(np.diff(rp)))
    ci = np.delete(ci, int(rp[v]))
    rp[v + 1:] -= 1
    with pytest.raises(gc.GCError) as ei:
        create(rp, ci, e.n, len(ci))
    assert "one direction only" in str(ei.value)


def test_round_cap_reports_erounds(gc):
    g = graphgen.path(200)
    rp, ci = _dev(g)
    for mode in ("host", "persistent", "chunked"):
        with gc.Graph(rp, ci, mode=mode, max_rounds=5) as G:
            G.color()
            with pytest.raises(gc.GCError) as ei:
                G.stats()
            assert ei.value.code == gc.GC_EROUNDS


def test_repeated_calls_and_reuse(gc):
    g = graphgen.er(20000, 200000, 9)
    ref = oracle.rsc(g.rowptr, g.colidx)
    rp, ci = _dev(g)
    with gc.Graph(rp, ci, mode="persistent") as G:
        out = torch.empty(g.n, dtype=torch.int32, device="cuda")
        for i in range(20):
            out.fill_(12345)  # stale contents must not matter
            G.color(out)
            r, k = G.stats()
            assert r == ref.rounds and np.array_equal(out.cpu().numpy(), ref.colors)
        for mode in MODES:
            G.set("mode", mode)
            G.color(out)
            assert G.stats()[0] == ref.rounds
            assert np.array_equal(out.cpu().numpy(), ref.colors)


def test_other_stream(gc):
    g = graphgen.er(20000, 150000, 4)
    ref = oracle.rsc(g.rowptr, g.colidx)
    rp, ci = _dev(g)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        with gc.Graph(rp, ci, mode="persistent") as G:
            out = G.color(stream=s)
            G.stats()
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), ref.colors)


def test_state_widths(gc):
    # the working state is 1, 2 or 4 bytes by maximum degree; all give the
    # oracle's bits
    cases = [(graphgen.star(126, 0), 1), (graphgen.star(127, 0), 2),
             (graphgen.complete(300), 2), (graphgen.star(40000, 7), 4)]
    for g, width in cases:
        rp, ci = _dev(g)
        with gc.Graph(rp, ci) as G:
            assert G.get(gc.GC_OPT_STATE_BYTES) == width
        for mode in ("graph", "host", "persistent"):
            for algo in ALGOS:
                assert_parity(gc, g, mode=mode, algorithm=algo)


def test_changed_graph_is_reported(gc):
    # same rowptr, different edges: (0,2),(1,2),(1,3) needs 2 rounds, the
    # path 0-1-2-3 needs 3.  After the first call the handle knows R = 2; a
    # graph changed in place against the contract must not pass silently.
    rp = torch.tensor([0, 1, 3, 5, 6], dtype=torch.int32, device="cuda")
    ci = torch.tensor([2, 2, 3, 0, 1, 1], dtype=torch.int32, device="cuda")
    with gc.Graph(rp, ci, mode="graph") as G:
        G.color()
        assert G.stats()[0] == 2
        ci.copy_(torch.tensor([1, 0, 2, 1, 3, 2], dtype=torch.int32))
        G.color()
        with pytest.raises(gc.GCError) as ei:
            G.stats()
        assert ei.value.code == gc.GC_EINVAL and "changed" in str(ei.value)
        out = G.color()   # the handle re-learns the round count
        assert G.stats()[0] == 3
        assert out.cpu().tolist() == [0, 1, 0, 1]


def test_profiled_calls(gc):
    g = graphgen.er(30000, 300000, 12)
    ref = oracle.rsc(g.rowptr, g.colidx)
    rp, ci = _dev(g)
    with gc.Graph(rp, ci, profile=1) as G:
        for i in range(3):
            out = G.color()
            assert G.stats()[0] == ref.rounds
            assert np.array_equal(out.cpu().numpy(), ref.colors)
        prof = G.profile(reset=True)
        # the first call discovers R (round 1 and finish timed only)
        assert prof["round1"][1] == 3 and prof["finish"][1] == 3
        assert prof["speculate"][1] == 2 * (ref.rounds - 1)
        assert prof["detect"][1] == 2 * (ref.rounds - 1)
        assert all(ms > 0 for ms, _ in prof.values())
        assert G.profile()["speculate"] == (0.0, 0)


def test_star_with_million_leaves(gc):
    # one vertex of degree 10^6 on the workgroup path (and the leaves first)
    for centre in (0, 1_000_000):
        g = graphgen.star(1_000_000, centre)
        col, rounds, _, _ = gpu_color(gc, g, mode="persistent")
        expect = np.ones(g.n, np.int32) if centre == 0 else np.zeros(g.n, np.int32)
        expect[centre] = 0 if centre == 0 else 1
        assert rounds == 2 and np.array_equal(col, expect)


def test_long_path_many_rounds(gc):
    # natural-order path: floor(n/2) + 1 rounds, colour v mod 2
    n = 20001
    g = graphgen.path(n)
    for mode in ("persistent", "graph"):
        col, rounds, ncol, _ = gpu_color(gc, g, mode=mode)
        assert rounds == n // 2 + 1
        assert np.array_equal(col, np.arange(n, dtype=np.int32) % 2)


@pytest.mark.parametrize("algorithm", ALGOS)
def test_complete_2048(gc, algorithm):
    g = graphgen.complete(2048)
    col, rounds, ncol, _ = gpu_color(gc, g, mode="persistent", algorithm=algorithm)
    assert rounds == 2048 and ncol == 2048
    assert np.array_equal(col, np.arange(2048, dtype=np.int32))


# ------------------------------------------------------ full-size inputs --

def _full(gc, name, **kw):
    print(f"[case] workload {name} {kw}", flush=True)
    g = graphgen.workload(name)
    gold = GOLDEN[name]
    assert g.sha256() == gold["input_sha256"]
    rp64 = name == "rmat22_ef16"
    col, rounds, ncol, sizes = gpu_color(gc, g, rp64=rp64, validate=False, **kw)
    import hashlib
    assert rounds == gold["rounds"]
    assert ncol == gold["num_colors"]
    assert hashlib.sha256(col.astype(np.int32).tobytes()).hexdigest() == gold["colors_sha256"]
    assert list(sizes[:rounds]) == gold["round_sizes"]
    return g, col


@pytest.mark.slow
def test_workload_er_10k(gc):
    g, col = _full(gc, "er_10k_100k")
    ref = oracle.rsc(g.rowptr, g.colidx)
    assert np.array_equal(col, ref.colors)
    for mode in MODES:
        _full(gc, "er_10k_100k", mode=mode)


@pytest.mark.slow
def test_workload_er_1m(gc):
    _full(gc, "er_1m_16m", algorithm="pull")
    g, col = _full(gc, "er_1m_16m", algorithm="push")
    ref = oracle.rsc(g.rowptr, g.colidx)   # the oracle itself, a few seconds
    assert np.array_equal(col, ref.colors)
    assert oracle.check_proper(g.rowptr, g.colidx, col) == 0


@pytest.mark.slow
def test_workload_stencil(gc):
    _full(gc, "stencil27_160", algorithm="pull")
    g, col = _full(gc, "stencil27_160", algorithm="push")
    assert oracle.check_proper(g.rowptr, g.colidx, col) == 0
    assert oracle.check_grundy(g.rowptr, g.colidx, col) == 0


@pytest.mark.slow
def test_workload_rmat(gc):
    _full(gc, "rmat22_ef16", algorithm="pull")
    g, col = _full(gc, "rmat22_ef16", algorithm="push")
    assert oracle.check_proper(g.rowptr, g.colidx, col) == 0
    assert oracle.check_grundy(g.rowptr, g.colidx, col) == 0


def test_options_changed_between_calls_on_one_handle(gc):
    # a captured round graph carries its degree lists, flag blocks and grid:
    # every option change between calls must give the oracle's bits
    g = graphgen.rmat(14, 16, seed=3)
    ref = oracle.rsc(g.rowptr, g.colidx)
    rp, ci = _dev(g, rp64=True)
    steps = [{}, {"heavy_degree": 1024}, {"heavy_degree": 16384}, {"blocks_per_cu": 2},
             {"medium_degree": 32}, {"lanes": 4}, {"heavy_degree": 256, "medium_degree": 16},
             {"blocks_per_cu": 16}, {"algorithm": "pull"}, {"heavy_degree": 2048}]
    with gc.Graph(rp, ci, mode="graph") as G:
        for opts in steps:
            for k, v in opts.items():
                G.set(k, v)
            for _ in range(2):
                print(f"[case] live options {opts}", flush=True)
                out = G.color()
                r, _ = G.stats()
                assert r == ref.rounds, opts
                assert np.array_equal(out.cpu().numpy(), ref.colors), opts


def test_flag_layout_switch_between_calls(gc):
    # with no medium or heavy vertex the pushed flags are stored colour-major
    # per 64-vertex chunk, otherwise 32 bytes per vertex; the layout follows
    # the degree classes from call to call on one handle, and the flags left
    # by a call in the other layout must never count
    g = graphgen.er(20000, 200000, 17)
    ref = oracle.rsc(g.rowptr, g.colidx)
    rp, ci = _dev(g)
    steps = [({}, False), ({"medium_degree": 16}, True), ({"medium_degree": 0}, False),
             ({"medium_degree": 24}, True), ({"lanes": 32}, None)]
    with gc.Graph(rp, ci, mode="graph") as G:
        for opts, medium in steps:
            for k, v in opts.items():
                G.set(k, v)
            for _ in range(2):
                print(f"[case] flag layout, options {opts}", flush=True)
                out = G.color()
                r, _ = G.stats()
                if medium is not None:
                    assert (G.get(gc.GC_OPT_MEDIUM_COUNT) > 0) == medium, opts
                assert r == ref.rounds, opts
                assert np.array_equal(out.cpu().numpy(), ref.colors), opts


def test_option_values_are_checked(gc):
    # every option rejects values outside its range with GC_EINVAL and keeps
    # its previous value; the handle still colours correctly afterwards
    g = graphgen.er(3000, 20000, 13)
    ref = oracle.rsc(g.rowptr, g.colidx)
    rp, ci = _dev(g)
    bad = [(gc.GC_OPT_MODE, 9), (gc.GC_OPT_LANES, 3), (gc.GC_OPT_LANES, 128),
           (gc.GC_OPT_HEAVY_DEGREE, 0), (gc.GC_OPT_BLOCKS_PER_CU, 0),
           (gc.GC_OPT_BLOCKS_PER_CU, 65), (gc.GC_OPT_MAX_ROUNDS, -1),
           (gc.GC_OPT_CHUNK_ROUNDS, 0), (gc.GC_OPT_PERSISTENT_BLOCKS_PER_CU, 5),
           (gc.GC_OPT_PROFILE, 2), (gc.GC_OPT_ALGORITHM, 5), (gc.GC_OPT_ALGORITHM, -1),
           (gc.GC_OPT_PARTITIONS, -1), (gc.GC_OPT_ORDER, 3), (99, 0)]
    with gc.Graph(rp, ci) as G:
        before = {opt: G.get(opt) for opt, _ in bad if opt != 99}
        for opt, val in bad:
            with pytest.raises(gc.GCError) as e:
                gc.gc_set_option(G.h, opt, val)
            assert e.value.code == gc.GC_EINVAL, (opt, val)
        for opt, v in before.items():
            assert G.get(opt) == v, opt
        with pytest.raises(gc.GCError):
            G.get(99)
        out = G.color()
        assert G.stats()[0] == ref.rounds
        assert np.array_equal(out.cpu().numpy(), ref.colors)


@pytest.mark.parametrize("rp64", [False, True])
def test_persistent_kernel_on_a_full_grid(gc, rp64):
    # 400,000 vertices give 6,250 chunks of 64: more workgroups than every
    # CU can hold, so the cooperative grid is at its co-residency bound
    # (4 workgroups per CU with int32 row pointers, 3 with int64 ones, from
    # the kernel's register use), and every per-CU setting below it
    g = graphgen.er(400_000, 4_000_000, 21)
    ref = oracle.rsc(g.rowptr, g.colidx)
    for per_cu in (4, 3, 1):
        print(f"[case] persistent full grid rp64={rp64} per_cu={per_cu}", flush=True)
        assert_parity(gc, g, ref, mode="persistent", rp64=rp64, persistent_blocks_per_cu=per_cu)
