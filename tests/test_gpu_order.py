"""GPU: colouring in a vertex order (GC_OPT_ORDER) equals the oracle's
colouring of the relabelled graph mapped back, bit for bit (colours and
round count), for the largest-first and seeded random orders, under every
algorithm, with unsorted input rows, int64 row pointers, order changes on a
live handle and the 1M-vertex ER workload."""
import numpy as np
import pytest

import graphgen
import oracle
from oracle import ordering

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

ALGOS = {
    "push": lambda rp, ci: (oracle.rsc(rp, ci).colors, oracle.rsc(rp, ci).rounds),
    "pull": lambda rp, ci: (oracle.rsc(rp, ci).colors, oracle.rsc(rp, ci).rounds),
    "seq": lambda rp, ci: (oracle.seq(rp, ci), oracle.seq_rounds(rp, ci)[0]),
    "blocks": lambda rp, ci: oracle.blocks(rp, ci, 64)[:2],
}


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


def expected(g, kind, seed, algo):
    col, (c2, R) = ordering.colour_in_order(g.rowptr, g.colidx, kind, seed, ALGOS[algo])
    return col, R


def check(gc, G, g, kind, seed, algo):
    want, R = expected(g, kind, seed, algo)
    G.set("algorithm", algo)
    G.set("partitions", 64)
    G.set("order", kind)
    G.set("order_seed", seed)
    for _ in range(2):
        out = G.color()
        r, _ = G.stats()
        assert r == R, (kind, seed, algo, r, R)
        assert np.array_equal(out.cpu().numpy(), want), (kind, seed, algo)


@pytest.mark.parametrize("algo", list(ALGOS))
@pytest.mark.parametrize("kind,seed", [("largest_first", 0), ("random", 0), ("random", 12345)])
def test_orders_every_algorithm(gc, algo, kind, seed):
    for name, g in [("er", graphgen.er(5000, 60000, 3)), ("star", graphgen.star(3000, 1500)),
                    ("crown", graphgen.crown(20)), ("rmat12", graphgen.rmat(12, 16, seed=4))]:
        print(f"[case] order {kind}/{seed} {algo} {name}", flush=True)
        rp, ci = _dev(g, rp64=name.startswith("rmat"))
        with gc.Graph(rp, ci, validate=True) as G:
            check(gc, G, g, kind, seed, algo)


def test_orders_unsorted_rows_and_live_changes(gc):
    g = graphgen.er(8000, 90000, 6)
    u = graphgen.shuffle_rows(g, np.random.default_rng(2))
    rp, ci = _dev(u)
    with gc.Graph(rp, ci, validate=True, rows_sorted=False) as G:
        for kind, seed in [("largest_first", 0), ("random", 1), ("random", 2), ("natural", 0),
                           ("largest_first", 0)]:
            print(f"[case] live order {kind}/{seed}", flush=True)
            if kind == "natural":
                ref = oracle.rsc(g.rowptr, g.colidx)
                G.set("algorithm", "push")
                G.set("order", kind)
                out = G.color()
                assert G.stats()[0] == ref.rounds
                assert np.array_equal(out.cpu().numpy(), ref.colors)
            else:
                check(gc, G, g, kind, seed, "push")


@pytest.mark.parametrize("kind", ["largest_first", "random"])
def test_orders_workload_er_1m(gc, kind):
    g = graphgen.workload("er_1m_16m")
    rp, ci = _dev(g)
    with gc.Graph(rp, ci) as G:
        check(gc, G, g, kind, 0, "push")


@pytest.fixture(scope="module")
def dense():
    # dense ER: average degree 1000, 187 colours (past the 32 flag bytes, into
    # the wide blocks of the wavefront-per-vertex path)
    return graphgen.er(8000, 4000000, 17)


@pytest.mark.parametrize("algo", ["push", "pull", "seq"])
def test_dense_graph_natural_order(gc, dense, algo):
    g = dense
    want, R = ALGOS[algo](g.rowptr, g.colidx)
    rp, ci = _dev(g)
    with gc.Graph(rp, ci, algorithm=algo) as G:
        for _ in range(2):
            out = G.color()
            r, k = G.stats()
            assert r == R and np.array_equal(out.cpu().numpy(), want), algo


def test_dense_graph_largest_first(gc, dense):
    rp, ci = _dev(dense)
    with gc.Graph(rp, ci) as G:
        check(gc, G, dense, "largest_first", 0, "push")
