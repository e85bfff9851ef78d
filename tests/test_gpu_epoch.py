"""GPU: the pushed colour flags across the 8-bit epoch wrap.

Under the push algorithm a call marks "colour c is final on a neighbour" by
storing the call's epoch (1..255) into byte c of a vertex's flag block
(colours 0..31), or of its wide block (colours 32..511, vertices of the
wavefront and workgroup classes) -- the GPU form of Algorithm 1's update of
a neighbour's ForbiddenColors (Section 3.1).  Flags are cleared only on the
first call and when the epoch wraps, so a byte left from an earlier cycle
must never equal a later epoch.  These tests run more than 255 calls on one
handle and check every result bit for bit against the oracle, including
calls where the degree classes change between calls so that wide blocks
unused for a while are read again after the wrap.
"""
import numpy as np
import pytest

import graphgen
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def gc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1509_08267_amd import gc as gcmod
    gcmod.load()
    return gcmod


def _dev(g):
    return (torch.from_numpy(g.rowptr.astype(np.int32)).cuda(),
            torch.from_numpy(g.colidx).cuda())


@pytest.mark.parametrize("layout", ["by_chunk", "by_vertex"])
def test_three_hundred_calls_across_the_wrap(gc, layout):
    # ER graphs with no medium vertex use the chunk-major flag layout; a low
    # medium threshold moves the vertices of degree above it to the wavefront
    # path and the flags to the by-vertex layout
    g = graphgen.er(6000, 60000, 31)
    ref = oracle.rsc(g.rowptr, g.colidx)
    rp, ci = _dev(g)
    opts = {} if layout == "by_chunk" else {"medium_degree": 20}
    with gc.Graph(rp, ci, algorithm="push", **opts) as G:
        out = torch.empty(g.n, dtype=torch.int32, device="cuda")
        for call in range(300):
            G.color(out)
            rounds, _ = G.stats()
            if call == 0:  # the degree classes are rebuilt by the first call
                assert (G.get(gc.GC_OPT_MEDIUM_COUNT) > 0) == (layout == "by_vertex")
            if call < 5 or 250 <= call <= 260 or call % 37 == 0 or call == 299:
                assert rounds == ref.rounds, call
                assert np.array_equal(out.cpu().numpy(), ref.colors), call


def test_wide_blocks_reused_after_the_wrap(gc):
    # A dense graph needs colours beyond 31, which wavefront-class vertices
    # take from their wide blocks.  Call k runs with epoch (k mod 255) + 1.
    # Calls 0..9 run with every vertex in the wavefront class, so each wide
    # block ends up holding epoch 10 in the bytes of the colours pushed to
    # it; calls 10..259 run with 3 such vertices, so when the epoch wraps at
    # call 255 only 3 blocks are in use; calls 260..279 put every vertex back
    # in the class.  Call 264 runs with epoch 10 again: unless the clear at
    # the wrap covered every allocated block, the stale bytes equal to 10
    # hide free colours and the colouring stops being First Fit.
    g = graphgen.er(1500, 150_000, 32)
    ref = oracle.rsc(g.rowptr, g.colidx)
    assert ref.num_colors > 40
    rp, ci = _dev(g)
    many, few = 64, 240
    with gc.Graph(rp, ci, algorithm="push", medium_degree=many) as G:
        out = torch.empty(g.n, dtype=torch.int32, device="cuda")
        for call in range(280):
            if call == 10:
                G.set("medium_degree", few)
            elif call == 260:
                G.set("medium_degree", many)
            G.color(out)
            rounds, ncol = G.stats()
            # (the degree classes are rebuilt by the first call after a change)
            if call in (0, 260):
                assert G.get(gc.GC_OPT_MEDIUM_COUNT) == g.n, call
            elif call == 10:
                assert 0 < G.get(gc.GC_OPT_MEDIUM_COUNT) < 10
            assert rounds == ref.rounds, call
            assert np.array_equal(out.cpu().numpy(), ref.colors), call
