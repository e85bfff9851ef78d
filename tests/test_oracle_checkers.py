"""Pins of the oracle's two property checkers and of its batch wrapper.

The checkers are what the large-workload GPU tests assert beside bit
equality, so each must be seen to flag bad colourings with the exact count
its definition gives, not only to accept good ones:

* ``check_proper`` counts CSR entries (v, u) whose endpoints share a colour,
  plus vertices left without a colour: 0 exactly for a proper colouring
  (Section 2.1; Lemma 1 of Section 4);
* ``check_grundy`` counts vertices whose colour is not the least colour
  absent from their neighbourhood (First Fit, Section 3).

Every expected count below was worked by hand from those definitions, so a
checker stubbed to return 0, or one that is off by one (one direction of an
edge only, one candidate colour too few or too many, the vertex itself in
its own neighbourhood), fails at least one case.

``rsc_batch`` must colour every graph of a packed batch exactly as ``rsc``
colours it alone, with the per-graph offsets of the packed layout (local
rowptr of graph g at voff[g] + g).
"""
import numpy as np
import pytest

import graphgen
import oracle


def proper(g, colors):
    return oracle.check_proper(g.rowptr, g.colidx, np.asarray(colors, np.int32))


def grundy(g, colors):
    return oracle.check_grundy(g.rowptr, g.colidx, np.asarray(colors, np.int32))


# ------------------------------------------------------------ check_proper --

@pytest.mark.parametrize("graph, colors, expected", [
    # K3 = triangle 0-1-2
    ("k3", [0, 1, 2], 0),
    ("k3", [0, 0, 1], 2),      # edge 0-1 seen from both rows
    ("k3", [0, 0, 0], 6),      # all three edges, both directions
    ("k3", [5, 5, 1], 2),      # any colour values, not only small ones
    # path 0-1-2-3
    ("p4", [0, 1, 0, 1], 0),
    ("p4", [0, 0, 1, 0], 2),   # edge 0-1
    ("p4", [0, 0, 0, 0], 6),   # three edges
    ("p4", [1, 0, 0, 1], 2),   # edge 1-2
    # a vertex left uncoloured counts once, and two adjacent uncoloured
    # vertices also share the value -1 along their edge
    ("p4", [0, -1, 0, 1], 1),
    ("p4", [-1, -1, 0, 1], 4),
    # edgeless graph: only uncoloured vertices count
    ("e3", [0, 0, 0], 0),
    ("e3", [0, -1, -7], 2),
    # star with centre 0 and four leaves: a leaf sharing the centre's colour
    ("s4", [0, 1, 1, 1, 1], 0),
    ("s4", [1, 1, 0, 1, 0], 4),  # leaves 1 and 3 clash with the centre
])
def test_check_proper_exact_counts(graph, colors, expected):
    g = {"k3": graphgen.complete(3), "p4": graphgen.path(4), "e3": graphgen.empty(3),
         "s4": graphgen.star(4)}[graph]
    assert proper(g, colors) == expected


def test_check_proper_sees_a_single_bad_edge_anywhere():
    # C_10 properly 2-coloured, then one vertex at a time recoloured to its
    # neighbour's colour: exactly its clashing edge(s), counted from both
    # rows, must show
    g = graphgen.cycle(10)
    good = [v % 2 for v in range(10)]
    assert proper(g, good) == 0
    for v in range(10):
        bad = list(good)
        bad[v] = 1 - bad[v]   # now equal to both of its neighbours
        assert proper(g, bad) == 4, v


def test_check_proper_zero_vertices():
    g = graphgen.empty(0)
    assert oracle.check_proper(g.rowptr, g.colidx, np.zeros(0, np.int32)) == 0


# ------------------------------------------------------------ check_grundy --

@pytest.mark.parametrize("graph, colors, expected", [
    # path 0-1-2
    ("p3", [0, 1, 0], 0),      # the First-Fit colouring
    ("p3", [1, 0, 1], 0),      # also least-absent everywhere (mex{0}=1, mex{1}=0)
    ("p3", [0, 2, 0], 1),      # vertex 1: mex{0} = 1, not 2
    ("p3", [0, 1, 2], 1),      # vertex 2: mex{1} = 0, not 2
    ("p3", [1, 2, 1], 3),      # 0: mex{2}=0; 1: mex{1}=0; 2: mex{2}=0
    ("p3", [0, 0, 0], 3),      # improper: every vertex sees colour 0
    # K4 needs every colour 0..3: a vertex may take deg(v) + 1 - 1 = 3
    ("k4", [0, 1, 2, 3], 0),
    ("k4", [3, 2, 1, 0], 0),
    ("k4", [0, 1, 2, 4], 1),   # 4 exceeds the least absent (3)
    # isolated vertices: the least absent colour is 0
    ("e3", [0, 0, 0], 0),
    ("e3", [0, 1, -1], 2),
    # star with centre 0: leaves must take mex{centre}
    ("s4", [0, 1, 1, 1, 1], 0),
    ("s4", [1, 0, 0, 0, 0], 0),
])
def test_check_grundy_exact_counts(graph, colors, expected):
    g = {"p3": graphgen.path(3), "k4": graphgen.complete(4), "e3": graphgen.empty(3),
         "s4": graphgen.star(4)}[graph]
    assert grundy(g, colors) == expected


def test_check_grundy_star_worked_out():
    # star, centre 0, leaves 1..4, colours [2, 0, 1, 0, 0]:
    #   centre sees {0, 1, 0, 0}: least absent 2 -> fine
    #   leaf 1 sees {2}: least absent 0 -> fine
    #   leaf 2 sees {2}: least absent 0, has 1 -> flagged
    #   leaves 3, 4 as leaf 1 -> fine
    # and with leaf 2 recoloured 0 the centre's colour 2 is no longer the
    # least absent (colour 1 is now free), so the centre is flagged instead
    g = graphgen.star(4)
    assert grundy(g, [2, 0, 1, 0, 0]) == 1
    assert grundy(g, [2, 0, 0, 0, 0]) == 1       # centre: mex{0} = 1, not 2
    assert grundy(g, [1, 0, 0, 0, 0]) == 0


def test_check_grundy_flags_every_vertex_of_a_shifted_colouring():
    # C_10 coloured v mod 2 is First Fit.  Adding 1 to every colour gives the
    # even vertices colour 1 beside neighbours coloured 2, and the odd ones
    # colour 2 beside neighbours coloured 1: the least absent colour is 0 for
    # every vertex, so all ten are flagged
    g = graphgen.cycle(10)
    good = np.array([v % 2 for v in range(10)], np.int32)
    assert grundy(g, good) == 0
    assert grundy(g, good + 1) == 10


# -------------------------------------------------------------- rsc_batch --

def _pack(graphs):
    voff = np.zeros(len(graphs) + 1, np.int64)
    eoff = np.zeros(len(graphs) + 1, np.int64)
    rps, cis = [], []
    for i, g in enumerate(graphs):
        voff[i + 1] = voff[i] + g.n
        eoff[i + 1] = eoff[i] + g.nnz
        rps.append(g.rowptr.astype(np.int32))
        cis.append(g.colidx.astype(np.int32))
    rpl = np.concatenate(rps) if rps else np.zeros(0, np.int32)
    cil = np.concatenate(cis) if cis else np.zeros(0, np.int32)
    return voff, eoff, rpl, cil


def _mixed_batch():
    return [graphgen.path(5), graphgen.empty(0), graphgen.empty(3), graphgen.complete(4),
            graphgen.cycle(5), graphgen.er(200, 800, 1), graphgen.empty(0), graphgen.star(6, 6),
            graphgen.crown(4), graphgen.er(1000, 6000, 2), graphgen.empty(1)]


def test_rsc_batch_equals_per_graph_rsc():
    graphs = _mixed_batch()
    voff, eoff, rpl, cil = _pack(graphs)
    colors, rounds = oracle.rsc_batch(voff, eoff, rpl, cil)
    assert colors.shape[0] == voff[-1] and rounds.shape[0] == len(graphs)
    for i, g in enumerate(graphs):
        r = oracle.rsc(g.rowptr, g.colidx)
        got = colors[voff[i]:voff[i + 1]]
        assert np.array_equal(got, r.colors), i
        assert rounds[i] == r.rounds, i


def test_rsc_batch_closed_forms():
    # the hand-worked results of single graphs, read through the packed layout
    graphs = _mixed_batch()
    voff, eoff, rpl, cil = _pack(graphs)
    colors, rounds = oracle.rsc_batch(voff, eoff, rpl, cil)
    part = lambda i: list(colors[voff[i]:voff[i + 1]])
    assert part(0) == [0, 1, 0, 1, 0] and rounds[0] == 3      # path, R = floor(5/2) + 1
    assert part(1) == [] and rounds[1] == 0                   # n = 0
    assert part(2) == [0, 0, 0] and rounds[2] == 1            # edgeless
    assert part(3) == [0, 1, 2, 3] and rounds[3] == 4         # K4
    assert part(4) == [0, 1, 0, 2, 1] and rounds[4] == 3      # C5
    assert part(6) == [] and rounds[6] == 0
    assert part(7) == [0, 0, 0, 0, 0, 0, 1] and rounds[7] == 2  # star, centre highest
    assert part(8) == [0, 0, 1, 1, 2, 2, 3, 3] and rounds[8] == 4  # crown K_{4,4} - M
    assert part(10) == [0] and rounds[10] == 1


def test_rsc_batch_order_of_graphs_does_not_matter():
    graphs = _mixed_batch()
    perm = np.random.default_rng(3).permutation(len(graphs))
    voff, eoff, rpl, cil = _pack(graphs)
    c0, r0 = oracle.rsc_batch(voff, eoff, rpl, cil)
    pv, pe, prp, pci = _pack([graphs[i] for i in perm])
    c1, r1 = oracle.rsc_batch(pv, pe, prp, pci)
    for j, i in enumerate(perm):
        assert np.array_equal(c1[pv[j]:pv[j + 1]], c0[voff[i]:voff[i + 1]])
        assert r1[j] == r0[i]
