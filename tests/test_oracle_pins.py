"""Pins of the CPU oracle against what the paper and the mathematics fix.

The paper prints no worked example and no colouring (its figures are lost),
so the oracle is pinned by:

* closed forms worked by hand from Algorithm 1 (Section 3.1) with one vertex
  per block and the higher id recoloured on a conflict: complete graphs,
  paths, cycles, stars, crown graphs, empty graphs;
* properties fixed by the problem and the proofs: properness (Section 2.1,
  Lemma 1), First Fit's least-absent-colour property (Section 3), the
  Delta+1 bound (Section 2.1), termination and per-vertex recolouring bounds
  (Lemma 2 and its corollary, Section 4, with p = n);
* the brute-force chromatic number as a lower bound on any colour count;
* a second implementation written separately (``oracle.ref_py``);
* mutants of the definition (a flipped tie-break, sequential visibility,
  stale colours, an off-by-one First Fit, no conflict check) that each fail
  at least one of the pins above, showing the pins can see such mistakes.
"""
import numpy as np
import pytest

import graphgen
import oracle
from oracle import ref_py


def run(g):
    return oracle.rsc(g.rowptr, g.colidx)


def adj(g):
    return ref_py.adjacency(g.rowptr, g.colidx)


# ------------------------------------------------------------ closed forms --

@pytest.mark.parametrize("n", [1, 2, 3, 7, 31, 64, 65, 130])
def test_complete_graph_gets_n_colours(n):
    # K_n: in round r the vertices r-1..n-1 are uncoloured and all see colours
    # 0..r-2, so all try r-1 and only the lowest id keeps it.
    r = run(graphgen.complete(n))
    assert list(r.colors) == list(range(n))
    assert r.rounds == n
    assert r.num_colors == n


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 10, 11, 100, 1001])
def test_path_natural_order_gets_two_colours(n):
    # Path 0-1-...-(n-1): round 1 fixes vertex 0; each later round fixes the
    # next two vertices (colours 1 then 0), so colour v mod 2 and
    # R = floor(n/2) + 1.
    r = run(graphgen.path(n))
    assert list(r.colors) == [v % 2 for v in range(n)]
    assert r.rounds == n // 2 + 1
    assert r.num_colors == min(n, 2)


def test_cycle_5():
    # Round 1: only 0 keeps colour 0.  Round 2: 1 and 4 see colour 0 and try
    # 1; 2 and 3 try 0; 3 loses to 2.  Round 3: 3 sees 0 and 1, takes 2.
    r = run(graphgen.cycle(5))
    assert list(r.colors) == [0, 1, 0, 2, 1]
    assert r.rounds == 3
    assert list(r.round_of) == [1, 2, 2, 3, 2]


def test_cycle_9_and_10():
    # Rounds fix {0}, {1,2,8}, {3,4}, {5,6}, then the last vertex (odd n)
    # sees both 0 and 1 (colour 2) or the last two alternate (even n).
    r9 = run(graphgen.cycle(9))
    assert list(r9.colors) == [0, 1, 0, 1, 0, 1, 0, 2, 1]
    assert r9.rounds == 5
    r10 = run(graphgen.cycle(10))
    assert list(r10.colors) == [v % 2 for v in range(10)]
    assert r10.rounds == 5


def test_six_vertex_path_relabelled():
    # Edges 0-1, 1-2, 2-3, 3-5, 4-5 (a path 0-1-2-3-5-4).  Round 1 fixes 0
    # and 4 (no lower neighbour).  Round 2: 1 and 5 see colour 0 and try 1,
    # 2 and 3 try 0, 3 loses to 2.  Round 3: 3 sees 0 and 1 and takes 2.
    g = graphgen.from_edges(6, [(0, 1), (1, 2), (2, 3), (3, 5), (4, 5)])
    r = run(g)
    assert list(r.colors) == [0, 1, 0, 2, 0, 1]
    assert r.rounds == 3
    # sequential First Fit differs here (a round-synchronous build that
    # silently ran in sequential order would be caught)
    assert list(oracle.seq(g.rowptr, g.colidx)) == [0, 1, 0, 1, 0, 2]


@pytest.mark.parametrize("leaves", [1, 4, 50])
def test_star_centre_lowest(leaves):
    # Centre 0 has no lower neighbour: colour 0 in round 1; leaves take 1.
    r = run(graphgen.star(leaves, centre=0))
    assert list(r.colors) == [0] + [1] * leaves
    assert r.rounds == 2


@pytest.mark.parametrize("leaves", [1, 4, 50])
def test_star_centre_highest(leaves):
    # Leaves 0..k-1 have no lower neighbour: colour 0; the centre k loses
    # round 1 and takes 1 in round 2.  (With the lower id recoloured instead,
    # the leaves would be recoloured: this case pins the tie-break.)
    r = run(graphgen.star(leaves, centre=leaves))
    assert list(r.colors) == [0] * leaves + [1]
    assert r.rounds == 2


@pytest.mark.parametrize("k", [2, 3, 5, 8])
def test_crown_graph_first_fit_worst_case(k):
    # a_i = 2i, b_j = 2j+1, a_i ~ b_j iff i != j.  Round r fixes a_{r-1} and
    # b_{r-1} with colour r-1 (each sees colours 0..r-2 on its committed
    # opposite-side neighbours), so k colours for a 2-colourable graph.
    r = run(graphgen.crown(k))
    assert list(r.colors) == [i // 2 for i in range(2 * k)]
    assert r.rounds == k
    if 2 * k <= 10:
        assert ref_py.chromatic_number(adj(graphgen.crown(k))) == 2


@pytest.mark.parametrize("k", [1, 3, 600])
def test_hub_over_losers_worked_rounds(k):
    # Paths x1 - x2 - c - b, every b joined to the hub v, and v to w (ids in
    # that order, v last).  Round 1: x1 and w have no lower neighbour and
    # keep 0; x2, c, b and v lose to a lower neighbour also trying 0.  Round
    # 2: x2 tries 1 (x1 has 0) and keeps it; c and b try 0 (no final
    # neighbour), c keeps it over x2's 1, b loses to c; v tries 1 (w has 0)
    # and keeps it, since every b (lower) tries 0.  Round 3: b sees 0 on c and
    # 1 on v and takes 2.
    r = run(graphgen.hub_over_losers(k))
    assert list(r.colors) == [0] * k + [1] * k + [0] * k + [2] * k + [0, 1]
    assert r.rounds == 3
    assert list(r.trace[:, 0]) == [4 * k + 2, 3 * k + 1, k]


@pytest.mark.parametrize("n", [1, 5, 100])
def test_empty_graph(n):
    r = run(graphgen.empty(n))
    assert list(r.colors) == [0] * n
    assert r.rounds == 1


def test_no_vertices():
    r = oracle.rsc(np.zeros(1, np.int64), np.zeros(0, np.int32))
    assert r.rounds == 0 and r.colors.size == 0 and r.num_colors == 0


# ---------------------------------------------- sequential First Fit (SEQ) --

def test_seq_textbook_cases():
    assert list(oracle.seq(*_csr(graphgen.complete(6)))) == list(range(6))
    assert list(oracle.seq(*_csr(graphgen.path(9)))) == [v % 2 for v in range(9)]
    assert list(oracle.seq(*_csr(graphgen.cycle(5)))) == [0, 1, 0, 1, 2]
    # crown graph in the interleaved order is First Fit's worst case: k colours
    assert list(oracle.seq(*_csr(graphgen.crown(5)))) == [i // 2 for i in range(10)]


def _csr(g):
    return g.rowptr, g.colidx


# ------------------------------- id-priority schedule of SEQ (its rounds) --

def test_seq_rounds_closed_forms():
    # a path in natural order is one increasing path: round v + 1 for v
    R, ro = oracle.seq_rounds(*_csr(graphgen.path(9)))
    assert R == 9 and list(ro) == list(range(1, 10))
    # K_n: the ids themselves form the longest increasing path
    R, ro = oracle.seq_rounds(*_csr(graphgen.complete(7)))
    assert R == 7 and list(ro) == list(range(1, 8))
    # star: leaves before a high centre, or a low centre before its leaves
    R, ro = oracle.seq_rounds(*_csr(graphgen.star(5, centre=5)))
    assert R == 2 and list(ro) == [1] * 5 + [2]
    R, ro = oracle.seq_rounds(*_csr(graphgen.star(5, centre=0)))
    assert R == 2 and list(ro) == [1] + [2] * 5
    # no edges: one round; no vertices: none
    assert oracle.seq_rounds(*_csr(graphgen.empty(4)))[0] == 1
    assert oracle.seq_rounds(*_csr(graphgen.empty(0)))[0] == 0
    # path relabelled so the ids alternate low/high: every vertex is a local
    # extreme, two rounds
    p = graphgen.relabel(graphgen.path(8), [0, 4, 1, 5, 2, 6, 3, 7])
    assert oracle.seq_rounds(*_csr(p))[0] == 2


def test_seq_rounds_equal_longest_increasing_path_by_enumeration():
    for g in _random_graphs(500, 9, seed=21):
        R, ro = oracle.seq_rounds(g.rowptr, g.colidx)
        best = ref_py.longest_increasing_path(adj(g))
        assert list(ro) == best
        assert R == (max(best) if best else 0)


def test_seq_schedule_reproduces_sequential_first_fit():
    # the round-by-round schedule colours exactly like SEQ, in depth rounds
    for g in list(_random_graphs(300, 11, seed=22)) + [graphgen.er(300, 2000, 4)]:
        col, R, round_of = ref_py.seq_schedule(adj(g))
        assert col == list(oracle.seq(g.rowptr, g.colidx))
        R2, ro = oracle.seq_rounds(g.rowptr, g.colidx)
        assert R == R2 and round_of == list(ro)


def test_seq_rounds_pins_reject_a_reversed_dependency():
    # a plausible slip: depending on higher-id neighbours instead
    def wrong(g):
        n = g.n
        d = [0] * n
        a = adj(g)
        for v in reversed(range(n)):
            d[v] = 1 + max([d[u] for u in a[v] if u > v], default=0)
        return d
    g = graphgen.star(5, centre=0)
    assert wrong(g) != list(oracle.seq_rounds(*_csr(g))[1])


# ------------------------------- Algorithm 1 with p blocks, read literally --

def test_blocks_hand_worked_path():
    # path 0-1-2, p = 3: round 1 all take 0; 0 and 1 lose to their higher
    # neighbours; round 2 both take 1 (their slots hold 0), 0 loses to 1
    # again; round 3 vertex 0 sees 1 in its slot and takes 0
    col, R, rec = oracle.blocks(*_csr(graphgen.path(3)), 3)
    assert list(col) == [0, 1, 0] and R == 3 and list(rec) == [2, 1, 0]


def test_blocks_star_centre_in_lowest_block():
    # every vertex its own block: the centre (block 0) loses to every leaf
    # in round 1 and takes 1 in round 2
    col, R, rec = oracle.blocks(*_csr(graphgen.star(6, centre=0)), 7)
    assert list(col) == [1] + [0] * 6 and R == 2 and list(rec) == [1] + [0] * 6


def test_blocks_one_block_is_sequential_first_fit():
    for g in list(_random_graphs(300, 12, seed=31)) + [graphgen.er(2000, 16000, 2)]:
        col, R, rec = oracle.blocks(g.rowptr, g.colidx, 1)
        assert list(col) == list(oracle.seq(g.rowptr, g.colidx))
        assert R == (1 if g.n else 0) and not rec.any()


def test_blocks_lemma_bounds_and_properness():
    # Lemma 1: proper.  Lemma 2's argument: block V_p never loses, and each
    # lower block settles one round after the block above it, so R <= p and a
    # vertex of block b (0-based) is coloured again at most p - 1 - b times
    for g in list(_random_graphs(300, 14, seed=32)) + [graphgen.er(3000, 30000, 3)]:
        for p in (1, 2, 3, 5, 8, max(1, g.n)):
            col, R, rec = oracle.blocks(g.rowptr, g.colidx, p)
            if g.n == 0:
                continue
            assert oracle.check_proper(g.rowptr, g.colidx, col) == 0
            assert R <= p
            blk = np.arange(g.n) * p // g.n
            assert np.all(rec <= p - 1 - blk)
            assert np.all(col <= np.diff(g.rowptr))


def test_blocks_c_matches_python():
    for g in _random_graphs(1500, 11, seed=33):
        for p in (1, 2, 3, 4, 7, max(1, g.n)):
            col, R, rec = oracle.blocks(g.rowptr, g.colidx, p)
            c2, R2, rec2 = ref_py.blocks(adj(g), p)
            assert list(col) == c2 and R == R2 and list(rec) == rec2


def test_blocks_pins_reject_higher_partition_losing():
    # the opposite tie-break (the higher block recoloured) breaks the star pin
    def flipped(a, p):
        n = len(a)
        block = [v * p // n for v in range(n)]
        fb = {v: {u: -1 for u in a[v]} for v in range(n)}
        col = [-1] * n
        todo, R = set(range(n)), 0
        while todo:
            R += 1
            for v in sorted(todo):
                col[v] = ref_py.mex(fb[v].values())
                for u in a[v]:
                    if block[u] == block[v]:
                        fb[u][v] = col[v]
            again = set()
            for v in todo:
                for u in a[v]:
                    if block[u] != block[v]:
                        fb[v][u] = col[u]
                        if col[u] == col[v] and block[v] > block[u]:
                            again.add(v)
            todo = again
        return col, R
    g = graphgen.star(6, centre=0)
    assert flipped(adj(g), 7) != ([1] + [0] * 6, 2)


# ---------------------------------------------------- orderings (future work) --

def test_splitmix64_published_outputs():
    from oracle import ordering
    # the generator's first outputs from state 0 and from state 1234567, as
    # printed with its published reference implementation
    z = 0
    out = []
    for _ in range(3):
        z = (z + ordering.GOLDEN_GAMMA) & ((1 << 64) - 1)
        out.append(ordering.splitmix64_mix(z))
    assert out[0] == 0xE220A8397B1DCDAF
    assert out[1] == 0x6E789E6AA1B965F4
    assert out[2] == 0x06C45D188009454F
    z = 1234567
    z = (z + ordering.GOLDEN_GAMMA) & ((1 << 64) - 1)
    assert ordering.splitmix64_mix(z) == 6457827717110365317
    # the vectorised keys are the same function
    keys = ordering.random_keys(5, 99)
    assert [int(k) for k in keys] == [
        ordering.splitmix64_mix(99 + (v + 1) * ordering.GOLDEN_GAMMA) for v in range(5)]


def test_largest_first_order():
    from oracle import ordering
    g = graphgen.from_edges(6, [(0, 1), (1, 2), (1, 3), (3, 4), (3, 5), (4, 5)])
    # degrees 1,3,1,3,2,2: the two degree-3 vertices first (by id), then 4, 5, then 0, 2
    assert list(ordering.order(g.rowptr, g.colidx, "largest_first")) == [1, 3, 4, 5, 0, 2]
    for h in _random_graphs(200, 12, seed=41):
        s = ordering.order(h.rowptr, h.colidx, "largest_first")
        d = np.diff(h.rowptr)[s]
        assert sorted(s) == list(range(h.n))
        assert all(d[i] > d[i + 1] or (d[i] == d[i + 1] and s[i] < s[i + 1])
                   for i in range(h.n - 1))


def test_relabel_is_an_isomorphism_with_sorted_rows():
    from oracle import ordering
    for h in list(_random_graphs(100, 12, seed=42)) + [graphgen.er(500, 3000, 5)]:
        for kind in ("largest_first", "random"):
            s = ordering.order(h.rowptr, h.colidx, kind, seed=7)
            rp2, ci2, newid = ordering.relabel(h.rowptr, h.colidx, s)
            assert sorted(s) == list(range(h.n))
            e1 = {(int(newid[v]), int(u2)) for v in range(h.n)
                  for u2 in newid[h.colidx[h.rowptr[v]:h.rowptr[v + 1]]]}
            e2 = {(i, int(u)) for i in range(h.n) for u in ci2[rp2[i]:rp2[i + 1]]}
            assert e1 == e2
            assert all(np.all(np.diff(ci2[rp2[i]:rp2[i + 1]]) > 0) for i in range(h.n))


def test_largest_first_sequential_first_fit_on_a_star():
    # the centre goes first: colour 0, every leaf 1 (natural order with the
    # centre last gives the leaves 0 and the centre 1)
    from oracle import ordering
    g = graphgen.star(5, centre=5)
    col, _ = ordering.colour_in_order(g.rowptr, g.colidx, "largest_first", 0, oracle.seq)
    assert list(col) == [1, 1, 1, 1, 1, 0]
    assert list(oracle.seq(g.rowptr, g.colidx)) == [0, 0, 0, 0, 0, 1]


# ------------------------------------------------------ properties (random) --

def _random_graphs(count, nmax, seed):
    rng = np.random.default_rng(seed)
    for _ in range(count):
        n = int(rng.integers(0, nmax + 1))
        p = float(rng.choice([0.1, 0.3, 0.5, 0.8]))
        yield graphgen.random_small(n, p, rng)


def _check_all_properties(g, r):
    n = g.n
    deg = g.degrees()
    # P1 proper (Section 2.1; Lemma 1)
    assert oracle.check_proper(g.rowptr, g.colidx, r.colors) == 0
    # First Fit: each colour is the least absent from the final neighbourhood
    assert oracle.check_grundy(g.rowptr, g.colidx, r.colors) == 0
    if n == 0:
        assert r.rounds == 0
        return
    # colour <= deg(v), hence at most Delta + 1 colours (Section 2.1)
    assert np.all(r.colors <= deg)
    assert r.num_colors <= g.max_degree() + 1
    # Lemma 2 with p = n: a vertex is recoloured at most (number of higher
    # blocks) times; in the higher-id-loses orientation the lowest id still
    # uncoloured always keeps its colour, so v is final by round v + 1, and
    # the round count is at most n.
    assert np.all(r.round_of >= 1)
    assert np.all(r.round_of <= np.arange(n) + 1)
    assert 1 <= r.rounds <= n
    # each round shrinks the uncoloured set
    sizes = r.trace[:, 0]
    assert sizes[0] == n and np.all(np.diff(sizes) < 0)
    # a colour made final in round r is at most r - 1 (colours seen in round
    # r were made final in rounds < r)
    assert np.all(r.colors <= r.round_of - 1)
    # round 1: nothing is coloured, so every vertex tries 0 and exactly the
    # vertices with no lower neighbour keep it
    for v in range(n):
        row = g.colidx[g.rowptr[v]:g.rowptr[v + 1]]
        assert (r.round_of[v] == 1) == (not np.any(row < v))
    # trace columns recomputed from the per-vertex rounds
    for rr in range(1, r.rounds + 1):
        U = np.nonzero(r.round_of >= rr)[0]
        assert r.trace[rr - 1, 0] == U.size
        assert r.trace[rr - 1, 1] == deg[U].sum()
        lower = sum(int(np.sum(g.colidx[g.rowptr[v]:g.rowptr[v + 1]] < v)) for v in U)
        assert r.trace[rr - 1, 2] == lower


def test_properties_random_small():
    for g in _random_graphs(600, 12, seed=1):
        _check_all_properties(g, run(g))


def test_properties_medium_er():
    g = graphgen.er(3000, 30000, 5)
    _check_all_properties(g, run(g))


def test_properties_medium_rmat_and_stencil():
    for g in (graphgen.rmat(12, 8, 0.57, 0.19, 0.19, 3), graphgen.stencil27(12, 4)):
        r = run(g)
        assert oracle.check_proper(g.rowptr, g.colidx, r.colors) == 0
        assert oracle.check_grundy(g.rowptr, g.colidx, r.colors) == 0
        assert np.all(r.colors <= g.degrees())
        assert np.all(r.round_of <= np.arange(g.n) + 1)


def test_row_order_does_not_matter():
    rng = np.random.default_rng(7)
    for g in list(_random_graphs(100, 12, seed=2)) + [graphgen.er(2000, 20000, 1)]:
        a = run(g)
        b = run(graphgen.shuffle_rows(g, rng))
        assert np.array_equal(a.colors, b.colors) and a.rounds == b.rounds


def test_colour_count_against_chromatic_number():
    # chi <= K <= Delta + 1 for both the round-synchronous and the sequential
    # colourings (the objective of Section 2.1 is chi)
    for g in _random_graphs(400, 10, seed=3):
        if g.n == 0:
            continue
        chi = ref_py.chromatic_number(adj(g))
        k_rsc = run(g).num_colors
        k_seq = int(oracle.seq(g.rowptr, g.colidx).max()) + 1
        assert chi <= k_rsc <= g.max_degree() + 1
        assert chi <= k_seq <= g.max_degree() + 1


def test_brute_force_chromatic_number_itself():
    for n in range(1, 8):
        assert ref_py.chromatic_number(adj(graphgen.complete(n))) == n
    assert ref_py.chromatic_number(adj(graphgen.cycle(7))) == 3
    assert ref_py.chromatic_number(adj(graphgen.cycle(8))) == 2
    # Petersen graph: chi = 3
    outer = [(i, (i + 1) % 5) for i in range(5)]
    spokes = [(i, i + 5) for i in range(5)]
    inner = [(5 + i, 5 + (i + 2) % 5) for i in range(5)]
    assert ref_py.chromatic_number(adj(graphgen.from_edges(10, outer + spokes + inner))) == 3
    for g in _random_graphs(150, 7, seed=4):
        a = adj(g)
        assert ref_py.chromatic_number(a) == ref_py.chromatic_number_exhaustive(a)


# --------------------------------------------- two implementations agree --

def test_c_oracle_matches_python_oracle():
    for g in _random_graphs(3000, 11, seed=5):
        r = run(g)
        scans = []
        col, rounds, round_of = ref_py.rsc(adj(g), scans)
        assert list(r.colors) == col
        assert r.rounds == rounds
        assert list(r.round_of) == round_of
        assert list(r.trace[:, 3]) == scans
        assert list(oracle.seq(g.rowptr, g.colidx)) == ref_py.seq(adj(g))


def test_early_stop_scan_count_bounds():
    # the early-stop count lies between |losers with a lower neighbour| and
    # the full lower-prefix count, and equals the latter in the last round
    for g in list(_random_graphs(200, 12, seed=6)) + [graphgen.er(2000, 20000, 3)]:
        r = run(g)
        if g.n == 0:
            continue
        assert np.all(r.trace[:, 3] <= r.trace[:, 2])
        losers = r.trace[1:, 0] if r.rounds > 1 else np.zeros(0, np.int64)
        assert np.all(r.trace[:-1, 3] >= losers)
        assert r.trace[-1, 3] == r.trace[-1, 2]


# ------------------------------------------------------------ mutants ------
# Each mutant is a plausible misreading or slip in the definition.  The pins
# above are run against it; at least one must fail.

def _mutant_lower_loses(a):
    n = len(a)
    final, waiting, rounds = {}, set(range(n)), 0
    while waiting:
        rounds += 1
        t = {v: ref_py.mex(final[u] for u in a[v] if u in final) for v in waiting}
        losers = {v for v in waiting if any(u in waiting and u > v and t[u] == t[v] for u in a[v])}
        for v in waiting - losers:
            final[v] = t[v]
        waiting = losers
    return [final[v] for v in range(n)], rounds


def _mutant_sequential_visibility(a):
    # colours become visible to later vertices of the same round
    n = len(a)
    final, waiting, rounds = {}, set(range(n)), 0
    while waiting:
        rounds += 1
        t = {}
        for v in sorted(waiting):
            t[v] = ref_py.mex([final[u] for u in a[v] if u in final] +
                              [t[u] for u in a[v] if u in t])
        losers = {v for v in waiting if any(u in waiting and u < v and t[u] == t[v] for u in a[v])}
        for v in waiting - losers:
            final[v] = t[v]
        waiting = losers
    return [final[v] for v in range(n)], rounds


def _mutant_stale_colours(a):
    # a recoloured neighbour still forbids the colour it tried last round
    n = len(a)
    final, last, waiting, rounds = {}, {}, set(range(n)), 0
    while waiting:
        rounds += 1
        t = {v: ref_py.mex([final[u] for u in a[v] if u in final] +
                           [last[u] for u in a[v] if u in last and u not in final])
             for v in waiting}
        losers = {v for v in waiting if any(u in waiting and u < v and t[u] == t[v] for u in a[v])}
        for v in waiting:
            last[v] = t[v]
        for v in waiting - losers:
            final[v] = t[v]
        waiting = losers
    return [final[v] for v in range(n)], rounds


def _mutant_first_fit_from_one(a):
    n = len(a)
    final, waiting, rounds = {}, set(range(n)), 0
    while waiting:
        rounds += 1
        t = {}
        for v in waiting:
            s = {final[u] for u in a[v] if u in final}
            c = 1
            while c in s:
                c += 1
            t[v] = c
        losers = {v for v in waiting if any(u in waiting and u < v and t[u] == t[v] for u in a[v])}
        for v in waiting - losers:
            final[v] = t[v]
        waiting = losers
    return [final[v] for v in range(n)], rounds


def _mutant_no_conflict_check(a):
    n = len(a)
    col = [ref_py.mex([]) for _ in range(n)]
    return col, 1


def _mutant_both_endpoints_lose(a):
    # both ends of a conflicting edge are recoloured (no tie-break); K_2 then
    # never settles, so the loop is capped
    n = len(a)
    final, waiting, rounds = {}, set(range(n)), 0
    while waiting and rounds < 4 * n + 4:
        rounds += 1
        t = {v: ref_py.mex(final[u] for u in a[v] if u in final) for v in waiting}
        losers = {v for v in waiting if any(u in waiting and t[u] == t[v] for u in a[v])}
        for v in waiting - losers:
            final[v] = t[v]
        waiting = losers
    return [final.get(v, -1) for v in range(n)], rounds


def _pins_pass(impl) -> bool:
    """The closed-form and property pins, applied to an implementation
    returning (colours, rounds)."""
    cases = [
        (graphgen.complete(6), list(range(6)), 6),
        (graphgen.path(7), [v % 2 for v in range(7)], 4),
        (graphgen.cycle(5), [0, 1, 0, 2, 1], 3),
        (graphgen.from_edges(6, [(0, 1), (1, 2), (2, 3), (3, 5), (4, 5)]), [0, 1, 0, 2, 0, 1], 3),
        (graphgen.star(4, centre=4), [0, 0, 0, 0, 1], 2),
        (graphgen.crown(4), [i // 2 for i in range(8)], 4),
        (graphgen.empty(3), [0, 0, 0], 1),
    ]
    for g, want, rounds in cases:
        col, R = impl(adj(g))
        if list(col) != want or R != rounds:
            return False
    for g in _random_graphs(200, 10, seed=9):
        col, R = impl(adj(g))
        c = np.asarray(col, np.int32)
        if g.n and (oracle.check_proper(g.rowptr, g.colidx, c) != 0 or
                    oracle.check_grundy(g.rowptr, g.colidx, c) != 0):
            return False
    return True


def test_pins_accept_the_reference_definition():
    assert _pins_pass(lambda a: ref_py.rsc(a)[:2])


@pytest.mark.parametrize("mutant", [
    _mutant_lower_loses, _mutant_sequential_visibility, _mutant_stale_colours,
    _mutant_first_fit_from_one, _mutant_no_conflict_check,
    _mutant_both_endpoints_lose,
])
def test_pins_reject_mutant(mutant):
    assert not _pins_pass(mutant)
