"""Second, independent oracle in pure Python, for tiny graphs only.

TEST INFRASTRUCTURE ONLY.  Written separately from ``oracle.c`` from the same
passages, so that a slip in one is caught by the other:

* ``rsc`` -- Algorithm 1 (Section 3.1) with one vertex per block: each round
  every uncoloured vertex takes the least colour absent from its coloured
  neighbours (First Fit, Section 3); then of each pair of adjacent vertices
  that took the same colour this round the higher id is recoloured; repeat.
  Neighbours still waiting for a colour forbid nothing.
* ``seq`` -- sequential First Fit in id order (Section 5 baseline).
* ``seq_schedule`` -- the same colours by rounds: a vertex is coloured once
  its lower neighbours are; ``longest_increasing_path`` gives its round by
  enumeration.
* ``blocks`` -- Algorithm 1 read literally with p blocks of consecutive ids
  (per-edge forbidden slots, the lower-numbered block recoloured).
* ``chromatic_number`` -- brute force over all colourings, for n <= 10,
  the quantity the paper's objective minimises (Section 2.1).

Graphs are adjacency lists: ``adj[v]`` is an iterable of neighbours.
"""
from __future__ import annotations

import itertools


def adjacency(rowptr, colidx):
    n = len(rowptr) - 1
    return [[int(u) for u in colidx[int(rowptr[v]):int(rowptr[v + 1])]] for v in range(n)]


def mex(values) -> int:
    s = set(values)
    c = 0
    while c in s:
        c += 1
    return c


def rsc(adj, scan_counts=None):
    """Returns (colours, rounds, round_of).  If scan_counts is a list, the
    number of lower neighbours a row-order scan examines up to and including
    the first conflicting one (all of them without a conflict), summed over
    the round's vertices, is appended per round."""
    n = len(adj)
    final = {}            # v -> colour, once final
    round_of = [0] * n
    waiting = set(range(n))
    rounds = 0
    while waiting:
        rounds += 1
        trial = {v: mex(final[u] for u in adj[v] if u in final) for v in waiting}
        losers = {v for v in waiting
                  if any(u in waiting and u < v and trial[u] == trial[v] for u in adj[v])}
        if scan_counts is not None:
            total = 0
            for v in waiting:
                for u in adj[v]:
                    if u < v:
                        total += 1
                        if u in waiting and trial[u] == trial[v]:
                            break
            scan_counts.append(total)
        for v in waiting - losers:
            final[v] = trial[v]
            round_of[v] = rounds
        waiting = losers
    return [final[v] for v in range(n)], rounds, round_of


def seq(adj):
    n = len(adj)
    col = [None] * n
    for v in range(n):
        col[v] = mex(col[u] for u in adj[v] if u < v)
    return col


def longest_increasing_path(adj):
    """Per vertex v, the most vertices on a path whose ids increase and end
    at v, by exhaustive depth-first enumeration of such paths (tiny graphs)."""
    n = len(adj)
    best = [1] * n

    def walk(v, length):
        if length > best[v]:
            best[v] = length
        for u in adj[v]:
            if u > v:
                walk(u, length + 1)

    for v in range(n):
        walk(v, 1)
    return best


def seq_schedule(adj):
    """The id-priority schedule run round by round: in each round every
    uncoloured vertex whose lower neighbours are all coloured (at the round's
    start) takes the least colour absent among them.  Returns (colours,
    rounds, round_of)."""
    n = len(adj)
    col = [None] * n
    round_of = [0] * n
    waiting = set(range(n))
    r = 0
    while waiting:
        r += 1
        ready = [v for v in waiting if all(col[u] is not None for u in adj[v] if u < v)]
        picks = {v: mex(col[u] for u in adj[v] if u < v) for v in ready}
        for v, c in picks.items():
            col[v] = c
            round_of[v] = r
        waiting -= set(ready)
    return col, r, round_of


def blocks(adj, p):
    """Algorithm 1 with p blocks, from the pseudo-code: per-edge forbidden
    slots, phase 1 sequential inside each block (increasing id), phase 2
    refreshing the slots of foreign neighbours and recolouring the vertex of
    the lower-numbered block.  Returns (colours, rounds, recolours)."""
    n = len(adj)
    if n == 0:
        return [], 0, []
    block = [v * p // n for v in range(n)]
    forbidden = {v: {u: -1 for u in adj[v]} for v in range(n)}
    colour = [-1] * n
    recol = [0] * n
    todo = set(range(n))
    rounds = 0
    while todo:
        rounds += 1
        for b in sorted(set(block[v] for v in todo)):
            for v in sorted(x for x in todo if block[x] == b):
                c = mex(forbidden[v].values())
                if colour[v] >= 0:
                    recol[v] += 1
                colour[v] = c
                for u in adj[v]:
                    if block[u] == b:
                        forbidden[u][v] = c
        again = set()
        for v in todo:
            for u in adj[v]:
                if block[u] != block[v]:
                    forbidden[v][u] = colour[u]
                    if colour[u] == colour[v] and block[v] < block[u]:
                        again.add(v)
        todo = again
    return colour, rounds, recol


def is_proper(adj, col) -> bool:
    return all(col[v] != col[u] for v in range(len(adj)) for u in adj[v])


def chromatic_number(adj) -> int:
    """Smallest k admitting a proper colouring, by exhaustive search.

    Every assignment of k colours is enumerated by depth-first search over
    vertices 0..n-1, cutting a branch as soon as an edge is monochromatic and
    naming colours in order of first use (a relabelling of colour classes
    never changes properness)."""
    n = len(adj)
    if n == 0:
        return 0
    if n > 10:
        raise ValueError("brute force is for n <= 10")
    col = [-1] * n

    def extend(v, k, used):
        if v == n:
            return True
        for c in range(min(used + 1, k)):
            if all(col[u] != c for u in adj[v] if u < v):
                col[v] = c
                if extend(v + 1, k, max(used, c + 1)):
                    return True
                col[v] = -1
        return False

    for k in range(1, n + 1):
        if extend(0, k, 0):
            return k
    return n


def chromatic_number_exhaustive(adj) -> int:
    """The same quantity by plain enumeration of all k^n assignments (n <= 7),
    to check the pruned search above."""
    n = len(adj)
    if n == 0:
        return 0
    if n > 7:
        raise ValueError("plain enumeration is for n <= 7")
    edges = [(v, u) for v in range(n) for u in adj[v] if v < u]
    for k in range(1, n + 1):
        for col in itertools.product(range(k), repeat=n):
            if all(col[a] != col[b] for a, b in edges):
                return k
    return n
