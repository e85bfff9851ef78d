"""Vertex orderings applied before colouring (the paper's future work names
colouring and ordering schemes; its related work cites Jones and Plassmann's
random vertex order).

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle/``.

An ordering is a list sigma of all vertices; vertex sigma[i] gets the new id
i, the graph is relabelled (rows ascending), coloured, and each vertex takes
the colour of its new id.  Orders defined here:

* ``largest_first``: degree descending, ties by id ascending;
* ``random``: ascending by the output of the splitmix64 generator (Steele,
  Lea and Flood, 2014) at step v + 1 from state ``seed``, i.e.
  mix(seed + (v + 1) * 0x9E3779B97F4A7C15) with mix the generator's
  published finaliser; the mix is a bijection, so there are no ties.
"""
from __future__ import annotations

import numpy as np

GOLDEN_GAMMA = 0x9E3779B97F4A7C15
_M64 = (1 << 64) - 1


def splitmix64_mix(z: int) -> int:
    """The splitmix64 output function on one 64-bit state (Python ints)."""
    z &= _M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
    return z ^ (z >> 31)


def random_keys(n: int, seed: int) -> np.ndarray:
    """uint64 key of each vertex for the random order (vectorised)."""
    v = np.arange(n, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & _M64) + (v + np.uint64(1)) * np.uint64(GOLDEN_GAMMA)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return z


def order(rowptr, colidx, kind: str, seed: int = 0) -> np.ndarray:
    """sigma: the vertices in their new order."""
    rp = np.asarray(rowptr, dtype=np.int64)
    n = rp.shape[0] - 1
    ids = np.arange(n, dtype=np.int64)
    if kind == "natural":
        return ids
    if kind == "largest_first":
        deg = np.diff(rp)
        return np.lexsort((ids, -deg))  # last key is primary: -deg, then id
    if kind == "random":
        return np.argsort(random_keys(n, seed), kind="stable").astype(np.int64)
    raise ValueError(kind)


def relabel(rowptr, colidx, sigma):
    """(rowptr', colidx') of the graph with vertex sigma[i] renamed i, rows
    ascending."""
    rp = np.asarray(rowptr, dtype=np.int64)
    ci = np.asarray(colidx, dtype=np.int64)
    n = rp.shape[0] - 1
    newid = np.empty(n, dtype=np.int64)
    newid[sigma] = np.arange(n, dtype=np.int64)
    deg = np.diff(rp)
    src = np.repeat(np.arange(n, dtype=np.int64), deg)
    a, b = newid[src], newid[ci]
    idx = np.lexsort((b, a))
    rp2 = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(a, minlength=n), out=rp2[1:])
    return rp2, b[idx].astype(np.int32), newid


def colour_in_order(rowptr, colidx, kind: str, seed: int, colour_fn):
    """Colour with ``colour_fn(rowptr', colidx')`` on the relabelled graph and
    return each original vertex's colour (and colour_fn's full result)."""
    sigma = order(rowptr, colidx, kind, seed)
    rp2, ci2, newid = relabel(rowptr, colidx, sigma)
    res = colour_fn(rp2, ci2)
    colours = res[0] if isinstance(res, tuple) else res
    return np.asarray(colours)[newid], res
