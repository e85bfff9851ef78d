"""Seeded synthetic inputs: graphs in CSR form and request arrival times.

This package constructs inputs only and holds no colouring arithmetic; the
CPU oracle (``oracle``) and the GPU library both take their inputs from it.
The large generators are C (``graphgen.c``, one splitmix64 stream per seed and
stream number); the tiny named graphs used by the hand-checked cases are
plain Python.

Every graph is simple and undirected, as the problem statement requires
(paper, Section 2.1): symmetric CSR, no self-loops, no duplicate entries,
ascending rows.  ``rowptr`` is int64 and ``colidx`` int32 as numpy arrays.
"""
from __future__ import annotations

import ctypes
import hashlib
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "graphgen.c")
_LIB = os.path.join(_HERE, "libgraphgen.so")


def build() -> str:
    """Compile ``libgraphgen.so`` with gcc (OpenMP for the big generators)."""
    cmd = ["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-std=c11", "-Wall",
           "-o", _LIB + ".tmp", _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class _Graph(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("rowptr", ctypes.POINTER(ctypes.c_int64)),
                ("colidx", ctypes.POINTER(ctypes.c_int32))]


class _Batch(ctypes.Structure):
    _fields_ = [("num_graphs", ctypes.c_int64),
                ("voff", ctypes.POINTER(ctypes.c_int64)),
                ("eoff", ctypes.POINTER(ctypes.c_int64)),
                ("rowptr_local", ctypes.POINTER(ctypes.c_int32)),
                ("colidx_local", ctypes.POINTER(ctypes.c_int32))]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        i64, u64, dbl = ctypes.c_int64, ctypes.c_uint64, ctypes.c_double
        lib.gg_er.restype = ctypes.POINTER(_Graph)
        lib.gg_er.argtypes = [i64, i64, u64]
        lib.gg_rmat.restype = ctypes.POINTER(_Graph)
        lib.gg_rmat.argtypes = [ctypes.c_int, i64, dbl, dbl, dbl, u64]
        lib.gg_stencil27.restype = ctypes.POINTER(_Graph)
        lib.gg_stencil27.argtypes = [i64, u64]
        lib.gg_free.argtypes = [ctypes.POINTER(_Graph)]
        lib.gg_er_batch.restype = ctypes.POINTER(_Batch)
        lib.gg_er_batch.argtypes = [i64, u64, i64, i64, dbl, dbl]
        lib.gg_batch_free.argtypes = [ctypes.POINTER(_Batch)]
        lib.gg_batch_sizes.restype = ctypes.c_int
        lib.gg_batch_sizes.argtypes = [i64, u64, i64, i64, dbl, dbl,
                                       ctypes.c_void_p, ctypes.c_void_p]
        lib.gg_poisson_arrivals.restype = ctypes.c_int
        lib.gg_poisson_arrivals.argtypes = [i64, dbl, u64, ctypes.c_void_p]
        lib.gg_stream.argtypes = [u64, u64, i64, ctypes.c_void_p]
        _lib = lib
    return _lib


@dataclass
class CSR:
    """A simple undirected graph in CSR form (int64 rowptr, int32 colidx)."""
    rowptr: np.ndarray
    colidx: np.ndarray

    @property
    def n(self) -> int:
        return int(self.rowptr.shape[0] - 1)

    @property
    def nnz(self) -> int:
        return int(self.colidx.shape[0])

    @property
    def m(self) -> int:
        """Undirected edges (each counted once)."""
        return self.nnz // 2

    def degrees(self) -> np.ndarray:
        return np.diff(self.rowptr)

    def max_degree(self) -> int:
        return int(self.degrees().max()) if self.n else 0

    def sha256(self) -> str:
        h = hashlib.sha256()
        h.update(np.int64(self.n).tobytes())
        h.update(np.ascontiguousarray(self.rowptr, dtype=np.int64).tobytes())
        h.update(np.ascontiguousarray(self.colidx, dtype=np.int32).tobytes())
        return h.hexdigest()


@dataclass
class Batch:
    """Independent graphs packed with per-graph offsets and local ids."""
    voff: np.ndarray          # int64[G+1]
    eoff: np.ndarray          # int64[G+1]
    rowptr_local: np.ndarray  # int32[sum(n_g+1)], graph g at voff[g] + g
    colidx_local: np.ndarray  # int32[sum(nnz_g)], graph g at eoff[g]

    @property
    def num_graphs(self) -> int:
        return int(self.voff.shape[0] - 1)

    def graph(self, g: int) -> CSR:
        n = int(self.voff[g + 1] - self.voff[g])
        r0 = int(self.voff[g] + g)
        rp = self.rowptr_local[r0:r0 + n + 1].astype(np.int64)
        ci = self.colidx_local[int(self.eoff[g]):int(self.eoff[g + 1])]
        return CSR(rp, ci)

    def sha256(self) -> str:
        h = hashlib.sha256()
        for a in (self.voff, self.eoff, self.rowptr_local, self.colidx_local):
            h.update(np.ascontiguousarray(a).tobytes())
        return h.hexdigest()


def _take_graph(ptr) -> CSR:
    if not ptr:
        raise ValueError("graph generator rejected its parameters or ran out of memory")
    g = ptr.contents
    n, nnz = int(g.n), int(g.nnz)
    rp = np.ctypeslib.as_array(g.rowptr, shape=(n + 1,)).copy()
    ci = (np.ctypeslib.as_array(g.colidx, shape=(nnz,)).copy() if nnz
          else np.zeros(0, np.int32))
    _load().gg_free(ptr)
    return CSR(rp, ci)


def er(n: int, m: int, seed: int = 0) -> CSR:
    """Erdos-Renyi G(n, m): uniform endpoint pairs, loops and repeats
    dropped, drawn until exactly m distinct edges exist."""
    return _take_graph(_load().gg_er(n, m, seed))


def rmat(scale: int, edge_factor: int = 16, a: float = 0.57, b: float = 0.19,
         c: float = 0.19, seed: int = 0) -> CSR:
    """R-MAT with 2**scale vertices and edge_factor * 2**scale samples,
    symmetrised, loops and duplicates dropped, ids not permuted."""
    return _take_graph(_load().gg_rmat(scale, edge_factor, a, b, c, seed))


def stencil27(L: int, seed: int = 0) -> CSR:
    """27-point stencil on an L^3 grid, vertex ids a seeded permutation."""
    return _take_graph(_load().gg_stencil27(L, seed))


def er_batch_sizes(G: int, seed: int = 0, nmin: int = 100, nmax: int = 50_000,
                   dmin: float = 4.0, dmax: float = 64.0):
    """(n_g, m_g) of each graph of ``er_batch`` without generating edges."""
    ns = np.zeros(G, np.int64)
    ms = np.zeros(G, np.int64)
    rc = _load().gg_batch_sizes(G, seed, nmin, nmax, dmin, dmax,
                                ns.ctypes.data, ms.ctypes.data)
    if rc != 0:
        raise ValueError("bad batch parameters")
    return ns, ms


def er_batch(G: int, seed: int = 0, nmin: int = 100, nmax: int = 50_000,
             dmin: float = 4.0, dmax: float = 64.0) -> Batch:
    """G independent ER graphs: n_g log-uniform in [nmin, nmax], average
    degree uniform in [dmin, dmax]."""
    p = _load().gg_er_batch(G, seed, nmin, nmax, dmin, dmax)
    if not p:
        raise ValueError("batch generator rejected its parameters or ran out of memory")
    b = p.contents
    G = int(b.num_graphs)
    voff = np.ctypeslib.as_array(b.voff, shape=(G + 1,)).copy()
    eoff = np.ctypeslib.as_array(b.eoff, shape=(G + 1,)).copy()
    nv, ne = int(voff[G]), int(eoff[G])
    rpl = np.ctypeslib.as_array(b.rowptr_local, shape=(nv + G + 1,))[: nv + G].copy()
    cil = (np.ctypeslib.as_array(b.colidx_local, shape=(ne,)).copy() if ne
           else np.zeros(0, np.int32))
    _load().gg_batch_free(p)
    return Batch(voff, eoff, rpl, cil)


def poisson_arrivals(count: int, rate: float, seed: int = 1) -> np.ndarray:
    """Arrival times (seconds) of a Poisson stream of the given rate."""
    out = np.zeros(count, np.float64)
    if _load().gg_poisson_arrivals(count, rate, seed, out.ctypes.data) != 0:
        raise ValueError("bad arrival parameters")
    return out


def raw_stream(seed: int, stream: int, count: int) -> np.ndarray:
    out = np.zeros(count, np.uint64)
    _load().gg_stream(seed, stream, count, out.ctypes.data)
    return out


# --------------------------------------------------------- tiny graphs --

def from_edges(n: int, edges) -> CSR:
    """CSR of the simple graph on vertices 0..n-1 with the given edges."""
    adj = [set() for _ in range(n)]
    for a, b in edges:
        a, b = int(a), int(b)
        if not (0 <= a < n and 0 <= b < n):
            raise ValueError(f"edge ({a},{b}) out of range")
        if a == b:
            raise ValueError("self-loop in a simple graph")
        adj[a].add(b)
        adj[b].add(a)
    rp = np.zeros(n + 1, np.int64)
    cols = []
    for v in range(n):
        row = sorted(adj[v])
        cols.extend(row)
        rp[v + 1] = rp[v] + len(row)
    return CSR(rp, np.asarray(cols, dtype=np.int32))


def complete(n: int) -> CSR:
    return from_edges(n, [(i, j) for i in range(n) for j in range(i + 1, n)])


def path(n: int) -> CSR:
    return from_edges(n, [(i, i + 1) for i in range(n - 1)])


def cycle(n: int) -> CSR:
    return from_edges(n, [(i, (i + 1) % n) for i in range(n)])


def star(leaves: int, centre: int = 0) -> CSR:
    n = leaves + 1
    return from_edges(n, [(centre, v) for v in range(n) if v != centre])


def crown(k: int) -> CSR:
    """K_{k,k} minus a perfect matching, a_i = 2i, b_j = 2j + 1."""
    return from_edges(2 * k, [(2 * i, 2 * j + 1) for i in range(k) for j in range(k) if i != j])


def empty(n: int) -> CSR:
    return from_edges(n, [])


def hub_over_losers(k: int) -> CSR:
    """k paths x1_i - x2_i - c_i - b_i (ids x1 in [0, k), x2 in [k, 2k), c in
    [2k, 3k), b in [3k, 4k)), every b_i joined to a hub v = 4k + 1, and v
    joined to w = 4k.  The hub is the only vertex of high degree, and it
    commits (round 2) while all k of its lower neighbours b_i are still
    uncoloured."""
    edges = []
    for i in range(k):
        x1, x2, c, b = i, k + i, 2 * k + i, 3 * k + i
        edges += [(x1, x2), (x2, c), (c, b), (b, 4 * k + 1)]
    edges.append((4 * k, 4 * k + 1))
    return from_edges(4 * k + 2, edges)


def random_small(n: int, p: float, rng: np.random.Generator) -> CSR:
    """Tiny G(n, p) for randomized property tests (numpy Generator)."""
    edges = [(i, j) for i in range(n) for j in range(i + 1, n) if rng.random() < p]
    return from_edges(n, edges)


def shuffle_rows(g: CSR, rng: np.random.Generator) -> CSR:
    """Same graph with each row's entries permuted (unsorted rows)."""
    ci = g.colidx.copy()
    for v in range(g.n):
        s, e = int(g.rowptr[v]), int(g.rowptr[v + 1])
        ci[s:e] = rng.permutation(ci[s:e])
    return CSR(g.rowptr.copy(), ci)


def relabel(g: CSR, perm: np.ndarray) -> CSR:
    """Graph with vertex v renamed perm[v]."""
    n = g.n
    edges = []
    for v in range(n):
        for u in g.colidx[g.rowptr[v]:g.rowptr[v + 1]]:
            if v < u:
                edges.append((int(perm[v]), int(perm[u])))
    return from_edges(n, edges)


# ------------------------------------------------------- named workloads --

WORKLOADS = {
    "er_10k_100k": "Erdos-Renyi G(n=10,000, m=100,000), seed 0",
    "er_1m_16m": "Erdos-Renyi G(n=1,048,576, m=16,777,216), seed 0",
    "rmat22_ef16": "R-MAT scale 22, edge factor 16, (a,b,c,d)=(.57,.19,.19,.05), seed 0",
    "stencil27_160": "27-point stencil on a 160^3 grid, ids permuted with seed 0",
    "er_batch_4096": "4,096 ER graphs, n log-uniform in [100, 50,000], avg degree U[4, 64], seed 0",
}


def workload(name: str):
    """The named full-size inputs (CSR, or Batch for the batched workload)."""
    if name == "er_10k_100k":
        return er(10_000, 100_000, 0)
    if name == "er_1m_16m":
        return er(1 << 20, 1 << 24, 0)
    if name == "rmat22_ef16":
        return rmat(22, 16, 0.57, 0.19, 0.19, 0)
    if name == "stencil27_160":
        return stencil27(160, 0)
    if name == "er_batch_4096":
        return er_batch(4096, 0, 100, 50_000, 4.0, 64.0)
    raise KeyError(name)
