"""CPU oracle for round-synchronous speculative graph colouring.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg use it; the GPU library never imports it and shares no code
with it.

Two independent implementations of the same definitions live here:

* ``oracle.c`` (loaded through ctypes): ``rsc`` follows Algorithm 1 of
  Section 3.1 with one vertex per block, ``seq`` the sequential First-Fit
  baseline of Section 5, ``seq_rounds`` the rounds in which an id-priority
  schedule reproduces it, ``check_proper`` / ``check_grundy`` the properties
  of Section 2.1 and Lemma 1 (Section 4);
* ``ref_py`` (pure Python, tiny graphs): the same definitions written again
  from the paper, used to cross-check the C code, plus a brute-force
  chromatic number.

Readings of the paper that both implementations take are listed at the top
of ``oracle.c``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_lib = None


def build() -> str:
    """Compile ``liboracle.so`` (plain C, -O2, single-threaded)."""
    cmd = ["gcc", "-O2", "-fPIC", "-shared", "-std=c11", "-Wall", "-o",
           _LIB + ".tmp", _SRC]
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        p = ctypes.c_void_p
        i64 = ctypes.c_int64
        lib.oracle_rsc.restype = i64
        lib.oracle_rsc.argtypes = [i64, p, p, p, p, p, i64]
        lib.oracle_seq.restype = ctypes.c_int
        lib.oracle_seq.argtypes = [i64, p, p, p]
        lib.oracle_seq_rounds.restype = i64
        lib.oracle_seq_rounds.argtypes = [i64, p, p, p]
        lib.oracle_blocks.restype = i64
        lib.oracle_blocks.argtypes = [i64, p, p, i64, p, p]
        lib.oracle_check_proper.restype = i64
        lib.oracle_check_proper.argtypes = [i64, p, p, p]
        lib.oracle_check_grundy.restype = i64
        lib.oracle_check_grundy.argtypes = [i64, p, p, p]
        lib.oracle_rsc_batch.restype = ctypes.c_int
        lib.oracle_rsc_batch.argtypes = [i64, p, p, p, p, p, p]
        _lib = lib
    return _lib


def _csr(rowptr, colidx):
    rp = np.ascontiguousarray(rowptr, dtype=np.int64)
    ci = np.ascontiguousarray(colidx, dtype=np.int32)
    if ci.size == 0:
        ci = np.zeros(1, np.int32)  # keep a valid pointer
    return rp, ci


class RSCResult:
    def __init__(self, colors, rounds, round_of, trace):
        self.colors = colors          # int32[n]
        self.rounds = rounds          # R
        self.round_of = round_of      # int32[n]: round in which v became final
        self.trace = trace            # int64[R, 4]: |U_r|, sum deg, sum deg<, early-stop scan

    @property
    def num_colors(self) -> int:
        return int(self.colors.max()) + 1 if self.colors.size else 0


def rsc(rowptr, colidx, trace_cap: int = 1 << 16) -> RSCResult:
    """Round-synchronous speculative colouring (Algorithm 1, p = n)."""
    rp, ci = _csr(rowptr, colidx)
    n = rp.shape[0] - 1
    colors = np.zeros(max(n, 1), np.int32)
    round_of = np.zeros(max(n, 1), np.int32)
    trace = np.zeros((trace_cap, 4), np.int64)
    R = _load().oracle_rsc(n, rp.ctypes.data, ci.ctypes.data, colors.ctypes.data,
                           round_of.ctypes.data, trace.ctypes.data, trace_cap)
    if R < 0:
        raise ValueError("oracle_rsc rejected its input")
    return RSCResult(colors[:n], int(R), round_of[:n], trace[:min(R, trace_cap)].copy())


def seq(rowptr, colidx) -> np.ndarray:
    """Sequential First Fit in vertex-id order (Section 5 baseline)."""
    rp, ci = _csr(rowptr, colidx)
    n = rp.shape[0] - 1
    colors = np.zeros(max(n, 1), np.int32)
    if _load().oracle_seq(n, rp.ctypes.data, ci.ctypes.data, colors.ctypes.data) != 0:
        raise ValueError("oracle_seq rejected its input")
    return colors[:n]


def seq_rounds(rowptr, colidx):
    """(R, round_of) of the id-priority schedule that reproduces ``seq``:
    round_of[v] = vertices on the longest id-increasing path ending at v."""
    rp, ci = _csr(rowptr, colidx)
    n = rp.shape[0] - 1
    rounds = np.zeros(max(n, 1), np.int32)
    R = _load().oracle_seq_rounds(n, rp.ctypes.data, ci.ctypes.data, rounds.ctypes.data)
    if R < 0:
        raise ValueError("oracle_seq_rounds rejected its input")
    return int(R), rounds[:n]


def blocks(rowptr, colidx, p: int):
    """(colours, R, recolours) of Algorithm 1 with p blocks, read literally."""
    rp, ci = _csr(rowptr, colidx)
    n = rp.shape[0] - 1
    colors = np.zeros(max(n, 1), np.int32)
    rec = np.zeros(max(n, 1), np.int32)
    R = _load().oracle_blocks(n, rp.ctypes.data, ci.ctypes.data, int(p), colors.ctypes.data,
                              rec.ctypes.data)
    if R < 0:
        raise ValueError("oracle_blocks rejected its input")
    return colors[:n], int(R), rec[:n]


def check_proper(rowptr, colidx, colors) -> int:
    """Count of monochromatic CSR entries plus uncoloured vertices (0 = proper)."""
    rp, ci = _csr(rowptr, colidx)
    c = np.ascontiguousarray(colors, dtype=np.int32)
    n = rp.shape[0] - 1
    if c.shape[0] != n:
        raise ValueError("colour vector has the wrong length")
    if n == 0:
        return 0
    return int(_load().oracle_check_proper(n, rp.ctypes.data, ci.ctypes.data, c.ctypes.data))


def check_grundy(rowptr, colidx, colors) -> int:
    """Count of vertices whose colour is not the least absent neighbour colour."""
    rp, ci = _csr(rowptr, colidx)
    c = np.ascontiguousarray(colors, dtype=np.int32)
    n = rp.shape[0] - 1
    if c.shape[0] != n:
        raise ValueError("colour vector has the wrong length")
    if n == 0:
        return 0
    return int(_load().oracle_check_grundy(n, rp.ctypes.data, ci.ctypes.data, c.ctypes.data))


def rsc_batch(voff, eoff, rowptr_local, colidx_local):
    """oracle ``rsc`` applied to every graph of a packed batch."""
    voff = np.ascontiguousarray(voff, dtype=np.int64)
    eoff = np.ascontiguousarray(eoff, dtype=np.int64)
    rpl = np.ascontiguousarray(rowptr_local, dtype=np.int32)
    cil = np.ascontiguousarray(colidx_local, dtype=np.int32)
    if cil.size == 0:
        cil = np.zeros(1, np.int32)
    G = voff.shape[0] - 1
    colors = np.zeros(max(int(voff[-1]), 1), np.int32)
    rounds = np.zeros(max(G, 1), np.int64)
    rc = _load().oracle_rsc_batch(G, voff.ctypes.data, eoff.ctypes.data, rpl.ctypes.data,
                                  cil.ctypes.data, colors.ctypes.data, rounds.ctypes.data)
    if rc != 0:
        raise ValueError("oracle_rsc_batch failed")
    return colors[: int(voff[-1])], rounds[:G]
