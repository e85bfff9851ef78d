"""Thin ctypes binding of libgc (include/gc.h).

Argument marshalling only: every step of the colouring runs in the HIP
kernels of ``libgc.so``.  Torch provides device memory and streams.  The
library is never replaced by a host fallback: if ``libgc.so`` is missing or
fails to load, the calls raise.

``torch`` is imported before the library is loaded so that libgc binds to
the HIP runtime torch has already loaded (both carry the same soname).
"""
from __future__ import annotations

import contextlib
import ctypes
import os

import numpy as np
import torch  # noqa: F401  (loads the HIP runtime libgc binds to)

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgc.so")

# enum gc_status
GC_OK, GC_EINVAL, GC_ENOMEM, GC_EDEVICE, GC_EROUNDS, GC_EBUSY, GC_ETOOBIG = 0, -1, -2, -3, -4, -5, -6
STATUS_NAMES = {0: "GC_OK", -1: "GC_EINVAL", -2: "GC_ENOMEM", -3: "GC_EDEVICE",
                -4: "GC_EROUNDS", -5: "GC_EBUSY", -6: "GC_ETOOBIG"}
# enum gc_flags
GC_ROWPTR_I64, GC_VALIDATE, GC_ROWS_SORTED = 1, 2, 4
# enum gc_option
(GC_OPT_MODE, GC_OPT_LANES, GC_OPT_HEAVY_DEGREE, GC_OPT_BLOCKS_PER_CU, GC_OPT_MAX_ROUNDS,
 GC_OPT_CHUNK_ROUNDS, GC_OPT_MEDIUM_DEGREE, GC_OPT_MAX_DEGREE, GC_OPT_MEDIUM_COUNT,
 GC_OPT_HEAVY_COUNT, GC_OPT_PERSISTENT_BLOCKS_PER_CU, GC_OPT_STATE_BYTES,
 GC_OPT_PROFILE, GC_OPT_ALGORITHM, GC_OPT_PARTITIONS, GC_OPT_ORDER,
 GC_OPT_ORDER_SEED) = range(1, 18)
GC_ORDER_NATURAL, GC_ORDER_LARGEST_FIRST, GC_ORDER_RANDOM = range(3)
ORDERS = {"natural": GC_ORDER_NATURAL, "largest_first": GC_ORDER_LARGEST_FIRST,
          "random": GC_ORDER_RANDOM}
GC_ALGO_AUTO, GC_ALGO_PULL, GC_ALGO_PUSH, GC_ALGO_SEQ, GC_ALGO_BLOCKS = range(5)
ALGORITHMS = {"auto": GC_ALGO_AUTO, "pull": GC_ALGO_PULL, "push": GC_ALGO_PUSH,
              "seq": GC_ALGO_SEQ, "blocks": GC_ALGO_BLOCKS}
PROFILE_KINDS = ("round1", "speculate", "detect", "finish")
# enum gc_mode
GC_MODE_AUTO, GC_MODE_HOST, GC_MODE_CHUNKED, GC_MODE_PERSISTENT, GC_MODE_GRAPH = range(5)
MODES = {"auto": GC_MODE_AUTO, "host": GC_MODE_HOST, "chunked": GC_MODE_CHUNKED,
         "persistent": GC_MODE_PERSISTENT, "graph": GC_MODE_GRAPH}
GC_TRACE_ROUNDS = 65536

# Every symbol the header declares, for the load check.
EXPORTS = ["gc_create", "gc_color", "gc_get_stats", "gc_get_round_sizes", "gc_set_option",
           "gc_get_option", "gc_get_profile", "gc_destroy", "gc_last_error",
           "gc_batch_workspace_bytes",
           "gc_color_batch", "gc_batch_step_workspace_bytes", "gc_batch_step", "gc_copy_segments",
           "gc_version", "gc_color_batch_noalloc"]


class GCError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


class gc_graph_desc(ctypes.Structure):
    _fields_ = [("rowptr_off", ctypes.c_int64), ("colidx_off", ctypes.c_int64),
                ("color_off", ctypes.c_int64), ("n", ctypes.c_int32),
                ("rounds", ctypes.c_int32), ("active", ctypes.c_int32),
                ("max_degree", ctypes.c_int32)]


_lib = None


def load():
    """Load libgc.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_1509_08267_amd.build` (hipcc, gfx950)")
    lib = ctypes.CDLL(LIB_PATH)
    p, i64, i32, u32, sz = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_uint32, ctypes.c_size_t
    lib.gc_create.argtypes = [ctypes.POINTER(p), p, p, i64, i64, u32, p]
    lib.gc_color.argtypes = [p, p, p]
    lib.gc_get_stats.argtypes = [p, ctypes.POINTER(i64), ctypes.POINTER(i32)]
    lib.gc_get_round_sizes.argtypes = [p, p, i64, ctypes.POINTER(i64)]
    lib.gc_set_option.argtypes = [p, ctypes.c_int, i64]
    lib.gc_get_option.argtypes = [p, ctypes.c_int, ctypes.POINTER(i64)]
    lib.gc_get_profile.argtypes = [p, p, p, ctypes.c_int]
    lib.gc_destroy.argtypes = [p]
    lib.gc_last_error.argtypes = [p]
    lib.gc_last_error.restype = ctypes.c_char_p
    lib.gc_batch_workspace_bytes.argtypes = [i64, p, p]
    lib.gc_batch_workspace_bytes.restype = sz
    lib.gc_color_batch.argtypes = [i64, p, p, p, p, p, p, p, sz, p]
    lib.gc_color_batch_noalloc.argtypes = [i64, p, p, p, p, p, p, p]
    lib.gc_batch_step_workspace_bytes.argtypes = [i64, i64]
    lib.gc_batch_step_workspace_bytes.restype = sz
    lib.gc_batch_step.argtypes = [i64, p, p, p, p, i32, p, sz, p]
    lib.gc_copy_segments.argtypes = [i64, p, i64, p]
    lib.gc_version.restype = ctypes.c_char_p
    for name in ("gc_create", "gc_color", "gc_get_stats", "gc_get_round_sizes", "gc_set_option",
                 "gc_get_option", "gc_get_profile", "gc_destroy", "gc_color_batch", "gc_batch_step",
                 "gc_color_batch_noalloc"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _check(rc: int, h=None):
    if rc != GC_OK:
        msg = load().gc_last_error(h).decode(errors="replace")
        raise GCError(rc, msg)
    return rc


def _ptr(t) -> int:
    if t is None:
        return 0
    if isinstance(t, int):
        return t
    return t.data_ptr()


def _stream(stream) -> int:
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


# ----------------------------------------------------- C-ABI, same names --

def gc_create(rowptr, colidx, n: int, m: int, flags: int, stream=None) -> int:
    h = ctypes.c_void_p()
    _check(load().gc_create(ctypes.byref(h), _ptr(rowptr), _ptr(colidx), n, m, flags,
                            _stream(stream)))
    return h.value


def gc_color(h: int, colors_out, stream=None) -> None:
    _check(load().gc_color(h, _ptr(colors_out), _stream(stream)), h)


def gc_get_stats(h: int):
    r = ctypes.c_int64()
    k = ctypes.c_int32()
    _check(load().gc_get_stats(h, ctypes.byref(r), ctypes.byref(k)), h)
    return int(r.value), int(k.value)


def gc_get_round_sizes(h: int, cap: int = GC_TRACE_ROUNDS):
    import numpy as np
    out = np.zeros(max(cap, 1), np.int64)
    r = ctypes.c_int64()
    _check(load().gc_get_round_sizes(h, out.ctypes.data, cap, ctypes.byref(r)), h)
    return out[: min(int(r.value), cap)]


def gc_set_option(h: int, option: int, value: int) -> None:
    _check(load().gc_set_option(h, option, int(value)), h)


def gc_get_option(h: int, option: int) -> int:
    v = ctypes.c_int64()
    _check(load().gc_get_option(h, option, ctypes.byref(v)), h)
    return int(v.value)


def gc_get_profile(h: int, reset: bool = False):
    """{kind: (total_ms, launches)} for round1, speculate, detect, finish."""
    import numpy as np
    ms = np.zeros(4, np.float64)
    n = np.zeros(4, np.int64)
    _check(load().gc_get_profile(h, ms.ctypes.data, n.ctypes.data, int(reset)), h)
    return {k: (float(ms[i]), int(n[i])) for i, k in enumerate(PROFILE_KINDS)}


def gc_destroy(h: int) -> None:
    _check(load().gc_destroy(h))


def gc_last_error(h: int = 0) -> str:
    return load().gc_last_error(h).decode(errors="replace")


def gc_version() -> str:
    return load().gc_version().decode()


def gc_batch_workspace_bytes(num_graphs: int, voff_host, eoff_host) -> int:
    import numpy as np
    v = np.ascontiguousarray(voff_host, dtype=np.int64)
    e = np.ascontiguousarray(eoff_host, dtype=np.int64)
    return int(load().gc_batch_workspace_bytes(num_graphs, v.ctypes.data, e.ctypes.data))


def gc_color_batch(num_graphs, voff, eoff, rowptr_local, colidx_local, colors_out, rounds_out,
                   workspace, workspace_bytes, stream=None) -> None:
    _check(load().gc_color_batch(num_graphs, _ptr(voff), _ptr(eoff), _ptr(rowptr_local),
                                 _ptr(colidx_local), _ptr(colors_out), _ptr(rounds_out),
                                 _ptr(workspace), workspace_bytes, _stream(stream)))


GC_STATIC_BATCH_MAX_GRAPHS = 65536


def gc_color_batch_noalloc(num_graphs, voff, eoff, rowptr_local, colidx_local, colors_out,
                           rounds_out, stream=None) -> None:
    _check(load().gc_color_batch_noalloc(num_graphs, _ptr(voff), _ptr(eoff), _ptr(rowptr_local),
                                         _ptr(colidx_local), _ptr(colors_out), _ptr(rounds_out),
                                         _stream(stream)))


def gc_batch_step_workspace_bytes(num_graphs: int, total_vertices: int) -> int:
    return int(load().gc_batch_step_workspace_bytes(num_graphs, total_vertices))


def gc_batch_step(num_graphs, descs, rowptr_base, colidx_base, colors_base, max_rounds,
                  workspace, workspace_bytes, stream=None) -> None:
    _check(load().gc_batch_step(num_graphs, _ptr(descs), _ptr(rowptr_base), _ptr(colidx_base),
                                _ptr(colors_base), max_rounds, _ptr(workspace), workspace_bytes,
                                _stream(stream)))


COPY_PIECE_WORDS = 4096  # GC_COPY_PIECE_WORDS


def gc_copy_segments(count: int, segs, pieces: int, stream=None) -> None:
    _check(load().gc_copy_segments(count, _ptr(segs), pieces, _stream(stream)))


# ------------------------------------------------------ convenience ------

def copy_segments_raw(src_ptrs, dst_ptrs, words, device, stream=None, host_buf=None,
                      dev_buf=None):
    """Copy segment i (words[i] int32 words from device address src_ptrs[i]
    to dst_ptrs[i]) with one gc_copy_segments launch on `stream`; the
    addresses are trusted (numpy int64 arrays).  `host_buf` (optional) is a
    pinned int64 tensor of at least 4 entries per segment that stages the
    descriptors instead of a new pinned allocation; the caller must not
    rewrite it before the stream has run the copy.  `dev_buf` (optional) is
    the same for the device copy of the descriptors (a buffer used only on
    `stream` can be reused by every call).  Returns the descriptor tensors,
    which must stay alive until the stream has run the copy."""
    words = np.asarray(words, dtype=np.int64)
    keep = words > 0
    if not keep.any():
        return None
    src = np.asarray(src_ptrs, dtype=np.int64)[keep]
    dst = np.asarray(dst_ptrs, dtype=np.int64)[keep]
    words = words[keep]
    per = (words + COPY_PIECE_WORDS - 1) // COPY_PIECE_WORDS
    first = np.zeros_like(per)
    np.cumsum(per[:-1], out=first[1:])
    desc = np.stack([src, dst, words, first], axis=1)
    if host_buf is not None and host_buf.numel() >= desc.size:
        h_desc = host_buf[:desc.size].view(-1, 4)
        h_desc.numpy()[:] = desc
    else:
        h_desc = torch.from_numpy(np.ascontiguousarray(desc)).pin_memory()
    with torch.cuda.stream(stream) if stream is not None else contextlib.nullcontext():
        if dev_buf is not None and dev_buf.numel() >= desc.size:
            d_desc = dev_buf[:desc.size].view(-1, 4)
            d_desc.copy_(h_desc, non_blocking=True)
        else:
            d_desc = h_desc.to(device, non_blocking=True)
        gc_copy_segments(int(words.size), d_desc, int(per.sum()), stream)
    return h_desc, d_desc


def copy_segments(pairs, stream=None):
    """Copy each (src, dst) pair of int32 device tensors (src.numel() words
    into the start of dst) with one gc_copy_segments launch on `stream`.
    Returns the descriptor tensors (pinned host copy, device copy), which
    must stay alive until the stream has run the copy."""
    pairs = [(s, d) for s, d in pairs if s.numel() > 0]
    if not pairs:
        return None
    for s, d in pairs:
        if s.dtype != torch.int32 or d.dtype != torch.int32 or not s.is_cuda or not d.is_cuda:
            raise ValueError("copy_segments takes int32 device tensors")
        if d.numel() < s.numel() or not s.is_contiguous() or not d.is_contiguous():
            raise ValueError("copy_segments: destination too small or not contiguous")
    return copy_segments_raw([s.data_ptr() for s, _ in pairs], [d.data_ptr() for _, d in pairs],
                             [s.numel() for s, _ in pairs], pairs[0][1].device, stream)


class Graph:
    """A graph bound on the GPU (gc_create) that can be coloured repeatedly.

    rowptr: int32 or int64 CUDA tensor of n + 1 entries; colidx: int32 CUDA
    tensor.  The tensors are kept referenced for the handle's lifetime (the
    library borrows them)."""

    def __init__(self, rowptr: torch.Tensor, colidx: torch.Tensor, *, validate: bool = False,
                 rows_sorted: bool = True, stream=None, **options):
        if not (rowptr.is_cuda and colidx.is_cuda):
            raise ValueError("rowptr and colidx must be device tensors")
        if rowptr.dtype not in (torch.int32, torch.int64) or colidx.dtype != torch.int32:
            raise ValueError("rowptr must be int32/int64 and colidx int32")
        self.rowptr = rowptr.contiguous()
        self.colidx = colidx.contiguous()
        self.n = int(rowptr.numel()) - 1
        self.m = int(colidx.numel())
        flags = (GC_ROWPTR_I64 if rowptr.dtype == torch.int64 else 0)
        flags |= GC_VALIDATE if validate else 0
        flags |= GC_ROWS_SORTED if rows_sorted else 0
        self.h = gc_create(self.rowptr, self.colidx, self.n, self.m, flags, stream)
        for k, v in options.items():
            self.set(k, v)

    _OPTS = {"mode": GC_OPT_MODE, "lanes": GC_OPT_LANES, "heavy_degree": GC_OPT_HEAVY_DEGREE,
             "blocks_per_cu": GC_OPT_BLOCKS_PER_CU, "max_rounds": GC_OPT_MAX_ROUNDS,
             "chunk_rounds": GC_OPT_CHUNK_ROUNDS, "medium_degree": GC_OPT_MEDIUM_DEGREE,
             "persistent_blocks_per_cu": GC_OPT_PERSISTENT_BLOCKS_PER_CU,
             "profile": GC_OPT_PROFILE, "algorithm": GC_OPT_ALGORITHM,
             "partitions": GC_OPT_PARTITIONS, "order": GC_OPT_ORDER,
             "order_seed": GC_OPT_ORDER_SEED}

    def set(self, name: str, value):
        if name == "mode" and isinstance(value, str):
            value = MODES[value]
        if name == "algorithm" and isinstance(value, str):
            value = ALGORITHMS[value]
        if name == "order" and isinstance(value, str):
            value = ORDERS[value]
        gc_set_option(self.h, self._OPTS[name], value)

    def get(self, option: int) -> int:
        return gc_get_option(self.h, option)

    def color(self, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        if out is None:
            out = torch.empty(max(self.n, 0), dtype=torch.int32, device=self.colidx.device)
        gc_color(self.h, out, stream)
        return out

    def stats(self):
        """(rounds, num_colors) of the last colouring; waits for it."""
        return gc_get_stats(self.h)

    def round_sizes(self):
        return gc_get_round_sizes(self.h)

    def profile(self, reset: bool = False):
        return gc_get_profile(self.h, reset)

    def close(self):
        if getattr(self, "h", None):
            gc_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def color(rowptr: torch.Tensor, colidx: torch.Tensor, **kw) -> torch.Tensor:
    """Colour one graph; returns the int32 colour tensor (synchronised)."""
    with Graph(rowptr, colidx, **{k: v for k, v in kw.items() if k in ("validate", "rows_sorted")}) as g:
        for k, v in kw.items():
            if k not in ("validate", "rows_sorted"):
                g.set(k, v)
        out = g.color()
        g.stats()
        return out


def color_batch(voff, eoff, rowptr_local, colidx_local, *, voff_host=None, eoff_host=None,
                stream=None):
    """Colour every graph of a packed batch in one launch (gc_color_batch).

    voff/eoff/rowptr_local/colidx_local are device tensors (int64, int64,
    int32, int32); voff_host/eoff_host (numpy) size the workspace and are
    copied from the device when not given.  Returns (colors, rounds) device
    tensors; the work is queued on `stream` (not synchronised)."""
    import numpy as np
    G = int(voff.numel()) - 1
    vh = np.asarray(voff_host if voff_host is not None else voff.cpu().numpy(), dtype=np.int64)
    eh = np.asarray(eoff_host if eoff_host is not None else eoff.cpu().numpy(), dtype=np.int64)
    nbytes = gc_batch_workspace_bytes(G, vh, eh)
    if nbytes == 0 and G > 0:
        raise GCError(GC_EINVAL, "gc_batch_workspace_bytes rejected the offsets")
    dev = colidx_local.device if colidx_local.numel() else rowptr_local.device
    ws = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=dev)
    colors = torch.empty(max(int(vh[-1]), 1), dtype=torch.int32, device=dev)
    rounds = torch.empty(max(G, 1), dtype=torch.int32, device=dev)
    gc_color_batch(G, voff, eoff, rowptr_local, colidx_local, colors, rounds, ws, nbytes, stream)
    return colors[: int(vh[-1])], rounds[:G]


DESC_DTYPE = None


def desc_array(rows):
    """numpy structured array of gc_graph_desc from (rowptr_off, colidx_off,
    color_off, n, rounds) tuples."""
    import numpy as np
    global DESC_DTYPE
    if DESC_DTYPE is None:
        DESC_DTYPE = np.dtype([("rowptr_off", "<i8"), ("colidx_off", "<i8"), ("color_off", "<i8"),
                               ("n", "<i4"), ("rounds", "<i4"), ("active", "<i4"),
                               ("max_degree", "<i4")])
        assert DESC_DTYPE.itemsize == ctypes.sizeof(gc_graph_desc)
    return np.array([(r[0], r[1], r[2], r[3], r[4] if len(r) > 4 else 0, 0, 0) for r in rows],
                    dtype=DESC_DTYPE)


def batch_step(descs_dev, rowptr_base, colidx_base, colors_base, max_rounds, *, workspace=None,
               stream=None):
    """Advance the graphs described by `descs_dev` (a uint8 device tensor
    holding gc_graph_desc records) by at most max_rounds rounds."""
    G = int(descs_dev.numel()) // ctypes.sizeof(gc_graph_desc)
    need = gc_batch_step_workspace_bytes(G, 0)
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=descs_dev.device)
    gc_batch_step(G, descs_dev, rowptr_base, colidx_base, colors_base, max_rounds, workspace,
                  int(workspace.numel()), stream)
    return workspace
