"""C-ABI checks that need no GPU: the library loads, exports every symbol
the header declares, and rejects bad arguments before touching a device."""
import ctypes
import os
import re

import pytest

from conftest import ROOT

HEADER = os.path.join(ROOT, "include", "gc.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(gc_[a-z_]+)\s*\(", text)
    return sorted(set(names))


@pytest.fixture(scope="module")
def gc():
    from paper_1509_08267_amd import gc as gcmod
    if not os.path.exists(gcmod.LIB_PATH):
        from paper_1509_08267_amd import build
        build.build()
    gcmod.load()
    return gcmod


def test_header_declares_the_boundary():
    names = _declared_functions()
    for must in ("gc_create", "gc_color", "gc_color_batch", "gc_get_stats", "gc_destroy",
                 "gc_last_error", "gc_batch_workspace_bytes"):
        assert must in names


def test_library_exports_every_declared_symbol(gc):
    lib = gc.load()
    names = _declared_functions()
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert sorted(gc.EXPORTS) == names


def test_one_hip_runtime_in_process(gc):
    # libgc must bind to the HIP runtime torch loaded, not a second copy
    maps = open("/proc/self/maps").read()
    paths = {line.split()[-1] for line in maps.splitlines() if "libamdhip64" in line}
    assert len(paths) <= 1, paths


def test_version(gc):
    assert re.match(r"^\d+\.\d+\.\d+$", gc.gc_version())


def _create(gc, rowptr, colidx, n, m, flags):
    lib = gc.load()
    h = ctypes.c_void_p(123)
    rc = lib.gc_create(ctypes.byref(h), rowptr, colidx, n, m, flags, None)
    return rc, h.value


def test_create_rejects_bad_arguments_on_host(gc):
    lib = gc.load()
    assert lib.gc_create(None, 1, 1, 1, 0, 0, None) == gc.GC_EINVAL
    rc, h = _create(gc, 8, 8, -1, 0, 0)
    assert rc == gc.GC_EINVAL and h is None
    assert "negative" in gc.gc_last_error()
    rc, _ = _create(gc, 8, 8, 4, -5, 0)
    assert rc == gc.GC_EINVAL
    rc, _ = _create(gc, 8, 8, 1 << 31, 0, 0)
    assert rc == gc.GC_ETOOBIG
    rc, _ = _create(gc, 8, 8, 10, 1 << 31, 0)      # needs int64 rowptr
    assert rc == gc.GC_ETOOBIG
    rc, _ = _create(gc, 8, 8, 10, 10, 1 << 7)      # unknown flag
    assert rc == gc.GC_EINVAL and "flag" in gc.gc_last_error()
    rc, _ = _create(gc, None, 8, 10, 10, 0)        # NULL rowptr
    assert rc == gc.GC_EINVAL
    rc, _ = _create(gc, 8, None, 10, 10, 0)        # NULL colidx with m > 0
    assert rc == gc.GC_EINVAL


def test_calls_on_null_handle(gc):
    lib = gc.load()
    assert lib.gc_color(None, 8, None) == gc.GC_EINVAL
    r, k = ctypes.c_int64(), ctypes.c_int32()
    assert lib.gc_get_stats(None, ctypes.byref(r), ctypes.byref(k)) == gc.GC_EINVAL
    assert lib.gc_set_option(None, gc.GC_OPT_MODE, 1) == gc.GC_EINVAL
    assert lib.gc_destroy(None) == gc.GC_OK
    assert "NULL" in gc.gc_last_error()


def test_batch_sizing_rejects_bad_offsets(gc):
    import numpy as np
    assert gc.gc_batch_workspace_bytes(-1, np.zeros(1, np.int64), np.zeros(1, np.int64)) == 0
    bad = np.array([0, 5, 3], np.int64)   # decreasing vertex offsets
    assert gc.gc_batch_workspace_bytes(2, bad, np.array([0, 2, 4], np.int64)) == 0
