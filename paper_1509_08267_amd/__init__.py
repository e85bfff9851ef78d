"""MI355X-native round-synchronous speculative graph colouring.

The colouring runs in hand-written gfx950 HIP kernels behind the C ABI of
``libgc.so`` (``include/gc.h``); ``gc`` is its thin ctypes binding.  Import
``paper_1509_08267_amd.gc`` to use it (importing this package alone loads
nothing)."""

__all__ = ["gc"]
