"""libpss: Parallel Space Saving (k-majority) on one MI355X.

The hot path is hand-written HIP for gfx950 behind the C-ABI declared in
``include/pss.h`` (``csrc/``, built into ``libpss.so`` by ``build.py``).
``binding`` is a thin ctypes layer with the same function names; importing
it loads the library and fails loudly when it has not been built.
"""
