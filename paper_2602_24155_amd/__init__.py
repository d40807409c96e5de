"""Controlled reduction for hypersurface zeta functions on MI355X (gfx950).

The compute lives in the C-ABI library ``libcrfrob.so`` (host C++ setup and
HIP kernels); ``crfrob`` is the thin ctypes binding with the same names as
``include/crfrob.h``.  ``workload`` produces seeded synthetic inputs.
"""
