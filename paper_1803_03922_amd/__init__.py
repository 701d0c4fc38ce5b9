"""Degree-separated direction-optimized BFS for MI355X (gfx950).

The compute path is the HIP library ``libdsbfs.so`` (sources in ``csrc/``,
C-ABI in ``include/dsbfs.h``); ``dsbfs`` is its thin ctypes binding. Import
of this package is lazy: nothing is loaded until ``dsbfs`` is used.
"""
