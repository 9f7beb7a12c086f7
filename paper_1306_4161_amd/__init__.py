"""Hierarchical SUMMA local update on one MI355X (gfx950).

The compute path lives in the HIP library ``libhsumma.so`` built from
``csrc/`` and declared in ``include/hsumma.h``; ``hsumma`` is its thin ctypes
binding (argument marshalling only).  Importing this package loads nothing;
the first call into ``hsumma`` loads the library and fails loudly if it is
missing.
"""
__all__ = ["hsumma", "inputs"]
