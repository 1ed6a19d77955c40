"""sqh -- segmented QuickHull for planar point sets on AMD MI355X (gfx950).

The compute path is the C-ABI library ``libsqh.so`` built from ``csrc/``
(hand-written HIP); ``sqh`` is its thin ctypes binding and ``workloads``
holds the seeded input generators. Importing this package loads nothing
native; ``sqh.load()`` does, and fails loudly if the library is missing.
"""
__all__ = ["workloads", "sqh"]
