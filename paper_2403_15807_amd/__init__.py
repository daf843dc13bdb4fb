"""Filtered exact top-k vector search on MI355X (gfx950).

The scan-based access path for mixed vector-relational search of Sanca &
Ailamaki (Section 3): a relational predicate over int32 columns, distances
between a batch of queries and the qualifying vectors, and each query's
exact top-k -- behind the C ABI of ``include/vrs.h`` (``libvrs.so``), with
``vrs.py`` as its ctypes binding.

Importing the package loads nothing; ``paper_2403_15807_amd.vrs`` loads the
library on first use.
"""

__all__ = ["vrs", "inputs"]
