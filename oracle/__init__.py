"""CPU oracle for the dual-layer lossless Radiance encoder.

TEST INFRASTRUCTURE ONLY.  Imported by ``tests/``, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py``; never by the product package.
"""
from . import oracle  # noqa: F401
