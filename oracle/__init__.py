"""CPU oracle of the oblique-projection FEAST method -- test infrastructure only.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product path never does.
"""
from . import gfeast  # noqa: F401
