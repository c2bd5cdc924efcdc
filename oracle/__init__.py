"""FP64 CPU oracle for entropic partial optimal transport.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  It shares no code
with the HIP solver library, and the solver never calls it.
"""
from .potref import *  # noqa: F401,F403
