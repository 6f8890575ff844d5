"""Plain FP64 CPU oracle for the DGSEM compressible-Euler right-hand side.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py``; never by the product package.  The C source
(``orc.c``) shares no code with the HIP library.
"""
from .orc import *  # noqa: F401,F403
