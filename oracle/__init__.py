"""CPU FP64 oracle for the L-ACE exchange path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
link this package: it exists so that ``tests/``, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py`` can check and time the GPU library
against a plain, slow, obviously correct implementation written from the
paper.  It shares no code with the HIP library.
"""
from .lace_oracle import *  # noqa: F401,F403
