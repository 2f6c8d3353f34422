"""MI355X (gfx950) implementation of the L-ACE exact-exchange hot path
(Carnimeo, Baroni, Giannozzi, arXiv:1801.09263).

The compute path is the HIP library ``liblace.so`` behind the C ABI of
``include/lace.h``; ``lace`` is its ctypes binding and ``session`` keeps the
device buffers of one cell together.
"""
from . import lace  # noqa: F401
