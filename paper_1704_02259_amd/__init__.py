"""hybfs: hybrid (direction-optimising) breadth-first search for MI355X.

The traversal runs in hand-written gfx950 HIP kernels behind the C ABI of
libhybfs.so (include/hybfs.h); this package only binds it.
"""
from .hybfs import *  # noqa: F401,F403
from .hybfs import Graph, HybfsError, load  # noqa: F401
