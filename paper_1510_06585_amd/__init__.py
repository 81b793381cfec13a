"""MI355X (gfx950) skeleton library: Map / Pipeline / MapReduce / Loop over
device buffers, fused into hand-written HIP kernels behind a C-ABI
(``include/skel.h``).  This package is the thin Python binding."""
from .skel import *  # noqa: F401,F403
from .skel import lib, Plan, Node, SkelError  # noqa: F401
