"""MI355X (gfx950) asynchronous discontinuous Galerkin right-hand side with
asynchrony-tolerant neighbour traces (arXiv 2603.28710), behind the C ABI of
include/adg.h. `binding` is the ctypes layer (same names as the C ABI);
`solver.Solver` holds a context and its torch-allocated device buffers.
"""
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libadg.so")
INCLUDE = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
