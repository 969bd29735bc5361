"""MI355X (gfx950) implementation of the semi-implicit step of the 4D
generalized subjective-surface segmentation (arXiv 2111.11866).

The compute path is libsubsurf4d.so (hand-written HIP, C ABI in
include/subsurf4d.h); ``binding`` is its ctypes wrapper.
"""
from paper_2111_11866_amd import binding  # noqa: F401
