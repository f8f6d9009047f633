"""MI355X (gfx950) hot path of the POD-augmented conjugate-gradient method.

The work happens in libpodcg.so (HIP kernels behind the C ABI of
include/podcg.h).  This package only loads it and marshals torch tensors.
If the library has not been built, using it raises: there is no CPU fallback.
"""

from ._lib import LIB_PATH, load
from .solver import PodCG, PodCGBatch, PodCGError

__all__ = ["PodCG", "PodCGBatch", "PodCGError", "LIB_PATH", "load"]
