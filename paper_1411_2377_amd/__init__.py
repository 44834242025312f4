"""Multiple-precision CSR SpMV, transposed product and BiCG/GPBiCG on one MI355X.

The compute path is libmpspmv.so (hand-written HIP kernels for gfx950, C ABI in
include/mpspmv.h); this package is its binding.  Importing it fails when the library is not
built.
"""
from .api import *  # noqa: F401,F403
from .mparray import CSRMatrix, MPArray  # noqa: F401
from . import autograd  # noqa: F401,E402
