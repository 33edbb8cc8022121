"""MI355X-native relational operators as tensor programs (exact and relaxed),
after "The Tensor Data Platform" (arXiv 2211.02753).

The compute path is libtdp.so (hand-written HIP kernels for gfx950, C ABI in
include/tdp.h); this package only marshals arguments to it.
"""
from . import _lib  # noqa: F401
from ._lib import load as load_library  # noqa: F401
