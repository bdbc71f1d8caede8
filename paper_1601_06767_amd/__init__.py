"""MI355X-native band sum of the RPA polarizability chi0 (arXiv:1601.06767).

The compute lives in libgwchi0.so (HIP kernels for gfx950 behind the C ABI of
include/gwchi0.h).  ``_lib`` is the ctypes binding with the ABI's names;
``autograd`` wraps the differentiable entry points for torch.
"""
from . import _lib  # noqa: F401  (raises ImportError if the library was not built)
from ._lib import *  # noqa: F401,F403
