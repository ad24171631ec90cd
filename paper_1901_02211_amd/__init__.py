"""Overlap topological charge density by symmetric multi-probing on AMD MI355X.

Thin ctypes binding of libsmpq.so (declared in include/smpq.h): every function has
the name of the C entry point it marshals arguments for; all computation runs in
the library's HIP kernels.  Importing this package fails when the library has not
been built (``python paper_1901_02211_amd/build.py``).
"""
from .binding import *  # noqa: F401,F403
from .binding import __all__  # noqa: F401
