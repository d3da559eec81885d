"""MI355X (gfx950) SFFT image subtraction: HIP kernels behind a C ABI.

The compute path is libsfft.so (built from csrc/ by build.py); ``binding``
exposes its C entry points to Python.
"""
from . import binding  # noqa: F401
from .binding import Plan, SFFT_MODE_F32C, SFFT_MODE_F64  # noqa: F401
