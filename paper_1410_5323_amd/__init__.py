"""MI355X (gfx950) propagation of charged nuclei through gridded turbulent fields.

The computation lives in libcrp.so (HIP kernels behind the C ABI of
include/crp.h); ``crp`` is its ctypes binding.
"""
from . import crp  # noqa: F401

__all__ = ["crp"]
