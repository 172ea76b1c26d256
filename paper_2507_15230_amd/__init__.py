"""MI355X localized-relation builder (VT / VV / TT blocks per vertex cluster).

The computation lives in ``libgale.so`` (HIP kernels for gfx950 behind the C
ABI of ``include/gale.h``); ``gale`` is its ctypes binding.
"""
from .gale import (REL_ALL, REL_TT, REL_VT, REL_VV, Context, GaleError, load_library)  # noqa: F401

__all__ = ["Context", "GaleError", "load_library", "REL_VT", "REL_VV", "REL_TT", "REL_ALL"]
