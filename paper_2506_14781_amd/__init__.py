"""Two-dimensional parallel tempering on MI355X (gfx950).

The sampling path is the HIP library libtdpt.so behind the C ABI in
include/tdpt.h; `tdpt` is its Python binding.
"""
from .tdpt import (NO_PSWAP, Batch, Instance, Problem, RunConfig, TdptError, load_library,
                   workspace_bytes)

__all__ = ["Instance", "Problem", "RunConfig", "Batch", "TdptError", "NO_PSWAP", "load_library",
           "workspace_bytes"]
