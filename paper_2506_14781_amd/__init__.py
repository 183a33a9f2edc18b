"""Two-dimensional parallel tempering on MI355X (gfx950).

The sampling path is the HIP library libtdpt.so behind the C ABI in
include/tdpt.h; `tdpt` is its Python binding.
"""
from .tdpt import (E_BUSY, E_DEVICE, E_INVALID, E_NOMEM, E_RANGE, E_STATE, NO_PSWAP, OK, Batch, Instance,
                   Problem, RunConfig, TdptError, load_library, workspace_bytes)

__all__ = ["Instance", "Problem", "RunConfig", "Batch", "TdptError", "NO_PSWAP", "load_library",
           "workspace_bytes", "OK", "E_INVALID", "E_RANGE", "E_NOMEM", "E_DEVICE", "E_STATE", "E_BUSY"]
