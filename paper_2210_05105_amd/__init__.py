"""Randomized sparse CP-ALS on MI355X (gfx950): Python binding of libcpr.

The work is done by the HIP library `libcpr.so` (C ABI in include/cpr.h);
this package only marshals arguments.  PyTorch supplies device memory and
the HIP stream.  There is no CPU fallback: if the library is missing the
import of `Context` fails.
"""
from .binding import (Batch, CprError, Context, load_library, PHASES, SAMPLERS,
                      PRECISIONS, declared_symbols, pinv, pinv_noalloc)

__all__ = ["Batch", "CprError", "Context", "load_library", "PHASES", "SAMPLERS",
           "PRECISIONS", "declared_symbols", "pinv", "pinv_noalloc"]
