"""MI355X (gfx950) hot path of the phase-averaged bubbly-flow solver.

Thin Python binding of ``libbubbly.so`` (C ABI in ``include/bubbly.h``).  It
only marshals arguments: every step of the path runs in the HIP kernels of
the library.  PyTorch provides device memory and streams.

The library is built in-tree by ``python -m paper_2511_21031_amd.build``;
importing the binding without it raises ``ImportError`` (there is no CPU
fallback).
"""
from __future__ import annotations

from ._binding import (BubblyError, Batch, Context, lib, library_path, BC_PERIODIC, BC_REFLECTIVE,
                       PREC_FP64, PREC_MIXED, BUBBLES_UNSPLIT, BUBBLES_SPLIT, CONTENTS_POLYTROPIC,
                       CONTENTS_TRANSFER, context_from_case, ctx_buffer_bytes)

__all__ = ["BubblyError", "Batch", "Context", "lib", "library_path", "context_from_case", "BC_PERIODIC",
           "BC_REFLECTIVE", "PREC_FP64", "PREC_MIXED", "BUBBLES_UNSPLIT", "BUBBLES_SPLIT",
           "CONTENTS_POLYTROPIC", "CONTENTS_TRANSFER", "ctx_buffer_bytes"]
