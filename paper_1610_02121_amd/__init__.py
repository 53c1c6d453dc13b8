"""MI355X (gfx950) Chebyshev-filtered subspace iteration for the enriched
spectral finite-element Kohn-Sham problem.

The compute path is the HIP library `libchebfilter.so` (C ABI in
include/chebfilter.h); this package only binds it.  Importing the binding
never falls back to any other implementation: if the library is missing,
`load_library()` raises.
"""
from .binding import (Batch, ChebFilterError, Context, Mlp, empty_block, fermi_level,  # noqa: F401
                      load_library)

__all__ = ["Batch", "Context", "ChebFilterError", "Mlp", "empty_block", "fermi_level", "load_library"]
