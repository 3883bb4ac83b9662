"""lMBD on AMD Instinct MI355X: atom-wise many-body dispersion energies and forces.

The hot path lives in the HIP library ``liblmbd.so`` (C ABI: include/lmbd.h);
this package only marshals arguments.  Build the library with
``python -m paper_2407_06409_amd.build``.
"""
from .api import (MethodParams, Context, Server, compute, compute_batch, estimate_footprint, LMBDEnergy,
                  default_context, release_default_context)
from ._lib import LmbdError, lib as load_library, LIB_PATH

__all__ = ["MethodParams", "Context", "Server", "compute", "compute_batch", "estimate_footprint", "LMBDEnergy",
           "default_context", "release_default_context", "LmbdError", "load_library", "LIB_PATH"]
