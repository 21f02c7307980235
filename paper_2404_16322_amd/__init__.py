"""MI355X (gfx950) library for PCA-based, data-driven, incrementally pruned distance
comparison inside IVF nearest-neighbour search.

The compute path is the HIP library ``libddc.so`` (C ABI in ``include/ddc.h``); this
package only marshals arguments to it.  Importing the package does not load the
library; the first call does, and raises if it has not been built.
"""
from .binding import (CORR, DTYPE, PROJ, ROT, CALIB, DdcError, Index, Server, lib_path,  # noqa: F401
                      load_library)

__all__ = ["Index", "Server", "DdcError", "CORR", "DTYPE", "PROJ", "ROT", "CALIB", "lib_path", "load_library"]
