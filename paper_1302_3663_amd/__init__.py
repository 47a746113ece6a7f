"""MI355X-native immersed-boundary biofilm step (multigrid projection on a
staggered grid, delta spread/interpolation, springs) behind a C interface.

The numerical work runs in the HIP library ``libibmg.so`` built for gfx950;
this package only marshals arguments (``_lib``) and wraps a context
(``ibmg.Context``).  Importing it does not touch the GPU.
"""
from ._lib import (ABI_FUNCTIONS, IBB_AXIS_INOUT, IBB_AXIS_PERIODIC, IBB_AXIS_WALLS, IBB_FP32_REFINED, IBB_FP64,
                   IbbError, library_path, load)

__all__ = ["ABI_FUNCTIONS", "IBB_AXIS_INOUT", "IBB_AXIS_PERIODIC", "IBB_AXIS_WALLS", "IBB_FP32_REFINED", "IBB_FP64",
           "IbbError", "library_path", "load"]
