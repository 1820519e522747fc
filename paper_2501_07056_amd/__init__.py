"""gfx950 (MI355X) sparse matrix-matrix product C = A*B in CSR by Gustavson's
row-wise method with the intermediate products of long rows reordered into
LDS-sized column chunks (MAGNUS, ICS '25).  The computation runs in the HIP
library libmagnus.so; this package only marshals arguments."""
from .api import (CATEGORY, BatchPlan, Context, DeviceCSR, Plan, Server,  # noqa: F401
                  gpu_chunk_shift, paper_chunk_model)
from ._lib import MagnusError, declared_symbols, load  # noqa: F401
