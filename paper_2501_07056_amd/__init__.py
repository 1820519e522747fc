"""gfx950 (MI355X) sparse matrix-matrix product C = A*B in CSR by Gustavson's
row-wise method with the intermediate products of long rows reordered into
LDS-sized column chunks (MAGNUS, ICS '25).  The computation runs in the HIP
library libmagnus.so; this package only marshals arguments."""
from .api import CATEGORY, Context, DeviceCSR, Plan, gpu_chunk_shift, paper_chunk_model  # noqa: F401
from ._lib import MagnusError, declared_symbols, load  # noqa: F401
