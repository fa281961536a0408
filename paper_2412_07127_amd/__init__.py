"""IC(0)-preconditioned conjugate gradients on MI355X (gfx950).

The numerical work runs in the HIP library libicpcg.so (C ABI in
include/icpcg.h); this package is its thin Python binding. torch supplies
device memory and the stream. Importing the package does not touch the GPU;
the library is loaded when a Context is created and its absence is an error.
"""

from ._lib import LIB_PATH, declared_symbols, load  # noqa: F401
from .solver import CSR, Context, IcpcgError, Matrix, Preconditioner  # noqa: F401
from .autograd import PrecApply, prec_apply  # noqa: F401
from . import gnn  # noqa: F401

__all__ = ["CSR", "Context", "Matrix", "Preconditioner", "IcpcgError", "PrecApply", "prec_apply", "load",
           "declared_symbols", "LIB_PATH", "gnn"]
