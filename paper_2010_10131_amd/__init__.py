"""MI355X (gfx950) st-HOSVD: matricization-free Gram / TTM / TTT kernels, an
FP64 eigensolver and the mode-wise EIG/ALS driver of Alg. 2, behind the C ABI
declared in include/sthosvd.h.  ``api`` is the thin Python binding."""
from ._lib import SthError, load  # noqa: F401

__version__ = "0.1.0"
