"""MI355X block-sparse PINVIT: Python binding of the HIP library (libpinvit.so).

The compute path lives entirely in the HIP/C++ library; this package only marshals
arguments (``native``) and builds the library (``build``).
"""
from .native import Context, PvError, mpo_bond_dims, mpo_dense  # noqa: F401
