"""IFGF-accelerated apply of the 3-D Helmholtz combined-field operator on
MI355X (gfx950).

The compute path is the HIP library `libifgf.so` (C ABI in include/ifgf.h);
this package only marshals arguments to it.  Importing the package does not
load the library; `Plan` loads it on first use and raises if it is missing.
"""
from .api import Batch, IFGFApply, Plan, library_path, load_library  # noqa: F401

__all__ = ["Plan", "Batch", "IFGFApply", "load_library", "library_path"]
