"""tyee for MI355X: leap-frog Maxwell stepping on unstructured triangular Yee-like meshes.

The solver lives in the native library libtyee.so (C ABI in include/tyee.h); this package
is its Python binding.  Importing it fails loudly when the library has not been built.
"""
from .tyee import (Mesh, Sim, Batch, Learner, TyeeError, ORDER, PREC, FIELD, EXPORTS, LIB_PATH,  # noqa: F401
                   copy_bandwidth, flip, Open, open_frame, pml, Tet, TetSim)

__all__ = ["Mesh", "Sim", "Batch", "Learner", "TyeeError", "ORDER", "PREC", "FIELD", "EXPORTS", "LIB_PATH",
           "copy_bandwidth", "flip", "Open", "open_frame", "pml", "Tet", "TetSim"]
