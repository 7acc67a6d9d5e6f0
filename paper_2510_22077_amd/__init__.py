"""MI355X gPLMM Newton-Krylov solver for Navier-Stokes flow in porous voxel images.

The solver itself is the HIP library ``libgplmm.so`` (C ABI in
``include/gplmm.h``); this package only binds it (``binding.Solver``) and builds
it (``build.build``).
"""
from .binding import Solver, BatchSolver, Mlp, GplmmError, load, EXPORTS, LIB_PATH

__all__ = ["Solver", "BatchSolver", "Mlp", "GplmmError", "load", "EXPORTS", "LIB_PATH"]
