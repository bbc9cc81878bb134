"""MI355X-native fast multipole periodic BEM (arXiv 2201.12050): Python binding.

The operator and the solver live in the HIP library ``libfmbem.so`` (C ABI in
``include/fmbem.h``); this package only marshals arguments.  Build the
library with ``python -m paper_2201_12050_amd.build``.
"""
from ._lib import (Plan, FmbemError, load, LIB_PATH, EXPORTS, FP64, FP32, STATUS, solve_batch, Engine, Solver,
                   insertion_loss)

__all__ = ["Plan", "FmbemError", "load", "LIB_PATH", "EXPORTS", "FP64", "FP32", "STATUS", "solve_batch", "Engine",
           "Solver", "insertion_loss"]
