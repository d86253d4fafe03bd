"""MI355X-native inner loop of randomised-LMP preconditioned forcing-formulation
weak-constraint 4D-Var: a HIP library (libwc4d.so, C-ABI in include/wc4d.h) and
its thin Python binding."""
from . import wc4d  # noqa: F401
from .wc4d import (Lmp, Problem, SketchNet, Wc4dError, batch_solve, batch_solve_persistent,  # noqa: F401
                   corr_sqrt, gaussian_block, l96_trajectory, lib)
