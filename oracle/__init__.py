"""CPU FP64 oracle of SuperSCS (arXiv 1903.06477).

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow reference that the
GPU library is checked against.  Only the test-suite, the smoke check and the
CPU-baseline leg of the benchmark may import it; the product path never does.
It shares no code with the GPU library.  Every function cites the passage of
the paper it follows; see each module's docstring.
"""
from .cones import (proj_zero_dual, proj_nonneg, proj_soc, proj_psd, proj_exp,
                    proj_exp_dual, proj_dual_cone, proj_C, svec, smat)
from .linsys import DirectLinSys
from .superscs import Settings, solve, solve_scs, residual, termination, RestartedBroyden, Anderson

__all__ = [
    "proj_zero_dual", "proj_nonneg", "proj_soc", "proj_psd", "proj_exp", "proj_exp_dual",
    "proj_dual_cone", "proj_C", "svec", "smat", "DirectLinSys", "Settings", "solve",
    "residual", "termination", "RestartedBroyden", "Anderson", "solve_scs",
]
