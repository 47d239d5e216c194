"""MI355X (gfx950) HIP implementation of the entropy-stable SBP-SAT residual of the compressible
Navier-Stokes equations (Rojas et al., arXiv 1911.10966): C-ABI library ``libsbp_hip.so`` plus a
thin ctypes binding.  The library must be built (``python -m paper_1911_10966_amd.build``); there is
no CPU fallback."""
from .api import (Problem, ProblemSet, SBPResidual, lgl_operator, metrics,
                  metrics_optimized, profile_collect,  # noqa: F401
                  schedule_count)
from ._lib import LIB_PATH, SBPError, lib  # noqa: F401
