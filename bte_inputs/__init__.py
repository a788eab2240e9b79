"""Seeded synthetic inputs for the phonon-BTE source-iteration solver.

This package is shared by the FP64 CPU oracle (``oracle/``) and by the HIP
library's Python binding. It holds input recipes only (geometry masks, boundary
tables, band tables, angular quadrature tables, heat sources, probe sets,
batch specifications) and none of the solver's arithmetic.
"""
from .generators import *  # noqa: F401,F403
